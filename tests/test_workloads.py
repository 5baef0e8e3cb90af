"""The synthetic workloads follow the shapes the paper states."""
import json
import math
import os

import numpy as np

from synth.scenes import MULTI_AGENT_SIZES, multi_agent, room_plain, small_plain

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def test_replica_frame_intrinsics():
    """1200x680 frames with a 90 degree HFOV give f = W/2 = 600."""
    W = GOLD["frame_width"]["value"]
    H = GOLD["frame_height"]["value"]
    f = (W / 2) / math.tan(math.radians(GOLD["hfov_deg"]["value"] / 2))
    wl = room_plain(n=1000)
    assert (wl.views.width, wl.views.height) == (W, H)
    np.testing.assert_allclose(wl.views.intrinsics[0], [f, f, W / 2, H / 2], rtol=1e-6)


def test_small_workload_draws():
    wl = small_plain(0)
    sc = wl.scene
    assert sc.n == 2000 and sc.means.dtype == np.float32
    assert np.all(np.abs(sc.means[:, :2]) <= 1) and np.all((sc.means[:, 2] >= 2) & (sc.means[:, 2] <= 4))
    np.testing.assert_allclose(np.linalg.norm(sc.quats, axis=1), 1, rtol=1e-6)
    assert abs(sc.log_scales.mean() + 3) < 0.05 and abs(sc.log_scales.std() - 0.5) < 0.05
    np.testing.assert_allclose(wl.views.intrinsics[0], [100, 100, 64, 48])


def test_multi_agent_structure():
    wl = multi_agent(scale=0.01)
    sizes = np.diff(wl.scene.set_offsets)
    np.testing.assert_array_equal(sizes, [round(s * 0.01) for s in MULTI_AGENT_SIZES])
    assert wl.views.n == 48 and list(np.bincount(wl.views.view_set)) == [8] * 6
    R = wl.views.viewmats[:, :, :3].astype(np.float64)
    np.testing.assert_allclose(R @ np.swapaxes(R, 1, 2), np.broadcast_to(np.eye(3), R.shape), atol=1e-6)
    centers = -np.einsum("vji,vj->vi", R, wl.views.viewmats[:, :, 3])
    np.testing.assert_allclose(np.hypot(centers[:, 0], centers[:, 2]), 1.5, rtol=1e-5)
