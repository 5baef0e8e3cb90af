"""GPU parity of the occupancy-aware deduplication (Eqs. (envelope),
(free_carve), (dedup)) against the oracle, through the C ABI."""
import numpy as np
import pytest

from gpu_harness import announce
from oracle.dedup import dedup, free, occupied, voxel_of
from synth.scenes import look_at, pinhole

pytestmark = pytest.mark.gpu


def _case(seed):
    rng = np.random.default_rng(seed)
    n_t, n_s = 1500, 2500
    tm = rng.uniform(-1.5, 1.5, (n_t, 3)).astype(np.float32)
    tls = rng.normal(-3.2, 0.5, (n_t, 3)).astype(np.float32)
    sm = rng.uniform(-1.6, 1.6, (n_s, 3)).astype(np.float32)
    sm[:300] = tm[:300] + rng.normal(0, 0.01, (300, 3)).astype(np.float32)  # duplicates
    vms, intr = [], []
    for k in range(2):
        c = np.array([2.2 * np.cos(1.3 * k + 0.4), 0.1 * k, 2.2 * np.sin(1.3 * k + 0.4)])
        vms.append(look_at(c, (0.0, 0.0, 0.0), 0.0))
        intr.append(pinhole(40, 30, 20.0))
    depth = (0.8 + 2.5 * rng.random((2, 30, 40))).astype(np.float32)
    depth[0, :3, :5] = 0.0  # holes carve nothing
    return tm, tls, sm, np.array(vms, np.float32), np.array(intr, np.float32), depth


def test_dedup_matches_oracle():
    announce("dedup")
    import torch
    from paper_2605_10760_amd import dedup as gpu_dedup
    tm, tls, sm, vms, intr, depth = _case(3)
    v, k = 0.05, 1.0
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    keep, nvox = gpu_dedup(t(sm), t(tm), t(tls), t(depth), t(vms), t(intr), v, k)
    ref, n_amb = dedup(sm, tm, tls, depth, vms, intr, v, k)
    assert n_amb == 0
    # no box bound sits within 1e-9 of a voxel plane (where FP64 exp may differ
    # by an ulp between libraries), so every decision is exact
    s = np.exp(tls.astype(np.float64))
    for x in ((tm - k * s) / v, (tm + k * s) / v, sm.astype(np.float64) / v):
        assert np.min(np.abs(x - np.round(x))) > 1e-9
    np.testing.assert_array_equal(keep.cpu().numpy().astype(bool), ref)
    occ = occupied(tm, tls, v, k)
    fr, _ = free(depth, vms, intr, v)
    assert nvox == len(occ | fr)
    assert 0 < ref.sum() < ref.shape[0] and not ref[:300].any()


def test_dedup_overflow_reported():
    """A hash set too small for the target's voxels reports GSR_E_OVERFLOW."""
    announce("dedup overflow")
    import torch
    from paper_2605_10760_amd import GsrError, dedup as gpu_dedup
    tm, tls, sm, _, _, _ = _case(4)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    with pytest.raises(GsrError):
        gpu_dedup(t(sm), t(tm), t(tls), None, None, None, 0.05, 1.0, table_slots=1 << 10)


def test_dedup_table_grows_on_overflow():
    """The binding's default hash set starts from the input counts; one large
    box (about 21^3 voxels) overflows it, and the call grows the set and
    still matches the oracle."""
    announce("dedup table growth")
    import torch
    from paper_2605_10760_amd import dedup as gpu_dedup
    rng = np.random.default_rng(9)
    tm = np.array([[0.013, -0.021, 0.007]], np.float32)
    tls = np.full((1, 3), np.log(0.5), np.float32)
    sm = rng.uniform(-0.7, 0.7, (3000, 3)).astype(np.float32)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    keep, nvox = gpu_dedup(t(sm), t(tm), t(tls), None, None, None, 0.05, 1.0)
    occ = occupied(tm, tls, 0.05, 1.0)
    assert nvox == len(occ) > 4096
    ref = np.array([tuple(q) not in occ for q in voxel_of(sm, 0.05)])
    np.testing.assert_array_equal(keep.cpu().numpy().astype(bool), ref)


def _slab_hits(c, r, lo, hi, margin):
    """Segments c + t (r - c), t in [0, 1], that pass within `margin` of the
    box [lo, hi] (a conservative prefilter: the oracle's walk decides)."""
    d = r - c
    with np.errstate(divide="ignore", invalid="ignore"):
        t0 = (lo - margin - c) / d
        t1 = (hi + margin - c) / d
    tmin = np.where(d == 0, -np.inf, np.minimum(t0, t1))
    tmax = np.where(d == 0, np.inf, np.maximum(t0, t1))
    inside = np.all((d != 0) | ((c >= lo - margin) & (c <= hi + margin)), axis=-1)
    a = np.max(tmin, axis=-1)
    b = np.min(tmax, axis=-1)
    return inside & (a <= b) & (b >= -1e-9) & (a <= 1.0 + 1e-9)


def test_dedup_full_size_sampled():
    """A keyframe-sized case: 300k target Gaussians in the part of the room
    with x < 0.5 m, 200k borrowed Gaussians uniform in the room, eight
    640 x 480 keyframe depth maps (slanted planes, holes) from cameras on a
    circle around the room.  Sampled borrowed Gaussians, kept and dropped,
    against the oracle's definition: the target boxes and keyframe segments
    that could meet the Gaussian's voxel are preselected with a margin, and
    the oracle's box rule and segment walk decide."""
    announce("dedup full size 300k / 200k / 8 x 640x480")
    import torch
    from oracle.dedup import occupied, ray_ends, segment_voxels
    from paper_2605_10760_amd import dedup as gpu_dedup
    from synth.scenes import slanted_depth
    rng = np.random.default_rng(21)
    v, k = 0.05, 1.0
    lo_room, hi_room = np.array([-3.0, -1.5, -2.0]), np.array([3.0, 1.5, 2.0])
    tm = rng.uniform(lo_room, [0.5, 1.5, 2.0], (300_000, 3)).astype(np.float32)
    tls = rng.normal(-3.6, 0.4, (300_000, 3)).astype(np.float32)
    sm = rng.uniform(lo_room, hi_room, (200_000, 3)).astype(np.float32)
    K, H, W = 8, 480, 640
    depth, _, intr = slanted_depth(rng, K, W, H, f=320.0, hole_frac=0.02)
    depth = (0.6 * depth).astype(np.float32)
    vms = []
    for kf in range(K):
        th = 2 * np.pi * kf / K + 0.3
        c = np.array([2.6 * np.cos(th), 0.2 * np.sin(3 * th), 1.8 * np.sin(th)])
        vms.append(look_at(c, (0.0, 0.0, 0.0), 0.1 * np.sin(kf)))
    vms = np.array(vms, np.float32)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    keep, nvox = gpu_dedup(t(sm), t(tm), t(tls), t(depth), t(vms), t(intr.astype(np.float32)), v, k)
    keep = keep.cpu().numpy().astype(bool)
    assert 0.05 * keep.size < keep.sum() < 0.95 * keep.size
    ends = [ray_ends(depth[kf], vms[kf], intr[kf]) for kf in range(K)]
    s_t = np.exp(tls.astype(np.float64))
    m_t = tm.astype(np.float64)
    pick = np.concatenate([rng.choice(np.nonzero(keep)[0], 40, replace=False),
                           rng.choice(np.nonzero(~keep)[0], 40, replace=False)])
    for i in pick:
        q = np.floor(sm[i].astype(np.float64) / v).astype(np.int64)
        lo, hi = q * v, (q + 1) * v
        # target Gaussians whose box may reach the voxel
        near = np.all((m_t + k * s_t >= lo - 1e-6) & (m_t - k * s_t <= hi + 1e-6), axis=1)
        in_occ = tuple(q) in occupied(tm[near], tls[near], v, k) if near.any() else False
        in_free = False
        if not in_occ:
            for c, r, ok in ends:
                cand = np.nonzero(ok & _slab_hits(c, r, lo, hi, 1e-6))
                for j, ii in zip(*cand):
                    vox, amb = segment_voxels(c, r[j, ii], v)
                    assert not amb
                    if tuple(q) in vox:
                        in_free = True
                        break
                if in_free:
                    break
        assert keep[i] == (not in_occ and not in_free), (int(i), in_occ, in_free)
