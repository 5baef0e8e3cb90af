"""Pins of the oracle's occupancy-aware deduplication (Eqs. (envelope),
(free_carve), (dedup)): box/voxel overlap by brute force, segments against
dense sampling and a closed-form ray, and constructed keep/drop cases."""
import numpy as np

from oracle.dedup import dedup, free, occupied, segment_voxels, voxel_of

V = 0.05


def test_occupied_is_box_voxel_overlap():
    rng = np.random.default_rng(0)
    m = rng.normal(0, 0.3, (20, 3))
    ls = rng.normal(-3.0, 0.6, (20, 3))
    occ = occupied(m, ls, V, 1.5)
    s = np.exp(ls)
    lo, hi = m - 1.5 * s, m + 1.5 * s
    want = set()
    for a, b in zip(lo, hi):
        base = np.floor(a / V).astype(int) - 2
        top = np.floor(b / V).astype(int) + 2
        for x in range(base[0], top[0] + 1):
            for y in range(base[1], top[1] + 1):
                for z in range(base[2], top[2] + 1):
                    vlo = np.array([x, y, z]) * V
                    # voxel [vlo, vlo + V) meets the closed box [a, b]
                    if np.all(vlo <= b) and np.all(vlo + V > a):
                        want.add((x, y, z))
    assert occ == want


def _slab_length(c, r, vox):
    """Length of the segment c->r inside voxel vox (slab method)."""
    d = r - c
    t0, t1 = 0.0, 1.0
    lo = np.array(vox) * V
    for ax in range(3):
        if d[ax] == 0:
            if not lo[ax] <= c[ax] < lo[ax] + V:
                return 0.0
            continue
        a = (lo[ax] - c[ax]) / d[ax]
        b = (lo[ax] + V - c[ax]) / d[ax]
        t0, t1 = max(t0, min(a, b)), min(t1, max(a, b))
    return max(0.0, t1 - t0) * np.linalg.norm(d)


def test_segment_against_dense_sampling():
    rng = np.random.default_rng(1)
    for _ in range(40):
        c = rng.normal(0, 0.3, 3)
        r = c + rng.normal(0, 0.4, 3)
        exact, amb = segment_voxels(c, r, V)
        assert not amb
        t = np.arange(200000) / 200000.0
        pts = c[None] + t[:, None] * (r - c)[None]
        sampled = set(map(tuple, voxel_of(pts, V)))
        assert sampled <= exact
        for vox in exact - sampled:
            assert _slab_length(c, r, vox) < 1e-5


def test_axis_ray_closed_form():
    # camera at the origin looking down +z; the centre pixel's ray is the z axis
    vm = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0]], np.float64)
    intr = np.array([100.0, 100.0, 0.5, 0.5])  # pixel (0, 0) centre -> (0, 0, 1)
    fr, amb = free(np.full((1, 1, 1), 0.26), vm[None], intr[None], V)
    assert amb == 0
    assert fr == {(0, 0, z) for z in range(6)}
    # no depth, no carving
    fr, _ = free(np.zeros((1, 1, 1)), vm[None], intr[None], V)
    assert fr == set()


def test_dedup_constructed_cases():
    vm = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0]], np.float64)
    intr = np.array([100.0, 100.0, 0.5, 0.5])
    depth = np.full((1, 1, 1), 0.26)
    tgt = np.array([[1.0, 1.0, 1.0]])
    tls = np.log(np.array([[0.01, 0.01, 0.01]]))
    src = np.array([[1.003, 1.004, 1.002],   # occupied voxel (20, 20, 20)
                    [0.01, 0.02, 0.12],      # carved voxel (0, 0, 2)
                    [0.5, 0.5, 0.5],         # untouched
                    [0.01, 0.02, 0.31]])     # past the depth: voxel (0, 0, 6)
    keep, amb = dedup(src, tgt, tls, depth, vm[None], intr[None], V, 1.0)
    assert amb == 0
    np.testing.assert_array_equal(keep, [False, False, True, True])


def test_start_on_a_plane_moving_down():
    """t in [0, 1) (Eq. (free_carve)): a segment starting on the plane z = 0
    and moving to z = -0.12 meets voxel 0 at t = 0, then -1, -2 and -3."""
    vox, amb = segment_voxels(np.zeros(3), np.array([0.0, 0.0, -0.12]), V)
    assert not amb
    assert vox == {(0, 0, 0), (0, 0, -1), (0, 0, -2), (0, 0, -3)}
    # moving up from the same plane: voxels 0, 1, 2
    vox, _ = segment_voxels(np.zeros(3), np.array([0.0, 0.0, 0.12]), V)
    assert vox == {(0, 0, 0), (0, 0, 1), (0, 0, 2)}
