"""Pins of the oracle's refinement extras (Sec. III-C, Eq. (refine_loss)):
finite differences of the exposure-compensated L1 loss, the reduction to the
plain L1 gradient, and opacity pruning against a direct recount."""
import numpy as np

from oracle.refine import exposure, l1_loss, l1_loss_grad, prune


def _case(seed, V=2, H=5, W=6):
    rng = np.random.default_rng(seed)
    c = rng.random((V, 3, H, W))
    d = 0.5 + 3 * rng.random((V, H, W))
    tc = rng.random((V, 3, H, W))
    td = 0.5 + 3 * rng.random((V, H, W))
    a = rng.normal(0, 0.3, V)
    b = rng.normal(0, 0.1, V)
    return c, d, tc, td, a, b


def test_exposure_closed_form():
    c, _, _, _, a, b = _case(0)
    e = exposure(c, a, b)
    for k in range(c.shape[0]):
        np.testing.assert_allclose(e[k], np.exp(a[k]) * c[k] + b[k], rtol=1e-15)


def test_l1_grad_matches_central_differences():
    """Away from the kinks of |.| the loss is linear in each input, so central
    differences are exact up to rounding."""
    c, d, tc, td, a, b = _case(1)
    g = l1_loss_grad(c, d, tc, td, a, b, 1.75, 0.25)
    h = 1e-7
    f = lambda c_, d_, a_, b_: l1_loss(c_, d_, tc, td, a_, b_, 1.75, 0.25)
    rng = np.random.default_rng(2)
    for _ in range(20):
        idx = tuple(rng.integers(0, s) for s in c.shape)
        cp, cm = c.copy(), c.copy()
        cp[idx] += h
        cm[idx] -= h
        fd = (f(cp, d, a, b) - f(cm, d, a, b)) / (2 * h)
        assert abs(fd - g["d_color"][idx]) <= 1e-7 * max(1e-3, abs(fd)) + 1e-12
        jdx = tuple(rng.integers(0, s) for s in d.shape)
        dp, dm = d.copy(), d.copy()
        dp[jdx] += h
        dm[jdx] -= h
        fd = (f(c, dp, a, b) - f(c, dm, a, b)) / (2 * h)
        assert abs(fd - g["d_depth"][jdx]) <= 1e-7 * max(1e-3, abs(fd)) + 1e-12
    for k in range(c.shape[0]):
        for key, arr in (("d_a", a), ("d_b", b)):
            p, m = arr.copy(), arr.copy()
            p[k] += h
            m[k] -= h
            fd = ((f(c, d, p, b) - f(c, d, m, b)) if key == "d_a"
                  else (f(c, d, a, p) - f(c, d, a, m))) / (2 * h)
            assert abs(fd - g[key][k]) <= 1e-6 * max(1e-3, abs(fd)), key


def test_no_exposure_is_plain_l1():
    c, d, tc, td, _, _ = _case(3)
    z = np.zeros(c.shape[0])
    g = l1_loss_grad(c, d, tc, td, z, z, 0.95, 0.25)
    np.testing.assert_array_equal(g["d_color"], 0.95 * np.sign(c - tc) / c.size)
    np.testing.assert_array_equal(g["d_depth"], 0.25 * np.sign(d - td) / d.size)


def test_prune_recount():
    o = np.array([-6.0, -5.0, -5.4, 0.0, -5.29, 2.0, -5.3], np.float32)
    idx, offs = prune(o, [0, 3, 7], 0.005)
    # sigmoid(-5.29) = 0.005015 > 0.005 > sigmoid(-5.3) = 0.004965
    np.testing.assert_array_equal(idx, [1, 3, 4, 5])
    np.testing.assert_array_equal(offs, [0, 1, 4])
    rng = np.random.default_rng(4)
    o = rng.normal(-5.3, 0.2, 5000).astype(np.float32)
    idx, offs = prune(o, [0, 1234, 5000])
    keep = 1 / (1 + np.exp(-o.astype(np.float64))) >= 0.005
    np.testing.assert_array_equal(idx, np.nonzero(keep)[0])
    assert offs[1] == keep[:1234].sum() and offs[2] == keep.sum()
