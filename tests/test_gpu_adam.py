"""GPU parity of the library's Adam update (gsr_adam) with the oracle's:
several arrays of ragged sizes in one launch (vector and scalar element
paths), five eager steps, then three replays of a captured step with eager
work in between (the device step count advances every replay)."""
import numpy as np
import pytest

from gpu_harness import announce
from oracle.adam import adam_step

pytestmark = pytest.mark.gpu

# ragged against the kernel's 1024-element chunks
SIZES = (1, 5, 1023, 1025, 8195, 100_003)
LRS = (1e-3, 5e-2, 2.5e-3, 1.6e-4, 3e-3, 1e-2)


def _check(P, G_hist, p0, lrs, got_p, got_m, got_v, steps, b1, b2, eps):
    for k, n in enumerate(SIZES):
        q, m, v = p0[k].astype(np.float64), np.zeros(n), np.zeros(n)
        # magnitudes of the moments' terms: FP32 rounds each running sum
        # relative to these, so a moment that cancels to a small value keeps
        # an absolute error of a few ulps of its largest term
        am, av = np.zeros(n), np.zeros(n)
        for t in range(1, steps + 1):
            g = G_hist[t - 1][k].astype(np.float64)
            q, m, v = adam_step(q, g, m, v, t, lrs[k], b1, b2, eps)
            am = b1 * am + (1 - b1) * np.abs(g)
            av = b2 * av + (1 - b2) * g * g
        # the FP32 parameter carries an ulp of |p| per step; the update itself
        # is exact to FP32 rounding of m, v and the quotient
        tol = 4e-7 * np.abs(q) * steps + 1e-4 * lrs[k] * steps
        assert np.all(np.abs(got_p[k] - q) <= tol), (n, np.abs(got_p[k] - q).max())
        assert np.all(np.abs(got_m[k] - m) <= 3e-7 * steps * am), (n, np.abs(got_m[k] - m).max())
        assert np.all(np.abs(got_v[k] - v) <= 3e-7 * steps * av), (n, np.abs(got_v[k] - v).max())


def test_adam_matches_oracle_eager_and_graph():
    announce("adam eager + graph")
    import torch
    from paper_2605_10760_amd import Adam
    rng = np.random.default_rng(3)
    b1, b2, eps = 0.9, 0.999, 1e-15
    p0 = [rng.normal(size=n).astype(np.float32) for n in SIZES]
    # the last array starts one element into its buffer: unaligned rows take
    # the scalar path
    bufs = [torch.from_numpy(a).cuda() for a in p0[:-1]]
    big = torch.zeros(SIZES[-1] + 1, device="cuda")
    big[1:] = torch.from_numpy(p0[-1]).cuda()
    params = bufs + [big[1:]]
    grads = [torch.zeros_like(p) for p in params]
    for p, g in zip(params, grads):
        p.grad = g
    opt = Adam(list(zip(params, LRS)), betas=(b1, b2), eps=eps)
    hist = []
    for _ in range(5):
        gs = [rng.normal(size=n).astype(np.float32) * 10 ** rng.uniform(-6, 2) for n in SIZES]
        for g, a in zip(grads, gs):
            g.copy_(torch.from_numpy(a).cuda())
        hist.append(gs)
        opt.step()
    torch.cuda.synchronize()
    assert int(opt.t.item()) == 5
    _check(None, hist, p0, LRS, [p.cpu().numpy() for p in params],
           [m.cpu().numpy() for m in opt.m], [v.cpu().numpy() for v in opt.v], 5, b1, b2, eps)
    # capture one step; replay with new gradients written in between
    graph = torch.cuda.CUDAGraph()
    saved = ([p.clone() for p in params], [m.clone() for m in opt.m], [v.clone() for v in opt.v],
             opt.t.clone())
    with torch.cuda.graph(graph):
        opt.step()
    # capturing records the step without running it
    for a, b in zip(saved[0], params):
        assert torch.equal(a, b)
    for _ in range(3):
        gs = [rng.normal(size=n).astype(np.float32) for n in SIZES]
        for g, a in zip(grads, gs):
            g.copy_(torch.from_numpy(a).cuda())
        hist.append(gs)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
    assert int(opt.t.item()) == 8
    _check(None, hist, p0, LRS, [p.cpu().numpy() for p in params],
           [m.cpu().numpy() for m in opt.m], [v.cpu().numpy() for v in opt.v], 8, b1, b2, eps)


def test_adam_rejects_bad_arguments():
    announce("adam args")
    import ctypes as C
    import torch
    from paper_2605_10760_amd import _lib
    lib = _lib.load()
    t = torch.zeros(1, dtype=torch.int32, device="cuda")
    g = (_lib.AdamGroup * 1)()
    g[0] = _lib.AdamGroup(None, None, None, None, 4, 1e-3, 0)
    assert lib.gsr_adam(g, 1, 0.9, 0.999, 1e-8, C.c_void_p(t.data_ptr()), None) == _lib.GSR_E_INVALID_ARG
    assert lib.gsr_adam(g, 0, 0.9, 0.999, 1e-8, C.c_void_p(t.data_ptr()), None) == _lib.GSR_E_INVALID_ARG
    assert lib.gsr_adam(g, 9, 0.9, 0.999, 1e-8, C.c_void_p(t.data_ptr()), None) == _lib.GSR_E_INVALID_ARG
    g[0] = _lib.AdamGroup(None, None, None, None, 0, 1e-3, 0)  # empty array: only the tick
    assert lib.gsr_adam(g, 1, 0.9, 0.999, 1e-8, C.c_void_p(t.data_ptr()), None) == _lib.GSR_OK
    torch.cuda.synchronize()
    assert int(t.item()) == 1
