"""Float64 coarsest-level solve (conjugate gradients in one workgroup per
channel) against the oracle's exact solution, and full solves that use it.

Tolerance of the coarse solve: the kernel runs CG in float64 to a relative
residual of 1e-12 and rounds the result to float32 once, so it must match
the exact float64 solution to float32 rounding (<= 255 * 2^-24) plus the
CG error (relative residual 1e-12 times the conditioning of these small
grids, far below that): 1e-4 absolute on the 0-255 scale.
"""
import numpy as np
import pytest

import oracle
from paper_2110_03946_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def ddi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2110_03946_amd import ddi as mod
    mod.lib()
    return mod


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("C,H,W,d,kind", [
    (1, 1, 1, 0.5, "bernoulli"), (1, 5, 3, 0.3, "bernoulli"), (3, 64, 128, 0.05, "bernoulli"),
    (2, 67, 113, 0.02, "clustered"), (3, 68, 120, 0.1, "clustered"), (1, 90, 91, 0.01, "bernoulli"),
    (1, 1, 8192, 0.01, "bernoulli"), (4, 8192, 1, 0.05, "bernoulli")])
def test_coarse_solve_parity(ddi, C, H, W, d, kind):
    f, c = synth.make_workload(H, W, C, d, kind, workload=11, index=H + W)
    say("coarse solve", C, H, W, d, kind)
    u = host(ddi.coarse_solve(dev(f), dev(c), max_iter=20000, tol=1e-12))
    ex = oracle.solve_exact(f.astype(np.float64), c)
    np.testing.assert_allclose(u, ex, atol=1e-4, rtol=0)
    np.testing.assert_array_equal(u[:, c == 1], f[:, c == 1])


def test_coarse_solve_iteration_cap(ddi):
    """max_iter bounds the work: one step from u = c ? f : 0 moves the
    unknowns but does not solve a system with large holes."""
    f, c = synth.make_workload(80, 100, 1, 0.01, "clustered", workload=11, index=3)
    u1 = host(ddi.coarse_solve(dev(f), dev(c), max_iter=1, tol=0.0))
    ex = oracle.solve_exact(f.astype(np.float64), c)
    assert np.abs(u1 - ex).max() > 1.0
    np.testing.assert_array_equal(u1[:, c == 1], f[:, c == 1])


def test_coarse_solve_rejects_large(ddi):
    f = torch.zeros((1, 91, 91), dtype=torch.float32, device="cuda")
    c = torch.ones((91, 91), dtype=torch.uint8, device="cuda")
    with pytest.raises(ddi.DDIError):
        ddi.coarse_solve(f, c)


@pytest.mark.parametrize("C,H,W,d,kind,prm", [
    (3, 2160, 3840, 0.04, "bernoulli", dict(levels=6)),
    (3, 1080, 1920, 0.03, "clustered", dict(levels=5, local_iters=24, local_tol=0.0005,
                                            coarse_sweeps=2, coarse_local_iters=16)),
    (1, 200, 300, 0.05, "bernoulli", dict(levels=3, block=32)),
    (2, 90, 91, 0.05, "bernoulli", dict(levels=1, block=32))])
def test_solve_with_float64_coarsest_level(ddi, C, H, W, d, kind, prm):
    f, c = synth.make_workload(H, W, C, d, kind, workload=12, index=H)
    say("solve coarse_solver=1", C, H, W, d, kind, prm)
    p = dict(dict(rel_tol=5e-5, max_sweeps=60, coarse_solver=1, coarse_cg_tol=1e-10), **prm)
    with ddi.Plan(H, W, C, **p) as plan:
        u_t, st = plan.solve(dev(f), dev(c))
    u = host(u_t)
    ex = oracle.solve_exact(f.astype(np.float64), c)
    err = float(np.abs(u - ex).max())
    say("  sweeps", st["sweeps"], "rel", st["rel_residual"], "err", err)
    assert err <= 0.5
    np.testing.assert_array_equal(u[:, c == 1], f[:, c == 1])


def test_batch_with_float64_coarsest_level(ddi):
    """Images with and without the float64 coarse solve in one batch equal
    their single-image solves bit for bit."""
    C = 3
    specs = [(120, 160, 0.05, "bernoulli", 1), (96, 96, 0.04, "clustered", 0),
             (130, 70, 0.05, "bernoulli", 1)]
    data = [synth.make_workload(h, w, C, d, k, workload=13, index=i)
            for i, (h, w, d, k, _) in enumerate(specs)]
    prms = [ddi.default_params(levels=3, block=32, rel_tol=1e-5, max_sweeps=60, coarse_solver=cs)
            for *_, cs in specs]
    say("batch coarse_solver mix")
    with ddi.Batch([c.shape for _, c in data], C, params=prms) as b:
        us, st, codes = b.solve([dev(f) for f, _ in data], [dev(c) for _, c in data])
    assert codes == [0, 0, 0]
    for (f, c), p, u_t, s in zip(data, prms, us, st):
        q = ddi.Params.from_buffer_copy(p)
        with ddi.Plan(c.shape[0], c.shape[1], C, params=q) as plan:
            u_ref, s_ref = plan.solve(dev(f), dev(c))
        assert s["sweeps"] == s_ref["sweeps"]
        np.testing.assert_array_equal(host(u_t), host(u_ref))
