"""Float64 coarsest-level solve (conjugate gradients in one workgroup per
channel, or on a grid of workgroups for levels of any size) against the
oracle's exact solution, and full solves that use it.

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


SMALL = [(1, 1, 1, 0.5, "bernoulli"), (1, 5, 3, 0.3, "bernoulli"), (3, 64, 128, 0.05, "bernoulli"),
         (2, 67, 113, 0.02, "clustered"), (3, 68, 120, 0.1, "clustered"),
         (1, 90, 91, 0.01, "bernoulli"), (1, 1, 8192, 0.01, "bernoulli"),
         (4, 8192, 1, 0.05, "bernoulli")]


@pytest.mark.parametrize("wgs", [1, 3, 0, 64])
@pytest.mark.parametrize("C,H,W,d,kind", SMALL)
def test_coarse_grid_parity(ddi, C, H, W, d, kind, wgs):
    """The grid solve on 1, 3, the default and 64 workgroups: the exact
    solution to the same bound as the one-workgroup solve, and that solve's
    result to twice the bound (the same CG with the dot products summed in
    another order)."""
    f, c = synth.make_workload(H, W, C, d, kind, workload=11, index=H + W)
    say("coarse grid solve", C, H, W, d, kind, "workgroups", wgs)
    u_t, steps = ddi.coarse_solve_grid(dev(f), dev(c), max_iter=20000, tol=1e-12,
                                       workgroups=wgs, steps=True)
    u = host(u_t)
    ex = oracle.solve_exact(f.astype(np.float64), c)
    np.testing.assert_allclose(u, ex, atol=1e-4, rtol=0)
    np.testing.assert_array_equal(u[:, c == 1], f[:, c == 1])
    assert len(steps) == C and all(0 <= k < 20000 for k in steps)
    u1 = host(ddi.coarse_solve(dev(f), dev(c), max_iter=20000, tol=1e-12))
    np.testing.assert_allclose(u, u1, atol=2e-4, rtol=0)


def _coarsened(H, W, C, d, kind, times, index):
    """A workload subsampled `times` times like the pyramid (a coarse pixel
    is known if one of its 2 x 2 fine pixels is, with their mean): input
    shaping only, vectorised; the expected values come from the oracle."""
    f, c = synth.make_workload(H, W, C, d, kind, workload=14, index=index)
    f = f.astype(np.float64)
    for _ in range(times):
        h, w = c.shape
        hp, wp = h + h % 2, w + w % 2
        cp = np.zeros((hp, wp)); cp[:h, :w] = c
        fp = np.zeros((f.shape[0], hp, wp)); fp[:, :h, :w] = f * c
        n = cp.reshape(hp // 2, 2, wp // 2, 2).sum(axis=(1, 3))
        s = fp.reshape(f.shape[0], hp // 2, 2, wp // 2, 2).sum(axis=(2, 4))
        c = (n > 0).astype(np.uint8)
        f = np.where(n > 0, s / np.maximum(n, 1), 0.0)
    return np.ascontiguousarray(f.astype(np.float32)), np.ascontiguousarray(c)


@pytest.mark.parametrize("H,W,d,kind,times", [
    (2160, 3840, 0.04, "bernoulli", 3),   # the coarsest level of 4K with 4 levels
    (1080, 1920, 0.03, "clustered", 2),   # large holes: many CG steps
    (1600, 520, 0.002, "bernoulli", 1)])  # few known pixels: a far-reaching solve
def test_coarse_grid_large_levels(ddi, H, W, d, kind, times):
    """Levels over 8192 pixels, which only the grid solve takes, against the
    oracle's exact solution (sparse direct solve in float64)."""
    f, c = _coarsened(H, W, 3, d, kind, times, index=times)
    say("coarse grid solve of a coarsened level", f.shape, kind, "known", float(c.mean()))
    u_t, steps = ddi.coarse_solve_grid(dev(f), dev(c), max_iter=20000, tol=1e-12, steps=True)
    u = host(u_t)
    ex = oracle.solve_exact(f.astype(np.float64), c)
    say("  steps", steps, "max err", float(np.abs(u - ex).max()))
    np.testing.assert_allclose(u, ex, atol=1e-4, rtol=0)
    np.testing.assert_array_equal(u[:, c == 1], f[:, c == 1])


def test_coarse_grid_iteration_cap_and_tolerance(ddi):
    """max_iter bounds the steps of every channel; a tolerance the start
    already meets takes no step (u = c ? f : 0)."""
    f, c = synth.make_workload(300, 200, 2, 0.01, "clustered", workload=11, index=5)
    u1, s1 = ddi.coarse_solve_grid(dev(f), dev(c), max_iter=1, tol=0.0, steps=True)
    assert s1 == [1, 1]
    ex = oracle.solve_exact(f.astype(np.float64), c)
    assert np.abs(host(u1) - ex).max() > 1.0
    u0, s0 = ddi.coarse_solve_grid(dev(f), dev(c), max_iter=100, tol=10.0, steps=True)
    assert s0 == [0, 0]
    np.testing.assert_array_equal(host(u0), np.where(c == 1, f, 0).astype(np.float32))


def test_coarse_grid_rejects_bad_workspace(ddi):
    f = torch.zeros((1, 100, 100), dtype=torch.float32, device="cuda")
    c = torch.ones((100, 100), dtype=torch.uint8, device="cuda")
    need = ddi.coarse_grid_bytes(100, 100, 1)
    short = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(ddi.DDIError):
        ddi.coarse_solve_grid(f, c, work=short)
    big = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(ddi.DDIError):  # not 256-byte aligned
        ddi.coarse_solve_grid(f, c, work=big[8:])
    with pytest.raises(ddi.DDIError):
        ddi.coarse_solve_grid(f, c, workgroups=257)


def test_coarse_grid_stall_reported(ddi):
    """A barrier wait that exceeds its bound ends the solve on every
    workgroup and is reported: forced from the host with a bound of zero
    polls, the entry point, a plan and a batch return DDI_ESTALL; with the
    default bound the same calls succeed again."""
    f, c = synth.make_workload(120, 160, 3, 0.05, "bernoulli", workload=11, index=9)
    prm = dict(levels=1, block=32, rel_tol=1e-4, max_sweeps=40, coarse_solver=1)
    lib = ddi.lib()
    try:
        lib.ddi_coarse_grid_debug_spin_limit(0)
        say("stall: entry point")
        with pytest.raises(ddi.DDIError) as e:
            ddi.coarse_solve_grid(dev(f), dev(c), workgroups=16, steps=True)
        assert e.value.code == ddi.DDI_ESTALL
        say("stall: plan")
        with ddi.Plan(120, 160, 3, **prm) as plan:
            with pytest.raises(ddi.DDIError) as e:
                plan.solve(dev(f), dev(c))
            assert e.value.code == ddi.DDI_ESTALL
        say("stall: batch")
        with ddi.Batch([(120, 160)], 3, params=[ddi.default_params(**prm)]) as b:
            with pytest.raises(ddi.DDIError) as e:
                b.solve([dev(f)], [dev(c)])
            assert e.value.code == ddi.DDI_ESTALL
    finally:
        lib.ddi_coarse_grid_debug_spin_limit(-1)
    say("stall: default bound again")
    u = host(ddi.coarse_solve_grid(dev(f), dev(c), workgroups=16, tol=1e-12, max_iter=20000))
    np.testing.assert_allclose(u, oracle.solve_exact(f.astype(np.float64), c), atol=1e-4, rtol=0)
    with ddi.Plan(120, 160, 3, **prm) as plan:
        plan.solve(dev(f), dev(c))


def test_coarse_solve_rejects_large(ddi):
    f = torch.zeros((1, 91, 91), dtype=torch.float32, device="cuda")
    c = torch.ones((91, 91), dtype=torch.uint8, device="cuda")
    with pytest.raises(ddi.DDIError):
        ddi.coarse_solve(f, c)


@pytest.mark.parametrize("C,H,W,d,kind,prm", [
    (3, 2160, 3840, 0.04, "bernoulli", dict(levels=6)),
    (3, 2160, 3840, 0.04, "bernoulli", dict(levels=4)),
    (2, 600, 900, 0.02, "clustered", dict(levels=2, block=32)),
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
    # the last image's coarsest level (its only level, 220 x 210) takes the
    # grid solve
    specs = [(120, 160, 0.05, "bernoulli", 1, 3), (96, 96, 0.04, "clustered", 0, 3),
             (130, 70, 0.05, "bernoulli", 1, 3), (220, 210, 0.05, "bernoulli", 1, 1)]
    data = [synth.make_workload(h, w, C, d, k, workload=13, index=i)
            for i, (h, w, d, k, _, _) in enumerate(specs)]
    prms = [ddi.default_params(levels=lv, block=32, rel_tol=1e-5, max_sweeps=60,
                               coarse_solver=cs) for *_, cs, lv in specs]
    say("batch coarse_solver mix")
    with ddi.Batch([c.shape for _, c in data], C, params=prms) as b:
        us, st, codes = b.solve([dev(f) for f, _ in data], [dev(c) for _, c in data])
    assert codes == [0, 0, 0, 0]
    for (f, c), p, u_t, s in zip(data, prms, us, st):
        q = ddi.Params.from_buffer_copy(p)
        with ddi.Plan(c.shape[0], c.shape[1], C, params=q) as plan:
            u_ref, s_ref = plan.solve(dev(f), dev(c))
        assert s["sweeps"] == s_ref["sweeps"]
        np.testing.assert_array_equal(host(u_t), host(u_ref))
