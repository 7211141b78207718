"""Mixed precision (storage = 1): bfloat16 storage of the correction and
its right-hand side, float32 arithmetic, float32 iterative refinement,
float64 norms.

Tolerances:
  refine residual   u_next = u + d is one float32 addition: bit-exact.
                    rhs is the float32 stencil (1e-4 from the float64
                    definition, as for the plain residual) rounded to
                    bfloat16: within one bfloat16 ulp (2^-7 relative) of
                    the float64 value rounded to bfloat16.
  correction sweep  the float32 sweep's 2e-3 plus the bfloat16 rounding of
                    the stored correction, 2^-8 relative.
  full solve        0.5 grey levels max-abs against the exact float64
                    solution in every channel, u = f bit for bit on the mask.
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
    return t.float().cpu().numpy() if t.dtype == torch.bfloat16 else t.cpu().numpy()


def bf16(x):
    """float64/32 array -> bfloat16 tensor (round to nearest even) on the GPU."""
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(torch.bfloat16).cuda()


def bf16_value(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(
        torch.bfloat16).float().numpy().astype(np.float64)


def case(C, H, W, d=0.06, kind="bernoulli", seed=0):
    f, c = synth.make_workload(H, W, C, d, kind, workload=30, index=seed)
    rng = np.random.default_rng(seed + 100)
    u = np.where(c == 1, f, rng.uniform(0, 255, f.shape).astype(np.float32)).astype(np.float32)
    dd = np.where(c == 1, 0.0, rng.normal(0, 20, f.shape)).astype(np.float32)
    return f, c, u, dd


@pytest.mark.parametrize("C,H,W", [(1, 1, 1), (1, 17, 5), (3, 67, 131), (2, 64, 64),
                                   (1, 130, 1)])
@pytest.mark.parametrize("with_d", [False, True])
def test_refine_residual_parity(ddi, C, H, W, with_d):
    f, c, u, dd = case(C, H, W, seed=H + W)
    say("refine residual", C, H, W, with_d)
    d_t = bf16(dd) if with_d else None
    un_t, rhs_t, rsq = ddi.refine_residual(dev(f), dev(c), dev(u), d_t)
    if with_d:
        dv = d_t.float().cpu().numpy()
        un_exp = (u + dv).astype(np.float32)
        un = host(un_t)
        np.testing.assert_array_equal(un, un_exp)
    else:
        assert un_t is None
        un_exp = u
    r64 = oracle.residual(f.astype(np.float64), c, un_exp.astype(np.float64))
    rhs = host(rhs_t).astype(np.float64)
    ulp = np.maximum(np.abs(bf16_value(r64)), 1e-30) * 2.0 ** -7
    assert np.all(np.abs(rhs - bf16_value(r64)) <= ulp + 1e-4)
    np.testing.assert_allclose(rsq, (r64 ** 2).reshape(C, -1).sum(1), rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("C,H,W", [(1, 1, 1), (1, 2, 3), (1, 17, 5), (3, 67, 131), (2, 64, 64),
                                   (1, 130, 1), (3, 33, 200), (3, 1079, 1921), (3, 2160, 3840)])
def test_refine_start_bit_exact(ddi, C, H, W):
    """The first refinement residual built with the coarse-to-fine start
    equals the prolongation followed by the refinement residual, bit for bit
    (iterate, right-hand side and norms); odd sizes clamp the last coarse
    row and column."""
    f, c, _, _ = case(C, H, W, seed=H + 2 * W)
    hc, wc = (H + 1) // 2, (W + 1) // 2
    uc = np.random.default_rng(H * W + 5).uniform(0, 255, (C, hc, wc)).astype(np.float32)
    say("refine start", C, H, W)
    u_ref = ddi.prolong(dev(uc), dev(f), dev(c))
    _, rhs_ref, rsq_ref = ddi.refine_residual(dev(f), dev(c), u_ref)
    u, rhs, rsq = ddi.refine_start(dev(uc), dev(f), dev(c))
    np.testing.assert_array_equal(host(u), host(u_ref))
    torch.cuda.synchronize()
    assert torch.equal(rhs.view(torch.int16), rhs_ref.view(torch.int16))
    np.testing.assert_array_equal(rsq, rsq_ref)


SWEEP_CASES = [(1, 64, 64, 64, 4, 0.25, 8), (3, 67, 131, 32, 4, 0.5, 6), (2, 100, 75, 24, 6, 1.0, 5),
               (1, 130, 70, 64, 4, 0.25, 12), (1, 20, 200, 16, 2, 0.3, 4), (1, 7, 9, 8, 2, 0.5, 3)]


@pytest.mark.parametrize("C,H,W,S,o,alpha,k", SWEEP_CASES)
@pytest.mark.parametrize("start", ["zero", "given"])
def test_correction_sweep_parity(ddi, C, H, W, S, o, alpha, k, start):
    f, c, u, dd = case(C, H, W, seed=3 * H + W)
    say("correction sweep", C, H, W, S, o, alpha, k, start)
    r64 = oracle.residual(f.astype(np.float64), c, u.astype(np.float64))
    rhs_t = bf16(r64)
    rhs = rhs_t.float().cpu().numpy().astype(np.float64)
    d_t = bf16(dd) if start == "given" else None
    d_in = d_t.float().cpu().numpy().astype(np.float64) if d_t is not None else np.zeros_like(r64)
    out = host(ddi.correction_sweep(d_t, rhs_t, dev(c), S, o, alpha, k)).astype(np.float64)
    for ch in range(C):
        exp = oracle.correction_step(d_in[ch], rhs[ch], c, S, o, alpha, k)
        tol = 2e-3 + np.abs(exp) * 2.0 ** -8
        err = np.abs(out[ch] - exp)
        assert np.all(err <= tol), (ch, float((err - tol).max()))
        assert np.all(out[ch][c == 1] == 0.0)


def _bench_precision():
    import bench
    return bench.precision_params()


@pytest.mark.parametrize("C,H,W,d,kind,prm", [
    (3, 2160, 3840, 0.03, "bernoulli", dict()),
    (3, 2160, 3840, 0.03, "bernoulli", "bench"),
    (3, 1080, 1920, 0.03, "clustered", dict(levels=5, local_iters=24, local_tol=0.0005,
                                            coarse_sweeps=2, coarse_local_iters=16)),
    (1, 200, 300, 0.05, "bernoulli", dict(levels=3, block=32)),
    (2, 61, 90, 0.1, "bernoulli", dict(levels=1, block=16, inner_sweeps=3)),
])
def test_precision_variant_solve(ddi, C, H, W, d, kind, prm):
    """storage = 1 reaches the same fixed point: within 0.5 grey levels in
    every channel, u = f on the mask."""
    if prm == "bench":  # the benchmark's parameters on a frame it does not time
        prm = _bench_precision()
    f, c = synth.make_workload(H, W, C, d, kind, workload=31, index=H)
    say("storage=1 solve", C, H, W, d, kind, prm)
    p = dict(dict(levels=4, local_iters=16, robin_alpha=0.25, coarse_sweeps=1, coarsest_sweeps=1,
                  coarse_local_iters=4, local_tol=0.0005, rel_tol=3e-5, min_sweeps=1,
                  max_sweeps=40, storage=1, inner_sweeps=2), **prm)
    with ddi.Plan(H, W, C, **p) as plan:
        u_t, st = plan.solve(dev(f), dev(c), allow_noconv=True)
        say("  first solve", st)
        assert st["converged"] == 1
        u = host(u_t)
        u2_t, st2 = plan.solve(dev(f), dev(c))  # second solve: start buffers from the first
        np.testing.assert_array_equal(host(u2_t), u)
    ex = oracle.solve_exact(f.astype(np.float64), c)
    errs = [float(np.abs(u[k] - ex[k]).max()) for k in range(C)]
    say("  refinements", st["refinements"], "sweeps", st["sweeps"], "rel", st["rel_residual"],
        "err per channel", errs)
    assert st["converged"] == 1 and st["sweeps"] == st["refinements"] * p["inner_sweeps"]
    assert max(errs) <= 0.5
    np.testing.assert_array_equal(u[:, c == 1], f[:, c == 1])
    # the reported residual is that of the returned iterate: max over
    # channels of ||b - A u|| / ||b||, from float32 stencil values (their
    # rounding, ~255 * 2^-24 per pixel, is a few % of residuals this small)
    rel = max(oracle.rel_residual(f[k].astype(np.float64), c, u[k].astype(np.float64))
              for k in range(C))
    assert abs(rel - st["rel_residual"]) <= 0.05 * rel + 1e-9


def test_precision_variant_errors(ddi):
    f, c = synth.make_workload(40, 48, 1, 0.05, "bernoulli", workload=32)
    with ddi.Plan(40, 48, 1, storage=1, block=16, levels=2) as plan:
        with pytest.raises(ddi.DDIError) as ei:
            plan.solve(dev(f), dev(np.zeros_like(c)))
        assert ei.value.code == ddi.DDI_ESINGULAR
        bad = c.copy()
        bad[3, 3] = 7
        with pytest.raises(ddi.DDIError) as ei:
            plan.solve(dev(f), dev(bad))
        assert ei.value.code == ddi.DDI_EINVAL
    with ddi.Plan(40, 48, 1, storage=1, block=16, levels=2, rel_tol=0.0, max_sweeps=3) as plan:
        u_t, st = plan.solve(dev(f), dev(c), allow_noconv=True)
        assert st["converged"] == 0 and st["refinements"] == 3
    with pytest.raises(ddi.DDIError):
        ddi.Batch([(40, 48)], 1, params=ddi.default_params(storage=1))


@pytest.mark.parametrize("storage", [0, 1])
def test_sweep_times_per_sweep(ddi, storage):
    """With timing = 1 the plan reports one device time per finest-level
    sweep of the last solve (the correction sweeps for storage = 1), and
    they add up to the solve's sweep time."""
    f, c = synth.make_workload(256, 384, 3, 0.04, "bernoulli", workload=33)
    say("sweep times", storage)
    p = dict(levels=3, block=32, local_iters=12, rel_tol=1e-4, min_sweeps=2, max_sweeps=40,
             storage=storage, inner_sweeps=2, timing=1)
    with ddi.Plan(256, 384, 3, **p) as plan:
        plan.solve(dev(f), dev(c))
        _, st = plan.solve(dev(f), dev(c))
        t = plan.sweep_times()
    assert len(t) == st["sweeps"] >= 2
    assert all(x > 0.0 for x in t)
    assert abs(sum(t) - st["sweep_ms"]) <= 1e-6 + 1e-6 * st["sweep_ms"]
