"""Multilevel CG (method = 1), the comparator of Sec. 5: same fixed point as
ORAS, checked against the oracle's exact solution."""
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


@pytest.mark.parametrize("C,H,W,d,kind,levels", [
    (1, 1, 1, 0.5, "bernoulli", 1), (1, 17, 5, 0.2, "bernoulli", 1), (3, 67, 131, 0.05, "bernoulli", 3),
    (2, 120, 96, 0.02, "clustered", 4), (3, 540, 960, 0.04, "bernoulli", 4)])
def test_mlcg_matches_exact(ddi, C, H, W, d, kind, levels):
    f, c = synth.make_workload(H, W, C, d, kind, workload=60, index=H)
    say("mlcg", C, H, W, d, kind, levels)
    with ddi.Plan(H, W, C, method=1, levels=levels, rel_tol=1e-6, max_sweeps=5000,
                  final_residual=0) as plan:
        u_t, st = plan.solve(dev(f), dev(c))
        u = u_t.cpu().numpy()
        u2_t, st2 = plan.solve(dev(f), dev(c))
        np.testing.assert_array_equal(u2_t.cpu().numpy(), u)
    ex = oracle.solve_exact(f.astype(np.float64), c)
    err = float(np.abs(u - ex).max())
    say("  iters", st["sweeps"], "all levels", st["cg_steps"], "rel", st["rel_residual"], "err", err)
    assert st["converged"] == 1 and st["rel_residual"] <= 1e-6
    assert err <= 0.02
    np.testing.assert_array_equal(u[:, c == 1], f[:, c == 1])


def test_mlcg_errors(ddi):
    f, c = synth.make_workload(40, 48, 1, 0.05, "bernoulli", workload=61)
    with ddi.Plan(40, 48, 1, method=1, levels=2) as plan:
        with pytest.raises(ddi.DDIError) as ei:
            plan.solve(dev(f), dev(np.zeros_like(c)))
        assert ei.value.code == ddi.DDI_ESINGULAR
        u = torch.empty((1, 40, 48), dtype=torch.float32, device="cuda")
        with pytest.raises(ddi.DDIError):
            plan.solve_async(dev(f), dev(c), u)
    with ddi.Plan(40, 48, 1, method=1, levels=1, rel_tol=1e-12, max_sweeps=3) as plan:
        _, st = plan.solve(dev(f), dev(c), allow_noconv=True)
        assert st["converged"] == 0 and st["sweeps"] == 3
    assert ddi.check_params(40, 48, 1, ddi.default_params(method=1, storage=1)) == ddi.DDI_EINVAL
