"""Dispatch order of the finest level's first sweep (order_blocks = 1: the
blocks whose level-2 blocks ran the most CG steps first, the table built
inside the level-1 sweep launch) against logical order (order_blocks = 0).

The order only decides which workgroup runs which block: every block reads
the same input buffer, writes only its owned pixels of the other one and
its own partial slot, so the solves must agree bit for bit -- returned
image, sweep count, residual -- with and without the skips, through the
synchronous, asynchronous and graph paths. The output buffers start as NaN,
so a block that no workgroup ran (or one run twice in place of another)
would show. The converged results are also checked against the oracle.
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


BENCH = dict(block=64, overlap=4, levels=4, local_iters=16, robin_alpha=0.25, coarse_sweeps=1,
             coarsest_sweeps=1, coarse_local_iters=8, local_tol=0.004, rel_tol=5e-4,
             min_sweeps=3, max_sweeps=30, final_residual=0)

CASES = [
    # the benchmark workload
    (3, 2160, 3840, 0.04, "bernoulli", BENCH),
    # clustered mask, odd sizes, many sweeps (late sweeps skip most blocks)
    (3, 1081, 1923, 0.03, "clustered", dict(BENCH, rel_tol=1e-6, local_tol=0.001,
                                            max_sweeps=80)),
    # two levels: no level 2, so no table (the plans must still agree);
    # four channels
    (4, 540, 960, 0.04, "bernoulli", dict(BENCH, levels=2, coarsest_sweeps=2, rel_tol=1e-5,
                                          max_sweeps=40)),
    # one level: logical order
    (1, 700, 1000, 0.05, "bernoulli", dict(levels=1, overlap=8, local_tol=0.003, rel_tol=1e-5,
                                           max_sweeps=80, check_every=2, final_residual=1)),
    # no fused prolongation, a float64 coarsest solve
    (3, 128, 250, 0.05, "bernoulli", dict(BENCH, levels=2, fuse_prolong=0, coarse_solver=1,
                                          rel_tol=1e-5, max_sweeps=40)),
    # no fused prolongation, three levels: the table is built in a plain
    # level-1 sweep and used by a plain finest sweep
    (3, 700, 1300, 0.05, "clustered", dict(BENCH, levels=3, fuse_prolong=0, rel_tol=1e-6,
                                           local_tol=0.001, max_sweeps=80)),
    # odd sizes, the last block row and column shifted back on every level
    (2, 1111, 2222, 0.04, "bernoulli", dict(BENCH, rel_tol=1e-5, max_sweeps=40)),
]


def _solve(ddi, f, c, prm, mode="sync"):
    C, H, W = f.shape
    u = torch.full((C, H, W), float("nan"), dtype=torch.float32, device="cuda")
    with ddi.Plan(H, W, C, **prm) as plan:
        if mode == "sync":
            _, st = plan.solve(dev(f), dev(c), u, allow_noconv=True)
        elif mode == "async":
            plan.solve_async(dev(f), dev(c), u)
            _, st = plan.wait(allow_noconv=True)
        else:  # graph: capture, then two replays
            fd, cd = dev(f), dev(c)
            for _ in range(3):
                u.fill_(float("nan"))
                _, st = plan.solve(fd, cd, u, allow_noconv=True)
    torch.cuda.synchronize()
    return u.cpu().numpy(), st


@pytest.mark.parametrize("C,H,W,d,kind,prm", CASES)
def test_order_matches_logical_order(ddi, C, H, W, d, kind, prm):
    f, c = synth.make_workload(H, W, C, d, kind, workload=76, index=H + W)
    for skip in (1, 0):
        say("order vs logical", C, H, W, kind, "skip", skip)
        ref, st0 = _solve(ddi, f, c, dict(prm, skip_unchanged=skip, order_blocks=0))
        got, st1 = _solve(ddi, f, c, dict(prm, skip_unchanged=skip, order_blocks=1))
        assert not np.isnan(got).any()
        assert np.array_equal(got, ref), f"max diff {np.nanmax(np.abs(got - ref))}"
        assert (st1["sweeps"], st1["rel_residual"]) == (st0["sweeps"], st0["rel_residual"])
    if H * W <= 1_000_000:
        ex = oracle.solve_exact(f.astype(np.float64), c)
        assert np.abs(got - ex).max() <= 0.5


@pytest.mark.parametrize("mode", ["async", "graph"])
def test_order_async_and_graph(ddi, mode):
    C, H, W = 3, 540, 960
    f, c = synth.make_workload(H, W, C, 0.04, "bernoulli", workload=76, index=1)
    prm = dict(BENCH, rel_tol=1e-5, max_sweeps=40)
    ref, st0 = _solve(ddi, f, c, dict(prm, order_blocks=0))
    extra = dict(use_graph=1) if mode == "graph" else {}
    say("order", mode)
    got, st1 = _solve(ddi, f, c, dict(prm, order_blocks=1, **extra), mode=mode)
    assert np.array_equal(got, ref)
    assert st1["sweeps"] == st0["sweeps"]
