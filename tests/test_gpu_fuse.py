"""Prolongation fused into the first sweep of a level (fuse_prolong = 1)
against the separate prolongation kernel (fuse_prolong = 0), and one fused
sweep against the oracle.

The fused tile load and the separate prolongation kernels evaluate the same
float32 mix (3/4 of the nearer and 1/4 of the farther sample, columns then
rows, one rounding each), so both paths give the same iterates: the solves
must agree bit for bit, in the returned image and in the statistics. The
separate path is itself pinned to the oracle's prolongation and sweep; the
full solves are also checked against the oracle's exact solution, and one
fused first sweep at 1920 x 1080 x 3 against the oracle's prolongation and
sweep on sampled blocks.
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


BENCH = dict(block=64, overlap=4, levels=4, local_iters=16, robin_alpha=0.25, coarse_sweeps=1,
             coarsest_sweeps=1, coarse_local_iters=4, local_tol=0.002, rel_tol=5e-4,
             min_sweeps=2, max_sweeps=30, final_residual=0)

CASES = [
    # the benchmark workload: every level fused
    (3, 2160, 3840, 0.04, "bernoulli", BENCH),
    # odd sizes: the last block row and column start at odd pixels, the
    # coarse grids have a half-covered last row and column
    (3, 1081, 1923, 0.03, "clustered", dict(levels=4, rel_tol=1e-4, max_sweeps=60)),
    (1, 200, 300, 0.05, "bernoulli", dict(levels=3, coarse_sweeps=2, rel_tol=1e-5,
                                          max_sweeps=80)),
    # narrow levels: level 1 is 65 x 39 (blocks narrower than 64 columns)
    (2, 130, 77, 0.1, "bernoulli", dict(levels=2, rel_tol=1e-5, max_sweeps=80)),
    # level 1 has 50 rows: its blocks are not 64 high, only the finest
    # level fuses
    (1, 100, 500, 0.05, "clustered", dict(levels=3, rel_tol=1e-5, max_sweeps=120)),
    # coarse_sweeps = 0: the coarser levels keep the separate prolongation
    (3, 540, 960, 0.04, "bernoulli", dict(levels=4, coarse_sweeps=0, rel_tol=1e-4,
                                          max_sweeps=80)),
    # float64 coarsest level, 5 levels
    (3, 1080, 1920, 0.03, "bernoulli", dict(levels=5, coarse_solver=1, rel_tol=1e-4,
                                            max_sweeps=60)),
    # min_sweeps = 1: the stop test right after the fused sweep
    (3, 270, 480, 0.1, "bernoulli", dict(levels=3, min_sweeps=1, rel_tol=2e-3,
                                         max_sweeps=40)),
]


@pytest.mark.parametrize("C,H,W,d,kind,prm", CASES)
def test_fused_prolongation_matches_separate(ddi, C, H, W, d, kind, prm):
    f, c = synth.make_workload(H, W, C, d, kind, workload=70, index=H + W)
    say("fuse vs separate", C, H, W, d, kind, prm)
    out = {}
    for fuse in (0, 1):
        with ddi.Plan(H, W, C, fuse_prolong=fuse, **prm) as plan:
            u_t, st = plan.solve(dev(f), dev(c), allow_noconv=True)
            u2_t, st2 = plan.solve(dev(f), dev(c), allow_noconv=True)  # other start buffer
        out[fuse] = (host(u_t), st, host(u2_t), st2)
        say("  fuse", fuse, "sweeps", st["sweeps"], "rel", st["rel_residual"])
    u0, s0, v0, t0 = out[0]
    u1, s1, v1, t1 = out[1]
    assert s1["sweeps"] == s0["sweeps"] and s1["rel_residual"] == s0["rel_residual"]
    assert t1["sweeps"] == t0["sweeps"] and t1["rel_residual"] == t0["rel_residual"]
    np.testing.assert_array_equal(u1, u0)
    np.testing.assert_array_equal(v1, v0)
    np.testing.assert_array_equal(u1[:, c == 1], f[:, c == 1])
    if H * W <= 600_000 and s1["converged"]:
        ex = oracle.solve_exact(f.astype(np.float64), c)
        err = float(np.abs(u1 - ex).max())
        say("  max err vs exact", err)
        assert err <= 0.5


def test_fused_prolongation_graph_and_timing(ddi):
    """The fused first sweep inside a captured graph and under timing gives
    the separate path's result."""
    C, H, W = 3, 540, 960
    f, c = synth.make_workload(H, W, C, 0.04, "bernoulli", workload=71)
    say("fuse graph / timing")
    ref = None
    for fuse, extra in [(0, {}), (1, dict(use_graph=1)), (1, dict(timing=1))]:
        with ddi.Plan(H, W, C, fuse_prolong=fuse, **dict(BENCH, **extra)) as plan:
            for _ in range(3):
                u_t, st = plan.solve(dev(f), dev(c))
        u = host(u_t)
        if ref is None:
            ref = (u, st["sweeps"])
        else:
            assert st["sweeps"] == ref[1]
            np.testing.assert_array_equal(u, ref[0])
        if extra.get("timing"):
            # the first sweep's share of the timing statistics
            assert 0 < st["first_sweep_ms"] < st["sweep_ms"]
            assert 0 < st["first_cg_steps"] < st["cg_steps"]
        else:
            assert st["first_sweep_ms"] == 0 and st["first_cg_steps"] == 0



def test_fused_prolongation_in_batches(ddi):
    """Batched solves with per-image fuse_prolong settings (fused and
    separate images in the same launches, images whose finest blocks are
    not 64 rows high, one-level images) equal the separate path bit for
    bit."""
    C = 3
    specs = [(540, 960, 0.04, "bernoulli", 4, 1), (257, 333, 0.05, "clustered", 3, 1),
             (48, 200, 0.1, "bernoulli", 2, 1), (300, 300, 0.03, "bernoulli", 4, 0),
             (130, 77, 0.1, "clustered", 1, 1), (1080, 1920, 0.03, "bernoulli", 5, 1)]
    data = [synth.make_workload(h, w, C, d, k, workload=72, index=i)
            for i, (h, w, d, k, _, _) in enumerate(specs)]
    base = dict(rel_tol=1e-4, max_sweeps=60, final_residual=0)
    say("batch fuse mix")
    res = {}
    for fuse_on in (0, 1):
        prms = [ddi.default_params(levels=L, fuse_prolong=fz if fuse_on else 0, **base)
                for *_, L, fz in specs]
        with ddi.Batch([c.shape for _, c in data], C, params=prms) as b:
            for rep in range(2):  # the second solve starts in the other buffer
                us, st, codes = b.solve([dev(f) for f, _ in data], [dev(c) for _, c in data])
                assert codes == [0] * len(specs)
                res[(fuse_on, rep)] = ([host(u) for u in us], [s["sweeps"] for s in st])
        say("  fuse", fuse_on, "sweeps", res[(fuse_on, 0)][1])
    for rep in range(2):
        u0, s0 = res[(0, rep)]
        u1, s1 = res[(1, rep)]
        assert s1 == s0
        for a, b_ in zip(u1, u0):
            np.testing.assert_array_equal(a, b_)


def test_fused_first_sweep_vs_oracle_1080p(ddi):
    """One fused first finest sweep at 1920 x 1080 x 3, against the oracle
    on sampled blocks (the four corners and four inside). The plan has two
    levels and solves level 1 in float64 (the grid solve: 540 x 960 pixels),
    then runs exactly one finest sweep, whose tile is the prolongation of
    that solution built in the tile load. The oracle takes its own level 1
    (coarsen, exact float64 solve), fine_start and one oras_step.

    Tolerance 3e-3: the sweep's 2e-3 (float32 against float64 CG) plus the
    difference of the two starts, which is the prolongation's 2e-5 and the
    float64 coarse solve's 1e-4 carried through one local solve."""
    C, H, W = 3, 1080, 1920
    f, c = synth.make_workload(H, W, C, 0.04, "bernoulli", workload=15, index=0)
    p = dict(levels=2, coarse_solver=1, coarse_cg_tol=1e-10, coarse_cg_iters=20000,
             block=64, overlap=4, robin_alpha=0.25, local_iters=16, local_tol=0.0,
             min_sweeps=1, max_sweeps=1, rel_tol=0.0, final_residual=0)
    say("fused first sweep vs oracle", C, H, W)
    with ddi.Plan(H, W, C, **p) as plan:
        u_t, st = plan.solve(dev(f), dev(c), allow_noconv=True)
    out = host(u_t)
    assert st["sweeps"] == 1
    fd = f.astype(np.float64)
    fc, cc = oracle.coarsen(fd, c)
    start = oracle.fine_start(oracle.solve_exact(fc, cc), fd, c)
    oy, bh = oracle.block_origins(H, 64, 4)
    ox, bw = oracle.block_origins(W, 64, 4)
    ly, hy = oracle.owner_bounds(oy, bh, H)
    lx, hx = oracle.owner_bounds(ox, bw, W)
    nby, nbx = len(oy), len(ox)
    rng = np.random.default_rng(15)
    picks = [(0, 0), (nby - 1, nbx - 1), (0, nbx - 1), (nby - 1, 0)]
    picks += [(int(rng.integers(nby)), int(rng.integers(nbx))) for _ in range(4)]
    for i, (by, bx) in enumerate(picks):
        ch = i % C
        ref, _ = oracle.oras_step(start[ch], fd[ch], c, 64, 4, 0.25, 16, blocks=[(by, bx)])
        sl = (slice(ly[by], hy[by]), slice(lx[bx], hx[bx]))
        err = float(np.abs(out[ch][sl] - ref[sl]).max())
        say("  block", by, bx, "ch", ch, "dev", err)
        assert err <= 3e-3, (by, bx, err)
    np.testing.assert_array_equal(out[:, c == 1], f[:, c == 1])
