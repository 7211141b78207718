"""Finest-level sweeps that skip redundant work (skip_unchanged = 1)
against sweeps that do all of it (skip_unchanged = 0).

A block that the previous sweep left unchanged keeps its values in both
ping-pong buffers; if it runs no CG step again its write-back is skipped,
and if its whole 3 x 3 neighbourhood was left unchanged its input tile is
the previous one, so the block is skipped whole. Nothing the solver computes
may differ: the solves must agree bit for bit, in the returned image, the
sweep count and the residual. The cases run many sweeps with the local stop
on (so that most late blocks run no CG step and skipping is exercised), on
grids whose last block is shifted back to the border, through the
synchronous, asynchronous and graph paths; the timing counters show that
blocks were skipped. Converged results are also checked against the
oracle's exact solution.
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


# the benchmark's solver settings
BENCH = dict(block=64, overlap=4, levels=4, local_iters=16, robin_alpha=0.25, coarse_sweeps=1,
             coarsest_sweeps=1, coarse_local_iters=8, local_tol=0.004, rel_tol=5e-4,
             min_sweeps=3, max_sweeps=30, final_residual=0)

CASES = [
    # the benchmark workload (three sweeps: the third one skips)
    (3, 2160, 3840, 0.04, "bernoulli", BENCH),
    # many sweeps to a tight tolerance: most late blocks are skipped
    (3, 1080, 1920, 0.04, "bernoulli", dict(BENCH, rel_tol=2e-6, max_sweeps=40)),
    # clustered mask, odd sizes (last block row and column shifted back)
    (3, 1081, 1923, 0.03, "clustered", dict(BENCH, rel_tol=1e-5, max_sweeps=60)),
    # one level, one channel, overlap 8, single check every second sweep
    (1, 700, 1000, 0.05, "bernoulli", dict(levels=1, overlap=8, local_tol=0.003,
                                           rel_tol=1e-5, max_sweeps=80, check_every=2,
                                           final_residual=1)),
    # two channels, no local stop: blocks always run CG while r != 0
    (2, 300, 500, 0.1, "bernoulli", dict(levels=2, rel_tol=1e-6, max_sweeps=60)),
    # four channels (the most a plan takes)
    (4, 540, 960, 0.04, "clustered", dict(BENCH, rel_tol=1e-5, max_sweeps=40)),
    # overlap 15 on a 3840-wide level: the last block's tile reaches two
    # blocks back, so the plan keeps no flags and skips nothing
    (3, 256, 3840, 0.04, "bernoulli", dict(BENCH, overlap=15, rel_tol=1e-5, max_sweeps=40)),
]


@pytest.mark.parametrize("C,H,W,d,kind,prm", CASES)
def test_skip_matches_full_sweeps(ddi, C, H, W, d, kind, prm):
    f, c = synth.make_workload(H, W, C, d, kind, workload=75, index=H + W)
    say("skip vs full", C, H, W, d, kind, prm)
    out = {}
    for skip in (0, 1):
        with ddi.Plan(H, W, C, skip_unchanged=skip, **prm) as plan:
            u_t, st = plan.solve(dev(f), dev(c), allow_noconv=True)
            u2_t, st2 = plan.solve(dev(f), dev(c), allow_noconv=True)  # other start buffer
        out[skip] = (host(u_t), st, host(u2_t), st2)
        say("  skip", skip, "sweeps", st["sweeps"], "rel", st["rel_residual"])
    u0, s0, v0, t0 = out[0]
    u1, s1, v1, t1 = out[1]
    assert s1["sweeps"] == s0["sweeps"] and s1["rel_residual"] == s0["rel_residual"]
    assert t1["sweeps"] == t0["sweeps"] and t1["rel_residual"] == t0["rel_residual"]
    np.testing.assert_array_equal(u1, u0)
    np.testing.assert_array_equal(v1, v0)
    np.testing.assert_array_equal(u1[:, c == 1], f[:, c == 1])
    if H * W <= 800_000 and s1["converged"]:
        ex = oracle.solve_exact(f.astype(np.float64), c)
        err = float(np.abs(u1 - ex).max())
        say("  max err vs exact", err)
        assert err <= 0.5


def test_skip_counters_and_paths(ddi):
    """With timing the plan counts the blocks it skipped; the asynchronous
    solve and graph replays (several, with eager solves between them) equal
    the synchronous solve without skipping."""
    C, H, W = 3, 1080, 1920
    f, c = synth.make_workload(H, W, C, 0.04, "bernoulli", workload=76)
    # the local stop's residual floor lies above 2e-6: every solve runs all
    # 40 sweeps
    prm = dict(BENCH, rel_tol=2e-6, max_sweeps=40)
    say("skip counters / async / graph")
    fd, cd = dev(f), dev(c)
    with ddi.Plan(H, W, C, skip_unchanged=0, **prm) as plan:
        ref_t, ref_st = plan.solve(fd, cd, allow_noconv=True)
        ref = host(ref_t)
    nblk = ddi.block_count(H, 64, 4) * ddi.block_count(W, 64, 4) * C
    for skip in (0, 1):
        with ddi.Plan(H, W, C, skip_unchanged=skip, timing=1, **prm) as plan:
            u_t, st = plan.solve(fd, cd, allow_noconv=True)
        np.testing.assert_array_equal(host(u_t), ref)
        say("  timing skip", skip, "skipped", st["skipped_blocks"], "unwritten",
            st["unwritten_blocks"], "sweeps", st["sweeps"])
        if skip:
            # skips only from the third sweep on
            assert 0 < st["skipped_blocks"] + st["unwritten_blocks"] <= (st["sweeps"] - 2) * nblk
            assert st["skipped_blocks"] > 0 and st["unwritten_blocks"] > 0
        else:
            assert st["skipped_blocks"] == 0 and st["unwritten_blocks"] == 0
    with ddi.Plan(H, W, C, skip_unchanged=1, **prm) as plan:
        u = torch.empty_like(fd)
        for _ in range(2):
            plan.solve_async(fd, cd, u)
            _, st = plan.wait(allow_noconv=True)
            assert st["sweeps"] == ref_st["sweeps"]
            np.testing.assert_array_equal(host(u), ref)
    with ddi.Plan(H, W, C, skip_unchanged=1, use_graph=1, **prm) as plan:
        for rep in range(3):
            u_t, st = plan.solve(fd, cd, allow_noconv=True)
            assert st["sweeps"] == ref_st["sweeps"]
            np.testing.assert_array_equal(host(u_t), ref)
            # eager work of the program's own between the replays
            torch.cuda.synchronize()
            (fd * 0.5).sum().item()


def test_skip_ignored_where_it_does_not_apply(ddi):
    """Plans whose finest blocks are not 64 rows high, bfloat16 storage and
    the comparator methods run as before with skip_unchanged = 1."""
    C, H, W = 3, 270, 480
    f, c = synth.make_workload(H, W, C, 0.05, "bernoulli", workload=77)
    fd, cd = dev(f), dev(c)
    for extra in (dict(block=32), dict(storage=1, rel_tol=3e-5, coarse_solver=1),
                  dict(method=1), dict(method=2)):
        prm = dict(levels=3, rel_tol=1e-4, max_sweeps=60)
        prm.update(extra)
        say("skip ignored", extra)
        res = []
        for skip in (0, 1):
            with ddi.Plan(H, W, C, skip_unchanged=skip, **prm) as plan:
                u_t, st = plan.solve(fd, cd, allow_noconv=True)
                res.append((host(u_t), st["sweeps"]))
        assert res[0][1] == res[1][1]
        np.testing.assert_array_equal(res[0][0], res[1][0])


def test_skip_in_batches(ddi):
    """Batched solves (uneven sizes, mixed mask kinds, images that converge
    at different sweeps and drop out of the tables, an image whose finest
    blocks are not 64 rows high) equal the batch without skipping bit for
    bit, in images and sweep counts; with timing the skipped blocks are
    counted per image."""
    C = 3
    specs = [(540, 960, 0.04, "bernoulli"), (1081, 1923, 0.03, "clustered"),
             (720, 1280, 0.08, "bernoulli"), (48, 200, 0.1, "bernoulli"),
             (480, 640, 0.02, "clustered")]
    data = [synth.make_workload(h, w, C, d, k, workload=78, index=i)
            for i, (h, w, d, k) in enumerate(specs)]
    # a tolerance every image reaches (the batch reports counters for
    # converged images), after 3 to 10 sweeps
    base = dict(BENCH, rel_tol=3e-4, max_sweeps=40)
    say("skip in batches")
    res = {}
    for skip in (0, 1):
        for timing in (0, 1):
            prms = [ddi.default_params(skip_unchanged=skip, timing=timing, **base)
                    for _ in specs]
            with ddi.Batch([c.shape for _, c in data], C, params=prms) as b:
                for rep in range(2):  # the second solve starts in the other buffer
                    us, st, codes = b.solve([dev(f) for f, _ in data],
                                            [dev(c) for _, c in data], allow_noconv=True)
                    res[(skip, timing, rep)] = ([host(u) for u in us], st)
            say("  skip", skip, "timing", timing, "sweeps", [s["sweeps"] for s in st],
                "skipped", [s["skipped_blocks"] for s in st])
    for key, (us, st) in res.items():
        u0, s0 = res[(0, 0, key[2])]
        assert [s["sweeps"] for s in st] == [s["sweeps"] for s in s0]
        for a, b_ in zip(us, u0):
            np.testing.assert_array_equal(a, b_)
    st = res[(1, 1, 0)][1]
    assert sum(s["skipped_blocks"] for s in st) > 0
    assert sum(s["unwritten_blocks"] for s in st) > 0
    assert st[3]["skipped_blocks"] == 0 and st[3]["unwritten_blocks"] == 0  # 48 rows
    for s in res[(0, 1, 0)][1]:
        assert s["skipped_blocks"] == 0 and s["unwritten_blocks"] == 0
