"""HIP path vs the CPU oracle, element by element, through the C ABI.

Tolerances (grey levels, values in [0, 255]):
  residual      float32 stencil of float32 data vs the float64 definition:
                each of the four differences rounds once (<= 2^-17 * 255),
                sums of them twice more -> 1e-4 absolute.
  coarsen       bit-exact: the kernel sums <= 4 float32 values in float64
                (exact) and divides once, as the float64 oracle does.
  prolong       bilinear weights 3/4 and 1/4 per axis. The kernel mixes in
                float32, columns then rows, each mix one rounding of the
                exact weighted sum (the 1/4 product is exact, the 3/4 one
                fused): its result is within 0.5 ulp of the result plus
                0.5 ulp of the row values it mixes, i.e. within 1.6e-5 of
                the exact value for grey values below 256; the float64
                oracle is within 0.5 ulp (7.6e-6). The two float32 results
                differ by at most 2.3e-5 in exact terms, which in a float32
                binade below 256 is at most one ulp of 1.5e-5 (two of 7.6e-6
                below 128) -> 2e-5 absolute.
  ORAS sweep    k float32 CG steps vs float64 ones: 2e-3 absolute (the
                local corrections are at most a few hundred grey levels and
                CG on these well-conditioned blocks loses no more than a few
                float32 ulps per step).
  full solve    0.5 grey levels max-abs against the exact float64 solution,
                the accuracy bar of the solver; u = f bit for bit on the mask.
"""
import sys

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


def workload(C, H, W, d=0.05, kind="bernoulli", wl=0, idx=0):
    f, c = synth.make_workload(H, W, C, d, kind, workload=wl, index=idx)
    return f, c


# ---------------------------------------------------------------------------
# residual r = b - A u (eq. 7)
# ---------------------------------------------------------------------------

RES_SHAPES = [(1, 1, 1), (1, 17, 5), (3, 67, 131), (1, 256, 256), (2, 33, 64),
              (1, 130, 1), (1, 1, 130), (4, 70, 200)]


@pytest.mark.parametrize("C,H,W", RES_SHAPES)
def test_residual_parity(ddi, C, H, W):
    f, c = workload(C, H, W, 0.1, wl=1)
    rng = np.random.default_rng(H * 1000 + W)
    u = rng.uniform(0, 255, (C, H, W)).astype(np.float32)
    say("residual", C, H, W)
    r_t, rsq = ddi.residual(dev(f), dev(c), dev(u), r=dev(np.zeros_like(u)))
    r = host(r_t)
    ref = oracle.residual(f.astype(np.float64), c, u.astype(np.float64))
    np.testing.assert_allclose(r, ref, atol=1e-4, rtol=0)
    ref_sq = (ref ** 2).reshape(C, -1).sum(1)
    np.testing.assert_allclose(rsq, ref_sq, rtol=1e-5, atol=1e-6)


# ---------------------------------------------------------------------------
# coarsening and prolongation (Sec. 4)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("C,H,W,d", [(3, 256, 256, 0.05), (1, 67, 131, 0.2), (2, 5, 3, 0.5),
                                     (1, 1, 1, 1.0), (4, 100, 101, 0.03), (1, 9, 1, 0.3)])
def test_coarsen_bit_exact(ddi, C, H, W, d):
    f, c = workload(C, H, W, d, wl=2)
    say("coarsen", C, H, W)
    fc, cc = ddi.coarsen(dev(f), dev(c))
    ref_f, ref_c = oracle.coarsen(f.astype(np.float64), c)
    assert np.array_equal(host(cc), ref_c)
    assert np.array_equal(host(fc), ref_f.astype(np.float32))


@pytest.mark.parametrize("C,H,W", [(1, 64, 64), (3, 67, 131), (2, 6, 9), (1, 1, 7), (1, 130, 2)])
def test_prolong_parity(ddi, C, H, W):
    f, c = workload(C, H, W, 0.1, wl=3)
    hc, wc = (H + 1) // 2, (W + 1) // 2
    uc = np.random.default_rng(7).uniform(0, 255, (C, hc, wc)).astype(np.float32)
    say("prolong", C, H, W)
    u = host(ddi.prolong(dev(uc), dev(f), dev(c)))
    ref = oracle.fine_start(uc.astype(np.float64), f.astype(np.float64), c)
    np.testing.assert_allclose(u, ref.astype(np.float32), atol=2e-5, rtol=0)
    assert np.array_equal(u[:, c == 1], f[:, c == 1])


# ---------------------------------------------------------------------------
# one ORAS sweep (Sec. 3 eqs. 7-9)
# ---------------------------------------------------------------------------

SWEEP_CASES = [
    # C, H, W, S, o, alpha, k
    (1, 64, 64, 64, 4, 1.0, 16),      # one block: RAS = local solve
    (1, 200, 300, 64, 4, 0.25, 16),   # several 64-row blocks, clamped last ones
    (3, 130, 100, 32, 6, 0.5, 8),     # the paper's block size and overlap
    (1, 50, 70, 16, 4, 1.0, 4),
    (2, 40, 40, 8, 2, 0.25, 3),
    (1, 40, 120, 64, 4, 0.25, 16),    # 40-row blocks in 64-row registers
    (1, 20, 90, 32, 4, 0.5, 12),      # 20-row blocks in 32-row registers
    (1, 5, 70, 16, 2, 1.0, 6),        # 5-row blocks in 8-row registers
    (1, 64, 30, 64, 4, 0.25, 10),     # 30-wide blocks: idle lanes
    (1, 100, 100, 64, 0, 0.25, 5),    # no overlap
    (1, 131, 67, 64, 9, 0.75, 1),     # one CG step
]


@pytest.mark.parametrize("C,H,W,S,o,alpha,k", SWEEP_CASES)
@pytest.mark.parametrize("start", ["coarse", "near"])
def test_oras_sweep_parity(ddi, C, H, W, S, o, alpha, k, start):
    f, c = workload(C, H, W, 0.06, wl=4, idx=H + W)
    f64 = f.astype(np.float64)
    if start == "coarse":
        # the kind of start the multilevel scheme hands to a level
        fc, cc = oracle.coarsen(f64, c)
        uc = np.where(cc == 1, fc, fc[:, cc == 1].mean(axis=1)[:, None, None])
        u0 = oracle.fine_start(uc, f64, c).astype(np.float32)
    else:
        ex = oracle.solve_exact(f64, c)
        noise = np.random.default_rng(5).normal(0, 0.5, ex.shape)
        u0 = np.where(c == 1, f64, ex + noise).astype(np.float32)
    say("sweep", C, H, W, S, o, alpha, k, start)
    out_t, rsq = ddi.oras_sweep(dev(u0), dev(c), S, o, alpha, k)
    out = host(out_t)
    for ch in range(C):
        ref, ref_rsq = oracle.oras_step(u0[ch].astype(np.float64), f64[ch], c, S, o, alpha, k)
        err = np.abs(out[ch] - ref).max()
        corr = np.abs(ref - u0[ch]).max()
        assert err <= 2e-3, (ch, err, corr)
        assert rsq[ch] == pytest.approx(ref_rsq, rel=1e-5, abs=1e-8)
    assert np.array_equal(out[:, c == 1], u0[:, c == 1])


def test_sweep_sampled_blocks_at_4k(ddi):
    """Full 4K RGB shape in the solver's launch configuration (S = 64,
    o = 4): blocks sampled from the grid against the oracle, one by one."""
    C, H, W = 3, 2160, 3840
    f, c = synth.make_workload(H, W, C, 0.04, workload=1)
    rng = np.random.default_rng(11)
    u0 = np.where(c == 1, f, f.mean()).astype(np.float32)
    say("sweep 4k sampled")
    out = host(ddi.oras_sweep(dev(u0), dev(c), 64, 4, 0.25, 16)[0])
    nby = len(oracle.block_origins(H, 64, 4)[0])
    nbx = len(oracle.block_origins(W, 64, 4)[0])
    picks = [(0, 0), (nby - 1, nbx - 1), (0, nbx - 1), (nby - 1, 0)]
    picks += [(int(rng.integers(nby)), int(rng.integers(nbx))) for _ in range(4)]
    oy, bh = oracle.block_origins(H, 64, 4)
    ox, bw = oracle.block_origins(W, 64, 4)
    ly, hy = oracle.owner_bounds(oy, bh, H)
    lx, hx = oracle.owner_bounds(ox, bw, W)
    for by, bx in picks:
        ch = (by + bx) % C
        ref, _ = oracle.oras_step(u0[ch].astype(np.float64), f[ch].astype(np.float64), c,
                                  64, 4, 0.25, 16, blocks=[(by, bx)])
        sl = (slice(ly[by], hy[by]), slice(lx[bx], hx[bx]))
        err = np.abs(out[ch][sl] - ref[sl]).max()
        assert err <= 2e-3, (by, bx, err)


def test_large_image_sampled_blocks_and_solve(ddi):
    """8192 x 8192 x 2 (channel planes of 2^26 pixels, so 32-bit offsets
    reach 2^27 across both planes of a buffer): one full-size ORAS sweep
    against the oracle on sampled blocks (the four corners, where the
    last blocks are clamped, and two inside), then a multilevel solve that
    must converge, keep u = f on the mask bit for bit and stay within the
    range of the known values (discrete maximum principle, to the stop
    tolerance)."""
    C, H, W = 2, 8192, 8192
    rng = np.random.default_rng(12)
    yy = np.arange(H, dtype=np.float32)[:, None]
    xx = np.arange(W, dtype=np.float32)[None, :]
    f = np.stack([128.0 + 100.0 * np.sin(xx / (400.0 + 90 * k)) * np.cos(yy / (650.0 - 70 * k))
                  for k in range(C)]).astype(np.float32)
    c = (rng.random((H, W)) < 0.04).astype(np.uint8)
    say("large image", C, H, W)
    fd, cd = dev(f), dev(c)
    u0 = np.where(c == 1, f, np.float32(128.0)).astype(np.float32)
    out = host(ddi.oras_sweep(dev(u0), cd, 64, 4, 0.25, 16)[0])
    oy, bh = oracle.block_origins(H, 64, 4)
    ox, bw = oracle.block_origins(W, 64, 4)
    ly, hy = oracle.owner_bounds(oy, bh, H)
    lx, hx = oracle.owner_bounds(ox, bw, W)
    nby, nbx = len(oy), len(ox)
    picks = [(0, 0), (nby - 1, nbx - 1), (0, nbx - 1), (nby - 1, 0)]
    picks += [(int(rng.integers(nby)), int(rng.integers(nbx))) for _ in range(2)]
    for i, (by, bx) in enumerate(picks):
        ch = i % C
        ref, _ = oracle.oras_step(u0[ch].astype(np.float64), f[ch].astype(np.float64), c,
                                  64, 4, 0.25, 16, blocks=[(by, bx)])
        sl = (slice(ly[by], hy[by]), slice(lx[bx], hx[bx]))
        err = float(np.abs(out[ch][sl] - ref[sl]).max())
        say("  block", by, bx, "ch", ch, "dev", err)
        assert err <= 2e-3, (by, bx, err)
    del out
    with ddi.Plan(H, W, C, levels=5, rel_tol=1e-4, max_sweeps=60) as plan:
        u_t, st = plan.solve(fd, cd)
    u = host(u_t)
    say("  solve sweeps", st["sweeps"], "rel", st["rel_residual"])
    assert st["converged"] == 1
    np.testing.assert_array_equal(u[:, c == 1], f[:, c == 1])
    for ch in range(C):
        known = f[ch][c == 1]
        assert u[ch].min() >= known.min() - 0.5 and u[ch].max() <= known.max() + 0.5


# ---------------------------------------------------------------------------
# full multilevel solve vs the exact solution (Sec. 2-4)
# ---------------------------------------------------------------------------

def solve(ddi, f, c, **prm):
    C, H, W = f.shape
    with ddi.Plan(H, W, C, **prm) as plan:
        u, st = plan.solve(dev(f), dev(c))
        return host(u), st


def check_solution(f, c, u, bound=0.5):
    ex = oracle.solve_exact(f.astype(np.float64), c)
    err = np.abs(u - ex).max()
    assert np.array_equal(u[:, c == 1], f[:, c == 1]), "known pixels changed"
    assert err <= bound, err
    return err


def test_config0_256_grey(ddi):
    """256 x 256 grey, 5 % Bernoulli, two levels, overlap 4, stop at relative
    residual 1e-6 (64-pixel blocks: the on-chip block limit; 5 x 5 blocks)."""
    f, c = synth.make_workload(256, 256, 1, 0.05, workload=0)
    say("config0")
    u, st = solve(ddi, f, c, levels=2, block=64, overlap=4, rel_tol=1e-6)
    assert st["converged"] == 1 and st["rel_residual"] <= 1e-6
    rr = oracle.rel_residual(f.astype(np.float64), c, u.astype(np.float64))
    assert rr <= 2e-6, rr
    err = check_solution(f, c, u)
    assert err < 0.01, err


@pytest.mark.parametrize("C,H,W,d,kind,prm", [
    (3, 67, 131, 0.05, "bernoulli", {}),
    (1, 1, 1, 1.0, "bernoulli", {}),
    (1, 1, 200, 0.05, "bernoulli", {}),
    (1, 200, 1, 0.05, "bernoulli", {}),
    (2, 128, 96, 0.03, "clustered", {}),
    (1, 300, 500, 0.02, "bernoulli", {"block": 32, "overlap": 6, "local_iters": 8}),
    (3, 257, 255, 0.08, "clustered", {"levels": 3, "robin_alpha": 1.0}),
    (1, 64, 64, 0.1, "bernoulli", {"levels": 1}),
    # tall and narrow: more coarsening workgroups than coarse pixels / 256
    (1, 4096, 256, 0.05, "bernoulli", {"levels": 2}),
])
def test_solve_parity(ddi, C, H, W, d, kind, prm):
    f, c = workload(C, H, W, d, kind, wl=5, idx=H + W)
    say("solve", C, H, W, d, kind, prm)
    u, st = solve(ddi, f, c, rel_tol=1e-6, max_sweeps=200, **prm)
    assert st["converged"] == 1
    check_solution(f, c, u, bound=0.05)


def test_constant_data_reproduced(ddi):
    C, H, W = 2, 90, 150
    c = synth.make_mask(H, W, 0.03, "bernoulli", 3)
    f = np.full((C, H, W), 77.25, dtype=np.float32)
    u, st = solve(ddi, f, c, rel_tol=1e-7, max_sweeps=100)
    assert np.abs(u - 77.25).max() < 1e-4


def test_deterministic(ddi):
    f, c = workload(3, 150, 170, 0.04, wl=6)
    say("determinism")
    u1, _ = solve(ddi, f, c)
    u2, _ = solve(ddi, f, c)
    assert np.array_equal(u1, u2)


def test_error_paths(ddi):
    C, H, W = 1, 32, 32
    f = np.ones((C, H, W), np.float32)
    with ddi.Plan(H, W, C) as plan:
        say("empty mask")
        with pytest.raises(ddi.DDIError) as e:
            plan.solve(dev(f), dev(np.zeros((H, W), np.uint8)))
        assert e.value.code == ddi.DDI_ESINGULAR
        say("bad mask byte")
        bad = np.zeros((H, W), np.uint8)
        bad[3, 4] = 2
        with pytest.raises(ddi.DDIError) as e:
            plan.solve(dev(f), dev(bad))
        assert e.value.code == ddi.DDI_EINVAL
    f, c = workload(1, 128, 128, 0.02, wl=7)
    say("no convergence")
    with ddi.Plan(128, 128, 1, rel_tol=1e-12, min_sweeps=1, max_sweeps=1, levels=1) as plan:
        u, st = plan.solve(dev(f), dev(c), allow_noconv=True)
        assert st["converged"] == 0 and st["sweeps"] == 1
        with pytest.raises(ddi.DDIError) as e:
            plan.solve(dev(f), dev(c))
        assert e.value.code == ddi.DDI_ENOCONV


def test_aliased_buffers_rejected(ddi):
    """An output sharing memory with an input (u with f or c; in a batch also
    with another image's buffers) is DDI_EINVAL before any work is queued,
    and the plan still solves afterwards."""
    C, H, W = 2, 40, 56
    f, c = workload(C, H, W, 0.05, wl=7, idx=3)
    n = C * H * W
    buf = torch.zeros(2 * n, dtype=torch.float32, device="cuda")
    buf[:n] = dev(f).reshape(-1)
    fd = buf[:n].view(C, H, W)
    cd = dev(c)
    cases = {"u is f": fd, "u starts inside f": buf[n // 2:n // 2 + n].view(C, H, W),
             "u ends inside f": torch.zeros(2 * n, dtype=torch.float32, device="cuda")}
    with ddi.Plan(H, W, C) as plan:
        for name, u in cases.items():
            if name == "u ends inside f":
                # f placed in the upper half of a buffer whose lower part is u
                u[n // 2:n // 2 + n] = fd.reshape(-1)
                fo = u[n // 2:n // 2 + n].view(C, H, W)
                uo = u[:n].view(C, H, W)
                args = (fo, cd, uo)
            else:
                args = (fd, cd, u)
            say("alias", name)
            with pytest.raises(ddi.DDIError) as e:
                plan.solve(*args)
            assert e.value.code == ddi.DDI_EINVAL
            with pytest.raises(ddi.DDIError) as e:
                plan.solve_async(*args)
            assert e.value.code == ddi.DDI_EINVAL
        say("u overlapping c")
        # c in the first bytes of a float32 buffer whose first n floats are u
        fbuf = torch.zeros(n + H * W, dtype=torch.float32, device="cuda")
        cview = fbuf.view(torch.uint8)[:H * W].view(H, W)
        cview.copy_(cd)
        with pytest.raises(ddi.DDIError) as e:
            plan.solve(fd, cview, fbuf[:n].view(C, H, W))
        assert e.value.code == ddi.DDI_EINVAL
        # nothing was queued: a proper solve still works
        u, _ = plan.solve(fd, cd)
        ex = oracle.solve_exact(f.astype(np.float64), c)
        assert np.abs(host(u) - ex).max() <= 0.5
    say("batch: one image's output over another image's input")
    f2, c2 = workload(C, 24, 32, 0.05, wl=7, idx=4)
    with ddi.Batch([(H, W), (24, 32)], C) as b:
        f2d = dev(f2)
        u1 = torch.empty_like(f2d)
        with pytest.raises(ddi.DDIError) as e:
            b.solve([fd, f2d], [cd, dev(c2)], [torch.empty_like(fd), f2d])
        assert e.value.code == ddi.DDI_EINVAL
        with pytest.raises(ddi.DDIError) as e:
            big = torch.empty(n + C * 24 * 32, dtype=torch.float32, device="cuda")
            b.solve([fd, f2d], [cd, dev(c2)],
                    [big[:n].view(C, H, W), big[n - 8:n - 8 + C * 24 * 32].view(C, 24, 32)])
        assert e.value.code == ddi.DDI_EINVAL
        us, _, _ = b.solve([fd, f2d], [cd, dev(c2)], [torch.empty_like(fd), u1])
        assert np.abs(host(us[0]) - oracle.solve_exact(f.astype(np.float64), c)).max() <= 0.5


@pytest.mark.slow
def test_config1_4k_rgb_full_size(ddi):
    """4K RGB, 4 % Bernoulli shared mask, 64 x 64 blocks, overlap 4, four
    levels (coarsest 1/8): the benchmark's workload and parameters."""
    import bench
    C, H, W = 3, 2160, 3840
    f, c = synth.make_workload(H, W, C, 0.04, workload=1)
    say("config1 4K solve")
    u, st = solve(ddi, f, c, **bench.solver_params())
    say("config1 oracle", st)
    err = check_solution(f, c, u)
    say("config1 max err", err)


def test_graph_replays_match_eager(ddi):
    """use_graph = 1 captures the solve into a HIP graph and replays it; every
    replay (with eager work and synchronisations in between) must equal the
    eager solve bit for bit, also after a re-capture for other buffers and
    when the graph's first batch of sweeps is not enough."""
    f, c = workload(3, 300, 400, 0.04, wl=8)
    ft, ct = dev(f), dev(c)
    say("graph: eager reference")
    with ddi.Plan(300, 400, 3, levels=3) as plan:
        ref, st_ref = plan.solve(ft, ct)
        ref = host(ref)
    with ddi.Plan(300, 400, 3, levels=3, use_graph=1) as plan:
        u1 = torch.empty_like(ft)
        u2 = torch.empty_like(ft)
        for rep in range(4):
            say("graph replay", rep)
            out = u1 if rep < 3 else u2  # the last one re-captures
            _, st = plan.solve(ft, ct, out)
            junk = torch.randn(1 << 20, device="cuda").sum()  # eager work in between
            torch.cuda.synchronize()
            assert np.array_equal(host(out), ref), rep
            assert st["sweeps"] == st_ref["sweeps"]
        # a harder input needs more sweeps than the captured batch
        f2, c2 = workload(3, 300, 400, 0.02, "clustered", wl=9)
        say("graph: longer solve")
        out, st2 = plan.solve(dev(f2), dev(c2), u1)
        with ddi.Plan(300, 400, 3, levels=3) as p2:
            ref2, _ = p2.solve(dev(f2), dev(c2))
        assert np.array_equal(host(out), host(ref2))
