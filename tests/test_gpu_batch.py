"""Batched solve (ddi_batch_*) through the C ABI.

The batch runs the kernels of the single-image path over the work items of
all images at once, so each image's result must equal ddi_solve's on the
same image with the same parameters bit for bit (same arithmetic, same stop
decisions), and stay within 0.5 grey levels of the exact float64 solution
of the oracle.
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


# (H, W, density, kind): odd widths take the generic coarsening and
# prolongation launches beside the batched ones; 1 x 1 has a single level
MIXED = [(96, 160, 0.05, "bernoulli"), (64, 200, 0.08, "clustered"), (130, 70, 0.04, "bernoulli"),
         (33, 47, 0.1, "clustered"), (1, 1, 0.5, "bernoulli"), (200, 256, 0.03, "bernoulli"),
         (7, 300, 0.06, "bernoulli"), (150, 3, 0.2, "clustered")]
SMALL_PRM = dict(block=32, overlap=4, levels=3, local_iters=12, robin_alpha=0.3,
                 coarse_sweeps=2, coarsest_sweeps=3, rel_tol=1e-5, min_sweeps=1,
                 max_sweeps=80, final_residual=1)


def inputs(specs, C, wl=7):
    out = []
    for i, (h, w, d, kind) in enumerate(specs):
        out.append(synth.make_workload(h, w, C, d, kind, workload=wl, index=i))
    return out


def single_solves(ddi, data, C, prms):
    res = []
    for (f, c), p in zip(data, prms):
        h, w = c.shape
        with ddi.Plan(h, w, C, params=p) as plan:
            u, st = plan.solve(dev(f), dev(c))
            res.append((host(u), st))
    return res


@pytest.mark.parametrize("C", [1, 3])
def test_batch_bitwise_equals_single(ddi, C):
    data = inputs(MIXED, C)
    say("batch mixed", C, [s[:2] for s in MIXED])
    p = ddi.default_params(**SMALL_PRM)
    with ddi.Batch([c.shape for _, c in data], C, params=p) as b:
        us, st, codes = b.solve([dev(f) for f, _ in data], [dev(c) for _, c in data])
        assert codes == [0] * len(data)
        ref = single_solves(ddi, data, C, [ddi.default_params(**SMALL_PRM)] * len(data))
        for i, ((f, c), u_t, s, (u_ref, s_ref)) in enumerate(zip(data, us, st, ref)):
            u = host(u_t)
            assert s["sweeps"] == s_ref["sweeps"], i
            assert s["converged"] == 1
            np.testing.assert_array_equal(u, u_ref, err_msg=f"image {i}")
            assert s["rel_residual"] == s_ref["rel_residual"]
            ex = oracle.solve_exact(f.astype(np.float64), c)
            assert np.abs(u - ex).max() <= 0.5, i
            np.testing.assert_array_equal(u[:, c == 1], f[:, c == 1])
        # a second solve on the same batch (start buffers from the first)
        us2, st2, _ = b.solve([dev(f) for f, _ in data], [dev(c) for _, c in data])
        for u1, u2 in zip(us, us2):
            np.testing.assert_array_equal(host(u1), host(u2))


# Deeper pyramids whose level-1 widths are multiples of 8: the single-image
# solve makes levels 2-3 (and 4-5 with six levels) from level 1 in one
# launch, the batch one level per launch, so bit-equal results check that the
# two-level launch equals two one-level ones (ragged heights at every level).
DEEP = [(200, 256, 0.05, "bernoulli"), (131, 208, 0.06, "clustered"), (77, 160, 0.04, "bernoulli")]


@pytest.mark.parametrize("C,levels", [(1, 6), (3, 5), (2, 4)])
def test_batch_equals_single_deep_pyramid(ddi, C, levels):
    data = inputs(DEEP, C, wl=9)
    prm = {**SMALL_PRM, "levels": levels}
    say("batch deep pyramid", C, levels, [s[:2] for s in DEEP])
    with ddi.Batch([c.shape for _, c in data], C, params=ddi.default_params(**prm)) as b:
        us, st, codes = b.solve([dev(f) for f, _ in data], [dev(c) for _, c in data])
    assert codes == [0] * len(data)
    ref = single_solves(ddi, data, C, [ddi.default_params(**prm)] * len(data))
    for i, ((f, c), u_t, s, (u_ref, s_ref)) in enumerate(zip(data, us, st, ref)):
        u = host(u_t)
        assert s["sweeps"] == s_ref["sweeps"], i
        np.testing.assert_array_equal(u, u_ref, err_msg=f"image {i}")
        ex = oracle.solve_exact(f.astype(np.float64), c)
        assert np.abs(u - ex).max() <= 0.5, i


def test_batch_per_image_params(ddi):
    """Per-image parameters: several sweep instances (block heights) share
    each launch."""
    C = 2
    specs = [(120, 200, 0.05, "bernoulli"), (90, 90, 0.07, "clustered"), (64, 128, 0.05, "bernoulli"),
             (40, 36, 0.1, "bernoulli")]
    data = inputs(specs, C, wl=8)
    blocks = [64, 24, 16, 8]
    prms = [ddi.default_params(**{**SMALL_PRM, "block": b, "overlap": min(4, b // 4),
                                  "coarse_block": max(8, b // 2), "local_iters": 8 + i})
            for i, b in enumerate(blocks)]
    say("batch per-image params", blocks)
    with ddi.Batch([c.shape for _, c in data], C, params=prms) as b:
        us, st, codes = b.solve([dev(f) for f, _ in data], [dev(c) for _, c in data])
    assert codes == [0] * len(data)
    ref = single_solves(ddi, data, C, [ddi.default_params(**{**SMALL_PRM, "block": b,
                                                             "overlap": min(4, b // 4),
                                                             "coarse_block": max(8, b // 2),
                                                             "local_iters": 8 + i})
                                       for i, b in enumerate(blocks)])
    for i, (u_t, s, (u_ref, s_ref)) in enumerate(zip(us, st, ref)):
        assert s["sweeps"] == s_ref["sweeps"], i
        np.testing.assert_array_equal(host(u_t), u_ref, err_msg=f"image {i}")


def test_batch_error_images(ddi):
    """An empty mask (singular system) or a mask byte > 1 fails only its own
    image; the others are solved as usual."""
    C = 1
    specs = [(64, 96, 0.05, "bernoulli"), (64, 96, 0.05, "bernoulli"), (48, 80, 0.05, "bernoulli"),
             (40, 40, 0.05, "bernoulli")]
    data = inputs(specs, C, wl=9)
    data[1] = (data[1][0], np.zeros_like(data[1][1]))
    bad = data[2][1].copy()
    bad[5, 7] = 2
    data[2] = (data[2][0], bad)
    say("batch error images")
    p = ddi.default_params(**SMALL_PRM)
    with ddi.Batch([c.shape for _, c in data], C, params=p) as b:
        with pytest.raises(ddi.DDIError) as ei:
            b.solve([dev(f) for f, _ in data], [dev(c) for _, c in data])
        assert ei.value.code == ddi.DDI_ESINGULAR
        # the per-image codes, through the raw entry point
        import ctypes
        n = len(data)
        fs = [dev(f) for f, _ in data]
        cs = [dev(c) for _, c in data]
        us = [torch.empty_like(f) for f in fs]
        P = ctypes.c_void_p * n
        status = (ctypes.c_int * n)()
        st = (ddi.Stats * n)()
        rc = ddi.lib().ddi_batch_solve(b._h, P(*[t.data_ptr() for t in fs]),
                                       P(*[t.data_ptr() for t in cs]),
                                       P(*[t.data_ptr() for t in us]), st, status)
        assert rc == ddi.DDI_ESINGULAR
        assert list(status) == [0, ddi.DDI_ESINGULAR, ddi.DDI_EINVAL, 0]
        for i in (0, 3):
            f, c = data[i]
            ex = oracle.solve_exact(f.astype(np.float64), c)
            assert np.abs(host(us[i]) - ex).max() <= 0.5


def test_batch_create_errors(ddi):
    p = ddi.default_params()
    q = ddi.default_params(max_sweeps=10)
    with pytest.raises(ddi.DDIError):
        ddi.Batch([(10, 10), (0, 5)], 1, params=p)
    with pytest.raises(ddi.DDIError):
        ddi.Batch([(10, 10), (12, 5)], 1, params=[p, q])  # stop schedules differ
    with pytest.raises(ddi.DDIError):
        ddi.Batch([(10, 10)], 5, params=p)  # channels > 4


def test_batch_recipe_sample_vs_oracle(ddi):
    """Eight images of the batch recipe at their real sizes (4K included),
    solved with the benchmark's batch parameters: every image within 0.5 grey
    levels of the exact solution, u = f on the mask."""
    import bench
    C = 3
    specs = synth.batch_specs(n=8, seed=3)
    data = [synth.make_workload(s["h"], s["w"], C, s["density"], s["kind"], workload=3,
                                index=s["index"]) for s in specs]
    say("batch recipe sample", [(s["h"], s["w"], s["kind"], round(s["density"], 3)) for s in specs])
    prms = bench.batch_params(specs)
    with ddi.Batch([(s["h"], s["w"]) for s in specs], C, params=prms) as b:
        us, st, codes = b.solve([dev(f) for f, _ in data], [dev(c) for _, c in data])
    assert codes == [0] * len(data)
    for i, ((f, c), u_t) in enumerate(zip(data, us)):
        u = host(u_t)
        ex = oracle.solve_exact(f.astype(np.float64), c)
        err = np.abs(u - ex).max()
        say("image", i, specs[i]["h"], specs[i]["w"], specs[i]["kind"], "err", float(err),
            "sweeps", st[i]["sweeps"])
        assert err <= 0.5, i
        np.testing.assert_array_equal(u[:, c == 1], f[:, c == 1])


def test_batch_per_image_min_sweeps(ddi):
    """Images with different min_sweeps (a per-class sweep floor) share one
    batch: the stop tests start at the smallest, an image's test passes only
    from its own floor on, and each image equals its single-image solve bit
    for bit (same sweep count)."""
    C = 3
    data = inputs(MIXED[:4], C, wl=8)
    floors = [1, 3, 5, 2]
    prms = [ddi.default_params(**dict(SMALL_PRM, rel_tol=1e-2, min_sweeps=m)) for m in floors]
    say("batch per-image min_sweeps", floors)
    with ddi.Batch([c.shape for _, c in data], C, params=prms) as b:
        us, st, codes = b.solve([dev(f) for f, _ in data], [dev(c) for _, c in data])
        # a second solve starts from each image's previous sweep count: the
        # first batch of finest sweeps stops where the images holding three
        # quarters of the pixels converged last time, and the others go on
        # in tables of their own after a host check
        us2, st2, codes2 = b.solve([dev(f) for f, _ in data], [dev(c) for _, c in data])
    assert codes == [0] * len(data) and codes2 == [0] * len(data)
    ref = single_solves(ddi, data, C, prms)
    for i, (u_t, s, (u_ref, s_ref), m) in enumerate(zip(us, st, ref, floors)):
        assert s["sweeps"] == s_ref["sweeps"] and s["sweeps"] >= m, (i, s["sweeps"], m)
        np.testing.assert_array_equal(host(u_t), u_ref)
    for i, (u_t, s, (u_ref, s_ref)) in enumerate(zip(us2, st2, ref)):
        assert s["sweeps"] == s_ref["sweeps"], (i, s["sweeps"])
        np.testing.assert_array_equal(host(u_t), u_ref)
    # a loose tolerance every image meets early: each stops at its own floor
    assert [s["sweeps"] for s in st][1:3] == [3, 5]
