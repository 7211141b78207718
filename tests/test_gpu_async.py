"""ddi_solve_async / ddi_solve_wait: several plans in flight on one stream
give the same results as ddi_solve, bit for bit, including solves that
need more sweeps than their first batch (the continuation is enqueued by the
wait behind the other plans' work)."""
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


PRM = dict(block=32, overlap=4, levels=4, local_iters=12, rel_tol=1e-5, max_sweeps=200,
           final_residual=0)


@pytest.mark.parametrize("timing", [0, 1])
def test_async_pipeline_matches_sync(ddi, timing):
    C, H, W = 3, 160, 224
    frames = [synth.make_workload(H, W, C, d, k, workload=50, index=i)
              for i, (d, k) in enumerate([(0.05, "bernoulli"), (0.02, "clustered"),
                                          (0.08, "bernoulli"), (0.03, "clustered")])]
    say("async pipeline", len(frames), "frames, timing", timing)
    ref = []
    with ddi.Plan(H, W, C, **PRM) as p:
        for f, c in frames:
            u, st = p.solve(dev(f), dev(c))
            say("  sync sweeps", st["sweeps"])
            ref.append((host(u), st["sweeps"]))
    plans = [ddi.Plan(H, W, C, timing=timing, **PRM) for _ in range(2)]
    fs = [(dev(f), dev(c)) for f, c in frames]
    outs = [torch.empty((C, H, W), dtype=torch.float32, device="cuda") for _ in frames]
    # frames i and i + 1 in flight together; the clustered frames need more
    # sweeps than the plan's previous frame, so their waits enqueue more
    got = [None] * len(frames)
    plans[0].solve_async(*fs[0], outs[0])
    for i in range(len(frames)):
        if i + 1 < len(frames):
            plans[(i + 1) % 2].solve_async(*fs[i + 1], outs[i + 1])
        u, st = plans[i % 2].wait()
        got[i] = (host(u), st)
    for p in plans:
        p.close()
    for i, ((u, st), (u_ref, sw_ref)) in enumerate(zip(got, ref)):
        assert st["sweeps"] == sw_ref, i
        assert st["converged"] == 1
        np.testing.assert_array_equal(u, u_ref, err_msg=f"frame {i}")
        if timing:
            assert st["sweep_ms"] > 0 and st["cg_steps"] > 0
    f, c = frames[1]
    assert np.abs(got[1][0] - oracle.solve_exact(f.astype(np.float64), c)).max() <= 0.5


def test_async_errors(ddi):
    C, H, W = 1, 40, 48
    f, c = synth.make_workload(H, W, C, 0.05, "bernoulli", workload=51)
    with ddi.Plan(H, W, C, **PRM) as p:
        with pytest.raises(ddi.DDIError):
            p.wait()                                  # nothing pending
        u = torch.empty((C, H, W), dtype=torch.float32, device="cuda")
        p.solve_async(dev(f), dev(c), u)
        with pytest.raises(ddi.DDIError):
            p.solve_async(dev(f), dev(c), u)          # one pending solve per plan
        with pytest.raises(ddi.DDIError):
            p.solve(dev(f), dev(c), u)                # nor a synchronous one meanwhile
        _, st = p.wait()
        assert st["converged"] == 1
        with pytest.raises(ddi.DDIError) as ei:
            p.solve_async(dev(f), dev(np.zeros_like(c)), u)
            p.wait()
        assert ei.value.code == ddi.DDI_ESINGULAR
    with ddi.Plan(H, W, C, storage=1, block=16, levels=2) as p:
        u = torch.empty((C, H, W), dtype=torch.float32, device="cuda")
        with pytest.raises(ddi.DDIError):
            p.solve_async(dev(f), dev(c), u)
