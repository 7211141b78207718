"""ddi_solve_async / ddi_solve_wait: several plans in flight, on one stream
or each on a stream of its own, give the same results as ddi_solve, bit for
bit, including solves that need more sweeps than their first batch (the
continuation is enqueued by the wait behind the other plans' work); batch
plans on their own streams, driven by host threads at once, likewise."""
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


def test_frames_in_flight_on_own_streams(ddi):
    """Four plans, each on a stream of its own (chosen to sit on distinct
    hardware queues, as the benchmark does), with four frames in flight and
    timing on: every result equals the synchronous solve bit for bit, so
    plans running concurrently share no state."""
    import bench
    C, H, W = 3, 270, 480
    specs = [(0.05, "bernoulli"), (0.02, "clustered"), (0.08, "bernoulli"), (0.03, "clustered"),
             (0.04, "bernoulli"), (0.06, "clustered"), (0.03, "bernoulli"), (0.10, "bernoulli")]
    frames = [synth.make_workload(H, W, C, d, k, workload=52, index=i)
              for i, (d, k) in enumerate(specs)]
    say("frames in flight on own streams", len(frames))
    ref = []
    with ddi.Plan(H, W, C, **PRM) as p:
        for f, c in frames:
            u, st = p.solve(dev(f), dev(c))
            ref.append((host(u), st["sweeps"]))
    streams = bench.concurrent_streams(4)
    say("  concurrent streams", len(streams))
    plans = [ddi.Plan(H, W, C, timing=1, stream=streams[k % len(streams)], **PRM)
             for k in range(4)]
    fs = [(dev(f), dev(c)) for f, c in frames]
    outs = [torch.empty((C, H, W), dtype=torch.float32, device="cuda") for _ in range(4)]
    torch.cuda.synchronize()
    got = [None] * len(frames)
    for rnd in range(2):  # twice over: the second round starts in the other buffers
        for i in range(4):
            plans[i].solve_async(*fs[i], outs[i])
        for i in range(len(frames)):
            k = i % 4
            u, st = plans[k].wait()
            got[i] = (host(u), st)
            if i + 4 < len(frames):
                plans[k].solve_async(*fs[i + 4], outs[k])
        for i, ((u, st), (u_ref, sw_ref)) in enumerate(zip(got, ref)):
            assert st["sweeps"] == sw_ref, (rnd, i)
            assert st["converged"] == 1 and st["sweep_ms"] > 0
            np.testing.assert_array_equal(u, u_ref, err_msg=f"round {rnd} frame {i}")
    for p in plans:
        p.close()


def test_batches_in_flight_on_own_streams(ddi):
    """Two batch plans on streams of their own, driven by two host threads
    at once (the library call releases the interpreter lock): both equal a
    single batch plan's results bit for bit."""
    import threading
    import bench
    C = 3
    sizes = [(96, 160), (130, 70), (200, 256), (64, 200), (150, 3), (33, 47)]
    data = [synth.make_workload(h, w, C, 0.05, "clustered" if i % 2 else "bernoulli",
                                workload=53, index=i) for i, (h, w) in enumerate(sizes)]
    fs = [dev(f) for f, _ in data]
    cs = [dev(c) for _, c in data]
    prm = dict(block=32, overlap=4, levels=3, local_iters=12, rel_tol=1e-5, max_sweeps=120,
               final_residual=0)
    say("batches in flight", len(sizes))
    with ddi.Batch(sizes, C, **prm) as b:
        ref_u, ref_st, _ = b.solve(fs, cs)
        ref = [host(u) for u in ref_u]
    streams = bench.concurrent_streams(2)
    bs = [ddi.Batch(sizes, C, stream=streams[k % len(streams)], timing=1, **prm)
          for k in range(2)]
    uss = [[torch.empty_like(f) for f in fs] for _ in bs]
    torch.cuda.synchronize()
    results, errors = [[], []], []

    def worker(k):
        try:
            for _ in range(3):
                _, st, codes = bs[k].solve(fs, cs, uss[k])
                results[k].append(([s["sweeps"] for s in st], codes,
                                   [u.cpu().numpy() for u in uss[k]]))
        except Exception as e:
            errors.append(e)

    threads = [threading.Thread(target=worker, args=(k,)) for k in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    for b in bs:
        b.close()
    assert not errors, errors
    for k in range(2):
        for sweeps, codes, us in results[k]:
            assert codes == [0] * len(sizes)
            assert sweeps == [s["sweeps"] for s in ref_st]
            for a, r in zip(us, ref):
                np.testing.assert_array_equal(a, r)


def test_benchmark_launch_configuration_4k(ddi):
    """The 4K benchmark frame in the benchmark's own launch configuration:
    four plans with timing on, each on a stream of its own, four frames in
    flight through ddi_solve_async / ddi_solve_wait. Every result is the
    same bit for bit and within the 0.5 grey-level bar of the exact float64
    solution."""
    import bench
    C, H, W = 3, 2160, 3840
    f, c = synth.make_workload(H, W, C, bench.DENSITY, "bernoulli", workload=1)
    say("4K benchmark launch configuration")
    fd, cd = dev(f), dev(c)
    streams = bench.concurrent_streams(4)
    plans = [ddi.Plan(H, W, C, timing=1, stream=streams[k % len(streams)],
                      **bench.solver_params()) for k in range(4)]
    outs = [torch.empty_like(fd) for _ in range(4)]
    torch.cuda.synchronize()
    got = []
    for k in range(4):
        plans[k].solve_async(fd, cd, outs[k])
    for i in range(8):
        k = i % 4
        u, st = plans[k].wait()
        assert st["converged"] == 1
        got.append(host(u))
        if i + 4 < 8:
            plans[k].solve_async(fd, cd, outs[k])
    for p in plans:
        p.close()
    for u in got[1:]:
        np.testing.assert_array_equal(u, got[0])
    ex = oracle.solve_exact(f.astype(np.float64), c)
    err = float(np.abs(got[0] - ex).max())
    say("  max err vs exact", err)
    assert err <= 0.5
    np.testing.assert_array_equal(got[0][:, c == 1], f[:, c == 1])


def test_benchmark_settings_on_held_out_4k_frames(ddi):
    """The benchmark's solver settings were calibrated on its 4K workload
    class; frames of the same recipe with other seeds (indices 1-4) must
    also converge within the 0.5 grey-level bar of the exact float64
    solution, with the known pixels kept bit for bit."""
    import bench
    C, H, W = 3, 2160, 3840
    with ddi.Plan(H, W, C, **bench.solver_params()) as plan:
        for i in range(1, 5):
            f, c = synth.make_workload(H, W, C, bench.DENSITY, "bernoulli", workload=1, index=i)
            say("held-out 4K frame", i)
            u_t, st = plan.solve(dev(f), dev(c))
            u = host(u_t)
            ex = oracle.solve_exact(f.astype(np.float64), c)
            err = float(np.abs(u - ex).max())
            say("  sweeps", st["sweeps"], "max err vs exact", err)
            assert err <= 0.5
            np.testing.assert_array_equal(u[:, c == 1], f[:, c == 1])


def test_precision_plans_in_flight_from_threads(ddi):
    """Mixed-precision plans (storage = 1: synchronous refinement loop) on
    streams of their own, driven by host threads at once, as the precision
    benchmark does: every result equals the single plan's bit for bit."""
    import threading
    import bench
    C, H, W = 3, 270, 480
    prm = dict(bench.precision_params(), levels=4)
    frames = [synth.make_workload(H, W, C, 0.03, "bernoulli", workload=54, index=i)
              for i in range(2)]
    say("precision plans in flight")
    ref = []
    with ddi.Plan(H, W, C, **prm) as p:
        for f, c in frames:
            u, st = p.solve(dev(f), dev(c))
            ref.append((host(u), st["sweeps"]))
    streams = bench.concurrent_streams(2)
    plans = [ddi.Plan(H, W, C, timing=1, stream=streams[k % len(streams)], **prm)
             for k in range(2)]
    data = [(dev(f), dev(c)) for f, c in frames]
    torch.cuda.synchronize()
    res, errors = [[], []], []

    def worker(k):
        try:
            for _ in range(3):
                u, st = plans[k].solve(*data[k])
                res[k].append((u.cpu().numpy(), st["sweeps"]))
        except Exception as e:
            errors.append(e)

    threads = [threading.Thread(target=worker, args=(k,)) for k in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    for p in plans:
        p.close()
    assert not errors, errors
    for k in range(2):
        for u, sw in res[k]:
            assert sw == ref[k][1]
            np.testing.assert_array_equal(u, ref[k][0])


@pytest.mark.parametrize("method", [1, 2])
def test_comparator_plans_in_flight_from_threads(ddi, method):
    """Multilevel CG (method 1) and Krylov-accelerated ORAS (method 2)
    plans, whose solves wait on the host inside the call, driven from two
    host threads on streams of their own: results equal the single plan's
    bit for bit."""
    import threading
    import bench
    C, H, W = 3, 200, 320
    prm = dict(method=method, levels=3, rel_tol=1e-5, max_sweeps=200, final_residual=1)
    frames = [synth.make_workload(H, W, C, d, k, workload=55, index=i)
              for i, (d, k) in enumerate([(0.04, "bernoulli"), (0.03, "clustered")])]
    say("comparator plans in flight", method)
    ref = []
    with ddi.Plan(H, W, C, **prm) as p:
        for f, c in frames:
            u, st = p.solve(dev(f), dev(c))
            ref.append((host(u), st["sweeps"]))
    streams = bench.concurrent_streams(2)
    plans = [ddi.Plan(H, W, C, stream=streams[k % len(streams)], **prm) for k in range(2)]
    data = [(dev(f), dev(c)) for f, c in frames]
    torch.cuda.synchronize()
    res, errors = [[], []], []

    def worker(k):
        try:
            for _ in range(3):
                u, st = plans[k].solve(*data[k])
                res[k].append((u.cpu().numpy(), st["sweeps"]))
        except Exception as e:
            errors.append(e)

    threads = [threading.Thread(target=worker, args=(k,)) for k in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    for p in plans:
        p.close()
    assert not errors, errors
    for k in range(2):
        for u, sw in res[k]:
            assert sw == ref[k][1]
            np.testing.assert_array_equal(u, ref[k][0])
