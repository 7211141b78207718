"""Benchmark: homogeneous diffusion inpainting by multilevel ORAS on one
MI355X.

Default workload (--workload 4k): one step = one full solve (all levels,
every kernel of the path and the float64 stop tests) of a 3840 x 2160 x 3
float32 frame with a 4 % i.i.d. Bernoulli mask shared by the channels, 64 x
64 blocks with overlap 4, four levels (coarsest 1/8).

--workload precision: the 4K RGB frame with a 3 % Bernoulli mask, solved
with bfloat16 storage of the correction, float32 iterative refinement and a
float64 solve of the coarsest level; max error reported per channel.

--workload batch: one step = one batched solve of 48 RGB float32 images of
uneven size (sizes uniform over 640x480 .. 3840x2160, mask densities uniform
in 2-10 %, half of the masks clustered), each with the autotuned parameters
of its class; it also times the plain single-image path on the same images.

--workload serve: a Poisson stream (120 requests/s for 30 s) of 1080p / 4K /
720p RGB requests through the serving loop (paper_2110_03946_amd.serve),
then the same requests all at once (saturation) and through the plain
single-image path; p50/p99 latency from arrival to the result in host
memory.

--workload ablation: the 4K frame solved by multilevel ORAS, multilevel RAS
(alpha = 1), and their single-level forms, each to the same stop tolerance.
--workload psnr: PSNR of the 4K inpainting against the whole synthetic image
as the stop tolerance tightens.
--workload scaling: 960x540 to 3840x2160, multilevel ORAS against the
multilevel-CG comparator at the same stop tolerance.

Inputs are synthetic (paper_2110_03946_amd.synth) and already resident in
HBM when the timed region starts.

The timed region keeps several frames in flight (4k and precision: four
plans, each solving a seeded frame of its own; batch: three batch plans),
each on a stream of its own picked so that no two share a hardware queue:
one frame's latency-bound kernels run beside another's sweeps, and the
host's wait for a stop test never idles the GPU. A step of the 4k and
precision workloads is one frame on every plan (four frames). The timed
plans (and batch plans) carry no timing events; the per-sweep durations
come from separate passes on plans that record them (batch: batched solves
one at a time).

Prints one JSON line. Besides the driver's fields it carries
  roofline      the dominant kernel, the second finest-level ORAS sweep
                (one full outer iteration: every block runs and writes):
                its algorithmic bytes (float32 iterate read with the tile
                overlap re-read, written once, mask bits) over its own
                kernel duration, recorded by the launch at the kernel's
                start and end in synchronous solves with nothing else on
                the GPU; the later sweeps (which skip blocks), the fused
                first sweep and the same kernel in flight are sub-keys;
  cpu_baseline  the float64 CPU oracle on the first timed frame, all host
                threads and (single_core) one thread;
  max_err_grey  max |u - u_oracle| on the 0-255 scale over every plan's own
                timed result (batch: one image per autotuned class; serve:
                one served result per size);
  p50_ms/p99_ms 4k and precision: latency of one frame solved on its own
                (wall clock of a synchronous solve on a plan without timing
                events, after the timed region); batch: of a batched solve
                in flight;
  batch, precision, serve
                compact runs of those workloads (the 4k workload with
                --legs), each with its own value, error and comparison
                with the plain single-image path.

Usage: python bench.py [--gpus 1] [--steps 50] [--warmup 5] [--no-cpu]
                       [--workload 4k|batch|precision|serve|ablation|psnr|scaling]
                       [--frames-in-flight 4] [--batches-in-flight 3]
                       [--legs batch,precision,serve]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

H, W, C = 2160, 3840, 3
DENSITY = 0.04
FRAMES_IN_FLIGHT = 4
METRIC = "4K RGB frames/s at ≤0.5 grey-level err vs FP64; HBM GB/s frac; p99 ms"

# MI355X (gfx950) figures used for the roofline.
N_CU = 256
CLOCK_HZ = 2.4e9
HBM_PEAK_GBS = 8000.0
# float32 FMA on the vector ALU without packed instructions:
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz
VALU_F32_PEAK_TFLOPS = N_CU * 4 * 16 * 2 * CLOCK_HZ / 1e12
# algorithmic float32 flops per block pixel: residual (4 differences + 3
# sums) and, per CG step, the 5-point matvec (3 sums + multiply-subtract),
# two dot products (2 + 2) and three axpys (2 + 2 + 2)
FLOPS_RESIDUAL = 7
FLOPS_PER_CG_STEP = 15


def solver_params() -> dict:
    """Solver parameters of the benchmark workload (64 x 64 blocks, overlap
    4, coarsest level 1/8). The stop tolerance keeps the max error below
    0.5 grey levels on this workload class (0.38 at worst over eight
    frames). With frames in flight the VALU-bound local CG steps are the
    scarce resource: eight CG steps on the coarse levels buy a start good
    enough for a looser local stop (0.004) on the finest level. At least
    three finest-level sweeps: after two, the error on this workload class
    is 0.6-1.1 grey levels whatever the residual says, so no stop test is
    run before the third."""
    return dict(block=64, overlap=4, levels=4, local_iters=16, robin_alpha=0.25,
                coarse_sweeps=1, coarsest_sweeps=1, coarse_local_iters=8, local_tol=0.004,
                rel_tol=5e-4, min_sweeps=3, max_sweeps=30, check_every=1, final_residual=0)


def batch_params(specs):
    """Per-image solver parameters of the batched workload: the autotuner's
    entry for each image's class (size, mask kind, density)."""
    from paper_2110_03946_amd import autotune, ddi
    table = autotune.load_table()
    return [ddi.default_params(**autotune.params_for(table, s["h"], s["w"], s["kind"],
                                                     s["density"])) for s in specs]


def sweep_work(p: dict, sweeps: int, cg_steps: float, h: int = H, w: int = W, ch: int = C,
               skipped: float = 0.0, unwritten: float = 0.0):
    """Algorithmic flops and HBM bytes of the finest-level sweeps of a solve
    of an h x w x ch image (`sweeps` launches, `cg_steps` block CG steps
    actually run; `skipped` blocks skipped whole and `unwritten` blocks that
    skipped their write-back, summed over channels and launches)."""
    from paper_2110_03946_amd import ddi
    nby = ddi.block_count(h, p["block"], p["overlap"])
    nbx = ddi.block_count(w, p["block"], p["overlap"])
    bh, bw = min(p["block"], h), min(p["block"], w)
    blocks = nby * nbx * ch
    run = blocks * sweeps - skipped
    flops = bh * bw * (run * FLOPS_RESIDUAL + cg_steps * FLOPS_PER_CG_STEP)
    # per block that runs: its owned pixels of the iterate read once and
    # written once (float32; the write is skipped where the output already
    # holds the values), plus the transposed mask (one bit per pixel);
    # re-reads of the tile overlap are not algorithmic (the L2 serves them).
    # A block's owned pixels are taken as the mean, h * w / (nby * nbx).
    own = h * w / (nby * nbx)
    bytes_ = own * 4 * (2 * run - unwritten) + (run / ch) * own / 8
    return flops, bytes_


def roofline_of(flops: float, bytes_: float, sweep_ms: float, launches: int) -> dict:
    """Roofline object of the finest-level sweep: achieved rate against the
    bound its arithmetic intensity puts it under (ridge = peak flops / peak
    bytes per second)."""
    tflops = flops / (sweep_ms / 1e3) / 1e12
    gbs = bytes_ / (sweep_ms / 1e3) / 1e9
    intensity = flops / bytes_
    ridge = VALU_F32_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    if intensity >= ridge:
        r = {"bound": "alu", "achieved": round(tflops, 3), "peak": round(VALU_F32_PEAK_TFLOPS, 1),
             "unit": "TFLOP/s", "frac": round(tflops / VALU_F32_PEAK_TFLOPS, 4)}
    else:
        r = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
             "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)}
    r.update({"avg_launch_us": round(sweep_ms / max(launches, 1) * 1e3, 2),
              "flops_per_byte": round(intensity, 2), "ridge_flops_per_byte": round(ridge, 2),
              "valu_tflops": round(tflops, 3), "valu_frac": round(tflops / VALU_F32_PEAK_TFLOPS, 4),
              "hbm_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)})
    return r


SWEEP_SOURCES = ("sweep.hip", "device.h", "access.h", "internal.h")


def sweep_sources_sha256() -> str:
    """SHA-256 over the sources the finest-level sweep kernel is compiled
    from, in a fixed order."""
    import hashlib
    h = hashlib.sha256()
    for name in SWEEP_SOURCES:
        data = open(os.path.join(ROOT, "paper_2110_03946_amd", "csrc", name), "rb").read()
        h.update(name.encode() + b"\0" + str(len(data)).encode() + b"\0" + data)
    return h.hexdigest()


def measured_traffic():
    """HBM bytes of the second finest-level sweep launch (the kernel the
    roofline describes) from the committed rocprofv3 counter summary, or
    None when the sweep's sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "k_sweep2_4k_rgb_traffic.json")
    try:
        d = json.load(open(path))
        sha = sweep_sources_sha256()
    except (OSError, ValueError):
        return None
    return d["hbm_bytes_per_launch"] if d.get("sweep_sources_sha256") == sha else None


def summarize_trace(path: str) -> str:
    """Per (kernel, grid) duration table of a rocprofv3 --kernel-trace CSV:
    the same kernel runs on every level of the pyramid, and the grid size
    tells the levels apart (the finest-level sweep has 6912 workgroups)."""
    import csv
    import collections
    groups = collections.defaultdict(list)
    for row in csv.DictReader(open(path)):
        name = row["Kernel_Name"].replace("(anonymous namespace)::", "").split("(")[0]
        name = name.replace("void ", "")
        grid = (int(row["Grid_Size_X"]) * int(row["Grid_Size_Y"]) * int(row["Grid_Size_Z"]) //
                max(1, int(row["Workgroup_Size_X"]) * int(row["Workgroup_Size_Y"]) *
                    int(row["Workgroup_Size_Z"])))
        groups[(name, grid)].append(int(row["End_Timestamp"]) - int(row["Start_Timestamp"]))
    total = sum(sum(v) for v in groups.values())
    out = ["| kernel | workgroups | calls | avg us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    for (name, grid), v in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
        out.append(f"| {name} | {grid} | {len(v)} | {sum(v) / len(v) / 1e3:.2f} | "
                   f"{min(v) / 1e3:.2f} | {max(v) / 1e3:.2f} | {100 * sum(v) / total:.1f} |")
    return "\n".join(out)


def precision_params() -> dict:
    """Parameters of the mixed-precision workload: bfloat16 correction
    storage with float32 refinement steps of 2 correction sweeps, float64
    solve of the coarsest level (6 levels: 120 x 68 for 4K). The local stop
    0.002 leaves a refinement residual floor near 5e-5, so the stop
    tolerance sits above it (1e-4): two refinement steps, 0.21 grey levels
    at worst over eight frames."""
    return dict(block=64, overlap=4, levels=6, local_iters=16, robin_alpha=0.25,
                coarse_sweeps=1, coarsest_sweeps=1, coarse_local_iters=8, local_tol=0.002,
                rel_tol=1e-4, min_sweeps=1, max_sweeps=40, check_every=1, final_residual=0,
                coarse_solver=1, coarse_cg_iters=500, coarse_cg_tol=1e-10, storage=1,
                inner_sweeps=2)


PRECISION_DENSITY = 0.03
METRIC_PRECISION = ("4K RGB frames/s, bf16 storage + f32 refinement, ≤0.5 grey-level err vs "
                    "FP64 per channel")


def correction_bytes(m: int, refinements: int, h: int = H, w: int = W, ch: int = C) -> int:
    """Algorithmic HBM bytes of the correction sweeps of a mixed-precision
    solve: every sweep reads the bfloat16 right-hand side and writes the
    bfloat16 correction, all but the first of a step also read the previous
    correction; plus the transposed mask."""
    per_step = sum(ch * h * w * (4 if j == 0 else 6) + h * w // 8 for j in range(m))
    return refinements * per_step


def concurrent_streams(n: int, candidates: int = 24) -> list:
    """n torch streams (default priority) whose kernels run concurrently.

    HIP maps streams onto a few hardware queues (GPU_MAX_HW_QUEUES, 4 by
    default), and two streams on one queue execute one after the other;
    which streams share a queue is not exposed. Candidates are probed: a
    short single-thread spin kernel on the candidate and on every stream
    already chosen takes one spin's time only if none of them share a
    queue. Returns fewer than n streams if the candidates run out."""
    import torch
    if not hasattr(torch.cuda, "_sleep"):
        # no spin kernel to probe with: plain pool streams (consecutive pool
        # streams usually, but not always, sit on distinct queues)
        print("[bench] torch.cuda._sleep missing: streams not probed", file=sys.stderr)
        return [torch.cuda.Stream() for _ in range(n)]
    spin = int(0.5e-3 * CLOCK_HZ)

    def run(streams):
        torch.cuda.synchronize()
        t = time.perf_counter()
        for st in streams:
            with torch.cuda.stream(st):
                torch.cuda._sleep(spin)
        torch.cuda.synchronize()
        return time.perf_counter() - t

    pool = [torch.cuda.Stream() for _ in range(candidates)]
    run(pool[:1])
    one = min(run(pool[:1]) for _ in range(3))
    chosen = [pool[0]]
    for cand in pool[1:]:
        if len(chosen) == n:
            break
        if min(run(chosen + [cand]) for _ in range(2)) < 1.5 * one:
            chosen.append(cand)
    return chosen


def gen_workers() -> int:
    """Worker processes for input generation: the host's cores, at most 16."""
    return max(1, min(16, os.cpu_count() or 1))


def overlap_factor(p: dict) -> float:
    """(S / (S - o))^2: each block reads its S x S tile while owning a
    (S - o) x (S - o) core, so a full sweep reads every pixel this often."""
    return (p["block"] / (p["block"] - p["overlap"])) ** 2


def full_sweep_bytes(p: dict, h: int = H, w: int = W, ch: int = C) -> float:
    """Algorithmic HBM bytes of one full finest-level ORAS sweep (every
    block runs and writes): float32 iterate read with the tile overlap
    re-read, float32 iterate written once (Boolean partition of unity), and
    the transposed mask (one bit per pixel, shared by the channels)."""
    return ch * h * w * (4 * overlap_factor(p) + 4) + h * w / 8


def oracle_check(frames, outs):
    """Max |u - u_oracle| over frames (grey levels) and per channel, and the
    oracle's wall time and CG iterations on the first frame."""
    import oracle
    worst, per_ch, t_first, iters = 0.0, None, None, None
    for k, ((f, c), u) in enumerate(zip(frames, outs)):
        t0 = time.perf_counter()
        ex, info = oracle.solve_exact(f.astype(np.float64), c, return_info=True)
        t = time.perf_counter() - t0
        if k == 0:
            t_first, iters = t, [i["iters"] for i in info]
        d = np.abs(u.astype(np.float64) - ex)
        ch = [float(d[i].max()) for i in range(d.shape[0])]
        per_ch = ch if per_ch is None else [max(x, y) for x, y in zip(per_ch, ch)]
        worst = max(worst, max(ch))
    return worst, per_ch, t_first, iters


def oracle_one_core(h: int, w: int, density: float, wl: int, idx: int) -> float:
    """Seconds the float64 oracle takes on channel 0 of a frame with one
    OpenMP thread (a child process regenerates the frame from its seed)."""
    import subprocess
    code = ("import sys, time; sys.path.insert(0, %r)\n"
            "from paper_2110_03946_amd import synth\nimport oracle\n"
            "f, c = synth.make_workload(%d, %d, 1, %r, 'bernoulli', workload=%d, index=%d)\n"
            "assert oracle.threads() == 1\n"
            "t = time.perf_counter(); oracle.solve_exact(f[0].astype('float64'), c)\n"
            "print(time.perf_counter() - t)\n") % (ROOT, h, w, density, wl, idx)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                         check=True)
    return float(out.stdout.strip().splitlines()[-1])


def run_frame(args, workload: str) -> dict:
    """One 4K RGB frame per step: the float32 path (4k) or the mixed-precision
    path (precision). Every plan in flight solves a frame of its own."""
    import torch
    from paper_2110_03946_amd import ddi, synth
    precision = workload == "precision"
    density = PRECISION_DENSITY if precision else DENSITY
    wl = 3 if precision else 1
    nplans = args.frames_in_flight
    print(f"[bench] {workload}: generating {nplans} frames", file=sys.stderr, flush=True)
    frames = synth.make_workloads([(H, W, C, density, "bernoulli", wl, k) for k in range(nplans)],
                                  workers=gen_workers())
    fs = [torch.from_numpy(f).cuda() for f, _ in frames]
    cs = [torch.from_numpy(c).cuda() for _, c in frames]
    us = [torch.empty_like(f) for f in fs]
    prm = precision_params() if precision else solver_params()
    # several plans, each with a frame of its own in flight on a stream of
    # its own: one frame's latency-bound kernels (coarse levels, stop tests,
    # reductions) and the load phases of its sweeps run beside the other
    # frames' sweeps, and the host's wait for one plan's stop test never
    # leaves the GPU idle
    streams = concurrent_streams(nplans) if nplans > 1 else [None]
    if len(streams) < nplans:
        print(f"[bench] only {len(streams)} concurrent streams found", file=sys.stderr)
        streams = [streams[i % len(streams)] for i in range(nplans)]
    # the timed region runs the solver as a caller would: plans without
    # timing events (the per-sweep events, their counters' clears and
    # reductions are measured in a pass of their own below)
    plans = [ddi.Plan(H, W, C, timing=0, stream=s, **prm) for s in streams]
    plan = plans[0]
    for _ in range(args.warmup):
        for p, f, c, u in zip(plans, fs, cs, us):
            p.solve(f, c, u)
    torch.cuda.synchronize()
    sweeps_per_solve, rels = [], []
    inflight = {"ms": [], "nsweeps": []}

    def account(st, times):
        sweeps_per_solve.append(st["sweeps"])
        rels.append(st["rel_residual"])
        if times and len(times) > 1:
            inflight["ms"].append(times[1])

    # a step is one frame on every plan in flight (nplans frames)
    nframes = args.steps * nplans
    t0 = time.perf_counter()
    if nplans == 1:
        for _ in range(nframes):
            _, st = plan.solve(fs[0], cs[0], us[0])
            account(st, None)
    elif precision:
        # the refinement loop has no asynchronous entry point: one host
        # thread per plan drives synchronous solves (the library call
        # releases the interpreter lock)
        import threading
        lock = threading.Lock()
        errors = []

        def worker(k):
            try:
                for _ in range(args.steps):
                    _, st = plans[k].solve(fs[k], cs[k], us[k])
                    with lock:
                        account(st, None)
            except Exception as e:  # re-raised in the main thread
                errors.append(e)

        threads = [threading.Thread(target=worker, args=(k,)) for k in range(nplans)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        if errors:
            raise errors[0]
    else:
        for i in range(nplans):
            plans[i].solve_async(fs[i], cs[i], us[i])
        for i in range(nframes):
            k = i % nplans
            _, st = plans[k].wait()
            account(st, None)
            if i + nplans < nframes:
                plans[k].solve_async(fs[k], cs[k], us[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    fps = nframes / elapsed
    outs = [u.cpu().numpy() for u in us]  # each plan's own last timed result
    for p in plans:
        p.close()
    # the same frames in flight on plans with timing events (outside the
    # timed region): the second finest sweep's duration while it shares the
    # GPU with the other frames (roofline.in_flight)
    plans = [ddi.Plan(H, W, C, timing=1, stream=s, **prm) for s in streams]
    plan = plans[0]
    if not precision:
        n_t = nplans * max(2, min(args.steps, 10))
        for p, f, c, u in zip(plans, fs, cs, us):
            p.solve(f, c, u)
        for i in range(min(nplans, n_t)):
            plans[i].solve_async(fs[i], cs[i], us[i])
        for i in range(n_t):
            k = i % nplans
            plans[k].wait()
            t = plans[k].sweep_times()
            if t and len(t) > 1:
                inflight["ms"].append(t[1])
            if i + nplans < n_t:
                plans[k].solve_async(fs[k], cs[k], us[k])
        torch.cuda.synchronize()
    # the kernels with the GPU to themselves: synchronous solves, one frame
    # at a time, on a timed plan; the sweep launches record their kernels'
    # own start and end (no dispatch gap in the bracket)
    iso = {"t": [], "steps": 0.0, "first_steps": 0.0, "skipped": 0.0, "unwritten": 0.0,
           "refs": 0, "sweeps": 0}
    for _ in range(20):
        _, st = plan.solve(fs[0], cs[0], us[0])
        iso["t"].append(plan.sweep_times())
        iso["steps"] += st["cg_steps"] - st["first_cg_steps"]
        iso["first_steps"] += st["first_cg_steps"]
        iso["skipped"] += st["skipped_blocks"]
        iso["unwritten"] += st["unwritten_blocks"]
        iso["refs"] += st["refinements"]
        iso["sweeps"] += st["sweeps"]
    for p in plans[1:]:
        p.close()
    # latency of one frame on its own (no other frame queued): wall clock
    # of a synchronous solve on a plan without timing events
    lat = []
    with ddi.Plan(H, W, C, **prm) as lat_plan:
        for _ in range(3):
            lat_plan.solve(fs[0], cs[0], us[0])
        for _ in range(max(10, min(args.steps, 100))):
            ts = time.perf_counter()
            lat_plan.solve(fs[0], cs[0], us[0])
            lat.append((time.perf_counter() - ts) * 1e3)
    sync_fps = 1e3 / float(np.mean(lat))
    nb = ddi.block_count(H, prm["block"], prm["overlap"]) * ddi.block_count(W, prm["block"],
                                                                               prm["overlap"])
    if precision:
        roofline = precision_roofline(prm, iso)
        desc = ("4K RGB 3840x2160x3, 3% Bernoulli mask shared by the channels; bf16 storage of "
                "the correction and its right-hand side with f32 arithmetic, f32 iterative "
                "refinement (2 correction sweeps per step), f64 residual norm and f64 solve of "
                "the coarsest level")
        dtype = "bf16 storage / f32 compute"
    else:
        roofline = frame_roofline(prm, iso, inflight, nb, frames[0][1])
        desc = ("4K RGB 3840x2160x3 f32, 4% Bernoulli mask shared by the channels, multilevel "
                "ORAS (64x64 blocks, overlap 4, 4 levels: coarsest 1/8), CG local solves")
        dtype = "f32"
    out = {"metric": METRIC_PRECISION if precision else METRIC, "value": round(fps, 2),
           "unit": "frames/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(elapsed / args.steps * 1e3, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
           "config": {"workload": desc, "frames": f"{nplans} distinct seeded frames, one per "
                                                   "plan in flight",
                      "step": f"one frame on each of the {nplans} plans ({nplans} frames)",
                      **prm},
           "p50_ms": round(float(np.percentile(lat, 50)), 3),
           "p99_ms": round(float(np.percentile(lat, 99)), 3),
           "frames_in_flight": nplans,
           "single_frame_sync_fps": round(sync_fps, 2),
           "sweeps_per_solve": sorted(set(sweeps_per_solve)),
           "rel_residual_max": max(rels),
           "roofline": roofline}
    if precision:
        out["refinements_per_solve"] = round(iso["refs"] / 20, 2)
    else:
        out["coarsest_level"] = coarse_comparison(fs[0], cs[0], prm)
    if not args.no_cpu:
        print(f"[bench] {workload}: oracle on the {nplans} timed frames", file=sys.stderr,
              flush=True)
        err, per_ch, t_first, iters = oracle_check(frames, outs)
        out["max_err_grey"] = round(err, 4)
        out["max_err_grey_per_channel"] = [round(e, 4) for e in per_ch]
        out["max_err_frames"] = nplans
        if not precision:
            import oracle
            t1 = oracle_one_core(H, W, density, wl, 0)
            out["cpu_baseline"] = {
                "value": round(1.0 / t_first, 4), "unit": "frames/s", "cores": oracle.threads(),
                "kind": "oracle",
                "sample": "the first timed 3840x2160x3 frame: float64 CG on the reduced system "
                          f"to relative residual 1e-12 per channel ({iters} iterations), "
                          f"{t_first:.1f} s",
                "single_core": {"value": round(1.0 / (3 * t1), 4), "unit": "frames/s",
                                "cores": 1,
                                "sample": f"channel 0 of that frame on one thread, {t1:.1f} s, "
                                          "times 3 channels"}}
    return out


def coarse_comparison(f0, c0, prm: dict, reps: int = 20) -> dict:
    """The coarsest level of the 4K frame (1/8: 480 x 270 x 3) solved the two
    ways a plan offers: one float32 ORAS sweep from u = c ? f : 0 (what the
    benchmark plan runs there, coarse_solver = 0) and float64 conjugate
    gradients on a grid of workgroups (coarse_solver = 1, relative residual
    1e-10); then the whole 4K solve with each."""
    import torch
    from paper_2110_03946_amd import ddi
    f, c = f0, c0
    for _ in range(prm["levels"] - 1):
        f, c = ddi.coarsen(f, c)
    nc, hc, wc = f.shape
    work = torch.empty(ddi.coarse_grid_bytes(hc, wc, nc), dtype=torch.uint8, device="cuda")
    u64, u32 = torch.empty_like(f), torch.empty_like(f)
    start = torch.where(c.bool(), f, torch.zeros_like(f))
    sweep = dict(block=prm["block"], overlap=prm["overlap"], alpha=prm["robin_alpha"],
                 k=prm["coarse_local_iters"])
    _, steps = ddi.coarse_solve_grid(f, c, max_iter=500, tol=1e-10, u=u64, work=work,
                                     steps=True)
    ddi.oras_sweep_noalloc(start, c, u_out=u32, rsq=False, **sweep)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(reps):
        ddi.coarse_solve_grid(f, c, max_iter=500, tol=1e-10, u=u64, work=work)
    ev[1].record()
    ev[2].record()
    for _ in range(reps):
        ddi.oras_sweep_noalloc(start, c, u_out=u32, rsq=False, **sweep)
    ev[3].record()
    torch.cuda.synchronize()
    unk = ~c.bool()
    dev32 = float((u32 - u64).abs()[:, unk].max()) if bool(unk.any()) else 0.0
    out = {"level": f"{wc}x{hc}x{nc}", "known_frac": round(float(c.float().mean()), 4),
           "f64_grid_cg_us": round(ev[0].elapsed_time(ev[1]) / reps * 1e3, 1),
           "f64_grid_cg_steps": steps,
           "f32_oras_sweep_us": round(ev[2].elapsed_time(ev[3]) / reps * 1e3, 1),
           "f32_sweep_max_dev_from_f64_grey": round(dev32, 3),
           "timing": "CUDA events around back-to-back calls on one stream"}
    # the whole solve with each coarsest-level solver (synchronous, no timing
    # events)
    u = torch.empty_like(f0)
    for cs_ in (0, 1):
        q = dict(prm, coarse_solver=cs_)
        lat, sw = [], []
        with ddi.Plan(f0.shape[1], f0.shape[2], f0.shape[0], **q) as pl:
            for _ in range(3):
                pl.solve(f0, c0, u)
            for _ in range(reps):
                ts = time.perf_counter()
                _, st = pl.solve(f0, c0, u)
                lat.append((time.perf_counter() - ts) * 1e3)
                sw.append(st["sweeps"])
        out[f"solve_coarse_solver_{cs_}"] = {"p50_ms": round(float(np.percentile(lat, 50)), 3),
                                             "sweeps": sorted(set(sw))}
    return out


def frame_roofline(prm, iso, inflight, nb, c0) -> dict:
    """Roofline of the dominant kernel from its own launch durations (sweep
    launches record the kernel's start and end), alone on the GPU: the
    second finest sweep, one full outer ORAS iteration in which every block
    runs and writes (the third sweep skips blocks the second left
    unchanged and is reported apart)."""
    full_ms = float(np.mean([x[1] for x in iso["t"]]))
    first_ms = float(np.mean([x[0] for x in iso["t"]]))
    later = [v for x in iso["t"] for v in x[2:]]
    bfull = full_sweep_bytes(prm)
    gbs = bfull / (full_ms / 1e3) / 1e9
    # the first sweep: level-1 iterate read, f on the known pixels, the
    # transposed mask, u written
    hc, wc = (H + 1) // 2, (W + 1) // 2
    bfirst = C * H * W * 4 + C * hc * wc * 4 + C * int(c0.sum()) * 4 + H * W / 8
    r = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
         "kernel": "k_sweep2<false>: second finest-level ORAS sweep (one full outer iteration: "
                   "all 6912 blocks of 64x64 run and write)",
         "avg_launch_us": round(full_ms * 1e3, 2),
         "bytes_per_launch": round(bfull),
         "bytes_model": "C*H*W*(4*(S/(S-o))^2 + 4) + H*W/8: iterate read with the tile "
                        "overlap re-read (S=64, o=4: 1.138), iterate written once, mask bits",
         "timing": "kernel start/end recorded by the launch (hipExtLaunchKernel events), 20 "
                   "synchronous solves, nothing else on the GPU"}
    if later:
        # later sweeps skip blocks: credit only the blocks that run, and
        # the writes they do not skip
        n_later = len(later)
        own = H * W / nb
        # per block and channel: a whole skip saves its tile read, its write
        # and its share of the mask bits; a skipped write-back its write
        b_later = (n_later * bfull - iso["skipped"] * own * (4 * overlap_factor(prm) + 4)
                   - iso["skipped"] * own / 8 / C - iso["unwritten"] * own * 4)
        ms_later = float(np.sum(later))
        r["later_sweeps"] = {
            "avg_launch_us": round(ms_later / n_later * 1e3, 2),
            "achieved": round(b_later / (ms_later / 1e3) / 1e9, 1),
            "skipped_block_frac": round(iso["skipped"] / (n_later * nb * C), 4),
            "unwritten_block_frac": round(iso["unwritten"] / (n_later * nb * C), 4),
            "bytes_model": "the full-sweep bytes less the blocks skipped whole (their reads, "
                           "writes and mask bits) and the write-backs skipped"}
    r["first_sweep"] = {
        "kernel": "k_sweep2_pro: first finest sweep, bilinear prolongation in the tile load",
        "avg_launch_us": round(first_ms * 1e3, 2),
        "achieved": round(bfirst / (first_ms / 1e3) / 1e9, 1),
        "bytes_per_launch": round(bfirst),
        "cg_steps_per_block": round(iso["first_steps"] / 20 / (nb * C), 2)}
    steady_steps = iso["steps"] / 20
    r["cg_steps_per_block_steady_sweeps"] = round(steady_steps / (nb * C) /
                                                  max(1, iso["sweeps"] / 20 - 1), 2)
    if inflight["ms"]:
        ms = float(np.mean(inflight["ms"]))
        r["in_flight"] = {"avg_launch_us": round(ms * 1e3, 2),
                          "achieved": round(bfull / (ms / 1e3) / 1e9, 1),
                          "note": "the same second sweep with the other frames in flight, "
                                  "sharing the GPU with their kernels (a pass on plans with "
                                  "timing events after the timed region)"}
    r["valu_peak_basis"] = ("78.6 TFLOP/s float32 without packed instructions: 256 CU x 4 SIMD x "
                            "16 lanes x 2 flop (FMA) x 2.4 GHz; packed FP32 is disabled in this "
                            "build")
    return r


def precision_roofline(prm, iso) -> dict:
    """Correction sweeps of the mixed-precision path (k_sweep2<true>),
    against the bound their arithmetic intensity puts them under. Bytes:
    bfloat16 right-hand side read, correction written (and read, except in
    a step's first sweep), transposed mask. Flops: the residual of the
    correction equation on every block (one more add than the float32
    sweep's, for the right-hand side) plus the CG steps the blocks ran."""
    from paper_2110_03946_amd import ddi
    ms = [v for x in iso["t"] for v in x]
    if not ms:
        return None
    nby = ddi.block_count(H, prm["block"], prm["overlap"])
    nbx = ddi.block_count(W, prm["block"], prm["overlap"])
    bh, bw = min(prm["block"], H), min(prm["block"], W)
    flops = bh * bw * (len(ms) * nby * nbx * C * (FLOPS_RESIDUAL + 1)
                       + iso["steps"] * FLOPS_PER_CG_STEP)
    bytes_ = correction_bytes(prm["inner_sweeps"], 1) * iso["refs"]
    r = roofline_of(flops, bytes_, float(np.sum(ms)), len(ms))
    r.update({"traffic": None,
              "kernel": "k_sweep2<true> (finest-level correction sweep, bf16 storage)",
              "timing": "events recorded on the stream around each correction sweep's launch, "
                        "20 synchronous solves"})
    return r


SERVE_RATE, SERVE_SECONDS = 120.0, 30.0
METRIC_SERVE = "served frames/s and p50/p99 latency (Poisson 120 req/s, mixed resolution)"


def reference_solve(plan_kw, f, c):
    """The solver itself run to a tight tolerance (float64 norms, no local
    stop): the reference the ablation and PSNR studies measure against
    without the CPU oracle."""
    from paper_2110_03946_amd import ddi
    p = dict(plan_kw, local_tol=0.0, rel_tol=1e-6, max_sweeps=400, min_sweeps=1,
             final_residual=1)
    with ddi.Plan(H, W, C, **p) as plan:
        u, st = plan.solve(f, c, allow_noconv=True)
    return u, st


def timed_solves(plan, f, c, u, n: int):
    """Median device ms of n solves (after one warm-up) and the last stats."""
    plan.solve(f, c, u, allow_noconv=True)
    ms = []
    for _ in range(n):
        _, st = plan.solve(f, c, u, allow_noconv=True)
        ms.append(st["ms"])
    return float(np.median(ms)), st


def run_ablation(args):
    """RAS (alpha = 1) against ORAS (tuned alpha) and single- against
    multilevel, on the 4K frame, each solved to the benchmark's stop
    tolerance; error measured against a tight solve of the solver itself."""
    import torch
    from paper_2110_03946_amd import ddi, synth
    f_np, c_np = synth.make_workload(H, W, C, DENSITY, "bernoulli", workload=1)
    f = torch.from_numpy(f_np).cuda()
    c = torch.from_numpy(c_np).cuda()
    u = torch.empty_like(f)
    base = solver_params()
    ref, _ = reference_solve(base, f, c)
    rows = []
    for name, over in [("multilevel ORAS (alpha 0.25, 4 levels)", {}),
                       ("multilevel RAS (alpha 1)", dict(robin_alpha=1.0)),
                       ("single-level ORAS (alpha 0.25)", dict(levels=1)),
                       ("single-level RAS (alpha 1)", dict(levels=1, robin_alpha=1.0)),
                       # Krylov acceleration (not in the paper): flexible GMRES(8) over
                       # one ORAS sweep per step, after the same multilevel start
                       ("Krylov-accelerated multilevel ORAS (FGMRES(8))",
                        dict(method=2, krylov_restart=8)),
                       ("Krylov-accelerated multilevel ORAS (FGMRES(8)), rel_tol 5e-5",
                        dict(method=2, krylov_restart=8, rel_tol=5e-5)),
                       ("Krylov-accelerated single-level ORAS (FGMRES(8))",
                        dict(method=2, krylov_restart=8, levels=1))]:
        prm = dict(base, **over, max_sweeps=400, final_residual=1)
        with ddi.Plan(H, W, C, **prm) as plan:
            ms, st = timed_solves(plan, f, c, u, max(3, args.steps // 10))
        err = float((u - ref).abs().max())
        rows.append({"variant": name, "ms": round(ms, 3), "sweeps": st["sweeps"],
                     "converged": st["converged"], "rel_residual": st["rel_residual"],
                     "max_dev_from_tight_solve_grey": round(err, 4)})
        print(f"[bench] {name}: {ms:.3f} ms, {st['sweeps']} sweeps", file=sys.stderr, flush=True)
    out = {"metric": "4K RGB solve time to rel_tol 5e-4: ORAS vs RAS, multilevel vs single "
                     "level, stationary vs Krylov-accelerated",
           "value": rows[0]["ms"], "unit": "ms", "higher_is_better": False, "n_gpus": 1,
           "data": "synthetic", "dtype": "f32",
           "config": {"workload": "4K RGB 3840x2160x3, 4% Bernoulli; each variant stops at the "
                                  "benchmark's rel_tol 5e-4 (max 400 sweeps)"},
           "rows": rows, "roofline": None}
    print(json.dumps(out), flush=True)


def psnr(a, b) -> float:
    mse = float(((a.double() - b.double()) ** 2).mean())
    return float("inf") if mse == 0 else 10.0 * math.log10(255.0 ** 2 / mse)


def run_psnr(args):
    """PSNR of the inpainting against the full synthetic image (known
    everywhere, so the reconstruction quality is measurable) and its
    deviation from a tight solve, as the stop tolerance tightens."""
    import torch
    from paper_2110_03946_amd import ddi, synth
    f_np, c_np = synth.make_workload(H, W, C, DENSITY, "bernoulli", workload=1)
    f = torch.from_numpy(f_np).cuda()
    c = torch.from_numpy(c_np).cuda()
    u = torch.empty_like(f)
    base = solver_params()
    ref, _ = reference_solve(base, f, c)
    rows = []
    for tol in (1e-2, 3e-3, 1e-3, 5e-4, 3e-4, 1e-4, 3e-5, 1e-5):
        # the stop test after every sweep, so each tolerance stops where its
        # residual test first passes
        prm = dict(base, rel_tol=tol, min_sweeps=1, max_sweeps=200, final_residual=1,
                   local_tol=min(base["local_tol"], 0.002 if tol >= 1e-4 else 0.0))
        with ddi.Plan(H, W, C, **prm) as plan:
            ms, st = timed_solves(plan, f, c, u, 5)
        rows.append({"rel_tol": tol, "sweeps": st["sweeps"], "ms": round(ms, 3),
                     "rel_residual": st["rel_residual"], "psnr_db": round(psnr(u, f), 3),
                     "psnr_tight_db": round(psnr(ref, f), 3),
                     "max_dev_from_tight_solve_grey": round(float((u - ref).abs().max()), 4)})
        print(f"[bench] rel_tol {tol:g}: {rows[-1]}", file=sys.stderr, flush=True)
    out = {"metric": "PSNR (dB) of the 4K RGB inpainting vs the stop tolerance",
           "value": rows[2]["psnr_db"], "unit": "dB", "higher_is_better": True, "n_gpus": 1,
           "data": "synthetic", "dtype": "f32",
           "config": {"workload": "4K RGB 3840x2160x3, 4% Bernoulli; PSNR against the whole "
                                  "synthetic image (ground truth everywhere)"},
           "rows": rows, "roofline": None}
    print(json.dumps(out), flush=True)


SCALING_SIZES = ((540, 960), (1080, 1920), (2160, 3840))


def run_scaling(args):
    """Resolution sweep of multilevel ORAS against the multilevel-CG
    comparator (method = 1) on the same frames and stop tolerance: solve
    time, time per megapixel, and each result's deviation from a tight solve
    of the solver itself."""
    import torch
    from paper_2110_03946_amd import ddi, synth
    base = solver_params()
    rows = []
    for h, w in SCALING_SIZES:
        f_np, c_np = synth.make_workload(h, w, C, DENSITY, "bernoulli", workload=1)
        f = torch.from_numpy(f_np).cuda()
        c = torch.from_numpy(c_np).cuda()
        u = torch.empty_like(f)
        p_ref = dict(base, local_tol=0.0, rel_tol=1e-6, max_sweeps=400, min_sweeps=1,
                     final_residual=1)
        with ddi.Plan(h, w, C, **p_ref) as plan:
            ref, _ = plan.solve(f, c, allow_noconv=True)
        row = {"size": f"{w}x{h}", "megapixels": round(h * w / 1e6, 3)}
        # ML-CG at the same stop tolerance, and at a 10x tighter one (its
        # error at equal residual is larger: CG leaves smooth error that
        # the residual norm weighs little)
        for name, prm in [("oras", dict(base)),
                          ("mlcg", dict(base, method=1, max_sweeps=5000)),
                          ("mlcg_tight", dict(base, method=1, max_sweeps=5000,
                                              rel_tol=base["rel_tol"] / 10)),
                          ("krylov_oras", dict(base, method=2, krylov_restart=8,
                                               max_sweeps=200)),
                          ("krylov_oras_tight", dict(base, method=2, krylov_restart=8,
                                                     max_sweeps=200,
                                                     rel_tol=base["rel_tol"] / 10))]:
            with ddi.Plan(h, w, C, **prm) as plan:
                ms, st = timed_solves(plan, f, c, u, 5)
            row[name] = {"ms": round(ms, 3), "ms_per_mpx": round(ms / (h * w / 1e6), 4),
                         "finest_iterations": st["sweeps"],
                         "max_dev_from_tight_solve_grey": round(float((u - ref).abs().max()), 4)}
            if name.startswith("mlcg"):
                row[name]["cg_steps_all_levels"] = st["cg_steps"]
        row["mlcg_over_oras"] = round(row["mlcg"]["ms"] / row["oras"]["ms"], 2)
        row["mlcg_tight_over_oras"] = round(row["mlcg_tight"]["ms"] / row["oras"]["ms"], 2)
        row["krylov_over_oras"] = round(row["krylov_oras"]["ms"] / row["oras"]["ms"], 2)
        row["krylov_tight_over_oras"] = round(row["krylov_oras_tight"]["ms"] / row["oras"]["ms"],
                                              2)
        rows.append(row)
        print(f"[bench] {row}", file=sys.stderr, flush=True)
    out = {"metric": "solve time vs resolution: multilevel ORAS against multilevel CG",
           "value": rows[-1]["mlcg_over_oras"], "unit": "x (ML-CG time / ORAS time at 4K)",
           "higher_is_better": True, "n_gpus": 1, "data": "synthetic", "dtype": "f32",
           "config": {"workload": "RGB frames 960x540, 1920x1080, 3840x2160, 4% Bernoulli; both "
                                  "methods stop at rel_tol 5e-4 on the finest level (ML-CG on "
                                  "every level)"},
           "rows": rows, "roofline": None}
    print(json.dumps(out), flush=True)


def run_serve(args) -> dict:
    """Poisson stream of mixed-resolution requests through the serving loop
    (slot pools under an HBM budget, graph replays, results copied back to
    host memory), then the same requests all at once (saturation), then the
    plain single-image path on them. The first served result of every
    (size, frame) pair is kept and one per size is checked against the
    float64 oracle."""
    import torch
    from paper_2110_03946_amd import serve
    reqs, pool_dens = serve.poisson_stream(SERVE_RATE, args.serve_seconds)
    print(f"[bench] serve: {len(reqs)} requests; generating the frame pool", file=sys.stderr,
          flush=True)
    pool, host_pool = serve.frame_pool(pool_dens, workers=gen_workers(), keep_host=True)
    kept = {}

    def on_result(req, u):
        key = (req.size, req.frame)
        if key not in kept:
            kept[key] = u.numpy().copy()

    srv = serve.Server(budget_bytes=args.serve_budget_gb << 30, on_result=on_result)
    srv.warmup(pool)
    kept.clear()
    print("[bench] serve: the stream in real time", file=sys.stderr, flush=True)
    rt = srv.run(reqs, pool, realtime=True).summary()
    print("[bench] saturation", file=sys.stderr, flush=True)
    sat_reqs, _ = serve.poisson_stream(SERVE_RATE, args.serve_seconds)
    sat = srv.run(sat_reqs, pool, realtime=False).summary()
    srv.close()
    plain_reqs, _ = serve.poisson_stream(SERVE_RATE, args.serve_seconds)
    plain = serve.plain_path(plain_reqs, pool)
    out = {"metric": METRIC_SERVE, "value": rt["frames_per_s"], "unit": "frames/s", "n_gpus": 1,
           "steps": len(reqs), "warmup": 1, "ms_per_step": round(1e3 / rt["frames_per_s"], 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"Poisson arrivals {SERVE_RATE:.0f}/s for {args.serve_seconds:.0f} "
                                  "s: 50% 1920x1080, 30% 3840x2160, 20% 1280x720 RGB f32, "
                                  "Bernoulli masks 2-8 %; slot pools under an HBM budget, "
                                  "HIP-graph replays, results copied to host memory"},
           "p50_ms": rt["p50_ms"], "p99_ms": rt["p99_ms"], "realtime": rt, "saturation": sat,
           "plain_single_image_path": plain, "roofline": None}
    if not args.no_cpu:
        import oracle
        err, checked = 0.0, []
        for size in sorted({k[0] for k in kept}):
            k = min(kk for kk in kept if kk[0] == size)
            f, c = host_pool[k[0]][k[1]]
            ex = oracle.solve_exact(f.astype(np.float64), c)
            err = max(err, float(np.abs(kept[k].astype(np.float64) - ex).max()))
            checked.append(f"{size[1]}x{size[0]}")
        out["max_err_grey"] = round(err, 4)
        out["max_err_checked"] = f"one served result per size ({', '.join(checked)})"
    return out


BATCH_N, BATCH_SEED = 48, 2
BATCHES_IN_FLIGHT = 3
METRIC_BATCH = "batched uneven RGB frames/s at ≤0.5 grey-level err vs FP64"


def batch_class(s: dict) -> str:
    """Autotuner class of a batch image: size, mask kind, density bucket."""
    from paper_2110_03946_amd import autotune
    lo, hi = next((b for b in autotune.DENSITY_BUCKETS if b[0] <= s["density"] <= b[1]),
                  autotune.DENSITY_BUCKETS[-1])
    return f'{s["h"]}x{s["w"]}/{s["kind"]}/{lo:.2f}-{hi:.2f}'


def run_batch(args) -> dict:
    """48 uneven RGB images in one batched solve per step (autotuned
    parameters per image class), beside the plain single-image path on the
    same images; the result of one image per class is checked against the
    float64 oracle."""
    import torch
    from paper_2110_03946_amd import ddi, synth
    specs = synth.batch_specs(BATCH_N, BATCH_SEED)
    print(f"[bench] batch: generating {len(specs)} images", file=sys.stderr, flush=True)
    data = synth.make_workloads([(s["h"], s["w"], C, s["density"], s["kind"], BATCH_SEED,
                                  s["index"]) for s in specs], workers=gen_workers())
    fs = [torch.from_numpy(f).cuda() for f, _ in data]
    cs = [torch.from_numpy(c).cuda() for _, c in data]
    us = [torch.empty_like(f) for f in fs]
    prms = batch_params(specs)
    for p in prms:
        p.timing = 0  # the timed batches run as a caller would (no timing events)
        p.final_residual = 0
    sizes = [(s["h"], s["w"]) for s in specs]
    # several batched solves in flight, each batch plan on a stream of its
    # own and driven by a host thread of its own (the library call releases
    # the interpreter lock): one batch's coarse levels and stop tests run
    # beside another's sweeps
    import threading
    nb = args.batches_in_flight
    streams = concurrent_streams(nb) if nb > 1 else [None]
    streams = [streams[i % len(streams)] for i in range(nb)]
    bs = [ddi.Batch(sizes, C, params=[ddi.Params.from_buffer_copy(p) for p in prms], stream=s)
          for s in streams]
    uss = [us] + [[torch.empty_like(f) for f in fs] for _ in range(nb - 1)]
    b = bs[0]
    for _ in range(args.warmup):
        for bb, uu in zip(bs, uss):
            bb.solve(fs, cs, uu)
    torch.cuda.synchronize()
    lat, sweeps = [], []
    lock = threading.Lock()
    errors = []

    def worker(k):
        try:
            for _ in range(k, args.steps, nb):
                ts = time.perf_counter()
                _, st, _ = bs[k].solve(fs, cs, uss[k])
                dt = (time.perf_counter() - ts) * 1e3
                with lock:
                    lat.append(dt)
                    sweeps[:] = [x["sweeps"] for x in st]
        except Exception as e:  # re-raised in the main thread
            errors.append(e)

    threads = [threading.Thread(target=worker, args=(k,)) for k in range(nb)]
    t0 = time.perf_counter()
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if errors:
        raise errors[0]
    fps = args.steps * len(specs) / elapsed
    # the finest batched sweeps' durations and CG steps (roofline), outside
    # the timed region: batched solves one at a time on a plan with timing
    # events
    tprms = [ddi.Params.from_buffer_copy(p) for p in prms]
    for p in tprms:
        p.timing = 1
    sweep_ms = flops = bytes_ = 0.0
    launches = 0
    with ddi.Batch(sizes, C, params=tprms) as bt:
        bt.solve(fs, cs, uss[-1])
        for _ in range(5):
            _, st, _ = bt.solve(fs, cs, uss[-1])
            for (h, w), p, x in zip(sizes, tprms, st):
                a, bb = sweep_work(p.as_dict(), x["sweeps"], x["cg_steps"], h, w,
                                   skipped=x["skipped_blocks"], unwritten=x["unwritten_blocks"])
                flops += a
                bytes_ += bb
            sweep_ms += st[0]["sweep_ms"]
            launches += max(x["sweeps"] for x in st)
    # one batch at a time: the latency of a batched solve on its own
    lat1 = []
    for _ in range(max(3, min(args.steps // 2, 10))):
        ts = time.perf_counter()
        b.solve(fs, cs, us)
        lat1.append((time.perf_counter() - ts) * 1e3)
    for bb in bs[1:]:
        bb.close()

    # the plain single-image path on the same images and parameters
    plans = []
    for (h, w), p in zip(sizes, prms):
        q = ddi.Params.from_buffer_copy(p)
        q.timing = 0
        plans.append(ddi.Plan(h, w, C, params=q))
    for pl, f, c, u in zip(plans, fs, cs, us):
        pl.solve(f, c, u)
    torch.cuda.synchronize()
    reps = max(1, args.steps // 5)
    single_lat = []
    t1 = time.perf_counter()
    for _ in range(reps):
        for pl, f, c, u in zip(plans, fs, cs, us):
            ts = time.perf_counter()
            pl.solve(f, c, u)
            single_lat.append((time.perf_counter() - ts) * 1e3)
    torch.cuda.synchronize()
    single_fps = reps * len(specs) / (time.perf_counter() - t1)
    for pl in plans:
        pl.close()
    b.solve(fs, cs, us)  # us hold the batched results again

    roofline = roofline_of(flops, bytes_, sweep_ms, launches)
    roofline.update({"traffic": None,
                     "kernel": "k_sweep2_batch (finest-level ORAS sweep, all images)"})
    npix = sum(h * w for h, w in sizes)
    out = {"metric": METRIC_BATCH, "value": round(fps, 2), "unit": "frames/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(elapsed / args.steps * 1e3, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{len(specs)} RGB f32 images of uneven size "
                                  "(640x480/1280x720/1920x1080/3840x2160), masks 2-10 %, half "
                                  "clustered; batched multilevel ORAS, autotuned per class",
                      "images": len(specs), "megapixels": round(npix / 1e6, 2)},
           "p50_ms": round(float(np.percentile(lat, 50)), 3),
           "p99_ms": round(float(np.percentile(lat, 99)), 3),
           "batches_in_flight": nb,
           "one_batch_at_a_time": {"p50_ms": round(float(np.percentile(lat1, 50)), 3),
                                   "p99_ms": round(float(np.percentile(lat1, 99)), 3)},
           "single_image_path": {"frames_per_s": round(single_fps, 2),
                                 "p50_ms": round(float(np.percentile(single_lat, 50)), 3),
                                 "p99_ms": round(float(np.percentile(single_lat, 99)), 3)},
           "batch_speedup": round(fps / single_fps, 3),
           "sweeps_per_image": [min(sweeps), max(sweeps)],
           "roofline": roofline}
    if not args.no_cpu:
        # one image of every autotuned class (size x mask kind x density
        # bucket) present in the batch, against the float64 oracle
        import oracle
        seen, sample = set(), []
        for i, sp in enumerate(specs):
            k = batch_class(sp)
            if k not in seen:
                seen.add(k)
                sample.append(i)
        print(f"[bench] batch: oracle on {len(sample)} images (one per class)", file=sys.stderr,
              flush=True)
        t = 0.0
        err, per_class = 0.0, {}
        for i in sample:
            f, c = data[i]
            t0 = time.perf_counter()
            ex = oracle.solve_exact(f.astype(np.float64), c)
            t += time.perf_counter() - t0
            e = float(np.abs(us[i].cpu().numpy().astype(np.float64) - ex).max())
            per_class[batch_class(specs[i])] = round(e, 4)
            err = max(err, e)
        spix = sum(specs[i]["h"] * specs[i]["w"] for i in sample)
        out["cpu_baseline"] = {
            "value": round(spix / t / (npix / len(specs)), 4), "unit": "frames/s",
            "cores": oracle.threads(), "kind": "oracle",
            "sample": f"{len(sample)} images, one per autotuned class ({spix / 1e6:.1f} Mpx, "
                      f"{t:.1f} s): float64 CG to relative residual 1e-12; pixel rate scaled "
                      "to frames of the batch's mean size"}
        out["max_err_grey"] = round(err, 4)
        out["max_err_grey_per_class"] = per_class
    b.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle legs")
    ap.add_argument("--frames-in-flight", type=int, default=FRAMES_IN_FLIGHT,
                    help="4k and precision workloads: plans (one stream each) with a frame in flight")
    ap.add_argument("--batches-in-flight", type=int, default=BATCHES_IN_FLIGHT,
                    help="batch workload: batch plans (one stream and host thread each)")
    ap.add_argument("--workload", choices=["4k", "batch", "precision", "serve", "ablation", "psnr",
                                           "scaling"], default="4k")
    ap.add_argument("--legs", default="batch,precision,serve",
                    help="4k workload: compact runs of these workloads added to the line as "
                         "keys (comma list; empty for none)")
    ap.add_argument("--serve-seconds", type=float, default=SERVE_SECONDS)
    ap.add_argument("--serve-budget-gb", type=int, default=16)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain 256 MiB device-to-device copy (the known-size "
                         "reference for FETCH_SIZE / WRITE_SIZE counters) and exit")
    ap.add_argument("--summarize-trace", metavar="CSV",
                    help="print a per-kernel, per-grid table of a rocprofv3 kernel trace and exit")
    args = ap.parse_args()
    if args.summarize_trace:
        print(summarize_trace(args.summarize_trace))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); this solver has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        n = 64 << 20  # 64 Mi float32 = 256 MiB each way
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": 4 * n}), flush=True)
        return
    from paper_2110_03946_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    if not torch.cuda.is_available():
        print("no GPU", file=sys.stderr)
        sys.exit(1)
    if args.workload == "batch":
        print(json.dumps(run_batch(args)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(run_serve(args)), flush=True)
        return
    if args.workload == "ablation":
        run_ablation(args)
        return
    if args.workload == "psnr":
        run_psnr(args)
        return
    if args.workload == "scaling":
        run_scaling(args)
        return
    if args.workload == "precision":
        print(json.dumps(run_frame(args, "precision")), flush=True)
        return

    out = run_frame(args, "4k")
    # compact runs of the other workloads, each against the plain
    # single-image path on the same GPU where it has one
    legs = [x for x in args.legs.split(",") if x]
    for leg in legs:
        t0 = time.perf_counter()
        sub = argparse.Namespace(**vars(args))
        if leg == "batch":
            sub.steps, sub.warmup = 6, 1
            r = run_batch(sub)
        elif leg == "precision":
            sub.steps, sub.warmup = 20, 2
            r = run_frame(sub, "precision")
        elif leg == "serve":
            sub.serve_seconds = 5.0
            r = run_serve(sub)
        else:
            raise SystemExit(f"unknown leg {leg!r}")
        r["leg_wall_s"] = round(time.perf_counter() - t0, 1)
        out[leg] = r
        print(f"[bench] leg {leg}: {r['value']} {r['unit']} ({r['leg_wall_s']} s)",
              file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
