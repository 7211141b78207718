"""Autotuner of the solver parameters per workload class.

A class is an image size with a mask kind and a density range. For each
class the tuner takes four seeded tuning images at the hard end of the
density range: of 16 seeded mask draws, the four whose largest hole (the
largest distance from an unknown pixel to the nearest known one) is widest,
since the width of the widest hole is what the local solves and the coarse
levels must bridge; and in the last of them a quarter disk of radius 1.5
times the widest of those holes is cut into a corner (a hole at the border
is the hardest kind: the reflecting boundary gives it no known pixel on that
side; 1.5 covers the rare frames whose widest hole lies beyond every draw,
such as a 28-pixel corner hole at 640 x 480 and 2 % against at most 19 in 64
draws), computes a reference solution with the solver itself run to
a tight tolerance (no oracle is involved), and searches the parameters --
block size and overlap, CG steps per local solve on the finest and coarser
levels, the local stop tolerance, the number of levels and the coarse-level
sweeps -- by coordinate descent. A candidate is scored by

  * its error curve: for n = 1 .. n_max finest-level sweeps, the returned
    iterate's float64 relative residual and its max-abs distance to the
    reference;
  * its sweep floor: the number of finest-level sweeps from which every
    tuning image's error stays below `target` (a margin under the 0.5
    grey-level bar) up to n_max. It becomes the class's min_sweeps, so the
    bar rests on a sweep count measured for the class and not on the
    residual alone (after few sweeps a small residual can come with a large
    error);
  * the stop tolerance it needs from there: the largest relative residual
    tolerance such that on every tuning image the first sweep from the floor
    on that meets it has an error below `target` and lies clear of the
    residual floor the local stop tolerance leaves; an image whose residual
    at the floor is larger than the tuning images' goes on sweeping;
  * its cost: the measured device time per image of a batched solve of
    copies of the tuning images with that tolerance (enough copies to fill
    the GPU, as in the batched workload, so small images are not scored by
    their launch latency).

The search covers the tile shape on every level: the finest block size and
overlap, and the block size and overlap of the coarser levels.

The table the tuner writes (JSON) maps each class to the winning parameters
including rel_tol and min_sweeps; `params_for` looks an image up in it.

  python -m paper_2110_03946_amd.autotune --out table.json [--quick]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import ddi, synth

# parameters shared by every class: the batched solve runs the finest-level
# sweeps of all images in lock step, so the sweep cap and the test spacing
# are common (min_sweeps, the sweep floor, is per class)
SCHEDULE = dict(max_sweeps=60, check_every=1)

# starting points of the search: a light one (fast where the mask is easy),
# one with more coarse CG work and a looser finest-level local stop, and a
# robust one (large holes: more levels and coarse work, longer local solves,
# a tighter local stop)
STARTS = [
    dict(block=64, overlap=4, levels=4, local_iters=16, robin_alpha=0.25,
         coarse_sweeps=1, coarsest_sweeps=1, coarse_local_iters=4, local_tol=0.002,
         coarse_block=0, coarse_overlap=-1),
    dict(block=64, overlap=4, levels=4, local_iters=16, robin_alpha=0.25,
         coarse_sweeps=1, coarsest_sweeps=1, coarse_local_iters=8, local_tol=0.004,
         coarse_block=0, coarse_overlap=-1),
    dict(block=64, overlap=4, levels=5, local_iters=24, robin_alpha=0.25,
         coarse_sweeps=2, coarsest_sweeps=4, coarse_local_iters=16, local_tol=0.0005,
         coarse_block=0, coarse_overlap=-1),
]

SPACE = [
    ("local_iters", [12, 16, 24, 32]),
    ("local_tol", [0.0, 0.0005, 0.001, 0.002, 0.003, 0.004, 0.006]),
    ("levels", [3, 4, 5, 6]),
    ("coarse_local_iters", [4, 8, 16]),
    ("coarse_sweeps", [1, 2, 3]),
    ("coarsest_sweeps", [1, 2, 4]),
    ("overlap", [2, 4, 8]),
    ("block", [32, 48, 64]),
    ("coarse_block", [0, 32, 48]),
    ("coarse_overlap", [-1, 2, 8]),
    ("robin_alpha", [0.15, 0.25, 0.4]),
]

# classes of the batched workload: sizes x mask kinds x density ranges
DENSITY_BUCKETS = ((0.02, 0.05), (0.05, 0.10))
KINDS = ("bernoulli", "clustered")

REF_PARAMS = dict(block=64, overlap=8, levels=5, local_iters=32, robin_alpha=0.25,
                  coarse_sweeps=3, coarsest_sweeps=6, coarse_local_iters=16, local_tol=0.0,
                  rel_tol=2e-7, min_sweeps=1, max_sweeps=400, check_every=4, final_residual=1)


def class_key(h: int, w: int, kind: str, lo: float, hi: float) -> str:
    return f"{h}x{w}/{kind}/{lo:.2f}-{hi:.2f}"


def _torch():
    import torch
    return torch


def reference(f, c, channels):
    """Tight solve with the solver itself (the tuning reference)."""
    torch = _torch()
    h, w = c.shape
    with ddi.Plan(h, w, channels, **REF_PARAMS) as plan:
        u, st = plan.solve(f, c, allow_noconv=True)
    torch.cuda.synchronize()
    return u, st


def curve(prm: dict, imgs, n_max: int, repeats: int = 1):
    """Per image: arrays rel[n], err[n], ms[n] for n = 1 .. n_max sweeps
    (ms: the solo solve's device time)."""
    torch = _torch()
    out = []
    for f, c, uref in imgs:
        h, w = c.shape
        C = f.shape[0]
        rel, err, ms = [], [], []
        u = torch.empty_like(f)
        for n in range(1, n_max + 1):
            p = dict(prm, min_sweeps=n, max_sweeps=n, rel_tol=0.0, final_residual=1)
            with ddi.Plan(h, w, C, **p) as plan:
                best = float("inf")
                for _ in range(repeats):
                    _, st = plan.solve(f, c, u, allow_noconv=True)
                    best = min(best, st["ms"])
            rel.append(st["rel_residual"])
            err.append(float((u - uref).abs().max()))
            ms.append(best)
        out.append((np.array(rel), np.array(err), np.array(ms)))
    return out


def batch_cost(prm: dict, tol: float, imgs, values: float = 2.0e7, repeats: int = 3,
               min_sweeps: int = 1) -> float:
    """Device ms per image of a batched solve of copies of the tuning
    images (about `values` float32 values per batch)."""
    torch = _torch()
    per = sum(f.numel() for f, _, _ in imgs)
    reps = max(1, int(round(values / per)))
    fs = [f for f, _, _ in imgs] * reps
    cs = [c for _, c, _ in imgs] * reps
    us = [torch.empty_like(f) for f in fs]
    p = ddi.default_params(**dict(prm, rel_tol=tol, final_residual=0, min_sweeps=min_sweeps,
                                  **SCHEDULE))
    with ddi.Batch([tuple(c.shape) for c in cs], fs[0].shape[0], params=p) as b:
        b.solve(fs, cs, us, allow_noconv=True)
        best = float("inf")
        for _ in range(repeats):
            _, st, _ = b.solve(fs, cs, us, allow_noconv=True)
            best = min(best, st[0]["ms"])
    return best / len(fs)


def sweep_floor(curves, target: float):
    """Smallest n such that from sweep n on every image's error stays below
    target up to the last sweep of its curve; None when none does."""
    n_max = min(len(err) for _, err, _ in curves)
    for n in range(1, n_max + 1):
        if all(float(np.max(err[n - 1:n_max])) <= target for _, err, _ in curves):
            return n
    return None


def pick_tol(curves, target: float, min_sweeps: int = 2):
    """Largest tolerance meeting the error target on every image, its mean
    cost and stop sweeps; None when no tolerance does."""
    floor = max(float(r[-1]) for r, _, _ in curves)
    cands = sorted({float(x) for r, _, _ in curves for x in r[min_sweeps - 1:]}, reverse=True)
    for tol in cands:
        if tol < 1.5 * floor:
            break
        stops, ok = [], True
        for rel, err, _ in curves:
            idx = [i for i in range(min_sweeps - 1, len(rel)) if rel[i] <= tol]
            if not idx or err[idx[0]] > target:
                ok = False
                break
            stops.append(idx[0])
        if ok:
            cost = float(np.mean([ms[i] for (_, _, ms), i in zip(curves, stops)]))
            return tol, cost, [i + 1 for i in stops]
    return None


TUNE_WORKLOAD = 90  # workload seed of the tuning draws


def widest_holes(h, w, kind, density, n_pick=4, n_draw=16, workload=TUNE_WORKLOAD):
    """Indices of the n_pick masks, among n_draw seeded draws, whose largest
    hole (distance from an unknown pixel to the nearest known pixel) is
    widest, widest first."""
    from scipy import ndimage
    scores = []
    for i in range(n_draw):
        c = synth.make_mask(h, w, density, kind, synth.mask_seed(workload, i))
        scores.append((float(ndimage.distance_transform_edt(c == 0).max()), i))
    scores.sort(key=lambda t: (-t[0], t[1]))
    return [i for _, i in scores[:n_pick]]


def corner_hole(c, masks, factor: float = 1.5):
    """c with a quarter disk of radius `factor` times the widest hole of
    `masks` cleared at the top-left corner (at least one known pixel is
    kept elsewhere); returns (mask, radius)."""
    from scipy import ndimage
    r = factor * max(float(ndimage.distance_transform_edt(m == 0).max()) for m in masks)
    h, w = c.shape
    yy, xx = np.mgrid[0:h, 0:w]
    out = c.copy()
    out[yy * yy + xx * xx < r * r] = 0
    if not out.any():
        out[h - 1, w - 1] = 1
    return out, round(r, 1)


def tune_class(h, w, kind, lo, hi, channels=3, seeds=None, target=0.3, n_max=24,
               passes=2, log=print):
    torch = _torch()
    if seeds is None:
        seeds = widest_holes(h, w, kind, lo)
    imgs = []
    radius = None
    for k, s in enumerate(seeds):
        f, c = synth.make_workload(h, w, channels, lo, kind, workload=TUNE_WORKLOAD, index=s)
        if k == len(seeds) - 1 and len(seeds) > 1:
            c, radius = corner_hole(c, [synth.make_mask(h, w, lo, kind,
                                                        synth.mask_seed(TUNE_WORKLOAD, t))
                                        for t in seeds])
        fd = torch.from_numpy(f).cuda()
        cd = torch.from_numpy(c).cuda()
        uref, st = reference(fd, cd, channels)
        log(f"  reference seed {s}: {st['sweeps']} sweeps, rel {st['rel_residual']:.2e}")
        imgs.append((fd, cd, uref))

    def score(prm):
        """(rank, res): feasible candidates rank by cost; infeasible ones
        after them, by their worst error after n_max sweeps."""
        cb = prm.get("coarse_block", 0) or prm["block"]
        co = prm.get("coarse_overlap", -1)
        co = prm["overlap"] if co < 0 else co
        if prm["overlap"] >= prm["block"] or co >= cb or \
                ddi.check_params(h, w, channels, ddi.default_params(**prm, **SCHEDULE)) != 0:
            return (2, float("inf")), None
        cv = curve(prm, imgs, n_max)
        floor = sweep_floor(cv, target)
        res = pick_tol(cv, target, min_sweeps=floor) if floor else None
        if res is None:
            return (1, max(float(err[-1]) for _, err, _ in cv)), None
        cost = batch_cost(prm, res[0], imgs, min_sweeps=floor)
        return (0, cost), (res[0], cost, res[2], floor)

    best, best_rank, best_res = None, None, None
    for start in STARTS:
        rank, res = score(start)
        log(f"  start {start}: {rank}")
        if best_rank is None or rank < best_rank:
            best, best_rank, best_res = dict(start), rank, res
    for _ in range(passes):
        improved = False
        for key, values in SPACE:
            for v in values:
                if best.get(key) == v:
                    continue
                cand = dict(best, **{key: v})
                rank, res = score(cand)
                if rank < best_rank:
                    best, best_rank, best_res, improved = cand, rank, res, True
                    log(f"  {key}={v}: {rank}" +
                        (f" tol {res[0]:.3g}, sweeps {res[2]}" if res else ""))
        if not improved:
            break
    if best_res is None:
        raise RuntimeError(f"no parameters meet the target for {h}x{w} {kind} {lo}-{hi}")
    tol, cost, stops, floor = best_res
    return dict(params=dict(best, rel_tol=tol, min_sweeps=floor, **SCHEDULE),
                tuning=dict(ms=round(cost, 4), sweeps=stops, floor=floor, target=target,
                            seeds=list(seeds), corner_hole_radius=radius, density=lo))


def load_table(path: str | None = None) -> dict:
    path = path or os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_params.json")
    with open(path) as fh:
        return json.load(fh)


def params_for(table: dict, h: int, w: int, kind: str, density: float) -> dict:
    """Parameters of the class nearest to (h, w, kind, density): same kind,
    the density bucket holding `density` (else the nearest), the size with
    the nearest pixel count."""
    best, key_best = None, None
    for key, entry in table["classes"].items():
        size, k, dens = key.split("/")
        if k != kind:
            continue
        ch, cw = (int(x) for x in size.split("x"))
        lo, hi = (float(x) for x in dens.split("-"))
        dd = 0.0 if lo <= density <= hi else min(abs(density - lo), abs(density - hi))
        ds = abs(np.log((ch * cw) / float(h * w)))
        score = (dd, ds)
        if best is None or score < best:
            best, key_best = score, key
    if key_best is None:
        raise KeyError(f"no tuned class for mask kind {kind!r}")
    return dict(table["classes"][key_best]["params"])


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--quick", action="store_true", help="one pass, smallest sizes only")
    ap.add_argument("--sizes", default=None, help="comma list of HxW (default: the batch sizes)")
    args = ap.parse_args(argv)
    torch = _torch()
    if not torch.cuda.is_available():
        print("the tuner needs a GPU", file=sys.stderr)
        return 1
    ddi.lib()
    sizes = synth.BATCH_SIZES
    if args.sizes:
        sizes = [tuple(int(v) for v in s.split("x")) for s in args.sizes.split(",")]
    if args.quick:
        sizes = sizes[:1]
    table = {"schedule": SCHEDULE, "classes": {},
             "command": "python -m paper_2110_03946_amd.autotune " + " ".join(argv or sys.argv[1:])}
    t0 = time.time()
    for h, w in sizes:
        for kind in KINDS:
            for lo, hi in DENSITY_BUCKETS:
                key = class_key(h, w, kind, lo, hi)
                print(f"class {key}", flush=True)
                table["classes"][key] = tune_class(h, w, kind, lo, hi,
                                                   passes=1 if args.quick else 2,
                                                   log=lambda s: print(s, flush=True))
                print(f"  -> {json.dumps(table['classes'][key])}  [{time.time() - t0:.0f} s]",
                      flush=True)
                with open(args.out, "w") as fh:
                    json.dump(table, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
