"""Seeded synthetic inputs for homogeneous diffusion inpainting.

This module only draws test data: images f and binary masks c. It holds none
of the inpainting arithmetic, so both the CPU oracle and the HIP path can be
fed from it without sharing any code of the method.

The paper evaluates on one 4K photograph with a 5 % mask obtained by Voronoi
densification (Sec. 5); neither is available, so these generators stand in for
them with the same shapes (H x W x 3, grey values in [0, 255]) and the same
density class (2-10 % known pixels).

Image recipe, per channel, numpy ``default_rng(seed + channel)``:
  * 8 Gaussian blobs, centre uniform over the image, sigma uniform in
    [0.02, 0.25] * min(H, W), amplitude uniform in [-1, 1];
  * 4 axis-aligned rectangles with uniform corners, each adding a constant
    uniform in [-0.5, 0.5] inside;
  * affine normalisation of the channel to [0, 255].

Mask recipes, numpy ``default_rng(seed)``:
  * ``bernoulli``: every pixel known independently with probability d;
  * ``clustered``: seeds drawn with probability s = 1 - (1 - d)**(1/9), then
    dilated by a 3x3 box (clipped at the border), so a pixel is known with
    probability d;
  * at least one known pixel is forced (pixel (0, 0)) so the system is
    never singular.

Seed convention used by the tests and the benchmark: image seed
``1000 * workload + index``, mask seed ``image seed + 500``.

Batch recipe (``batch_specs``), numpy ``default_rng(seed)``: n images, sizes
uniform over 640x480, 1280x720, 1920x1080 and 3840x2160, mask densities
uniform in [0.02, 0.10], exactly half of the masks clustered (a random half),
the rest Bernoulli.
"""
from __future__ import annotations

import numpy as np

__all__ = ["make_image", "make_mask", "make_workload", "make_workloads", "image_seed",
           "mask_seed", "batch_specs", "BATCH_SIZES"]


def image_seed(workload: int, index: int = 0) -> int:
    return 1000 * workload + index


def mask_seed(workload: int, index: int = 0) -> int:
    return image_seed(workload, index) + 500


def _channel(h: int, w: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    ys = np.arange(h, dtype=np.float64)
    xs = np.arange(w, dtype=np.float64)
    img = np.zeros((h, w), dtype=np.float64)
    m = float(min(h, w))
    for _ in range(8):
        cy = rng.uniform(0, h)
        cx = rng.uniform(0, w)
        sig = rng.uniform(0.02, 0.25) * m
        amp = rng.uniform(-1.0, 1.0)
        gy = np.exp(-0.5 * ((ys - cy) / sig) ** 2)
        gx = np.exp(-0.5 * ((xs - cx) / sig) ** 2)
        img += amp * np.outer(gy, gx)
    for _ in range(4):
        y0, y1 = np.sort(rng.integers(0, h + 1, size=2))
        x0, x1 = np.sort(rng.integers(0, w + 1, size=2))
        img[y0:y1, x0:x1] += rng.uniform(-0.5, 0.5)
    lo, hi = img.min(), img.max()
    if hi > lo:
        img = (img - lo) * (255.0 / (hi - lo))
    else:
        img[:] = 127.5
    return img


def make_image(h: int, w: int, channels: int = 1, seed: int = 0) -> np.ndarray:
    """Float32 image of shape (channels, h, w), values in [0, 255]."""
    out = np.empty((channels, h, w), dtype=np.float32)
    for ch in range(channels):
        out[ch] = _channel(h, w, seed + ch)
    return out


def make_mask(h: int, w: int, density: float, kind: str = "bernoulli",
              seed: int = 0) -> np.ndarray:
    """uint8 mask of shape (h, w): 1 = known pixel, 0 = to be inpainted."""
    rng = np.random.default_rng(seed)
    if kind == "bernoulli":
        c = rng.random((h, w)) < density
    elif kind == "clustered":
        s = 1.0 - (1.0 - density) ** (1.0 / 9.0)
        seeds = rng.random((h, w)) < s
        c = np.zeros((h + 2, w + 2), dtype=bool)
        for dy in range(3):
            for dx in range(3):
                c[dy:dy + h, dx:dx + w] |= seeds
        c = c[1:h + 1, 1:w + 1]
    else:
        raise ValueError(f"unknown mask kind {kind!r}")
    c = c.astype(np.uint8)
    if not c.any():
        c[0, 0] = 1
    return c


def make_workload(h: int, w: int, channels: int, density: float,
                  kind: str = "bernoulli", workload: int = 0, index: int = 0):
    """(f, c) pair with the seed convention above."""
    f = make_image(h, w, channels, image_seed(workload, index))
    c = make_mask(h, w, density, kind, mask_seed(workload, index))
    return f, c


def _workload_args(a):
    return make_workload(*a)


def make_workloads(args, workers: int = 0):
    """make_workload for each argument tuple of `args` (h, w, channels,
    density, kind, workload, index), in worker processes started fresh
    (spawn: they import numpy and this module only) when workers > 1;
    the results are identical to sequential calls."""
    args = [tuple(a) for a in args]
    if workers <= 1 or len(args) <= 1:
        return [make_workload(*a) for a in args]
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=min(workers, len(args)),
                             mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_workload_args, args))


# (height, width) of the batch recipe
BATCH_SIZES = ((480, 640), (720, 1280), (1080, 1920), (2160, 3840))


def batch_specs(n: int = 48, seed: int = 2, sizes=BATCH_SIZES,
                densities=(0.02, 0.10)):
    """List of n dicts (h, w, density, kind, index) for a batch of uneven
    images; the data of entry i is make_workload(h, w, C, density, kind,
    workload=seed, index=i)."""
    rng = np.random.default_rng(seed)
    pick = rng.integers(0, len(sizes), size=n)
    dens = rng.uniform(densities[0], densities[1], size=n)
    clustered = np.zeros(n, dtype=bool)
    clustered[rng.permutation(n)[: n // 2]] = True
    return [dict(h=int(sizes[k][0]), w=int(sizes[k][1]), density=float(d),
                 kind="clustered" if cl else "bernoulli", index=i)
            for i, (k, d, cl) in enumerate(zip(pick, dens, clustered))]
