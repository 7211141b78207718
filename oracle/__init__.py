"""CPU oracle for multilevel ORAS homogeneous diffusion inpainting.

TEST INFRASTRUCTURE ONLY. This package is imported by the test suite, by
``__graft_entry__.smoke()`` and by the CPU-baseline leg of ``bench.py`` and
by nothing else. It shares no code with the HIP path: no kernels, headers,
helpers, tables or constants. Both sides are fed from the seeded generators
in ``paper_2110_03946_amd.synth``, which hold none of the method's
arithmetic.

Everything here is plain and slow on purpose: float64 throughout, each
function written from the passage of Kaemper & Weickert, "Domain
decomposition algorithms for real-time homogeneous diffusion inpainting in
4K" (arXiv 2110.03946), that it cites.

Contents
  solve_exact      exact solution of eq. 6 (A u = b), plain C float64 CG on
                   the reduced SPD system (oracle.c).
  dense_matrix     the literal A = C - (I - C) L and b = C f of eq. 6 as
                   dense arrays, for images up to about 20 x 20.
  dense_solve      LU solve of the literal dense system.
  residual         r = b - A u (eq. 7), relative residual ||r|| / ||b||.
  coarsen          dyadic mask/value subsampling (Sec. 4).
  prolong          bilinear coarse-to-fine interpolation (a reading: the
                   paper does not say how the coarse solution initialises the
                   finer level); fine_start re-imposes u = f on the mask.
  block_origins, owner_bounds
                   overlapping block grid and the Boolean partition of unity
                   (Sec. 3 eq. 10, Sec. 4 block size / overlap).
  local_matrix     R_i A R_i^T of eq. 7 with the Robin interface modification
                   that makes RAS into ORAS (Sec. 3).
  local_cg         k steps of conjugate gradients on a local system (Sec. 4).
  oras_step        one ORAS iteration, eqs. 7-9.
  correction_step  one ORAS iteration on the residual-correction equation
                   A d = r (d = 0 on the mask) that iterative refinement
                   solves: the same local solves and partition of unity
                   applied to a general right-hand side.
  ml_oras          coarse-to-fine multilevel ORAS (Sec. 4).
  apply_matrix     A z for the matrix of eq. 6.
  fgmres_oras, krylov_oras
                   ORAS as a preconditioner of a Krylov method (not in the
                   paper): flexible GMRES(m) (Saad's flexible inner-outer
                   GMRES, 1993) on A u = b, each basis vector preconditioned
                   by one ORAS iteration on the correction equation
                   (correction_step from d = 0), after the coarse-to-fine
                   start of ml_oras.
  inverse_inf_norm ||K_UU^{-1}||_inf, which turns a residual bound into a
                   guaranteed bound on the error of an inpainting.

Parity pinning: every function here is checked in tests/test_oracle_pins.py
against closed forms, invariants, brute force or library routines.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (OpenMP, -O2)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-std=c99", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        lib.oracle_solve.restype = ctypes.c_int
        lib.oracle_solve.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_void_p, ctypes.c_double, ctypes.c_int,
            ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_threads.argtypes = []
        _lib = lib
    return _lib


def threads() -> int:
    """OpenMP threads the C solver uses (OMP_NUM_THREADS or all cores)."""
    return int(_load().oracle_threads())


# ---------------------------------------------------------------------------
# The exact solution (Sec. 2, eqs. 5-6)
# ---------------------------------------------------------------------------

class SingularMask(ValueError):
    """The mask has no known pixel: A is singular (pure Neumann problem)."""


def solve_exact(f, c, tol: float = 1e-12, max_iter: int = 200000,
                return_info: bool = False):
    """Exact inpainting u of eq. 6 for one channel (2-D f) or several
    channels sharing one mask (3-D f of shape (C, H, W)).

    float64 CG on the reduced system over the unknown pixels, from zero, to
    ||g - K u_U|| <= tol ||g||; u = f on the mask, bit for bit.
    """
    f = np.asarray(f)
    c = np.ascontiguousarray(c, dtype=np.uint8)
    if f.ndim == 3:
        outs = [solve_exact(f[k], c, tol, max_iter, True) for k in range(f.shape[0])]
        u = np.stack([o[0] for o in outs])
        info = [o[1] for o in outs]
        return (u, info) if return_info else u
    h, w = c.shape
    if f.shape != (h, w):
        raise ValueError("f and c shapes differ")
    fd = np.ascontiguousarray(f, dtype=np.float64)
    u = np.empty((h, w), dtype=np.float64)
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    st = _load().oracle_solve(h, w, fd.ctypes.data, c.ctypes.data,
                              u.ctypes.data, tol, max_iter,
                              ctypes.byref(it), ctypes.byref(rr))
    if st == 1:
        raise SingularMask("mask has no known pixel")
    if st < 0:
        raise ValueError("oracle_solve rejected its arguments")
    if st == 2:
        raise RuntimeError(f"oracle CG hit max_iter={max_iter}, relres={rr.value:g}")
    info = {"iters": it.value, "relres": rr.value}
    return (u, info) if return_info else u


# ---------------------------------------------------------------------------
# Literal operators (Sec. 2 eqs. 5-6, Sec. 3 eq. 7)
# ---------------------------------------------------------------------------

def laplacian_dense(h: int, w: int) -> np.ndarray:
    """Dense 5-point Laplacian L (Sec. 2) with reflecting boundaries.

    Reflection is half-sample mirroring: the mirrored neighbour of a border
    pixel is the pixel itself, so (u_q - u_p) vanishes for it and the row of
    L only holds the in-image neighbours.
    """
    n = h * w
    L = np.zeros((n, n))
    for i in range(h):
        for j in range(w):
            p = i * w + j
            for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                ii, jj = i + di, j + dj
                if 0 <= ii < h and 0 <= jj < w:
                    L[p, ii * w + jj] += 1.0
                    L[p, p] -= 1.0
    return L


def dense_matrix(f, c):
    """Literal A = C - (I - C) L and b = C f of eq. 6 (dense, float64)."""
    c = np.asarray(c)
    h, w = c.shape
    C = np.diag(c.reshape(-1).astype(np.float64))
    I = np.eye(h * w)
    A = C - (I - C) @ laplacian_dense(h, w)
    b = C @ np.asarray(f, dtype=np.float64).reshape(-1)
    return A, b


def dense_solve(f, c) -> np.ndarray:
    """Solve the literal system of eq. 6 by LU with partial pivoting."""
    A, b = dense_matrix(f, c)
    return np.linalg.solve(A, b).reshape(np.asarray(c).shape)


def residual(f, c, u) -> np.ndarray:
    """r = b - A u (eq. 7) with A, b of eq. 6, float64, elementwise.

    Known pixel p:   r_p = f_p - u_p.
    Unknown pixel p: r_p = (L u)_p = sum over in-image 4-neighbours q of
                     (u_q - u_p).
    """
    f = np.asarray(f, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    c = np.asarray(c)
    lu = np.zeros_like(u)
    lu[..., :, :-1] += u[..., :, 1:] - u[..., :, :-1]
    lu[..., :, 1:] += u[..., :, :-1] - u[..., :, 1:]
    lu[..., :-1, :] += u[..., 1:, :] - u[..., :-1, :]
    lu[..., 1:, :] += u[..., :-1, :] - u[..., 1:, :]
    return np.where(c == 1, f - u, lu)


def rel_residual(f, c, u) -> float:
    """||b - A u||_2 / ||b||_2 with b = C f (whole array, all channels)."""
    r = residual(f, c, u)
    b = np.where(np.asarray(c) == 1, np.asarray(f, dtype=np.float64), 0.0)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(r) / nb) if nb > 0 else float(np.linalg.norm(r))


def reduced_system(c) -> sp.csr_matrix:
    """K = -L restricted to rows and columns of unknown pixels (sparse)."""
    c = np.asarray(c)
    h, w = c.shape
    idx = -np.ones((h, w), dtype=np.int64)
    unk = np.flatnonzero(c.reshape(-1) == 0)
    idx.reshape(-1)[unk] = np.arange(unk.size)
    rows, cols, vals = [], [], []
    for i in range(h):
        for j in range(w):
            if c[i, j]:
                continue
            p = idx[i, j]
            deg = 0
            for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                ii, jj = i + di, j + dj
                if 0 <= ii < h and 0 <= jj < w:
                    deg += 1
                    if not c[ii, jj]:
                        rows.append(p); cols.append(idx[ii, jj]); vals.append(-1.0)
            rows.append(p); cols.append(p); vals.append(float(deg))
    return sp.csr_matrix((vals, (rows, cols)), shape=(unk.size, unk.size))


def inverse_inf_norm(c) -> float:
    """||K^{-1}||_inf for the reduced matrix K of eq. 6.

    K is a nonsingular M-matrix when the mask is nonempty, so K^{-1} >= 0
    entrywise and its row sums are the solution w of K w = 1; the norm is
    max w. With it, ||u - u*||_inf <= ||K^{-1}||_inf * ||r_U||_inf for any u
    that equals f on the mask.
    """
    import scipy.sparse.linalg as spl
    K = reduced_system(c)
    if K.shape[0] == 0:
        return 0.0
    wv = spl.spsolve(K.tocsc(), np.ones(K.shape[0]))
    return float(np.max(wv))


# ---------------------------------------------------------------------------
# Multilevel transfer (Sec. 4)
# ---------------------------------------------------------------------------

def coarsen(f, c):
    """One dyadic subsampling step of Sec. 4.

    Coarse pixel (I, J) covers fine pixels (2I + a, 2J + b), a, b in {0, 1},
    that lie inside the image (odd sizes give partial cells; coarse size is
    ceil(n / 2)). It is known iff at least one of them is known, and its
    value is the mean of the known fine values (the only ones a decoder
    holds). Unknown coarse pixels get value 0.
    """
    f = np.asarray(f, dtype=np.float64)
    c = np.asarray(c)
    h, w = c.shape[-2:]
    hc, wc = (h + 1) // 2, (w + 1) // 2
    shape = f.shape[:-2] + (hc, wc)
    fc = np.zeros(shape)
    cc = np.zeros((hc, wc), dtype=np.uint8)
    for I in range(hc):
        for J in range(wc):
            vals = []
            for a in (0, 1):
                for b in (0, 1):
                    i, j = 2 * I + a, 2 * J + b
                    if i < h and j < w and c[i, j]:
                        vals.append(f[..., i, j])
            if vals:
                cc[I, J] = 1
                fc[..., I, J] = sum(vals) / len(vals)
    return fc, cc


def prolong(uc, h: int, w: int) -> np.ndarray:
    """Bilinear interpolation of a coarse grid to an h x w fine grid.

    Pixel centres: fine pixel y sits at coarse coordinate (y + 0.5)/2 - 0.5,
    i.e. y/2 - 1/4. Interpolation between the two nearest coarse centres,
    with coordinates clamped to the coarse grid (so border pixels copy the
    nearest coarse value, consistent with reflecting boundaries).
    """
    uc = np.asarray(uc, dtype=np.float64)
    hc, wc = uc.shape[-2:]
    out = np.zeros(uc.shape[:-2] + (h, w))
    for y in range(h):
        ty = min(max((y + 0.5) / 2.0 - 0.5, 0.0), hc - 1.0)
        i0 = int(np.floor(ty)); i1 = min(i0 + 1, hc - 1); a = ty - i0
        for x in range(w):
            tx = min(max((x + 0.5) / 2.0 - 0.5, 0.0), wc - 1.0)
            j0 = int(np.floor(tx)); j1 = min(j0 + 1, wc - 1); b = tx - j0
            out[..., y, x] = ((1 - a) * ((1 - b) * uc[..., i0, j0] + b * uc[..., i0, j1])
                              + a * ((1 - b) * uc[..., i1, j0] + b * uc[..., i1, j1]))
    return out


def fine_start(uc, f, c) -> np.ndarray:
    """Initial guess of a finer level (Sec. 4): the coarse solution
    interpolated by prolong(), with u = f re-imposed on the mask."""
    f = np.asarray(f, dtype=np.float64)
    c = np.asarray(c)
    h, w = c.shape
    return np.where(c == 1, f, prolong(uc, h, w))


# ---------------------------------------------------------------------------
# Domain decomposition (Sec. 3, Sec. 4)
# ---------------------------------------------------------------------------

def block_origins(n: int, size: int, overlap: int):
    """Origins of the overlapping blocks along one axis of length n.

    Reading of "block size 32 with an overlap of 6" (Sec. 4): a block spans
    ``size`` pixels including the overlap, neighbours share ``overlap``
    pixels, so the stride is size - overlap; there are
    ceil((n - overlap) / (size - overlap)) blocks and the last one is
    shifted back to end at the border. This gives 148 x 83 blocks per channel
    for 3840 x 2160 at size 32, overlap 6, i.e. the paper's 36852 local
    problems for a colour image. A block longer than the axis is cut to n.
    Returns (origins, effective size).
    """
    if size >= n:
        return [0], n
    if not 0 <= overlap < size:
        raise ValueError("need 0 <= overlap < size")
    stride = size - overlap
    nb = -(-(n - overlap) // stride)
    return [min(k * stride, n - size) for k in range(nb)], size


def owner_bounds(origins, size: int, n: int):
    """Boolean partition of unity along one axis (the D_i of eq. 10).

    Block k owns [lo_k, hi_k): the overlap shared with block k+1 is split at
    its middle, the left half (rounded up) going to block k. Every pixel is
    owned by exactly one block, so sum_i R_i^T D_i R_i = I.
    """
    lo = [0]
    for k in range(len(origins) - 1):
        ov = origins[k] + size - origins[k + 1]
        lo.append(origins[k + 1] + (ov + 1) // 2)
    hi = lo[1:] + [n]
    return lo, hi


def local_matrix(c, y0: int, x0: int, bh: int, bw: int, alpha: float = 1.0):
    """Local matrix of block Omega_i = [y0, y0+bh) x [x0, x0+bw).

    Built row by row from A of eq. 6 restricted to the block's rows and
    columns, which is R_i A R_i^T of eq. 7: a known pixel keeps its identity
    row; an unknown pixel p has diagonal deg(p) (its in-image neighbours in
    the whole image) and -1 towards each neighbour inside the block.
    Neighbours outside the block are dropped -- the implicit homogeneous
    Dirichlet condition of RAS (Sec. 3).

    ORAS (Sec. 3): at the block interface the Dirichlet condition is replaced
    by a Robin condition. An interface neighbour q (in the image, outside the
    block) then enters the diagonal of p with weight alpha instead of 1:
    alpha = 1 is RAS, alpha -> 0 a Neumann condition. The weight is the same
    whatever the mask says at q.
    Returns a sparse (bh*bw) x (bh*bw) float64 matrix in row-major block
    order.
    """
    c = np.asarray(c)
    h, w = c.shape
    m = bh * bw
    M = sp.lil_matrix((m, m))
    for a in range(bh):
        for b in range(bw):
            i, j = y0 + a, x0 + b
            p = a * bw + b
            if c[i, j]:
                M[p, p] = 1.0
                continue
            for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                ii, jj = i + di, j + dj
                if not (0 <= ii < h and 0 <= jj < w):
                    continue  # reflecting image boundary: no neighbour
                aa, bb = a + di, b + dj
                if 0 <= aa < bh and 0 <= bb < bw:
                    M[p, p] += 1.0
                    M[p, aa * bw + bb] -= 1.0
                else:
                    M[p, p] += alpha
    return M.tocsr()


def local_cg(M, rhs, k: int):
    """k steps of conjugate gradients (Hestenes-Stiefel) on M v = rhs, v0 = 0.

    Stops early when r.r or p.Mp becomes zero (the local problem is then
    solved exactly, or the right-hand side vanished).
    """
    v = np.zeros_like(rhs)
    r = rhs.copy()
    p = r.copy()
    rho = float(r @ r)
    for _ in range(k):
        if rho == 0.0:
            break
        q = M @ p
        pq = float(p @ q)
        if pq <= 0.0:
            break
        a = rho / pq
        v = v + a * p
        r = r - a * q
        rho_new = float(r @ r)
        p = r + (rho_new / rho) * p
        rho = rho_new
    return v


def oras_step(u, f, c, size: int, overlap: int, alpha: float, k: int | None,
              blocks=None, size_y: int | None = None, overlap_y: int | None = None):
    """One (O)RAS iteration of Sec. 3 for one channel.

        r^n     = b - A u^n                                   (eq. 7)
        v_i^n   = (local matrix of block i)^{-1} R_i r^n      (eq. 7)
        u^{n+1} = u^n + sum_i R_i^T D_i v_i^n                 (eqs. 9, 10)

    The local solve is ``k`` CG steps from zero (Sec. 4), or an exact dense
    solve when k is None. D_i is the Boolean owner map of owner_bounds.
    ``blocks`` restricts the update to a list of (by, bx) block indices (for
    sampled comparisons on large images); other pixels keep u^n.
    Returns (u^{n+1}, ||r^n||_2^2 summed over the pixels the updated blocks own).
    """
    u = np.asarray(u, dtype=np.float64)
    c = np.asarray(c)
    h, w = c.shape
    sy = size if size_y is None else size_y
    oy_ = overlap if overlap_y is None else overlap_y
    oy, bh = block_origins(h, sy, oy_)
    ox, bw = block_origins(w, size, overlap)
    ly, hy = owner_bounds(oy, bh, h)
    lx, hx = owner_bounds(ox, bw, w)
    if blocks is None:
        blocks = [(i, j) for i in range(len(oy)) for j in range(len(ox))]
    r = residual(f, c, u)
    out = u.copy()
    rsq = 0.0
    for by, bx in blocks:
        y0, x0 = oy[by], ox[bx]
        rhs = r[y0:y0 + bh, x0:x0 + bw].reshape(-1)
        M = local_matrix(c, y0, x0, bh, bw, alpha)
        if k is None:
            import scipy.sparse.linalg as spl
            v = spl.spsolve(M.tocsc(), rhs)
        else:
            v = local_cg(M, rhs, k)
        v = v.reshape(bh, bw)
        ys, ye, xs, xe = ly[by], hy[by], lx[bx], hx[bx]
        out[ys:ye, xs:xe] += v[ys - y0:ye - y0, xs - x0:xe - x0]
        rsq += float(np.sum(r[ys:ye, xs:xe] ** 2))
    return out, rsq


def correction_step(d, rhs, c, size: int, overlap: int, alpha: float, k: int | None,
                    blocks=None):
    """One (O)RAS iteration of Sec. 3 (eqs. 7-9) on A d = rhs, where A is the
    matrix of eq. 6 and the mask rows carry d = 0 (rhs must vanish there).

    This is the correction equation of iterative refinement: if u has
    u = f on the mask and rhs = b - A u, then A (u + d) = b exactly when
    A d = rhs, and one iteration here from d equals oras_step from u + d
    minus u (the residual rhs - A d equals b - A (u + d)). Residual of d:
    0 on the mask, rhs_p + sum over in-image 4-neighbours q of (d_q - d_p)
    elsewhere.
    """
    d = np.asarray(d, dtype=np.float64)
    rhs = np.asarray(rhs, dtype=np.float64)
    c = np.asarray(c)
    h, w = c.shape
    oy, bh = block_origins(h, size, overlap)
    ox, bw = block_origins(w, size, overlap)
    ly, hy = owner_bounds(oy, bh, h)
    lx, hx = owner_bounds(ox, bw, w)
    if blocks is None:
        blocks = [(i, j) for i in range(len(oy)) for j in range(len(ox))]
    ld = np.zeros_like(d)
    ld[:, :-1] += d[:, 1:] - d[:, :-1]
    ld[:, 1:] += d[:, :-1] - d[:, 1:]
    ld[:-1, :] += d[1:, :] - d[:-1, :]
    ld[1:, :] += d[:-1, :] - d[1:, :]
    r = np.where(c == 1, 0.0, rhs + ld)
    out = d.copy()
    for by, bx in blocks:
        y0, x0 = oy[by], ox[bx]
        M = local_matrix(c, y0, x0, bh, bw, alpha)
        rhs_i = r[y0:y0 + bh, x0:x0 + bw].reshape(-1)
        if k is None:  # exact local solve, as in oras_step
            import scipy.sparse.linalg as spl
            v = spl.spsolve(M.tocsc(), rhs_i)
        else:
            v = local_cg(M, rhs_i, k)
        v = v.reshape(bh, bw)
        ys, ye, xs, xe = ly[by], hy[by], lx[bx], hx[bx]
        out[ys:ye, xs:xe] += v[ys - y0:ye - y0, xs - x0:xe - x0]
    return out


def ml_oras(f, c, levels: int, size: int, overlap: int, alpha: float,
            k: int | None, sweeps):
    """Coarse-to-fine multilevel ORAS (Sec. 4) for one channel.

    Build ``levels`` levels by repeated coarsen(); on the coarsest level
    start from u = f on the mask and 0 elsewhere; on every finer level start
    from the prolongated coarser solution with u = f re-imposed on the mask;
    run ``sweeps[l]`` ORAS iterations on level l (0 = finest).
    """
    fs, cs = [np.asarray(f, dtype=np.float64)], [np.asarray(c)]
    for _ in range(levels - 1):
        fc, cc = coarsen(fs[-1], cs[-1])
        fs.append(fc); cs.append(cc)
    u = None
    for lev in range(levels - 1, -1, -1):
        fl, cl = fs[lev], cs[lev]
        if u is None:
            u = np.where(cl == 1, fl, 0.0)
        else:
            u = fine_start(u, fl, cl)
        for _ in range(sweeps[lev]):
            u, _ = oras_step(u, fl, cl, size, overlap, alpha, k)
    return u


def apply_matrix(z, c):
    """A z for the matrix of eq. 6: z_p on the mask, the sum over in-image
    4-neighbours q of (z_p - z_q) elsewhere. Since residual(f, c, u) is
    b - A u, A z = -residual(0, c, z)."""
    z = np.asarray(z, dtype=np.float64)
    return -residual(np.zeros_like(z), c, z)


def fgmres_oras(f, c, u0, size: int, overlap: int, alpha: float, k: int | None,
                m: int, tol: float, max_iter: int):
    """Flexible GMRES(m) on A u = b (eq. 6) for one channel, from u0 (with
    u0 = f on the mask), right-preconditioned by one ORAS iteration on the
    correction equation: z_j = correction_step(0, v_j). Local CG with a fixed
    step count is not a linear map of its right-hand side, so the
    preconditioned vectors z_j are kept (flexible variant): the update is
    u = u0 + Z y with y minimising ||beta e_1 - H y||.

    Orthogonalisation by modified Gram-Schmidt; restart after m steps.
    Stops once ||b - A u|| <= tol ||b|| (the least-squares residual within a
    cycle, recomputed from u at each restart) or after max_iter steps.
    Returns (u, history): history[0] is the relative residual of u0, then
    one entry per step -- the least-squares residual, except that the last
    step of a cycle carries the residual of the updated u recomputed from
    scratch -- so len(history) - 1 is the number of steps.
    """
    f = np.asarray(f, dtype=np.float64)
    c = np.asarray(c)
    u = np.asarray(u0, dtype=np.float64).copy()
    bnorm = float(np.linalg.norm(np.where(c == 1, f, 0.0)))
    history = []
    steps = 0
    while True:
        r = residual(f, c, u)
        beta = float(np.linalg.norm(r))
        rel0 = beta / bnorm if bnorm > 0 else 0.0
        if history:
            history[-1] = rel0  # the cycle's last step, recomputed from u
        else:
            history.append(rel0)
        if beta <= tol * bnorm or steps >= max_iter or beta == 0.0:
            return u, history
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m))
        y = np.zeros(0)
        for j in range(m):
            z = correction_step(np.zeros_like(u), V[j], c, size, overlap, alpha, k)
            wv = apply_matrix(z, c)
            for i in range(j + 1):
                H[i, j] = float(np.sum(wv * V[i]))
                wv = wv - H[i, j] * V[i]
            H[j + 1, j] = float(np.linalg.norm(wv))
            Z.append(z)
            steps += 1
            g = np.zeros(j + 2)
            g[0] = beta
            y, *_ = np.linalg.lstsq(H[:j + 2, :j + 1], g, rcond=None)
            res = float(np.linalg.norm(g - H[:j + 2, :j + 1] @ y))
            history.append(res / bnorm)
            if res <= tol * bnorm or steps >= max_iter or H[j + 1, j] == 0.0:
                break
            V.append(wv / H[j + 1, j])
        for j, z in enumerate(Z):
            u = u + y[j] * z


def krylov_oras(f, c, levels: int, size: int, overlap: int, alpha: float,
                k: int | None, coarse_sweeps, m: int, tol: float, max_iter: int):
    """Krylov-accelerated multilevel ORAS for one channel: the coarse-to-fine
    start of ml_oras (coarse_sweeps[l] ORAS iterations on level l >= 1, none
    on the finest), then fgmres_oras on the finest level."""
    sweeps = [0] + list(coarse_sweeps)
    u0 = ml_oras(f, c, levels, size, overlap, alpha, k, sweeps)
    return fgmres_oras(f, c, u0, size, overlap, alpha, k, m, tol, max_iter)
