"""ctypes binding of libddi.so (include/ddi.h).

Argument marshalling only: every step runs in the HIP kernels of the
library. Tensors are torch tensors on the ROCm device (torch supplies device
memory and the current stream); shapes follow the C ABI:
  f, u : (channels, height, width) float32, contiguous
  c    : (height, width) uint8, contiguous, 1 = known pixel
There is no CPU fallback: if the library is not built, every call raises.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

from . import build as _build

_lib = None

DDI_OK = 0
DDI_EINVAL = -1
DDI_ESINGULAR = -2
DDI_ENOMEM = -3
DDI_ENOCONV = -4
DDI_EHIP = -5
DDI_ENODEV = -6
DDI_ESCRATCH = -7
DDI_ESTALL = -8
MAX_BLOCK = 64
NOALLOC_SCRATCH_BYTES = 4 << 20
COARSE_MAX_PIXELS = 8192


class Params(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int), ("overlap", ctypes.c_int),
                ("levels", ctypes.c_int), ("local_iters", ctypes.c_int),
                ("robin_alpha", ctypes.c_float), ("coarse_sweeps", ctypes.c_int),
                ("coarsest_sweeps", ctypes.c_int), ("rel_tol", ctypes.c_double),
                ("min_sweeps", ctypes.c_int), ("max_sweeps", ctypes.c_int),
                ("check_every", ctypes.c_int), ("final_residual", ctypes.c_int),
                ("timing", ctypes.c_int), ("coarse_block", ctypes.c_int),
                ("coarse_overlap", ctypes.c_int), ("coarse_local_iters", ctypes.c_int),
                ("local_tol", ctypes.c_float), ("use_graph", ctypes.c_int),
                ("coarse_solver", ctypes.c_int), ("coarse_cg_iters", ctypes.c_int),
                ("coarse_cg_tol", ctypes.c_double), ("storage", ctypes.c_int),
                ("inner_sweeps", ctypes.c_int), ("method", ctypes.c_int),
                ("fuse_prolong", ctypes.c_int), ("krylov_restart", ctypes.c_int),
                ("skip_unchanged", ctypes.c_int), ("order_blocks", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Stats(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int), ("converged", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("ms", ctypes.c_double),
                ("sweep_ms", ctypes.c_double), ("cg_steps", ctypes.c_double),
                ("refinements", ctypes.c_int), ("first_sweep_ms", ctypes.c_double),
                ("first_cg_steps", ctypes.c_double), ("skipped_blocks", ctypes.c_double),
                ("unwritten_blocks", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class DDIError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = lib().ddi_strerror(code).decode()
        if code == DDI_EHIP:
            msg += f" (hip error {lib().ddi_last_hip_error()})"
        super().__init__(f"{what}: {msg} [{code}]" if what else f"{msg} [{code}]")


def library_path() -> str:
    return _build.LIB


def lib():
    """Load libddi.so (built in tree by ``python -m paper_2110_03946_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            raise RuntimeError(
                f"{_build.LIB} is not built; run `python -m paper_2110_03946_amd.build` "
                "(the solver has no CPU fallback)")
        L = ctypes.CDLL(_build.LIB)
        vp, i, d, f = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_float
        ip = ctypes.POINTER(ctypes.c_int)
        sig = {
            "ddi_default_params": (i, [ctypes.POINTER(Params)]),
            "ddi_check_params": (i, [i, i, i, ctypes.POINTER(Params)]),
            "ddi_create": (i, [ctypes.POINTER(vp), i, i, i, ctypes.POINTER(Params), vp]),
            "ddi_solve": (i, [vp, vp, vp, vp, ctypes.POINTER(Stats)]),
            "ddi_destroy": (i, [vp]),
            "ddi_solve_async": (i, [vp, vp, vp, vp]),
            "ddi_solve_wait": (i, [vp, ctypes.POINTER(Stats)]),
            "ddi_strerror": (ctypes.c_char_p, [i]),
            "ddi_last_hip_error": (i, []),
            "ddi_sweep_times": (i, [vp, ctypes.POINTER(d), i, ip]),
            "ddi_block_count": (i, [i, i, i]),
            "ddi_block_range": (i, [i, i, i, i, ip, ip, ip]),
            "ddi_residual": (i, [vp, vp, vp, i, i, i, vp, vp, vp]),
            "ddi_coarsen": (i, [vp, vp, i, i, i, vp, vp, vp]),
            "ddi_prolong": (i, [vp, i, i, vp, vp, i, i, i, vp, vp]),
            "ddi_oras_sweep": (i, [vp, vp, vp, i, i, i, i, i, f, i, vp, vp]),
            "ddi_oras_sweep_noalloc": (i, [vp, vp, vp, i, i, i, i, i, f, i, vp, vp]),
            "ddi_noalloc_scratch_bytes": (i, [i, i, i, i, i, ctypes.POINTER(ctypes.c_size_t)]),
            "ddi_coarse_solve": (i, [vp, vp, i, i, i, vp, i, d, vp]),
            "ddi_coarse_grid_bytes": (i, [i, i, i, ctypes.POINTER(ctypes.c_size_t)]),
            "ddi_selfcheck_access": (i, [i, i, i, vp, ctypes.POINTER(ctypes.c_longlong),
                                         ctypes.POINTER(ctypes.c_longlong), ctypes.c_char_p, i]),
            "ddi_coarse_grid_debug_spin_limit": (i, [ctypes.c_long]),
            "ddi_coarse_solve_grid": (i, [vp, vp, i, i, i, vp, i, d, i, vp, ctypes.c_size_t, vp,
                                          vp]),
            "ddi_plan_footprint": (i, [i, i, i, ctypes.POINTER(Params),
                                       ctypes.POINTER(ctypes.c_size_t)]),
            "ddi_plan_bytes": (i, [vp, ctypes.POINTER(ctypes.c_size_t)]),
            "ddi_refine_residual": (i, [vp, vp, vp, vp, i, i, i, vp, vp, vp, vp]),
            "ddi_refine_start": (i, [vp, i, i, vp, vp, i, i, i, vp, vp, vp, vp]),
            "ddi_correction_sweep": (i, [vp, vp, vp, vp, i, i, i, i, i, f, i, vp]),
            "ddi_batch_create": (i, [ctypes.POINTER(vp), i, ip, ip, i, ctypes.POINTER(Params),
                                     i, vp]),
            "ddi_batch_solve": (i, [vp, vp, vp, vp, ctypes.POINTER(Stats), ip]),
            "ddi_batch_destroy": (i, [vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def header_symbols() -> list[str]:
    """Function names declared in include/ddi.h."""
    hdr = os.path.join(_build.ROOT, "include", "ddi.h")
    txt = open(hdr).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w[\w\s\*]*?\b(ddi_\w+)\s*\(", txt, re.M)))


def _check(rc: int, what: str):
    if rc != DDI_OK:
        raise DDIError(rc, what)


def default_params(**overrides) -> Params:
    p = Params()
    _check(lib().ddi_default_params(ctypes.byref(p)), "ddi_default_params")
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def check_params(h: int, w: int, channels: int, p: Params) -> int:
    return lib().ddi_check_params(h, w, channels, ctypes.byref(p))


def plan_footprint(h: int, w: int, channels: int, p: Params | None = None) -> int:
    """Device bytes a plan for (h, w, channels, p) allocates (no GPU needed)."""
    n = ctypes.c_size_t()
    _check(lib().ddi_plan_footprint(h, w, channels, ctypes.byref(p) if p is not None else None,
                                    ctypes.byref(n)), "ddi_plan_footprint")
    return n.value


def block_count(n: int, block: int, overlap: int) -> int:
    return lib().ddi_block_count(n, block, overlap)


def block_range(n: int, block: int, overlap: int, k: int):
    o, lo, hi = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(lib().ddi_block_range(n, block, overlap, k, ctypes.byref(o), ctypes.byref(lo),
                                 ctypes.byref(hi)), "ddi_block_range")
    return o.value, lo.value, hi.value


# ---------------------------------------------------------------------------
# device-tensor helpers (torch only as the owner of device memory / streams)
# ---------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _img(t, name, channels=None, hw=None):
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float32")
    if t.dim() == 2:
        t = t.unsqueeze(0)
    if t.dim() != 3:
        raise ValueError(f"{name} must be (channels, height, width)")
    if channels is not None and t.shape[0] != channels:
        raise ValueError(f"{name} has {t.shape[0]} channels, expected {channels}")
    if hw is not None and tuple(t.shape[1:]) != tuple(hw):
        raise ValueError(f"{name} is {tuple(t.shape[1:])}, expected {tuple(hw)}")
    return t


def _mask(t, hw=None):
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError("c must be a torch tensor on the GPU")
    if t.dtype != torch.uint8 or not t.is_contiguous() or t.dim() != 2:
        raise TypeError("c must be a contiguous (height, width) uint8 tensor")
    if hw is not None and tuple(t.shape) != tuple(hw):
        raise ValueError(f"c is {tuple(t.shape)}, expected {tuple(hw)}")
    return t


class Plan:
    """A solver plan for one image size (ddi_create / ddi_solve / ddi_destroy)."""

    def __init__(self, height: int, width: int, channels: int = 3,
                 params: Params | None = None, stream=None, **overrides):
        if params is None:
            params = default_params(**overrides)
        elif overrides:
            for k, v in overrides.items():
                setattr(params, k, v)
        self.height, self.width, self.channels = height, width, channels
        self.params = params
        self._stream = stream
        h = ctypes.c_void_p()
        _check(lib().ddi_create(ctypes.byref(h), height, width, channels,
                                ctypes.byref(params), _stream(stream)), "ddi_create")
        self._h = h

    def solve(self, f, c, u=None, allow_noconv: bool = False):
        """Inpaint f (C, H, W) with mask c (H, W) into u; returns (u, stats)."""
        torch = _torch()
        hw = (self.height, self.width)
        f = _img(f, "f", self.channels, hw)
        c = _mask(c, hw)
        if u is None:
            u = torch.empty_like(f)
        else:
            u = _img(u, "u", self.channels, hw)
        st = Stats()
        rc = lib().ddi_solve(self._h, _ptr(f), _ptr(c), _ptr(u), ctypes.byref(st))
        if rc != DDI_OK and not (allow_noconv and rc == DDI_ENOCONV):
            raise DDIError(rc, "ddi_solve")
        return u, st.as_dict()

    def solve_async(self, f, c, u):
        """Enqueue a solve (ddi_solve_async); f, c, u must stay alive until wait()."""
        hw = (self.height, self.width)
        f = _img(f, "f", self.channels, hw)
        c = _mask(c, hw)
        u = _img(u, "u", self.channels, hw)
        self._pending = (f, c, u)
        _check(lib().ddi_solve_async(self._h, _ptr(f), _ptr(c), _ptr(u)), "ddi_solve_async")
        return u

    def wait(self, allow_noconv: bool = False):
        """Finish the pending solve (ddi_solve_wait); returns (u, stats)."""
        st = Stats()
        rc = lib().ddi_solve_wait(self._h, ctypes.byref(st))
        u = self._pending[2] if getattr(self, "_pending", None) else None
        self._pending = None
        if rc != DDI_OK and not (allow_noconv and rc == DDI_ENOCONV):
            raise DDIError(rc, "ddi_solve_wait")
        return u, st.as_dict()

    def sweep_times(self) -> list:
        """Device ms of each finest-level sweep of the last solve (timing = 1)."""
        n = ctypes.c_int(0)
        _check(lib().ddi_sweep_times(self._h, None, 0, ctypes.byref(n)), "ddi_sweep_times")
        buf = (ctypes.c_double * max(n.value, 1))()
        _check(lib().ddi_sweep_times(self._h, buf, n.value, ctypes.byref(n)), "ddi_sweep_times")
        return list(buf[:n.value])

    def device_bytes(self) -> int:
        n = ctypes.c_size_t()
        _check(lib().ddi_plan_bytes(self._h, ctypes.byref(n)), "ddi_plan_bytes")
        return n.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ddi_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """A batch plan for many images of uneven size (ddi_batch_create /
    ddi_batch_solve / ddi_batch_destroy). `params` is one Params (or None
    for the defaults, with keyword overrides) or a list with one Params per
    image."""

    def __init__(self, sizes, channels: int = 3, params=None, stream=None, **overrides):
        self.sizes = [(int(h), int(w)) for h, w in sizes]
        n = len(self.sizes)
        self.channels = channels
        if params is None:
            plist = [default_params(**overrides)]
        elif isinstance(params, Params):
            plist = [params]
        else:
            plist = list(params)
        for p in plist:
            for k, v in overrides.items():
                setattr(p, k, v)
        self.params = plist
        arr = (Params * len(plist))(*plist)
        hs = (ctypes.c_int * n)(*[h for h, _ in self.sizes])
        ws = (ctypes.c_int * n)(*[w for _, w in self.sizes])
        h = ctypes.c_void_p()
        _check(lib().ddi_batch_create(ctypes.byref(h), n, hs, ws, channels, arr, len(plist),
                                      _stream(stream)), "ddi_batch_create")
        self._h = h

    def solve(self, fs, cs, us=None, allow_noconv: bool = False):
        """Inpaint every (f, c) pair into us; returns (us, stats list, status list)."""
        torch = _torch()
        n = len(self.sizes)
        if len(fs) != n or len(cs) != n:
            raise ValueError(f"expected {n} images and masks")
        fs = [_img(f, "f", self.channels, hw) for f, hw in zip(fs, self.sizes)]
        cs = [_mask(c, hw) for c, hw in zip(cs, self.sizes)]
        if us is None:
            us = [torch.empty_like(f) for f in fs]
        else:
            us = [_img(u, "u", self.channels, hw) for u, hw in zip(us, self.sizes)]
        P = ctypes.c_void_p * n
        st = (Stats * n)()
        status = (ctypes.c_int * n)()
        rc = lib().ddi_batch_solve(self._h, P(*[t.data_ptr() for t in fs]),
                                   P(*[t.data_ptr() for t in cs]),
                                   P(*[t.data_ptr() for t in us]), st, status)
        codes = list(status)
        if rc != DDI_OK and not (allow_noconv and all(x in (DDI_OK, DDI_ENOCONV) for x in codes)
                                 and rc == DDI_ENOCONV):
            raise DDIError(rc, "ddi_batch_solve")
        return us, [s.as_dict() for s in st], codes

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ddi_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(f, c, **params):
    """One-shot inpainting: creates a plan, solves, destroys it."""
    f3 = _img(f, "f")
    with Plan(f3.shape[1], f3.shape[2], f3.shape[0], **params) as plan:
        return plan.solve(f3, c)


def residual(f, c, u, r=None, stream=None):
    """r = b - A u (eq. 7); returns (r or None, per-channel sum of r^2)."""
    f = _img(f, "f")
    C, H, W = f.shape
    c = _mask(c, (H, W))
    u = _img(u, "u", C, (H, W))
    if r is not None:
        r = _img(r, "r", C, (H, W))
    rsq = np.zeros(C, dtype=np.float64)
    _check(lib().ddi_residual(_ptr(f), _ptr(c), _ptr(u), H, W, C,
                              _ptr(r) if r is not None else None,
                              rsq.ctypes.data_as(ctypes.c_void_p), _stream(stream)),
           "ddi_residual")
    return r, rsq


def coarsen(f, c, stream=None):
    """One dyadic subsampling step (Sec. 4); returns (fc, cc)."""
    torch = _torch()
    f = _img(f, "f")
    C, H, W = f.shape
    c = _mask(c, (H, W))
    hc, wc = (H + 1) // 2, (W + 1) // 2
    fc = torch.empty((C, hc, wc), dtype=torch.float32, device=f.device)
    cc = torch.empty((hc, wc), dtype=torch.uint8, device=f.device)
    _check(lib().ddi_coarsen(_ptr(f), _ptr(c), H, W, C, _ptr(fc), _ptr(cc), _stream(stream)),
           "ddi_coarsen")
    return fc, cc


def prolong(uc, f, c, u=None, stream=None):
    """Coarse-to-fine start: u = f on the mask, bilinear(uc) elsewhere."""
    torch = _torch()
    f = _img(f, "f")
    C, H, W = f.shape
    c = _mask(c, (H, W))
    uc = _img(uc, "uc", C)
    if u is None:
        u = torch.empty_like(f)
    _check(lib().ddi_prolong(_ptr(uc), uc.shape[1], uc.shape[2], _ptr(f), _ptr(c), H, W, C,
                             _ptr(u), _stream(stream)), "ddi_prolong")
    return u


def coarse_solve(f, c, max_iter: int = 500, tol: float = 1e-10, u=None, stream=None):
    """Float64 CG solve of a small grid (the coarsest-level solver)."""
    torch = _torch()
    f = _img(f, "f")
    C, H, W = f.shape
    c = _mask(c, (H, W))
    if u is None:
        u = torch.empty_like(f)
    _check(lib().ddi_coarse_solve(_ptr(f), _ptr(c), H, W, C, _ptr(u), max_iter, float(tol),
                                  _stream(stream)), "ddi_coarse_solve")
    return u


def selfcheck_access(h: int, w: int, channels: int, p: Params | None = None):
    """Host replay of every global-memory offset of a plan's kernels (no GPU):
    returns (offsets checked, offsets outside their buffer, first of those)."""
    checked, bad = ctypes.c_longlong(0), ctypes.c_longlong(0)
    buf = ctypes.create_string_buffer(512)
    _check(lib().ddi_selfcheck_access(h, w, channels, ctypes.byref(p) if p is not None else None,
                                      ctypes.byref(checked), ctypes.byref(bad), buf, 512),
           "ddi_selfcheck_access")
    return checked.value, bad.value, buf.value.decode()


def coarse_grid_bytes(h: int, w: int, channels: int) -> int:
    """Workspace bytes of coarse_solve_grid for an h x w x channels level."""
    n = ctypes.c_size_t()
    _check(lib().ddi_coarse_grid_bytes(h, w, channels, ctypes.byref(n)), "ddi_coarse_grid_bytes")
    return n.value


def coarse_solve_grid(f, c, max_iter: int = 500, tol: float = 1e-10, workgroups: int = 0,
                      u=None, work=None, steps: bool = False, stream=None):
    """Float64 CG solve of a level of any size on a grid of workgroups.

    work: a uint8 device tensor of at least coarse_grid_bytes bytes (one is
    allocated when None). Returns u, or (u, CG steps per channel) with
    steps=True, which waits for the stream."""
    torch = _torch()
    f = _img(f, "f")
    C, H, W = f.shape
    c = _mask(c, (H, W))
    if u is None:
        u = torch.empty_like(f)
    need = coarse_grid_bytes(H, W, C)
    if work is None:
        work = torch.empty(need, dtype=torch.uint8, device=f.device)
    if not (isinstance(work, torch.Tensor) and work.is_cuda and work.dtype == torch.uint8 and
            work.is_contiguous()):
        raise TypeError("work must be a contiguous uint8 tensor on the GPU")
    st = (ctypes.c_int * 4)() if steps else None
    _check(lib().ddi_coarse_solve_grid(_ptr(f), _ptr(c), H, W, C, _ptr(u), max_iter, float(tol),
                                       workgroups, _ptr(work), work.numel(),
                                       ctypes.cast(st, ctypes.c_void_p) if steps else None,
                                       _stream(stream)), "ddi_coarse_solve_grid")
    return (u, list(st)[:C]) if steps else u


def _bf16(t, name, channels=None, hw=None):
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.bfloat16 and
            t.is_contiguous() and t.dim() == 3):
        raise TypeError(f"{name} must be a contiguous (C, H, W) bfloat16 tensor on the GPU")
    if channels is not None and t.shape[0] != channels:
        raise ValueError(f"{name} has {t.shape[0]} channels, expected {channels}")
    if hw is not None and tuple(t.shape[1:]) != tuple(hw):
        raise ValueError(f"{name} is {tuple(t.shape[1:])}, expected {tuple(hw)}")
    return t


def refine_residual(f, c, u, d=None, stream=None):
    """Refinement step: returns (u_next or None, rhs bfloat16, per-channel ||r||^2)."""
    torch = _torch()
    f = _img(f, "f")
    C, H, W = f.shape
    c = _mask(c, (H, W))
    u = _img(u, "u", C, (H, W))
    un = None
    if d is not None:
        d = _bf16(d, "d", C, (H, W))
        un = torch.empty_like(u)
    rhs = torch.empty((C, H, W), dtype=torch.bfloat16, device=f.device)
    rsq = np.zeros(C, dtype=np.float64)
    _check(lib().ddi_refine_residual(_ptr(f), _ptr(c), _ptr(u), _ptr(d) if d is not None else None,
                                     H, W, C, _ptr(un) if un is not None else None, _ptr(rhs),
                                     rsq.ctypes.data_as(ctypes.c_void_p), _stream(stream)),
           "ddi_refine_residual")
    return un, rhs, rsq


def refine_start(uc, f, c, stream=None):
    """First refinement residual built with the coarse-to-fine start from the
    coarse grid uc: returns (u, rhs bfloat16, per-channel ||r||^2)."""
    torch = _torch()
    f = _img(f, "f")
    C, H, W = f.shape
    c = _mask(c, (H, W))
    uc = _img(uc, "uc", C, ((H + 1) // 2, (W + 1) // 2))
    u = torch.empty_like(f)
    rhs = torch.empty((C, H, W), dtype=torch.bfloat16, device=f.device)
    rsq = np.zeros(C, dtype=np.float64)
    _check(lib().ddi_refine_start(_ptr(uc), uc.shape[1], uc.shape[2], _ptr(f), _ptr(c), H, W, C,
                                  _ptr(u), _ptr(rhs), rsq.ctypes.data_as(ctypes.c_void_p),
                                  _stream(stream)),
           "ddi_refine_start")
    return u, rhs, rsq


def correction_sweep(d_in, rhs, c, block: int, overlap: int, alpha: float, k: int, stream=None):
    """One ORAS iteration on A d = rhs (bfloat16 d and rhs); returns d_out."""
    torch = _torch()
    rhs = _bf16(rhs, "rhs")
    C, H, W = rhs.shape
    c = _mask(c, (H, W))
    if d_in is not None:
        d_in = _bf16(d_in, "d_in", C, (H, W))
    d_out = torch.empty_like(rhs)
    _check(lib().ddi_correction_sweep(_ptr(d_in) if d_in is not None else None, _ptr(rhs), _ptr(c),
                                      _ptr(d_out), H, W, C, block, overlap, float(alpha), k,
                                      _stream(stream)), "ddi_correction_sweep")
    return d_out


def oras_sweep(u_in, c, block: int, overlap: int, alpha: float, k: int, u_out=None,
               stream=None):
    """One ORAS iteration (Sec. 3 eqs. 7-9); returns (u_out, per-channel ||r||^2 of u_in)."""
    torch = _torch()
    u_in = _img(u_in, "u_in")
    C, H, W = u_in.shape
    c = _mask(c, (H, W))
    if u_out is None:
        u_out = torch.empty_like(u_in)
    rsq = np.zeros(C, dtype=np.float64)
    _check(lib().ddi_oras_sweep(_ptr(u_in), _ptr(c), _ptr(u_out), H, W, C, block, overlap,
                                float(alpha), k, rsq.ctypes.data_as(ctypes.c_void_p),
                                _stream(stream)), "ddi_oras_sweep")
    return u_out, rsq


def noalloc_scratch_bytes(h: int, w: int, channels: int, block: int, overlap: int) -> int:
    """Scratch bytes ddi_oras_sweep_noalloc needs for these sizes (host only)."""
    n = ctypes.c_size_t(0)
    _check(lib().ddi_noalloc_scratch_bytes(h, w, channels, block, overlap, ctypes.byref(n)),
           "ddi_noalloc_scratch_bytes")
    return n.value


def oras_sweep_noalloc(u_in, c, block: int, overlap: int, alpha: float, k: int, u_out=None,
                       stream=None, rsq: bool = True):
    """ddi_oras_sweep without device allocation (fixed per-GPU scratch); returns
    (u_out, per-channel ||r||^2 of u_in, or None when rsq is False)."""
    torch = _torch()
    u_in = _img(u_in, "u_in")
    C, H, W = u_in.shape
    c = _mask(c, (H, W))
    if u_out is None:
        u_out = torch.empty_like(u_in)
    out = np.zeros(C, dtype=np.float64) if rsq else None
    _check(lib().ddi_oras_sweep_noalloc(_ptr(u_in), _ptr(c), _ptr(u_out), H, W, C, block, overlap,
                                        float(alpha), k,
                                        out.ctypes.data_as(ctypes.c_void_p) if rsq else None,
                                        _stream(stream)), "ddi_oras_sweep_noalloc")
    return u_out, out
