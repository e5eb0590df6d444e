"""SGP4 near-Earth propagation on MI355X: thin torch front end of libsgp4mi.

PyTorch supplies device memory and streams; every step of the computation runs
in the library's HIP kernels (see include/sgp4mi.h for the C ABI).

    rec = init(elem)                      # elem: float64 [8, n] on the GPU
    r, v, err = propagate(rec, t, "mixed")  # r, v: [3, n, T]; err: uint8 [n, T]

Element rows: no_kozai (rad/min), ecco, inclo, nodeo, argpo, mo (rad), bstar
(1/earth radii), epoch (days after the reference instant); times are minutes
after the reference instant.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from . import _native
from ._native import SGP4Error, PLAN_AUTOTUNE, PLAN_GRAPH, REC_CHECKSUM, REC_MISMATCH, REC_FIELD

__all__ = ["Record", "init", "propagate", "propagate_ragged", "RaggedPlan", "vjp", "vjp_ragged", "jacobian_ragged", "SGP4Function",
           "SGP4RaggedFunction", "PRECISIONS", "SGP4Error", "consts_bytes"]

PRECISIONS = {"fp64": _native.SGP4_FP64, "fp32": _native.SGP4_FP32, "mixed": _native.SGP4_FP32_MIXED}


def _prec(p) -> int:
    if isinstance(p, str):
        if p not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
        return PRECISIONS[p]
    return int(p)


def _out_dtype(p: int) -> torch.dtype:
    return torch.float64 if p == _native.SGP4_FP64 else torch.float32


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _need(t: torch.Tensor, dtype, name, device=None):
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} CUDA/HIP tensor")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")


def consts_bytes(n: int) -> int:
    return int(_native.lib().sgp4_consts_bytes(int(n)))


class Record:
    """Per-satellite constant record produced by :func:`init` (opaque bytes)."""

    def __init__(self, consts: torch.Tensor, n: int, flags: torch.Tensor, elem: torch.Tensor):
        self.consts, self.n, self.flags, self.elem = consts, n, flags, elem

    @property
    def device(self):
        return self.consts.device


def _ref(ref_jd):
    if ref_jd is None:
        return None
    w, f = (ref_jd, 0.0) if isinstance(ref_jd, (int, float)) else ref_jd
    return (ctypes.c_double * 2)(float(w), float(f))


def init(elem: torch.Tensor, grav: Optional[Sequence[float]] = None, ref_jd=None) -> Record:
    """Initialisation: elements float64 [8, n] (device) -> constant record.
    ref_jd: the reference instant of the epoch row and the times as a Julian
    date (a number or (whole, frac)); None = J2000.0.  Only the deep-space
    terms depend on it (sgp4_init_ex)."""
    _need(elem, torch.float64, "elem")
    if elem.dim() != 2 or elem.shape[0] != 8:
        raise ValueError("elem must have shape [8, n]")
    n = int(elem.shape[1])
    consts = torch.empty(max(consts_bytes(n), 1), dtype=torch.uint8, device=elem.device)
    flags = torch.empty(max(n, 1), dtype=torch.uint8, device=elem.device)
    g = None
    if grav is not None:
        g = (ctypes.c_double * 5)(*[float(x) for x in grav])
    with torch.cuda.device(elem.device):
        _native.check(_native.lib().sgp4_init_ex(g, _ref(ref_jd), n, _ptr(elem), _ptr(consts), _ptr(flags),
                                                 _stream(elem.device)), "sgp4_init_ex")
    return Record(consts, n, flags[:n], elem)


def propagate(rec: Record, t: torch.Tensor, precision="fp64", out=None, block: Optional[int] = None):
    """Dense grid: returns r [3, n, T], v [3, n, T] (km, km/s, TEME) and err uint8 [n, T].
    block: None for the library's default launch (sgp4_propagate), else the launch
    configuration word of sgp4_propagate_ex (workgroup size and flags)."""
    p = _prec(precision)
    _need(t, torch.float64, "t", rec.device)
    n, T = rec.n, int(t.numel())
    if out is None:
        dt = _out_dtype(p)
        r = torch.empty((3, n, T), dtype=dt, device=rec.device)
        v = torch.empty((3, n, T), dtype=dt, device=rec.device)
        err = torch.empty((n, T), dtype=torch.uint8, device=rec.device)
    else:
        r, v, err = out
    with torch.cuda.device(rec.device):
        if block is None:
            rc = _native.lib().sgp4_propagate(_ptr(rec.consts), n, _ptr(t), T, p, _ptr(r), _ptr(v), _ptr(err),
                                              _stream(rec.device))
        else:
            rc = _native.lib().sgp4_propagate_ex(_ptr(rec.consts), n, _ptr(t), T, p, _ptr(r), _ptr(v), _ptr(err),
                                                 int(block), _stream(rec.device))
        _native.check(rc, "sgp4_propagate")
    return r, v, err


def _ragged_out(p, nnz, device):
    dt = _out_dtype(p)
    return (torch.empty((3, nnz), dtype=dt, device=device), torch.empty((3, nnz), dtype=dt, device=device),
            torch.empty(nnz, dtype=torch.uint8, device=device))


class RaggedPlan:
    """A tuned (and optionally graph-captured) launch for one ragged batch."""

    def __init__(self, rec: Record, offsets: torch.Tensor, t: torch.Tensor, precision="fp64", out=None,
                 autotune: bool = True, graph: bool = True, config=None):
        """config: None (default or autotuned choice) or (mode, block, waves_per_cu)
        with mode 0 = tiles, 1 = flat."""
        self.p = _prec(precision)
        _need(offsets, torch.int64, "offsets", rec.device)
        _need(t, torch.float64, "t", rec.device)
        self.rec, self.offsets, self.t = rec, offsets, t
        self.nnz = int(t.numel())
        self.out = out if out is not None else _ragged_out(self.p, self.nnz, rec.device)
        r, v, err = self.out
        h = ctypes.c_void_p()
        flags = (PLAN_AUTOTUNE if autotune else 0) | (PLAN_GRAPH if graph else 0)
        with torch.cuda.device(rec.device):
            if config is None:
                rc = _native.lib().sgp4_plan_create(ctypes.byref(h), _ptr(rec.consts), rec.n, _ptr(offsets), _ptr(t),
                                                    self.nnz, self.p, _ptr(r), _ptr(v), _ptr(err), flags,
                                                    _stream(rec.device))
            else:
                mode, block, per_cu = (int(x) for x in config)
                rc = _native.lib().sgp4_plan_create_config(ctypes.byref(h), _ptr(rec.consts), rec.n, _ptr(offsets),
                                                           _ptr(t), self.nnz, self.p, _ptr(r), _ptr(v), _ptr(err),
                                                           mode, block, per_cu, flags, _stream(rec.device))
            _native.check(rc, "sgp4_plan_create")
        self.handle = h

    def launch(self):
        with torch.cuda.device(self.rec.device):
            _native.check(_native.lib().sgp4_plan_launch(self.handle, _stream(self.rec.device)), "sgp4_plan_launch")
        return self.out

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(512)
        _native.check(_native.lib().sgp4_plan_describe(self.handle, buf, 512), "sgp4_plan_describe")
        return buf.value.decode()

    def close(self):
        if getattr(self, "handle", None):
            _native.lib().sgp4_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def propagate_elements(elem: torch.Tensor, t: torch.Tensor, precision="fp64", grav: Optional[Sequence[float]] = None,
                       out=None, workspace: Optional[torch.Tensor] = None, flags: Optional[torch.Tensor] = None,
                       ref_jd=None):
    """Elements float64 [8, n] straight to r [3, n, T], v [3, n, T], err [n, T] in one
    call (sgp4_propagate_elements): a fused initialise-and-propagate launch for
    short time lists, initialisation into `workspace` (uint8, at least
    consts_bytes(n) bytes) and the dense launch for longer ones when given.
    flags: optional uint8 [n] tensor that receives the satellite flags.  ref_jd as
    for init."""
    p = _prec(precision)
    _need(elem, torch.float64, "elem")
    if elem.dim() != 2 or elem.shape[0] != 8:
        raise ValueError("elem must have shape [8, n]")
    _need(t, torch.float64, "t", elem.device)
    n, T = int(elem.shape[1]), int(t.numel())
    if out is None:
        dt = _out_dtype(p)
        r = torch.empty((3, n, T), dtype=dt, device=elem.device)
        v = torch.empty((3, n, T), dtype=dt, device=elem.device)
        err = torch.empty((n, T), dtype=torch.uint8, device=elem.device)
    else:
        r, v, err = out
    g = None
    if grav is not None:
        g = (ctypes.c_double * 5)(*[float(x) for x in grav])
    ws_bytes = 0
    if workspace is not None:
        _need(workspace, torch.uint8, "workspace", elem.device)
        ws_bytes = int(workspace.numel())
    if flags is not None:
        _need(flags, torch.uint8, "flags", elem.device)
        if flags.numel() < n:
            raise ValueError("flags must hold n entries")
    with torch.cuda.device(elem.device):
        _native.check(_native.lib().sgp4_propagate_elements_ex(
            g, _ref(ref_jd), n, _ptr(elem), _ptr(t), T, p, _ptr(r), _ptr(v), _ptr(err), _ptr(flags), _ptr(workspace),
            ws_bytes, _stream(elem.device)), "sgp4_propagate_elements_ex")
    return r, v, err


def screen(r: torch.Tensor, dist_km: float, err: Optional[torch.Tensor] = None, capacity: int = 1 << 20,
           mode: int = 0):
    """Conjunction screening of a dense output r [3, n, T] (float64 or float32,
    device): every pair i < j closer than dist_km at a common time index
    (sgp4_screen).  Returns (pairs int32 [m, 3] of (i, j, k), dist float64 [m]
    km, total) with m = min(total, capacity); event order is unspecified.
    mode: 0 automatic, 1 the on-chip path (n <= 12288), 2 the device-memory path."""
    if r.dim() != 3 or r.shape[0] != 3:
        raise ValueError("r must have shape [3, n, T]")
    if r.dtype not in (torch.float64, torch.float32):
        raise TypeError("r must be float64 or float32")
    _need(r, r.dtype, "r")
    n, T = int(r.shape[1]), int(r.shape[2])
    if err is not None:
        _need(err, torch.uint8, "err", r.device)
    cap = int(capacity)
    pairs = torch.empty((max(cap, 1), 3), dtype=torch.int32, device=r.device)
    dist = torch.empty(max(cap, 1), dtype=torch.float64, device=r.device)
    count = torch.empty(1, dtype=torch.int64, device=r.device)
    L = _native.lib()
    wsb = int(L.sgp4_screen_workspace_bytes(n, T))
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=r.device)
    prec = _native.SGP4_FP64 if r.dtype == torch.float64 else _native.SGP4_FP32
    with torch.cuda.device(r.device):
        _native.check(L.sgp4_screen_ex(_ptr(r), prec, _ptr(err), n, T, float(dist_km), cap, _ptr(pairs),
                                       _ptr(dist), _ptr(count), _ptr(ws), wsb, int(mode), _stream(r.device)),
                      "sgp4_screen")
    total = int(count.item())
    m = min(total, cap)
    return pairs[:m], dist[:m], total


def screen_noalloc(r: torch.Tensor, dist_km: float, err: Optional[torch.Tensor] = None, pairs=None, dist=None,
                   count=None):
    """As screen (automatic path) through sgp4_screen_noalloc: the workspace is
    the library's fixed per-GPU array, so the call allocates nothing when the
    caller passes the outputs pairs (int32 [capacity, 3]), dist (float64
    [capacity]) and count (int64 [1]); sgp4_screen_workspace_bytes(n, T) must
    not exceed NOALLOC_SCREEN_BYTES.  Returns (pairs[:m], dist[:m], total)."""
    if r.dim() != 3 or r.shape[0] != 3:
        raise ValueError("r must have shape [3, n, T]")
    if r.dtype not in (torch.float64, torch.float32):
        raise TypeError("r must be float64 or float32")
    _need(r, r.dtype, "r")
    n, T = int(r.shape[1]), int(r.shape[2])
    if err is not None:
        _need(err, torch.uint8, "err", r.device)
    if pairs is None:
        pairs = torch.empty((1 << 20, 3), dtype=torch.int32, device=r.device)
    if dist is None:
        dist = torch.empty(pairs.shape[0], dtype=torch.float64, device=r.device)
    if count is None:
        count = torch.empty(1, dtype=torch.int64, device=r.device)
    _need(pairs, torch.int32, "pairs", r.device)
    _need(dist, torch.float64, "dist", r.device)
    _need(count, torch.int64, "count", r.device)
    cap = int(min(pairs.shape[0], dist.shape[0]))
    prec = _native.SGP4_FP64 if r.dtype == torch.float64 else _native.SGP4_FP32
    with torch.cuda.device(r.device):
        _native.check(_native.lib().sgp4_screen_noalloc(_ptr(r), prec, _ptr(err), n, T, float(dist_km), cap,
                                                        _ptr(pairs), _ptr(dist), _ptr(count), _stream(r.device)),
                      "sgp4_screen_noalloc")
    total = int(count.item())
    m = min(total, cap)
    return pairs[:m], dist[:m], total


NOALLOC_SCREEN_BYTES = 64 << 20


def parse_text(text, fmt="tle", ref_jd=None, threads=0):
    """Element-set text (str or bytes; fmt "tle", "omm_kvn", "omm_csv" or
    "omm_json") to host numpy arrays: elem float64 [8, n] (rows as for init,
    epoch in days after ref_jd = (whole, frac), default J2000.0), satnum int64
    [n] and status int32 [n] (REC_* bits; elements NaN where REC_FIELD is set).
    Parsed by the library's native parser (sgp4_text_count / sgp4_text_parse)."""
    import numpy as np
    if fmt not in _native.TEXT_FORMATS:
        raise ValueError(f"unknown text format {fmt!r}")
    f = _native.TEXT_FORMATS[fmt]
    data = text.encode() if isinstance(text, str) else bytes(text)
    L = _native.lib()
    n = ctypes.c_int64(0)
    _native.check(L.sgp4_text_count(data, len(data), f, ctypes.byref(n)), "sgp4_text_count")
    n = int(n.value)
    elem = np.empty((8, n), dtype=np.float64)
    satnum = np.empty(n, dtype=np.int64)
    status = np.empty(n, dtype=np.int32)
    ref = None if ref_jd is None else (ctypes.c_double * 2)(float(ref_jd[0]), float(ref_jd[1]))
    _native.check(L.sgp4_text_parse(data, len(data), f, n, ref, ctypes.c_void_p(elem.ctypes.data),
                                    ctypes.c_void_p(satnum.ctypes.data), ctypes.c_void_p(status.ctypes.data),
                                    int(threads)), "sgp4_text_parse")
    return elem, satnum, status


def propagate_ragged(rec: Record, offsets: torch.Tensor, t: torch.Tensor, precision="fp64",
                     plan: Optional[RaggedPlan] = None, out=None):
    """CSR lists: returns r [3, nnz], v [3, nnz], err [nnz].  Without a plan the
    offsets are not checked: a point they place in no list gets code 8."""
    p = _prec(precision)
    _need(offsets, torch.int64, "offsets", rec.device)
    _need(t, torch.float64, "t", rec.device)
    if offsets.numel() != rec.n + 1:
        raise ValueError("offsets must have n + 1 entries")
    nnz = int(t.numel())
    if plan is not None:
        r, v, err = plan.out
        handle = plan.handle
    else:
        r, v, err = out if out is not None else _ragged_out(p, nnz, rec.device)
        handle = None
    with torch.cuda.device(rec.device):
        _native.check(_native.lib().sgp4_propagate_ragged(_ptr(rec.consts), rec.n, _ptr(offsets), _ptr(t), nnz, p,
                                                          _ptr(r), _ptr(v), _ptr(err), handle, _stream(rec.device)),
                      "sgp4_propagate_ragged")
    return r, v, err


def vjp(rec: Record, t: torch.Tensor, gr: torch.Tensor, gv: Optional[torch.Tensor] = None, precision="fp64"):
    """Vector-Jacobian product of the dense propagation: float64 [7, n]."""
    p = _prec(precision)
    _need(t, torch.float64, "t", rec.device)
    dt = _out_dtype(p)
    n, T = rec.n, int(t.numel())
    gr = gr.contiguous()
    _need(gr, dt, "gr", rec.device)
    if gr.numel() != 3 * n * T:
        raise ValueError("gr must have 3*n*T elements")
    if gv is not None:
        gv = gv.contiguous()
        _need(gv, dt, "gv", rec.device)
        if gv.numel() != 3 * n * T:
            raise ValueError("gv must have 3*n*T elements")
    out = torch.empty((7, n), dtype=torch.float64, device=rec.device)
    with torch.cuda.device(rec.device):
        _native.check(_native.lib().sgp4_vjp(n, _ptr(rec.elem), _ptr(rec.consts), _ptr(t), T, p, _ptr(gr), _ptr(gv),
                                             _ptr(out), _stream(rec.device)), "sgp4_vjp")
    return out


def vjp_ragged(rec: Record, offsets: torch.Tensor, t: torch.Tensor, gr: torch.Tensor,
               gv: Optional[torch.Tensor] = None, precision="fp64"):
    """Vector-Jacobian product over per-satellite time lists (CSR offsets
    int64 [n + 1], times float64 [nnz], cotangents [3, nnz]): float64 [7, n]."""
    p = _prec(precision)
    _need(offsets, torch.int64, "offsets", rec.device)
    _need(t, torch.float64, "t", rec.device)
    if offsets.numel() != rec.n + 1:
        raise ValueError("offsets must hold n + 1 entries")
    dt = _out_dtype(p)
    n, nnz = rec.n, int(t.numel())
    gr = gr.contiguous()
    _need(gr, dt, "gr", rec.device)
    if gr.numel() != 3 * nnz:
        raise ValueError("gr must have 3*nnz elements")
    if gv is not None:
        gv = gv.contiguous()
        _need(gv, dt, "gv", rec.device)
        if gv.numel() != 3 * nnz:
            raise ValueError("gv must have 3*nnz elements")
    out = torch.empty((7, n), dtype=torch.float64, device=rec.device)
    with torch.cuda.device(rec.device):
        _native.check(_native.lib().sgp4_vjp_ragged(n, _ptr(rec.elem), _ptr(rec.consts), _ptr(offsets), _ptr(t), nnz,
                                                    p, _ptr(gr), _ptr(gv), _ptr(out), _stream(rec.device)),
                      "sgp4_vjp_ragged")
    return out


def jacobian(rec: Record, t: torch.Tensor, precision="fp64", out: Optional[torch.Tensor] = None):
    """Jacobian of the dense propagation: float64 [6, 7, n, T], d(r, v)/d(elements),
    NaN at points whose code is 1, 2, 4 or 7."""
    p = _prec(precision)
    _need(t, torch.float64, "t", rec.device)
    n, T = rec.n, int(t.numel())
    if out is None:
        out = torch.empty((6, 7, n, T), dtype=torch.float64, device=rec.device)
    elif out.dtype != torch.float64 or out.numel() != 42 * n * T or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 tensor of 42*n*T elements")
    with torch.cuda.device(rec.device):
        _native.check(_native.lib().sgp4_jacobian(n, _ptr(rec.elem), _ptr(rec.consts), _ptr(t), T, p, _ptr(out),
                                                  _stream(rec.device)), "sgp4_jacobian")
    return out


def jacobian_ragged(rec: Record, offsets: torch.Tensor, t: torch.Tensor, precision="fp64",
                    out: Optional[torch.Tensor] = None):
    """Jacobian over per-satellite time lists (CSR offsets int64 [n + 1], times
    float64 [nnz]): float64 [6, 7, nnz], NaN at points whose code is 1, 2, 4 or 7."""
    p = _prec(precision)
    _need(offsets, torch.int64, "offsets", rec.device)
    _need(t, torch.float64, "t", rec.device)
    if offsets.numel() != rec.n + 1:
        raise ValueError("offsets must hold n + 1 entries")
    nnz = int(t.numel())
    if out is None:
        out = torch.empty((6, 7, nnz), dtype=torch.float64, device=rec.device)
    elif out.dtype != torch.float64 or out.numel() != 42 * nnz or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 tensor of 42*nnz elements")
    with torch.cuda.device(rec.device):
        _native.check(_native.lib().sgp4_jacobian_ragged(rec.n, _ptr(rec.elem), _ptr(rec.consts), _ptr(offsets),
                                                         _ptr(t), nnz, p, _ptr(out), _stream(rec.device)),
                      "sgp4_jacobian_ragged")
    return out


class SGP4Function(torch.autograd.Function):
    """(elem [8, n], t [T]) -> (r [3, n, T], v [3, n, T]); backward through the
    hand-written VJP kernel (no gradient for the epoch row or the times)."""

    @staticmethod
    def forward(ctx, elem, t, precision="fp64", grav=None):
        rec = init(elem.detach().contiguous(), grav)
        r, v, err = propagate(rec, t, precision)
        ctx.rec, ctx.t, ctx.precision = rec, t, precision
        ctx.mark_non_differentiable(err)
        return r, v, err

    @staticmethod
    def backward(ctx, gr, gv, _gerr):
        p = ctx.precision
        dt = _out_dtype(_prec(p))
        if gr is None:
            gr = torch.zeros((3, ctx.rec.n, ctx.t.numel()), dtype=dt, device=ctx.rec.device)
        g7 = vjp(ctx.rec, ctx.t, gr.to(dt), None if gv is None else gv.to(dt), p)
        g = torch.zeros((8, ctx.rec.n), dtype=torch.float64, device=ctx.rec.device)
        g[:7] = g7
        return g, None, None, None


class SGP4RaggedFunction(torch.autograd.Function):
    """(elem [8, n], offsets [n + 1], t [nnz]) -> (r [3, nnz], v [3, nnz], err
    [nnz]) over per-satellite time lists; backward through the ragged VJP
    kernel (no gradient for the epoch row, the offsets or the times)."""

    @staticmethod
    def forward(ctx, elem, offsets, t, precision="fp64", grav=None):
        rec = init(elem.detach().contiguous(), grav)
        r, v, err = propagate_ragged(rec, offsets, t, precision)
        ctx.rec, ctx.offsets, ctx.t, ctx.precision = rec, offsets, t, precision
        ctx.mark_non_differentiable(err)
        return r, v, err

    @staticmethod
    def backward(ctx, gr, gv, _gerr):
        p = ctx.precision
        dt = _out_dtype(_prec(p))
        if gr is None:
            gr = torch.zeros((3, ctx.t.numel()), dtype=dt, device=ctx.rec.device)
        g7 = vjp_ragged(ctx.rec, ctx.offsets, ctx.t, gr.to(dt), None if gv is None else gv.to(dt), p)
        g = torch.zeros((8, ctx.rec.n), dtype=torch.float64, device=ctx.rec.device)
        g[:7] = g7
        return g, None, None, None, None
