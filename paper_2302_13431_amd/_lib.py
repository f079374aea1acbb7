"""ctypes binding of libpisco (the C ABI declared in include/pisco.h).

Argument marshalling only: every computation runs in the HIP kernels of
libpisco.so.  Functions keep the C names; device arrays are passed as torch
tensors (their data pointers) and the stream is torch's current stream unless
given.  There is no CPU fallback: if the library is missing the import of the
functions raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpisco.so")

PISCO_OK = 0
STATUS_NAMES = {0: "ok", 1: "invalid argument", 2: "workspace too small", 3: "HIP error",
                4: "unsupported", 5: "numeric failure"}

FLAG_NONFINITE = 0x1
FLAG_NOT_CONVERGED = 0x2
FLAG_BLOCK_TOO_SMALL = 0x4
FLAG_ZERO_DATA = 0x8

STAGE_ALL, STAGE_GRAM, STAGE_NULLSPACE, STAGE_GX, STAGE_EIG, STAGE_MAPS, STAGE_MASK = range(7)
PREC_FP32, PREC_SPLIT_F16, PREC_SPLIT_BF16 = 0, 1, 2
PRODUCT_AUTO, PRODUCT_DENSE, PRODUCT_STRUCTURED = 0, 1, 2
SCHED_AUTO, SCHED_DEVICE = 0, 1


class Problem(ctypes.Structure):
    _fields_ = [("D", ctypes.c_int32), ("Q", ctypes.c_int32), ("acs", ctypes.c_int32 * 3),
                ("radius", ctypes.c_float), ("grid_lr", ctypes.c_int32 * 3),
                ("grid_out", ctypes.c_int32 * 3), ("thresh", ctypes.c_float),
                ("shape", ctypes.c_int32), ("gram_rows", ctypes.c_int32)]


class Opts(ctypes.Structure):
    _fields_ = [("power_iters", ctypes.c_int32), ("tol", ctypes.c_float),
                ("phase_rule", ctypes.c_int32), ("block", ctypes.c_int32),
                ("max_subspace_iters", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("product", ctypes.c_int32)]


class TraceEntry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 64), ("launches", ctypes.c_int32),
                ("total_ms", ctypes.c_double)]


class PiscoError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str = ""):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)} {msg}".strip())
        self.status = status


_lib = None

_P = ctypes.c_void_p
_SIGS = {
    "pisco_create": ([ctypes.POINTER(_P), _P], ctypes.c_int),
    "pisco_destroy": ([_P], ctypes.c_int),
    "pisco_set_stream": ([_P, _P], ctypes.c_int),
    "pisco_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "pisco_last_error": ([_P], ctypes.c_char_p),
    "pisco_get_status": ([_P, ctypes.POINTER(ctypes.c_uint32)], ctypes.c_int),
    "pisco_support": ([ctypes.c_int32, ctypes.c_float, ctypes.c_int32,
                       ctypes.POINTER(ctypes.c_int32), _P],
                      ctypes.c_int),
    "pisco_workspace_size": ([ctypes.POINTER(Problem), ctypes.POINTER(Opts), ctypes.c_int32,
                              ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "pisco_nullspace_block": ([ctypes.POINTER(Problem), ctypes.POINTER(Opts),
                               ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "pisco_gram": ([_P, ctypes.POINTER(Problem), _P, _P, _P, ctypes.c_size_t], ctypes.c_int),
    "pisco_gram_static": ([_P, ctypes.POINTER(Problem), _P, _P], ctypes.c_int),
    "pisco_gram_static_bytes": ([ctypes.POINTER(Problem), ctypes.POINTER(ctypes.c_size_t),
                                 ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "pisco_eig_sets_workspace_size": ([ctypes.c_int32, ctypes.c_int64,
                                       ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "pisco_eig_sets": ([_P, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_int32,
                        ctypes.c_int32, _P, _P, _P, _P, _P, ctypes.c_size_t], ctypes.c_int),
    "pisco_llr_workspace_size": ([ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "pisco_llr_svd": ([_P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P,
                       _P, _P, _P, _P, ctypes.c_size_t], ctypes.c_int),
    "pisco_support_mask": ([_P, ctypes.POINTER(Problem), _P, ctypes.c_float, _P, _P,
                            ctypes.c_size_t], ctypes.c_int),
    "pisco_espirit_operator": ([_P, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, _P, _P],
                               ctypes.c_int),
    "pisco_nullspace": ([_P, ctypes.POINTER(Problem), ctypes.POINTER(Opts), _P, _P, _P, _P, _P,
                         ctypes.c_size_t], ctypes.c_int),
    "pisco_gx": ([_P, ctypes.POINTER(Problem), ctypes.POINTER(Opts), _P, _P, _P, _P,
                  ctypes.c_size_t], ctypes.c_int),
    "pisco_eig": ([_P, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.POINTER(Opts), _P,
                   _P, _P, _P, _P, ctypes.c_size_t], ctypes.c_int),
    "pisco_maps": ([_P, ctypes.POINTER(Problem), ctypes.POINTER(Opts), _P, _P, _P, _P,
                    ctypes.c_size_t], ctypes.c_int),
    "pisco_estimate": ([_P, ctypes.POINTER(Problem), ctypes.POINTER(Opts), _P, _P, _P, _P,
                        ctypes.c_size_t], ctypes.c_int),
    "pisco_eig_from": ([_P, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.POINTER(Opts),
                        _P, _P, _P, _P, _P, _P, ctypes.c_size_t], ctypes.c_int),
    "pisco_eig_checked": ([_P, ctypes.c_int32, ctypes.c_int64, ctypes.c_float,
                           ctypes.POINTER(Opts), _P, _P, _P, _P, _P, _P, _P, _P,
                           ctypes.c_size_t], ctypes.c_int),
    "pisco_ws_param_count": ([ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "pisco_ws_workspace_size": ([ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)],
                                ctypes.c_int),
    "pisco_ws_init": ([_P, ctypes.c_int32, ctypes.c_uint64, _P, _P], ctypes.c_int),
    "pisco_ws_neighbor": ([_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), _P, _P],
                          ctypes.c_int),
    "pisco_ws_forward": ([_P, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, _P, _P, _P, _P, _P,
                          ctypes.c_size_t], ctypes.c_int),
    "pisco_ws_train_step": ([_P, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, _P, _P, _P, _P,
                             _P, _P, _P, ctypes.c_int32, ctypes.c_float, _P, _P, _P,
                             ctypes.c_size_t], ctypes.c_int),
    "pisco_batch_workspace_size": ([ctypes.c_int32, _P, _P, ctypes.POINTER(ctypes.c_size_t)],
                                   ctypes.c_int),
    "pisco_batch_create": ([_P, ctypes.c_int32, _P, _P, _P, _P, _P, _P, ctypes.c_size_t,
                            ctypes.POINTER(_P)], ctypes.c_int),
    "pisco_batch_launch": ([_P], ctypes.c_int),
    "pisco_batch_slice_info": ([_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)],
                               ctypes.c_int),
    "pisco_batch_destroy": ([_P], ctypes.c_int),
    "pisco_trace_enable": ([_P, ctypes.c_int32, ctypes.c_char_p], ctypes.c_int),
    "pisco_trace_read": ([_P, _P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
}


def lib():
    """Load libpisco.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} not built; run python -m paper_2302_13431_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


SHAPE_ELLIPSOID, SHAPE_RECTANGLE = 0, 1
ROWS_ALL, ROWS_VALID = 0, 1


def make_problem(D: int, Q: int, acs: Sequence[int], radius: float, grid_lr: Sequence[int],
                 grid_out: Sequence[int], thresh: float = 0.05, shape: int = SHAPE_ELLIPSOID,
                 gram_rows: int = ROWS_ALL) -> Problem:
    """Problem with extents given slowest-first; 2D shapes get z = 1."""
    def pad(v):
        v = list(v)
        return ([1] * (3 - len(v))) + v
    p = Problem()
    p.D, p.Q, p.radius, p.thresh = int(D), int(Q), float(radius), float(thresh)
    p.shape, p.gram_rows = int(shape), int(gram_rows)
    for name, val in (("acs", acs), ("grid_lr", grid_lr), ("grid_out", grid_out)):
        arr = getattr(p, name)
        for i, x in enumerate(pad(val)):
            arr[i] = int(x)
    return p


def make_opts(power_iters: int = 10, tol: float = 0.0, phase_rule: int = 0, block: int = 0,
              max_subspace_iters: int = 60, precision: int = PREC_FP32,
              schedule: int = 0, product: int = 0) -> Opts:
    o = Opts()
    o.power_iters, o.tol, o.phase_rule = int(power_iters), float(tol), int(phase_rule)
    o.block, o.max_subspace_iters = int(block), int(max_subspace_iters)
    o.precision, o.schedule, o.product = int(precision), int(schedule), int(product)
    return o


def _check(st: int, where: str, handle=None):
    if st != PISCO_OK:
        msg = ""
        if handle is not None:
            m = lib().pisco_last_error(handle)
            msg = m.decode() if m else ""
        raise PiscoError(st, where, msg)


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


# ---------------------------------------------------------------- host-only calls


def pisco_support(D: int, radius: float, shape: int = SHAPE_ELLIPSOID):
    """Support offsets as a list of (z, y, x) tuples in the library's order."""
    n = ctypes.c_int32()
    _check(lib().pisco_support(D, radius, shape, ctypes.byref(n), None), "pisco_support")
    buf = (ctypes.c_int32 * (3 * n.value))()
    _check(lib().pisco_support(D, radius, shape, ctypes.byref(n), ctypes.cast(buf, _P)),
           "pisco_support")
    return [tuple(buf[3 * i:3 * i + 3]) for i in range(n.value)]


def pisco_workspace_size(prob: Problem, opts: Optional[Opts], stage: int) -> int:
    out = ctypes.c_size_t()
    _check(lib().pisco_workspace_size(ctypes.byref(prob), ctypes.byref(opts) if opts else None,
                                      stage, ctypes.byref(out)), "pisco_workspace_size")
    return out.value


def pisco_nullspace_block(prob: Problem, opts: Optional[Opts]) -> int:
    out = ctypes.c_int32()
    _check(lib().pisco_nullspace_block(ctypes.byref(prob), ctypes.byref(opts) if opts else None,
                                       ctypes.byref(out)), "pisco_nullspace_block")
    return out.value


def pisco_status_string(st: int) -> str:
    return lib().pisco_status_string(st).decode()


# ---------------------------------------------------------------- handle and device calls


class Handle:
    """Owns a pisco handle bound to a HIP stream (torch's current by default)."""

    def __init__(self, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.h = _P()
        _check(lib().pisco_create(ctypes.byref(self.h), _P(stream.cuda_stream)), "pisco_create")

    def set_stream(self, stream=None):
        """Bind the handle to `stream` (None: the stream it was created with)."""
        s = self.stream if stream is None else stream
        _check(lib().pisco_set_stream(self.h, _P(s.cuda_stream)), "pisco_set_stream", self.h)

    def close(self):
        if self.h:
            lib().pisco_destroy(self.h)
            self.h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def status(self) -> int:
        f = ctypes.c_uint32()
        _check(lib().pisco_get_status(self.h, ctypes.byref(f)), "pisco_get_status", self.h)
        return f.value


def pisco_gram(h: Handle, prob: Problem, acs, gram, ws):
    _check(lib().pisco_gram(h.h, ctypes.byref(prob), _ptr(acs), _ptr(gram), _ptr(ws),
                            ws.numel() * ws.element_size()), "pisco_gram", h.h)


def pisco_gram_static(h: Handle, prob: Problem, acs, gram):
    """pisco_gram with the library's static scratch (no workspace argument)."""
    _check(lib().pisco_gram_static(h.h, ctypes.byref(prob), _ptr(acs), _ptr(gram)),
           "pisco_gram_static", h.h)


def pisco_gram_static_bytes(prob: Problem):
    """(scratch bytes needed, library limit) of pisco_gram_static."""
    need, limit = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().pisco_gram_static_bytes(ctypes.byref(prob), ctypes.byref(need),
                                         ctypes.byref(limit)), "pisco_gram_static_bytes")
    return need.value, limit.value


def pisco_nullspace(h: Handle, prob: Problem, opts: Opts, gram, eigvals, basis, counts, ws):
    _check(lib().pisco_nullspace(h.h, ctypes.byref(prob), ctypes.byref(opts), _ptr(gram),
                                 _ptr(eigvals), _ptr(basis), _ptr(counts), _ptr(ws),
                                 ws.numel() * ws.element_size()), "pisco_nullspace", h.h)


def pisco_gx(h: Handle, prob: Problem, opts: Opts, basis, counts, G, ws):
    _check(lib().pisco_gx(h.h, ctypes.byref(prob), ctypes.byref(opts), _ptr(basis), _ptr(counts),
                          _ptr(G), _ptr(ws), ws.numel() * ws.element_size()), "pisco_gx", h.h)


def pisco_eig(h: Handle, Q: int, N: int, bound: float, opts: Opts, G, maps, lam=None, iters=None):
    _check(lib().pisco_eig(h.h, Q, N, bound, ctypes.byref(opts), _ptr(G), _ptr(maps), _ptr(lam),
                           _ptr(iters), None, 0), "pisco_eig", h.h)


def pisco_eig_from(h: Handle, Q: int, N: int, bound: float, opts: Opts, G, init, maps, lam=None,
                   iters=None):
    _check(lib().pisco_eig_from(h.h, Q, N, bound, ctypes.byref(opts), _ptr(G), _ptr(init),
                                _ptr(maps), _ptr(lam), _ptr(iters), None, 0), "pisco_eig_from", h.h)


def pisco_eig_checked(h: Handle, Q: int, N: int, bound: float, opts: Opts, G, init, maps,
                      lam=None, iters=None, lam64=None, resid64=None):
    _check(lib().pisco_eig_checked(h.h, Q, N, bound, ctypes.byref(opts), _ptr(G), _ptr(init),
                                   _ptr(maps), _ptr(lam), _ptr(iters), _ptr(lam64),
                                   _ptr(resid64), None, 0), "pisco_eig_checked", h.h)


def pisco_eig_sets_workspace_size(Q: int, N: int) -> int:
    size = ctypes.c_size_t()
    _check(lib().pisco_eig_sets_workspace_size(Q, N, ctypes.byref(size)),
           "pisco_eig_sets_workspace_size")
    return size.value


def pisco_eig_sets(h: Handle, Q: int, N: int, bound: float, sets: int, krylov: int, G, maps,
                   lam, resid=None, ws=None):
    """ws: a 256-byte aligned device buffer of pisco_eig_sets_workspace_size
    bytes (allocated here through torch when None)."""
    if ws is None:
        import torch
        size = pisco_eig_sets_workspace_size(Q, N)
        raw = torch.empty(size + 256, dtype=torch.uint8, device=G.device)
        ws = raw[(-raw.data_ptr()) % 256:]
    _check(lib().pisco_eig_sets(h.h, Q, N, bound, sets, krylov, _ptr(G), _ptr(maps), _ptr(lam),
                                _ptr(resid), _ptr(ws), ws.numel() * ws.element_size()),
           "pisco_eig_sets", h.h)


def pisco_llr_svd(h: Handle, X, rank: int, V=None, Xr=None):
    """Partial SVDs of the B Casorati matrices X (torch complex64 [B][Q][m]):
    returns sigma [rank][B] (and fills V [rank][Q][B], Xr [B][Q][m] if given)."""
    import torch
    if X.dtype != torch.complex64 or X.dim() != 3 or not X.is_cuda:
        raise ValueError("X: need a CUDA complex64 tensor [B][Q][m]")
    B, Q, m = (int(v) for v in X.shape)
    for name, t, shape in (("V", V, (rank, Q, B)), ("Xr", Xr, (B, Q, m))):
        if t is not None and (t.dtype != torch.complex64 or tuple(t.shape) != shape
                              or not t.is_contiguous() or not t.is_cuda):
            raise ValueError(f"{name}: need a contiguous CUDA complex64 tensor {list(shape)}")
    size = ctypes.c_size_t()
    _check(lib().pisco_llr_workspace_size(B, Q, rank, ctypes.byref(size)),
           "pisco_llr_workspace_size")
    raw = torch.empty(size.value + 256, dtype=torch.uint8, device=X.device)
    ws = raw[(-raw.data_ptr()) % 256:]
    sigma = torch.empty((rank, B), dtype=torch.float32, device=X.device)
    _check(lib().pisco_llr_svd(h.h, B, m, Q, rank, _ptr(X.contiguous()), _ptr(sigma), _ptr(V),
                               _ptr(Xr), _ptr(ws), size.value), "pisco_llr_svd", h.h)
    return sigma


def pisco_support_mask(h: Handle, prob: Problem, lam, thresh: float, mask, ws):
    _check(lib().pisco_support_mask(h.h, ctypes.byref(prob), _ptr(lam), float(thresh),
                                    _ptr(mask), _ptr(ws), ws.numel() * ws.element_size()),
           "pisco_support_mask", h.h)


def pisco_espirit_operator(h: Handle, Q: int, N: int, bound: float, G, B):
    _check(lib().pisco_espirit_operator(h.h, Q, N, bound, _ptr(G), _ptr(B)),
           "pisco_espirit_operator", h.h)


def pisco_ws_param_count(Q: int) -> int:
    n = ctypes.c_int64()
    _check(lib().pisco_ws_param_count(Q, ctypes.byref(n)), "pisco_ws_param_count")
    return n.value


def pisco_ws_workspace_size(Q: int, N: int) -> int:
    n = ctypes.c_size_t()
    _check(lib().pisco_ws_workspace_size(Q, N, ctypes.byref(n)), "pisco_ws_workspace_size")
    return n.value


def pisco_ws_init(h: Handle, Q: int, seed: int, master, weights16):
    _check(lib().pisco_ws_init(h.h, Q, seed, _ptr(master), _ptr(weights16)), "pisco_ws_init", h.h)


def pisco_ws_neighbor(h: Handle, Q: int, grid_lr, coarse, neighbor):
    g = list(grid_lr)
    g = [1] * (3 - len(g)) + g
    arr = (ctypes.c_int32 * 3)(*g)
    _check(lib().pisco_ws_neighbor(h.h, Q, arr, _ptr(coarse), _ptr(neighbor)),
           "pisco_ws_neighbor", h.h)


def pisco_ws_forward(h: Handle, Q: int, N: int, bound: float, G, neighbor, weights16, init, ws):
    _check(lib().pisco_ws_forward(h.h, Q, N, bound, _ptr(G), _ptr(neighbor), _ptr(weights16),
                                  _ptr(init), _ptr(ws), ws.numel() * ws.element_size()),
           "pisco_ws_forward", h.h)


def pisco_ws_train_step(h: Handle, Q: int, N: int, bound: float, G, neighbor, target, master,
                        weights16, adam_m, adam_v, step: int, lr: float, loss_out, grad_out, ws):
    _check(lib().pisco_ws_train_step(h.h, Q, N, bound, _ptr(G), _ptr(neighbor), _ptr(target),
                                     _ptr(master), _ptr(weights16), _ptr(adam_m), _ptr(adam_v),
                                     int(step), float(lr), _ptr(loss_out), _ptr(grad_out),
                                     _ptr(ws), ws.numel() * ws.element_size()),
           "pisco_ws_train_step", h.h)


def pisco_maps(h: Handle, prob: Problem, opts: Opts, acs, maps_lr, maps_out, ws):
    _check(lib().pisco_maps(h.h, ctypes.byref(prob), ctypes.byref(opts), _ptr(acs), _ptr(maps_lr),
                            _ptr(maps_out), _ptr(ws), ws.numel() * ws.element_size()),
           "pisco_maps", h.h)


def pisco_estimate(h: Handle, prob: Problem, opts: Opts, acs, maps_out, lam, ws):
    _check(lib().pisco_estimate(h.h, ctypes.byref(prob), ctypes.byref(opts), _ptr(acs),
                                _ptr(maps_out), _ptr(lam), _ptr(ws),
                                ws.numel() * ws.element_size()), "pisco_estimate", h.h)


def pisco_trace_enable(h: Handle, enable: bool, filter: Optional[str] = None):
    _check(lib().pisco_trace_enable(h.h, 1 if enable else 0,
                                    filter.encode() if filter else None),
           "pisco_trace_enable", h.h)


def pisco_trace_read(h: Handle):
    """{kernel name: (launches, total_ms)} since the last read (synchronises)."""
    cap = 256
    buf = (TraceEntry * cap)()
    n = ctypes.c_int32()
    _check(lib().pisco_trace_read(h.h, ctypes.cast(buf, _P), cap, ctypes.byref(n)),
           "pisco_trace_read", h.h)
    return {buf[i].name.decode(): (buf[i].launches, buf[i].total_ms)
            for i in range(min(n.value, cap))}
