"""Stage-by-stage and end-to-end calls with torch-allocated device buffers.

torch provides device memory and the stream; every stage is one call into
libpisco (see include/pisco.h for the layouts).
"""
from __future__ import annotations

from typing import Optional, Sequence

from . import _lib as L


def _prod(v):
    out = 1
    for x in v:
        out *= int(x)
    return out


class Estimator:
    """Buffers and calls for one problem size."""

    def __init__(self, Q: int, acs_shape: Sequence[int], radius: float,
                 grid_lr: Sequence[int], grid_out: Sequence[int], thresh: float = 0.05,
                 power_iters: int = 10, tol: float = 0.0, phase_rule: int = 0,
                 block: int = 0, max_subspace_iters: int = 60, precision: int = 0,
                 schedule: int = 0, shape: int = 0, gram_rows: int = 0, stream=None,
                 product: int = 0):
        import torch
        self.torch = torch
        self.D = len(acs_shape)
        self.Q = int(Q)
        self.acs_shape = tuple(int(a) for a in acs_shape)
        self.grid_lr = tuple(int(a) for a in grid_lr)
        self.grid_out = tuple(int(a) for a in grid_out)
        self.radius = float(radius)
        self.prob = L.make_problem(self.D, Q, acs_shape, radius, grid_lr, grid_out, thresh,
                                   shape, gram_rows)
        self.opts = L.make_opts(power_iters, tol, phase_rule, block, max_subspace_iters,
                                precision, schedule, product)
        self.h = L.Handle(stream)
        self.support = L.pisco_support(self.D, radius, shape)
        self.nsup = len(self.support)
        self.n = self.Q * self.nsup
        self.P = self.Q * (self.Q + 1) // 2
        self.block = L.pisco_nullspace_block(self.prob, self.opts)
        self.Nlr = _prod(self.grid_lr)
        self.Nout = _prod(self.grid_out)
        dev = torch.device("cuda")
        ws_stage = max(L.pisco_workspace_size(self.prob, self.opts, s) for s in range(1, 7))
        self.ws_stage = torch.empty(ws_stage + 256, dtype=torch.uint8, device=dev)
        self.ws_all = None
        self.dev = dev

    # -------------------------------------------------------------- buffers
    def _alloc(self, shape, dtype):
        return self.torch.empty(tuple(shape), dtype=dtype, device=self.dev)

    def _need(self, x, nbytes: int, what: str):
        """The library takes raw device pointers: refuse a buffer that is not
        on the GPU or is smaller than the call reads or writes."""
        if x is None:
            return None
        if not (hasattr(x, "is_cuda") and x.is_cuda):
            raise ValueError(f"{what}: need a CUDA tensor")
        have = x.numel() * x.element_size()
        if have < nbytes:
            raise ValueError(f"{what}: {have} bytes, the call needs {nbytes}")
        return x.contiguous()

    def _need_out(self, x, nbytes: int, what: str):
        """An output buffer: as _need, and written in place, so contiguous."""
        if x is not None and hasattr(x, "is_contiguous") and not x.is_contiguous():
            raise ValueError(f"{what}: output must be contiguous")
        return self._need(x, nbytes, what)

    def _ws(self):
        # 256-byte aligned view of the stage workspace
        base = self.ws_stage.data_ptr()
        off = (-base) % 256
        return self.ws_stage[off:]

    # -------------------------------------------------------------- stages
    def gram(self, acs):
        t = self.torch
        out = self._alloc((self.n, self.n), t.complex64)
        acs = self._need(acs, 8 * self.Q * _prod(self.acs_shape), "acs")
        L.pisco_gram(self.h, self.prob, acs, out, self._ws())
        return out

    def nullspace(self, gram):
        t = self.torch
        b = self.block
        eig = self._alloc((b,), t.float64)
        basis = self._alloc((b, self.n), t.complex128)
        counts = self._alloc((4,), t.int32)
        gram = self._need(gram, 8 * self.n * self.n, "gram")
        L.pisco_nullspace(self.h, self.prob, self.opts, gram, eig, basis, counts, self._ws())
        return eig, basis, counts

    def gx(self, basis, counts):
        t = self.torch
        G = self._alloc((self.P, self.Nlr), t.complex64)
        basis = self._need(basis, 16 * self.block * self.n, "basis")
        counts = self._need(counts, 16, "counts")
        L.pisco_gx(self.h, self.prob, self.opts, basis, counts, G, self._ws())
        return G

    def eig(self, G, N: Optional[int] = None, opts: Optional[L.Opts] = None,
            Q: Optional[int] = None, bound: Optional[float] = None):
        t = self.torch
        N = self.Nlr if N is None else int(N)
        Q = self.Q if Q is None else int(Q)
        bound = float(self.nsup) if bound is None else float(bound)
        maps = self._alloc((Q, N), t.complex64)
        lam = self._alloc((N,), t.float32)
        it = self._alloc((N,), t.int32)
        G = self._need(G, 4 * Q * (Q + 1) * N, "G")
        L.pisco_eig(self.h, Q, N, bound, opts or self.opts, G, maps, lam, it)
        return maps, lam, it

    def eig_checked(self, G, init=None, opts: Optional[L.Opts] = None,
                    N: Optional[int] = None, Q: Optional[int] = None,
                    bound: Optional[float] = None):
        """Power iteration plus the FP64 Rayleigh check of the result:
        (maps, lam, iters, lam64, resid64)."""
        t = self.torch
        N = self.Nlr if N is None else int(N)
        Q = self.Q if Q is None else int(Q)
        bound = float(self.nsup) if bound is None else float(bound)
        maps = self._alloc((Q, N), t.complex64)
        lam = self._alloc((N,), t.float32)
        it = self._alloc((N,), t.int32)
        lam64 = self._alloc((N,), t.float64)
        res64 = self._alloc((N,), t.float64)
        G = self._need(G, 4 * Q * (Q + 1) * N, "G")
        init = self._need(init, 8 * Q * N, "init")
        L.pisco_eig_checked(self.h, Q, N, bound, opts or self.opts, G, init, maps, lam, it,
                            lam64, res64)
        return maps, lam, it, lam64, res64

    def eig_sets(self, G, sets: int = 1, krylov: Optional[int] = None, N: Optional[int] = None,
                 Q: Optional[int] = None, bound: Optional[float] = None):
        """The `sets` smallest eigenpairs per voxel by Lanczos (pisco_eig_sets):
        (maps [sets][Q][N], lam [sets][N], resid [sets][N])."""
        t = self.torch
        N = self.Nlr if N is None else int(N)
        Q = self.Q if Q is None else int(Q)
        K = Q if krylov is None else int(krylov)
        bound = float(self.nsup) if bound is None else float(bound)
        maps = self._alloc((sets, Q, N), t.complex64)
        lam = self._alloc((sets, N), t.float32)
        res = self._alloc((sets, N), t.float32)
        G = self._need(G, 4 * Q * (Q + 1) * N, "G")
        L.pisco_eig_sets(self.h, Q, N, bound, sets, K, G, maps, lam, res)
        return maps, lam, res

    def eig_from(self, G, init, opts: Optional[L.Opts] = None):
        """Power iteration from the given start vectors (float2 [Q][N_lr])."""
        t = self.torch
        N = self.Nlr
        maps = self._alloc((self.Q, N), t.complex64)
        lam = self._alloc((N,), t.float32)
        it = self._alloc((N,), t.int32)
        G = self._need(G, 4 * self.Q * (self.Q + 1) * N, "G")
        init = self._need(init, 8 * self.Q * N, "init")
        L.pisco_eig_from(self.h, self.Q, N, float(self.nsup), opts or self.opts, G, init, maps,
                         lam, it)
        return maps, lam, it

    def maps(self, acs, maps_lr):
        t = self.torch
        out = self._alloc((self.Q,) + self.grid_out, t.complex64)
        acs = self._need(acs, 8 * self.Q * _prod(self.acs_shape), "acs")
        maps_lr = self._need(maps_lr, 8 * self.Q * self.Nlr, "maps_lr")
        L.pisco_maps(self.h, self.prob, self.opts, acs, maps_lr, out, self._ws())
        return out

    def support_mask(self, lam, thresh: float = 0.1):
        """uint8 mask on grid_out from a low-res lambda_min map (pisco_support_mask)."""
        t = self.torch
        mask = self._alloc(self.grid_out, t.uint8)
        lam = self._need(lam, 4 * self.Nlr, "lam")
        L.pisco_support_mask(self.h, self.prob, lam, thresh, mask, self._ws())
        return mask

    def espirit_operator(self, G, Q: Optional[int] = None, N: Optional[int] = None,
                         bound: Optional[float] = None):
        """B = I - G / |Lambda| in G's packed layout (pisco_espirit_operator)."""
        Q = self.Q if Q is None else int(Q)
        N = self.Nlr if N is None else int(N)
        bound = float(self.nsup) if bound is None else float(bound)
        G = self._need(G, 4 * Q * (Q + 1) * N, "G")
        B = self.torch.empty_like(G)
        L.pisco_espirit_operator(self.h, Q, N, bound, G, B)
        return B

    def estimate(self, acs, out=None, lam=None):
        t = self.torch
        if self.ws_all is None:
            size = L.pisco_workspace_size(self.prob, self.opts, L.STAGE_ALL)
            self.ws_all = t.empty(size + 256, dtype=t.uint8, device=self.dev)
        base = self.ws_all.data_ptr()
        ws = self.ws_all[(-base) % 256:]
        if out is None:
            out = self._alloc((self.Q,) + self.grid_out, t.complex64)
        if lam is None:
            lam = self._alloc((self.Nlr,), t.float32)
        acs = self._need(acs, 8 * self.Q * _prod(self.acs_shape), "acs")
        self._need_out(out, 8 * self.Q * self.Nout, "out")
        self._need_out(lam, 4 * self.Nlr, "lam")
        L.pisco_estimate(self.h, self.prob, self.opts, acs, out, lam, ws)
        return out, lam

    def status(self) -> int:
        return self.h.status()
