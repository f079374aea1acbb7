"""Batches of problems in one graph launch (binding side of pisco_batch_*).

    b = Batch(specs, acs_list)   # plans, autotunes and captures
    b.launch()                   # one graph launch recomputes every slice
    b.outputs[i]                 # maps of slice i (torch, complex64)

Each spec is a dict with keys Q, acs (shape), radius, grid_lr, grid_out and
optionally precision, power_iters, tol, phase_rule, block.  torch only
allocates the outputs and the workspace; the ACS tensors must stay alive
(and keep their addresses) while the batch exists: a launch reads their
current contents.
"""
from __future__ import annotations

import ctypes
from typing import Dict, List, Sequence

from . import _lib as L


class Batch:
    def __init__(self, specs: Sequence[Dict], acs: Sequence, stream=None):
        import torch
        self.torch = torch
        self.h = L.Handle(stream)
        B = len(specs)
        assert B == len(acs) and B > 0
        self.acs = [a.contiguous() for a in acs]
        probs = (L.Problem * B)()
        opts = (L.Opts * B)()
        self.outputs, self.lam = [], []
        for i, sp in enumerate(specs):
            D = len(sp["acs"])
            probs[i] = L.make_problem(D, sp["Q"], sp["acs"], sp["radius"], sp["grid_lr"],
                                      sp["grid_out"], sp.get("thresh", 0.05))
            opts[i] = L.make_opts(sp.get("power_iters", 10), sp.get("tol", 0.0),
                                  sp.get("phase_rule", 0), sp.get("block", 0), 60,
                                  sp.get("precision", 0))
            self.outputs.append(torch.empty((sp["Q"],) + tuple(sp["grid_out"]),
                                            dtype=torch.complex64, device="cuda"))
            nlr = 1
            for g in sp["grid_lr"]:
                nlr *= int(g)
            self.lam.append(torch.empty((nlr,), dtype=torch.float32, device="cuda"))
        size = ctypes.c_size_t()
        L._check(L.lib().pisco_batch_workspace_size(B, ctypes.cast(probs, ctypes.c_void_p),
                                                     ctypes.cast(opts, ctypes.c_void_p),
                                                     ctypes.byref(size)),
                 "pisco_batch_workspace_size")
        self._ws_raw = torch.empty(size.value + 256, dtype=torch.uint8, device="cuda")
        ws = self._ws_raw[(-self._ws_raw.data_ptr()) % 256:]
        arrays = [(ctypes.c_void_p * B)(*[t.data_ptr() for t in ts])
                  for ts in (self.acs, self.outputs, self.lam)]
        self._keep = (probs, opts, arrays)
        ptr = [ctypes.cast(a, ctypes.c_void_p) for a in arrays]
        batch = ctypes.c_void_p()
        L._check(L.lib().pisco_batch_create(
            self.h.h, B, ctypes.cast(probs, ctypes.c_void_p), ctypes.cast(opts, ctypes.c_void_p),
            ptr[0], ptr[1], ptr[2], ctypes.c_void_p(ws.data_ptr()),
            size.value, ctypes.byref(batch)), "pisco_batch_create", self.h.h)
        self.b = batch
        self.B = B

    def launch(self):
        L._check(L.lib().pisco_batch_launch(self.b), "pisco_batch_launch", self.h.h)

    def info(self, i: int):
        """(block, planned products, product wave target) of slice i."""
        v = [ctypes.c_int32() for _ in range(3)]
        L._check(L.lib().pisco_batch_slice_info(self.b, i, *[ctypes.byref(x) for x in v]),
                 "pisco_batch_slice_info")
        return tuple(x.value for x in v)

    def status(self) -> int:
        return self.h.status()

    def close(self):
        if self.b:
            L.lib().pisco_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # pragma: no cover
            pass
