"""Learned warm start for the per-voxel power iteration (binding side).

Holds the network's parameters (FP32 master, FP16 copy, Adam moments) in
device memory and drives the library's kernels: pisco_ws_train_step,
pisco_ws_forward, pisco_ws_neighbor and pisco_eig_from.  torch only
allocates.  The network and its loss are described in include/pisco.h.

A learned solve of one scan (`LearnedSolver.solve`):
  1. G(x) on the estimation grid and on the grid coarser by two (the same
     nullspace basis serves both);
  2. the plain power iteration on the coarse grid (cheap: 1/4 or 1/8 of the
     voxels), giving each fine voxel a neighbour vector (its parent's);
  3. the network's start vector from G(x) and the neighbour vector;
  4. the power iteration on the estimation grid from that start.
"""
from __future__ import annotations

from typing import Optional, Sequence

from . import _lib as L


def coarse_grid(grid_lr: Sequence[int]):
    """The grid coarser by two per dimension (ceil)."""
    return tuple((int(g) + 1) // 2 for g in grid_lr)


class WarmStart:
    """Network parameters and training state for Q channels."""

    def __init__(self, Q: int, seed: int = 1, stream=None):
        import torch
        self.torch = torch
        self.Q = int(Q)
        self.h = L.Handle(stream)
        self.count = L.pisco_ws_param_count(self.Q)
        dev = "cuda"
        self.master = torch.empty(self.count, dtype=torch.float32, device=dev)
        self.w16 = torch.empty(self.count, dtype=torch.float16, device=dev)
        self.m = torch.zeros(self.count, dtype=torch.float32, device=dev)
        self.v = torch.zeros(self.count, dtype=torch.float32, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.step = 0
        self._ws = None
        self._ws_n = -1
        L.pisco_ws_init(self.h, self.Q, int(seed), self.master, self.w16)

    def _workspace(self, N: int):
        if N > self._ws_n:
            size = L.pisco_ws_workspace_size(self.Q, N)
            self._ws = self.torch.empty(size + 256, dtype=self.torch.uint8, device="cuda")
            self._ws_n = N
        base = self._ws.data_ptr()
        return self._ws[(-base) % 256:]

    def neighbor(self, grid_lr: Sequence[int], coarse_maps):
        """Neighbour vectors [Q][N] from eigenvectors on coarse_grid(grid_lr)."""
        N = 1
        for g in grid_lr:
            N *= int(g)
        nb = self.torch.empty((self.Q, N), dtype=self.torch.complex64, device="cuda")
        L.pisco_ws_neighbor(self.h, self.Q, grid_lr, coarse_maps.contiguous(), nb)
        return nb

    def forward(self, G, nb, bound: float):
        """Start vectors [Q][N] (unit norm)."""
        N = int(nb.shape[1])
        init = self.torch.empty((self.Q, N), dtype=self.torch.complex64, device="cuda")
        L.pisco_ws_forward(self.h, self.Q, N, float(bound), G.contiguous(), nb.contiguous(),
                           self.w16, init, self._workspace(N))
        return init

    def train_step(self, G, nb, target, bound: float, lr: float):
        """One Adam step on one batch; returns the device tensor of the mean
        loss before the step (not synchronised)."""
        N = int(nb.shape[1])
        self.step += 1
        L.pisco_ws_train_step(self.h, self.Q, N, float(bound), G.contiguous(), nb.contiguous(),
                              target.contiguous(), self.master, self.w16, self.m, self.v,
                              self.step, float(lr), self.loss, None, self._workspace(N))
        return self.loss

    def gradient(self, G, nb, target, bound: float):
        """(mean loss, gradient of the summed loss) without an update."""
        N = int(nb.shape[1])
        grad = self.torch.empty(self.count, dtype=self.torch.float32, device="cuda")
        loss = self.torch.empty(1, dtype=self.torch.float32, device="cuda")
        L.pisco_ws_train_step(self.h, self.Q, N, float(bound), G.contiguous(), nb.contiguous(),
                              target.contiguous(), None, self.w16, None, None, 0, 0.0, loss,
                              grad, self._workspace(N))
        return loss, grad


class LearnedSolver:
    """Estimation-grid and coarse-grid problems of one scan geometry."""

    def __init__(self, est, est_coarse, ws: WarmStart, coarse_iters: int = 10):
        self.est, self.est_c, self.ws = est, est_coarse, ws
        self.coarse_opts = L.make_opts(power_iters=coarse_iters, block=est.block)

    def fields(self, acs):
        """(G on the estimation grid, G on the coarse grid)."""
        gram = self.est.gram(acs)
        _, basis, counts = self.est.nullspace(gram)
        return self.est.gx(basis, counts), self.est_c.gx(basis, counts)

    def neighbour(self, Gc):
        maps_c, _, _ = self.est_c.eig(Gc, opts=self.coarse_opts)
        return self.ws.neighbor(self.est.grid_lr, maps_c)

    def solve(self, G, Gc, opts: Optional[L.Opts] = None):
        """Power iteration on G from the network's start vectors."""
        nb = self.neighbour(Gc)
        init = self.ws.forward(G, nb, float(self.est.nsup))
        return self.est.eig_from(G, init, opts)
