"""A periodic (3+1)D lattice split into z-slabs, the unit a multi-GPU run gives
each device (the paper's closing remark: sub-domains handled separately that
trade boundary values).  Each slab is a z-slab-mode lattice (DIRAC_SLAB_Z):
nz/S interior planes plus two halo planes on each side.  Each slab advances
as many steps as its halos allow (two per launch of the two-step kernel with
V(z) tables, else one), after which the halos of every slab's current buffers
are refilled with its neighbours' outermost two interior planes; with several
GPUs those copies are the point-to-point sends and receives of the same
planes, here they are device copies on the current stream.  Stepping the slabs
gives the bits of the whole periodic lattice stepped by the fused kernels.
"""
from __future__ import annotations

import torch

from .lattice import Lattice

HALO = 2          # halo planes per side of a z-slab


class SlabDecomposition:
    def __init__(self, nx: int, ny: int, nz: int, slabs: int, dtype=torch.complex128, dt: float = 0.5, d=None,
                 device="cuda"):
        if slabs < 1 or nz % slabs:
            raise ValueError("nz must split into equal slabs")
        self.nx, self.ny, self.nz, self.count = nx, ny, nz, slabs
        self.nzs = nz // slabs
        if self.nzs < HALO:
            raise ValueError("each slab needs at least %d interior planes" % HALO)
        self.parts = [Lattice((nx, ny, self.nzs), dtype=dtype, dt=dt, d=d, device=device, slab=True)
                      for _ in range(slabs)]
        self.device = self.parts[0].device

    def planes(self, s: int):
        """Global z of slab s's stored planes (halo below, interior, halo above)."""
        return [(s * self.nzs - HALO + q) % self.nz for q in range(self.nzs + 2 * HALO)]

    def load(self, arrays):
        """Global state (8 arrays (nz, ny, nx)): each slab takes its interior and halo planes."""
        for s, lat in enumerate(self.parts):
            idx = torch.tensor(self.planes(s), device=arrays[0].device if torch.is_tensor(arrays[0]) else "cpu")
            lat.load([torch.as_tensor(a)[idx] for a in arrays])

    def set_potential_z(self, m: float, v_int=None, v_half=None):
        """Global V(z) tables (nz entries): each slab gets the entries of its stored planes."""
        import numpy as np
        for s, lat in enumerate(self.parts):
            if v_int is None:
                lat.set_potential_z(m)
            else:
                idx = self.planes(s)
                lat.set_potential_z(m, np.asarray(v_int)[idx], np.asarray(v_half)[idx])

    def set_fields(self, m: float, v_site):
        """Global per-site V (8 arrays (nz, ny, nx)), split like the state."""
        for s, lat in enumerate(self.parts):
            idx = torch.tensor(self.planes(s))
            lat.set_fields(m, [torch.as_tensor(v)[idx] for v in v_site])

    def exchange(self):
        """Fill every slab's halo planes from its neighbours' current interiors."""
        n = self.nzs
        cur = [lat.state() for lat in self.parts]
        for s in range(self.count):
            below, above = cur[(s - 1) % self.count], cur[(s + 1) % self.count]
            for a in range(8):
                cur[s][a][0:HALO].copy_(below[a][n:n + HALO])
                cur[s][a][n + HALO:n + 2 * HALO].copy_(above[a][HALO:2 * HALO])

    def set_kernel(self, kind: str = "auto", zchunk: int = 0):
        """"auto" (two steps per halo refill where the two-step kernel applies) or "fused" (one)."""
        for lat in self.parts:
            lat.set_kernel(kind, 0, zchunk)

    @property
    def halo_steps(self) -> int:
        """Steps between halo refills (1 or 2)."""
        return self.parts[0].halo_steps

    def step(self, n: int = 1):
        n, k = int(n), self.halo_steps
        while n > 0:
            m = min(k, n)
            for lat in self.parts:
                lat.step(m)
            self.exchange()
            n -= m

    def norm(self):
        """(E_r, E_r on the C,D sites, plain norm) of the whole lattice: the slabs' sums added."""
        vals = [lat.norm() for lat in self.parts]
        return tuple(sum(v[q] for v in vals) for q in range(3))

    def state(self):
        """The global state assembled from the slab interiors (new tensors)."""
        return [torch.cat([lat.state()[a][HALO:HALO + self.nzs] for lat in self.parts], dim=0) for a in range(8)]
