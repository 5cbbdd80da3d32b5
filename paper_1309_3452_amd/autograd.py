"""Gradient of an observable with respect to a z-dependent potential, through
the hand-written adjoint of the leap-frog step (dirac_adjoint_vz): states are
rebuilt by reversing the scheme, not stored."""
from __future__ import annotations

import torch

from .lattice import Lattice


def potential_gradient(lat: Lattice, state0, m: float, v_int, v_half, nsteps: int, z0: float):
    """Forward nsteps from state0 with V(z) = (v_int, v_half), then the adjoint of
    L = sum_{z_s >= z0} |psi_s|^2.  Returns (L, dL/dv_int, dL/dv_half) as FP64
    tensors on the lattice's device; the lattice ends holding the rebuilt state0."""
    lat.load(state0)
    lat.set_potential_z(m, v_int, v_half)
    lat.step(nsteps)
    loss = lat.observables(z0)[0]
    lam = lat.seed_region(z0)
    dvi, dvh = lat.adjoint_vz(nsteps, lam)
    return loss, dvi, dvh


class DiracLoss(torch.autograd.Function):
    """L(p) = probability beyond z0 after nsteps, with V(z) = H_int p at integer z
    and H_half p at half-integer z (H: (nz, nodes) basis matrices, FP64 tensors)."""

    @staticmethod
    def forward(ctx, p, lat, state0, m, H_int, H_half, nsteps, z0):
        v_int = (H_int @ p.detach().to(torch.float64).cpu()).numpy()
        v_half = (H_half @ p.detach().to(torch.float64).cpu()).numpy()
        loss, dvi, dvh = potential_gradient(lat, state0, m, v_int, v_half, nsteps, z0)
        ctx.save_for_backward(dvi.cpu(), dvh.cpu(), H_int, H_half)
        ctx.p_dtype = p.dtype
        ctx.p_device = p.device
        return torch.tensor(loss, dtype=p.dtype, device=p.device)

    @staticmethod
    def backward(ctx, g):
        dvi, dvh, H_int, H_half = ctx.saved_tensors
        grad = H_int.t() @ dvi + H_half.t() @ dvh
        return (g.to(torch.float64).cpu() * grad).to(dtype=ctx.p_dtype, device=ctx.p_device), \
            None, None, None, None, None, None, None
