"""Exact discrete gradient of the 3D mean current density (FP64 oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).  As ``adjoint2d``
for the 3D model of ``lbm3d``: J is the current density summed over the
CL layers and averaged over the (x, y) area, on the state after ``nsteps``
steps from the equilibrium initial state; its gradient with respect to the
per-cell porosity, 1/K and effective O2 diffusivity (the three inputs the
paper varies independently, Section 5) is taken by reverse-mode
differentiation of the oracle itself (PyTorch autograd) with segment
recomputation.  Same convention at non-differentiable points (derivative of
|v| and of sqrt(1/K) is 0 where the argument is 0).
"""
from __future__ import annotations

import torch
from torch.utils.checkpoint import checkpoint

from . import lbm3d as L3


def _segment(geom, prm, nsteps):
    def run(state, phi, inv_k, d_eff):
        m = L3.Model3D(geom, prm, phi=phi, inv_k=inv_k, d_eff=d_eff)
        return m.run(state, nsteps)
    return run


def mean_current_density(geom: L3.Geometry3D, prm, phi, inv_k, d_eff, nsteps: int) -> torch.Tensor:
    """J after nsteps steps (differentiable in phi, inv_k, d_eff)."""
    m = L3.Model3D(geom, prm, phi=phi, inv_k=inv_k, d_eff=d_eff)
    s = m.run(m.initial_state(), nsteps)
    return m.observables(s)["current_density"]


def gradient(geom: L3.Geometry3D, prm, phi, inv_k, d_eff, nsteps: int, every: int = 100):
    """Return (J, dJ/dphi, dJ/d(1/K), dJ/dD_eff), float64 tensors [nz, ny, nx]."""
    leaves = [torch.as_tensor(a, dtype=L3.DT).clone().requires_grad_(True) for a in (phi, inv_k, d_eff)]
    m0 = L3.Model3D(geom, prm, phi=leaves[0], inv_k=leaves[1], d_eff=leaves[2])
    s = m0.initial_state()
    done = 0
    while done < nsteps:
        n = min(every, nsteps - done)
        s = checkpoint(_segment(geom, prm, n), s, *leaves, use_reentrant=False)
        done += n
    J = m0.observables(s)["current_density"]
    g = torch.autograd.grad(J, leaves)
    return J.detach(), g[0], g[1], g[2]
