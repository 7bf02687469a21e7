"""Exact discrete gradient of the mean current density (FP64 oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).  J is the mean
current density of Section 5, i.e. the x-average of the local current
density summed over the catalyst layer, evaluated on the state after
``nsteps`` steps from the equilibrium initial state.  Its gradient with
respect to the three per-cell inputs the paper varies independently
(porosity, permeability through 1/K, effective O2 diffusivity; Section 5,
permeability / porosity / diffusivity studies) is obtained by reverse-mode
differentiation of ``lbm2d`` itself (PyTorch autograd), with the run split
into segments that are recomputed during the backward pass so that memory
stays bounded; recomputation repeats the same float64 arithmetic, so the
gradient is that of the plain forward map (up to the order in which the
per-step contributions are summed).

Convention at non-differentiable points (shared with ``lbm2d._safe_sqrt``):
the derivative of |v| and of sqrt(1/K) is taken as 0 where the argument is
0 (the velocity recovery of Eq. 8 is C^1 there, and clear-fluid cells have
no permeability).
"""
from __future__ import annotations

import torch
from torch.utils.checkpoint import checkpoint

from . import lbm2d as L


def _segment(geom, prm, nsteps):
    def run(state, phi, inv_k, d_eff):
        m = L.Model(geom, prm, phi=phi, inv_k=inv_k, d_eff=d_eff)
        return m.run(state, nsteps)
    return run


def mean_current_density(geom: L.Geometry, prm: L.Params, phi, inv_k, d_eff, nsteps: int) -> torch.Tensor:
    """J after nsteps steps (differentiable in phi, inv_k, d_eff)."""
    m = L.Model(geom, prm, phi=phi, inv_k=inv_k, d_eff=d_eff)
    s = m.run(m.initial_state(), nsteps)
    return m.observables(s)["current_density"]


def gradient(geom: L.Geometry, prm: L.Params, phi, inv_k, d_eff, nsteps: int, every: int = 200):
    """Return (J, dJ/dphi, dJ/d(1/K), dJ/dD_eff) as float64 tensors [ny, nx]."""
    leaves = [torch.as_tensor(a, dtype=L.DT).clone().requires_grad_(True) for a in (phi, inv_k, d_eff)]
    m0 = L.Model(geom, prm, phi=leaves[0], inv_k=leaves[1], d_eff=leaves[2])
    s = m0.initial_state()
    done = 0
    while done < nsteps:
        n = min(every, nsteps - done)
        s = checkpoint(_segment(geom, prm, n), s, *leaves, use_reentrant=False)
        done += n
    J = m0.observables(s)["current_density"]
    g = torch.autograd.grad(J, leaves)
    return J.detach(), g[0], g[1], g[2]
