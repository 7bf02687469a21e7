"""Pin of the 3D oracle's discrete gradient (reverse-mode differentiation of
the oracle) against central finite differences of its forward map.  CPU only."""
import numpy as np
import torch

import workloads as W
from oracle import adjoint3d as A3
from oracle import lbm3d as L3

DT = torch.float64


def _case(seed=5):
    w = W.cathode3d_scaled(8, 4, 8, precision=64, nz_channel=4, nz_gdl=3, nz_cl=1, Re=0.8, V_op=0.45)
    rng = np.random.default_rng(seed)
    nz, ny, nx = 8, 4, 8
    phi = np.ones((nz, ny, nx))
    phi[4:] = rng.uniform(0.4, 0.8, size=(4, ny, nx))
    inv_k = np.where(phi < 1, (1 - phi) ** 2 / (0.0067 * phi ** 3 * 8.0 ** 2), 0.0)
    d_eff = phi ** 1.5 * w["D_f_lat"]
    return (L3.geometry_from_workload(w), L3.params_from_workload(w),
            [torch.tensor(a, dtype=DT) for a in (phi, inv_k, d_eff)])


def test_gradient_matches_central_differences_3d():
    g, p, fields = _case()
    nsteps = 24
    J, gphi, gk, gd = A3.gradient(g, p, *fields, nsteps=nsteps, every=10)
    assert float(J) > 0
    grads = [gphi, gk, gd]
    # CL, GDL, the inlet and outlet columns, and a channel cell next to the GDL
    cells = [(7, 1, 3), (6, 2, 5), (5, 0, 0), (7, 3, 7), (4, 1, 1), (3, 2, 4)]
    for f_idx in range(3):
        for (z, y, x) in cells:
            if f_idx == 1 and z < 4:
                continue  # clear channel: 1/K = 0, where sqrt(1/K) has no derivative (convention: 0)
            base = fields[f_idx][z, y, x].item()
            h = 1e-4 * max(abs(base), 1e-3)  # J rounding (~1e-14 relative) limits smaller steps
            vals = []
            for sgn in (1, -1):
                pert = [a.clone() for a in fields]
                pert[f_idx][z, y, x] = base + sgn * h
                vals.append(float(A3.mean_current_density(g, p, *pert, nsteps=nsteps)))
            fd = (vals[0] - vals[1]) / (2 * h)
            ad = float(grads[f_idx][z, y, x])
            scale = float(grads[f_idx].abs().max())
            assert abs(ad - fd) <= 1e-6 * scale + 1e-9 * abs(fd), (f_idx, z, y, x, ad, fd, scale)


def dense_direction3d(fields, nz_channel, seed=8):
    """A seeded random direction over the porous layers of the three
    fields, scaled by each field's own magnitude."""
    rng = np.random.default_rng(seed)
    dirs = []
    for f in fields:
        d = torch.tensor(rng.standard_normal(tuple(f.shape)), dtype=DT) * f.abs()
        d[:nz_channel] = 0.0
        dirs.append(d)
    return dirs


def forward_mode_derivative3d(g, p, fields, dirs, nsteps):
    """d/de J(fields + e dirs) at e = 0 by forward-mode differentiation."""
    import torch.autograd.forward_ad as fwAD
    with fwAD.dual_level():
        duals = [fwAD.make_dual(f.clone(), d) for f, d in zip(fields, dirs)]
        J = A3.mean_current_density(g, p, *duals, nsteps=nsteps)
        return float(fwAD.unpack_dual(J).tangent)


def test_gradient_along_a_dense_direction_3d():
    """<grad J, d> over every porous cell against forward-mode
    differentiation and a central difference along d."""
    g, p, fields = _case()
    nsteps = 24
    _, *grads = A3.gradient(g, p, *fields, nsteps=nsteps, every=10)
    dirs = dense_direction3d(fields, g.nz_channel)
    dot = sum(float((gr * d).sum()) for gr, d in zip(grads, dirs))
    jvp = forward_mode_derivative3d(g, p, fields, dirs, nsteps)
    h = 1e-5
    vals = [float(A3.mean_current_density(g, p, *[f + s * h * d for f, d in zip(fields, dirs)], nsteps=nsteps))
            for s in (1, -1)]
    fd = (vals[0] - vals[1]) / (2 * h)
    print(f"3d <grad, d> {dot:.15e}, forward mode {jvp:.15e}, central difference {fd:.15e}")
    assert abs(dot / jvp - 1) < 1e-12
    assert abs(dot / fd - 1) < 1e-6
