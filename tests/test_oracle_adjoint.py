"""Pin of the oracle's discrete gradient (reverse-mode differentiation of the
oracle) against central finite differences of the oracle's forward map,
which share no differentiation machinery.  CPU only."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import adjoint2d as A
from oracle import lbm2d as L

DT = torch.float64


def _case(nx=14, ny=10, layers=(5, 4, 1), seed=3, **over):
    w = W.adjoint2d(nx, ny)
    w.update(ny_channel=layers[0], ny_gdl=layers[1], ny_cl=layers[2], Re=2.0, V_op=0.45)
    w.update(over)
    rng = np.random.default_rng(seed)
    phi = np.ones((ny, nx))
    phi[layers[0]:] = rng.uniform(0.4, 0.8, size=(ny - layers[0], nx))
    dp = 0.3325 * layers[1]
    inv_k = np.where(phi < 1, (1 - phi) ** 2 / (0.0067 * phi ** 3 * dp * dp), 0.0)
    d_eff = phi ** 1.5 * w["D_f_lat"]
    g = L.geometry_from_workload(w)
    p = L.Params.from_workload(w)
    return g, p, [torch.tensor(a, dtype=DT) for a in (phi, inv_k, d_eff)]


def test_gradient_matches_central_differences():
    g, p, fields = _case()
    nsteps = 40
    J, gphi, gk, gd = A.gradient(g, p, *fields, nsteps=nsteps, every=15)
    assert float(J) > 0
    grads = [gphi, gk, gd]
    cells = [(9, 3), (8, 7), (6, 11), (9, 12), (5, 0), (7, 13)]  # CL, GDL, and the inlet / outlet columns
    for f_idx in range(3):
        for (y, x) in cells:
            base = fields[f_idx][y, x].item()
            h = 1e-6 * max(abs(base), 1e-3)
            vals = []
            for sgn in (1, -1):
                pert = [a.clone() for a in fields]
                pert[f_idx][y, x] = base + sgn * h
                vals.append(float(A.mean_current_density(g, p, *pert, nsteps=nsteps)))
            fd = (vals[0] - vals[1]) / (2 * h)
            ad = float(grads[f_idx][y, x])
            scale = float(grads[f_idx].abs().max())
            assert abs(ad - fd) <= 1e-6 * scale + 1e-9 * abs(fd), (f_idx, y, x, ad, fd, scale)


def test_checkpoint_segments_do_not_change_the_gradient():
    g, p, fields = _case(seed=4)
    a = A.gradient(g, p, *fields, nsteps=30, every=30)
    b = A.gradient(g, p, *fields, nsteps=30, every=7)
    assert torch.equal(a[0], b[0])  # same forward arithmetic
    for u, v in zip(a[1:], b[1:]):  # gradient terms summed in another order
        assert float((u - v).abs().max()) <= 1e-12 * float(v.abs().max())


def _dense_direction(fields, ny_channel, seed=7):
    """A seeded random direction over every porous cell of the three
    fields, scaled by each field's own magnitude."""
    rng = np.random.default_rng(seed)
    dirs = []
    for f in fields:
        porous = torch.zeros_like(f, dtype=torch.bool)
        porous[ny_channel:] = True
        d = torch.tensor(rng.standard_normal(tuple(f.shape)), dtype=DT)
        dirs.append(torch.where(porous, d * f.abs(), torch.zeros_like(f)))
    return dirs


def forward_mode_derivative(g, p, fields, dirs, nsteps):
    """d/de J(fields + e dirs) at e = 0 by forward-mode differentiation of
    the oracle's forward map (no reverse pass involved)."""
    import torch.autograd.forward_ad as fwAD
    with fwAD.dual_level():
        duals = [fwAD.make_dual(f.clone(), d) for f, d in zip(fields, dirs)]
        J = A.mean_current_density(g, p, *duals, nsteps=nsteps)
        return float(fwAD.unpack_dual(J).tangent)


def test_gradient_along_a_dense_direction():
    """The dot-product identity <grad J, d> = dJ(m + e d)/de over every
    porous cell at once: against forward-mode differentiation (exact up to
    rounding) and against a central difference along d (truncation
    O(h^2))."""
    g, p, fields = _case()
    nsteps = 40
    _, *grads = A.gradient(g, p, *fields, nsteps=nsteps, every=15)
    dirs = _dense_direction(fields, g.ny_channel)
    dot = sum(float((gr * d).sum()) for gr, d in zip(grads, dirs))
    jvp = forward_mode_derivative(g, p, fields, dirs, nsteps)
    h = 1e-6
    vals = [float(A.mean_current_density(g, p, *[f + s * h * d for f, d in zip(fields, dirs)], nsteps=nsteps))
            for s in (1, -1)]
    fd = (vals[0] - vals[1]) / (2 * h)
    print(f"<grad, d> {dot:.15e}, forward mode {jvp:.15e}, central difference {fd:.15e}")
    assert abs(dot / jvp - 1) < 1e-12
    assert abs(dot / fd - 1) < 1e-6


@pytest.mark.parametrize("option", [dict(butler_volmer=True, alpha_a=0.5, V_op=1.1, aj0_ref=1e5),
                                    dict(heat_physical=True)], ids=["butler_volmer", "heat_physical"])
def test_gradient_along_a_dense_direction_with_kinetics_or_heat_option(option):
    """The same identity with Butler-Volmer kinetics near the equilibrium
    potential (Eq. 13 with its anodic branch) and with the physically signed
    reaction heat, whose reverse terms the default case does not reach."""
    g, p, fields = _case(**option)
    assert p.butler_volmer == option.get("butler_volmer", False)
    assert p.heat_physical == option.get("heat_physical", False)
    nsteps = 40
    _, *grads = A.gradient(g, p, *fields, nsteps=nsteps, every=15)
    dirs = _dense_direction(fields, g.ny_channel, seed=8)
    dot = sum(float((gr * d).sum()) for gr, d in zip(grads, dirs))
    jvp = forward_mode_derivative(g, p, fields, dirs, nsteps)
    h = 1e-6
    vals = [float(A.mean_current_density(g, p, *[f + s * h * d for f, d in zip(fields, dirs)], nsteps=nsteps))
            for s in (1, -1)]
    fd = (vals[0] - vals[1]) / (2 * h)
    print(f"{option}: <grad, d> {dot:.15e}, forward mode {jvp:.15e}, central difference {fd:.15e}")
    assert abs(dot / jvp - 1) < 1e-12
    assert abs(dot / fd - 1) < 1e-6
