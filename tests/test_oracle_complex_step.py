"""Pin of the oracle's discrete gradient by complex-step differentiation.

The forward map is evaluated once in complex arithmetic with the inputs
moved by i h d; the imaginary part of J over h is the derivative along d
with no subtraction, hence no truncation or cancellation error, and no
differentiation machinery of its own (it runs the same forward code, whose
operations are analytic on the paths taken: wall and layer choices are
made on masks that do not depend on the inputs, and sqrt's zero convention
tests the real part).  The reverse-mode gradient that the GPU adjoint is
checked against must match it to rounding, per cell and along a dense
direction, for each option the GPU adjoint covers.  CPU only.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import adjoint2d as A
from oracle import adjoint3d as A3
from oracle import lbm2d as L
from oracle import lbm3d as L3

DT = torch.float64
CT = torch.complex128
H = 1e-30
OPTIONS_2D = {
    "printed": ({}, {}),
    "butler_volmer": (dict(butler_volmer=True, alpha_a=0.5, V_op=1.1, aj0_ref=1e5), {}),
    "heat_physical": (dict(heat_physical=True), {}),
    "periodic_x_body_force": (dict(Re=0.0), dict(periodic_x=True)),
    "periodic_y": (dict(Re=0.8), dict(periodic_y=True)),
    "outlet_pressure": (dict(p_out=3e-3), {}),
    "buoyancy": (dict(buoyancy=(3e-3, -5e-3)), {}),
    "sigma_energy": (dict(sigma_energy=True, heat_physical=True), {}),
    "pressure_inlet": (dict(pressure_inlet=True, p_in=4e-3), {}),
    "thin_cl": (dict(thin_cl=True, ny_gdl=5, ny_cl=0), {}),
    "thin_cl_all": (dict(thin_cl=True, ny_gdl=5, ny_cl=0, butler_volmer=True, alpha_a=0.5, V_op=1.1, aj0_ref=1e5,
                         heat_physical=True, buoyancy=(3e-3, -5e-3), sigma_energy=True, pressure_inlet=True,
                         p_in=4e-3), {}),
}


def _case2d(over, geo_flags):
    w = W.adjoint2d(14, 10)
    w.update(ny_channel=5, ny_gdl=4, ny_cl=1, Re=2.0, V_op=0.45)
    w.update(over)
    p = L.Params.from_workload(w)
    if geo_flags.get("periodic_x"):
        p.body_force = (2e-5, 0.0)
    g = L.Geometry(14, 10, w["ny_channel"], w["ny_gdl"], w["ny_cl"], **geo_flags)
    phi = torch.as_tensor(W.porosity_field(w), dtype=DT)
    m = L.Model(g, p, phi=phi)
    return g, p, [phi, m.inv_k.detach().clone(), m.d_eff.detach().clone()]


def _direction(fields, porous, seed):
    rng = np.random.default_rng(seed)
    return [torch.where(porous, torch.tensor(rng.standard_normal(tuple(f.shape)), dtype=DT) * f.abs(),
                        torch.zeros_like(f)) for f in fields]


def _complex_step(J_of, fields, dirs):
    """d/de J(fields + e dirs) at e = 0 as Im J(fields + i H dirs) / H."""
    J = J_of(*[f.to(CT) + 1j * H * d.to(CT) for f, d in zip(fields, dirs)])
    return float(J.imag) / H


@pytest.mark.parametrize("option", list(OPTIONS_2D))
def test_gradient_along_a_dense_direction_equals_complex_step_2d(option):
    over, flags = OPTIONS_2D[option]
    g, p, fields = _case2d(over, flags)
    nsteps = 40
    _, *grads = A.gradient(g, p, *fields, nsteps=nsteps, every=15)
    porous = torch.zeros_like(fields[0], dtype=torch.bool)
    porous[g.ny_channel:] = True
    dirs = _direction(fields, porous, seed=11)
    dot = sum(float((gr * d).sum()) for gr, d in zip(grads, dirs))
    cs = _complex_step(lambda *f: A.mean_current_density(g, p, *f, nsteps=nsteps), fields, dirs)
    print(f"2d {option}: <grad, d> {dot:.15e}, complex step {cs:.15e}, rel {abs(dot / cs - 1):.1e}")
    assert abs(dot / cs - 1) < 1e-12


def test_gradient_per_cell_equals_complex_step_2d():
    """Single cells of the CL, the GDL and the inlet and outlet columns, for
    each of the three fields: the reverse-mode entry against the complex-step
    derivative along that cell's unit vector."""
    g, p, fields = _case2d({}, {})
    nsteps = 40
    _, *grads = A.gradient(g, p, *fields, nsteps=nsteps, every=15)
    J_of = lambda *f: A.mean_current_density(g, p, *f, nsteps=nsteps)
    for i, name in enumerate(("phi", "inv_k", "d_eff")):
        scale = float(grads[i].abs().max())
        for (y, x) in ((9, 3), (6, 7), (8, 0), (5, 13)):
            dirs = [torch.zeros_like(f) for f in fields]
            dirs[i][y, x] = 1.0
            cs = _complex_step(J_of, fields, dirs)
            ad = float(grads[i][y, x])
            assert abs(ad - cs) <= 1e-12 * scale, (name, y, x, ad, cs, scale)


def _case3d(over, geo_flags):
    w = W.cathode3d_scaled(8, 4, 8, precision=64, nz_channel=4, nz_gdl=3, nz_cl=1, Re=0.8, V_op=0.45,
                           sphere_radius=1.5, filter_box=5)
    w.update(over)
    g = L3.geometry_from_workload(w, **geo_flags)
    p = L3.params_from_workload(w)
    phi = torch.as_tensor(W.sphere_pack_porosity(w), dtype=DT)
    m = L3.Model3D(g, p, phi=phi)
    return g, p, [phi, m.inv_k.detach().clone(), m.d_eff.detach().clone()]


@pytest.mark.parametrize("option", ["printed", "butler_volmer", "periodic_y"])
def test_gradient_along_a_dense_direction_equals_complex_step_3d(option):
    over = dict(butler_volmer=True, alpha_a=0.5, V_op=1.1, aj0_ref=1e5) if option == "butler_volmer" else {}
    flags = dict(periodic_y=True) if option == "periodic_y" else {}
    g, p, fields = _case3d(over, flags)
    nsteps = 24
    _, *grads = A3.gradient(g, p, *fields, nsteps=nsteps, every=10)
    porous = torch.zeros_like(fields[0], dtype=torch.bool)
    porous[g.nz_channel:] = True
    dirs = _direction(fields, porous, seed=12)
    dot = sum(float((gr * d).sum()) for gr, d in zip(grads, dirs))
    cs = _complex_step(lambda *f: A3.mean_current_density(g, p, *f, nsteps=nsteps), fields, dirs)
    print(f"3d {option}: <grad, d> {dot:.15e}, complex step {cs:.15e}, rel {abs(dot / cs - 1):.1e}")
    assert abs(dot / cs - 1) < 1e-12


def test_complex_step_sees_a_planted_error():
    """The check is not vacuous: a reverse-mode gradient of a forward map
    with a perturbed constant (the Tafel transfer coefficient) fails it."""
    g, p, fields = _case2d({}, {})
    nsteps = 20
    porous = torch.zeros_like(fields[0], dtype=torch.bool)
    porous[g.ny_channel:] = True
    dirs = _direction(fields, porous, seed=13)
    cs = _complex_step(lambda *f: A.mean_current_density(g, p, *f, nsteps=nsteps), fields, dirs)
    wrong = L.Params(**{**p.__dict__, "alpha_c": p.alpha_c * (1 + 1e-6)})
    _, *grads = A.gradient(g, wrong, *fields, nsteps=nsteps, every=7)
    dot = sum(float((gr * d).sum()) for gr, d in zip(grads, dirs))
    assert abs(dot / cs - 1) > 1e-9
