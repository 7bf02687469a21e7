"""Pins of the pressure-driven inlet (Section 4: flow induced by a pressure
difference between inlet and outlet) in the oracle.  CPU only."""
import pytest
import torch

from oracle import lbm2d as L

DT = torch.float64


@pytest.mark.parametrize("p_in,p_out", [(2e-3, 0.0), (5e-3, 3e-3)])
def test_pressure_driven_channel_is_exact_poiseuille(p_in, p_out):
    # Clear channel, inlet pressure p_in at x = 0, p_out at x = nx - 1: the
    # steady state is plane Poiseuille flow with gradient (p_in - p_out) /
    # (nx - 1) and a linear pressure, to round-off.
    nx, H = 40, 9
    m = L.Model(L.Geometry(nx, H, H, 0, 0),
                L.Params(tau_f=1.0, reaction=False, pressure_inlet=True, p_in=p_in, p_out=p_out, dx_cm=1e-3))
    f = m.fields(m.run(m.initial_state(), 6000))
    y = torch.arange(H, dtype=DT)
    exact = (p_in - p_out) / (nx - 1) / (2 * m.nu) * (y + 0.5) * (H - 0.5 - y)
    assert float((f["ux"] - exact.view(H, 1)).abs().max() / exact.max()) < 1e-11
    x = torch.arange(nx, dtype=DT)
    assert float((f["p"] - (p_in + (p_out - p_in) * x / (nx - 1))).abs().max()) < 1e-13
    assert float(f["uy"].abs().max()) < 1e-15


def test_pressure_driven_cathode_steady_state():
    # Channel over a porous GDL / CL, no reaction: the inlet nodes carry
    # p_in, the run reaches a steady state, the volume flux through the
    # columns x >= 1 is the same to 1e-3 (the model is weakly compressible
    # in p), and the reported inlet flux is the sum of the inlet nodes' u_x.
    nx, ny, H = 30, 12, 6
    m = L.Model(L.Geometry(nx, ny, H, 5, 1),
                L.Params(tau_f=0.8, reaction=False, pressure_inlet=True, p_in=3e-3, phi_gdl=0.6, Da_gdl=1e-2))
    s = m.run(m.initial_state(), 8000)
    f = m.fields(s)
    assert float((f["p"][:H, 0] - 3e-3).abs().max()) < 1e-15
    f2 = m.fields(m.run(s, 100))
    assert float((f2["ux"] - f["ux"]).abs().max()) < 1e-12
    flux = f["ux"][:, 1:].sum(0)
    assert float((flux - flux.mean()).abs().max() / flux.mean()) < 1e-3
    o = m.observables(s)
    assert abs(float(o["inlet_flux"] - f["ux"][:H, 0].sum())) < 1e-15
    assert float(o["inlet_flux"]) > 0


def test_velocity_inlet_flux_equals_the_prescribed_profile():
    m = L.Model(L.Geometry(20, 10, 5, 4, 1), L.Params(Re=3.0, V_op=0.6))
    o = m.observables(m.run(m.initial_state(), 30))
    assert abs(float(o["inlet_flux"] - m.inlet_velocity().sum())) < 1e-15
    # and the utilisation is consumption over the advected O2
    assert abs(float(o["o2_utilisation"] - o["consumed_c"] / (m.inlet_velocity().sum() * m.p.c_in))) < 1e-15


def test_pressure_inlet_utilisation_uses_the_measured_flux():
    m = L.Model(L.Geometry(20, 10, 5, 4, 1), L.Params(V_op=0.5, pressure_inlet=True, p_in=1e-3))
    o = m.observables(m.run(m.initial_state(), 40))
    assert float(o["inlet_flux"]) > 0
    assert abs(float(o["o2_utilisation"] - o["consumed_c"] / (o["inlet_flux"] * m.p.c_in))) < 1e-15
