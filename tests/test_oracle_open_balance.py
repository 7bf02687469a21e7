"""Pins of the oracle's current density and heat rate (Section 5
observables; Eq. 13 integrated over the CL, Eq. 15) by the O2 and heat
budgets of an open cathode, with no use of the oracle's observable
formulas on the other side.  CPU only.

The current density is the charge the cathode reaction passes per unit
membrane area and time: four electrons per O2 molecule (Eq. 12), so
I = 4 F (moles of O2 consumed per second per cm^2 of membrane).  The O2
consumed is measured here from the populations alone: streaming with
bounce-back only permutes populations, the open-boundary columns inject
(or remove) what they overwrite, and the CL removes the rest, so per step

    consumed = (O2 the boundary columns inject) - (change of the O2 stored),

both read off sums of the post-collision states and of their streamed,
boundary-completed populations.  A lattice cell holds C_ref dx^2 mol of
O2 per unit depth at c = 1 and a step lasts dt, so over a membrane of
nx cells

    I = 4 F C_ref dx consumed / (dt nx).

The same budget of the temperature-rise lattice gives the heat rate:
H = (rho c_p)_CL dx heat_added / (dt nx), (rho c_p)_CL the mixture heat
capacity of Eq. 19 in the CL.  The lattice scales are those of the
problem statement: dx is the GDL thickness over its rows (Table 2's
length scale) and dt makes the lattice O2 diffusivity D_f_lat equal to
D_O2 dt / dx^2.  Altering the unit conversion of the observables (dx, dt,
4 F C_ref, the mean over the membrane) breaks these identities.
"""
import pytest
import torch

import workloads as W
from oracle import lbm2d as L
from oracle import lbm3d as L3

DT = torch.float64


def _scales(p: L.Params, n_gdl: int):
    dx = p.gdl_thickness_cm / n_gdl
    dt = p.D_f_lat * dx * dx / p.D_O2
    return dx, dt


EPS = torch.finfo(DT).eps


def _budget(model, post, planes):
    """(injected by the boundary columns, change of the stored amount) over
    the step that starts from the state ``post``, and the round-off bound of
    their difference: each is a difference of sums of N populations, and
    pairwise summation errs by at most about log2(N) eps sum|g| per sum
    (three sums, log2 N < 21 here: 64 eps sum|g|)."""
    pre = model.pre_collision(post)
    nxt = model.collide(pre)
    injected = float(pre[planes].sum() - post[planes].sum())
    stored = float(nxt[planes].sum() - post[planes].sum())
    bound = 64 * EPS * float(post[planes].abs().sum())
    return injected, stored, nxt, bound


def _check_2d(model, post, steps, heat=True):
    p, g = model.p, model.g
    dx, dt = _scales(p, g.ny_gdl)
    four_f_cref = 4.0 * p.faraday * p.C_ref
    phi_cl = float(model.phi[-1, 1])
    rhocp_cl = phi_cl * p.rhocp_f + (1.0 - phi_cl) * p.rhocp_s
    for _ in range(steps):
        o = model.observables(post)
        inj_c, sto_c, _, err_c = _budget(model, post, slice(14, 19))
        inj_t, sto_t, post, err_t = _budget(model, post, slice(9, 14))
        consumed = inj_c - sto_c
        I = four_f_cref * dx * consumed / (dt * g.nx)
        assert consumed > 0
        tol = 1e-13 + err_c / consumed
        print(f"I {float(o['current_density']):.10e} budget {I:.10e} (tol {tol:.1e})")
        assert abs(float(o["current_density"]) / I - 1.0) < tol
        if heat:
            heat_added = sto_t - inj_t
            H = rhocp_cl * dx * heat_added / (dt * g.nx)
            tol = 1e-13 + err_t / heat_added
            print(f"H {float(o['heat_rate']):.10e} budget {H:.10e} (tol {tol:.1e})")
            assert abs(float(o["heat_rate"]) / H - 1.0) < tol
    return post


def test_current_density_is_the_o2_budget_of_the_200x40_cathode():
    """The 200x40 FP64 workload (layered GDL, parabolic inlet, Tafel
    kinetics at 0.6 V): every step of a developing run, the current density
    and heat rate equal the O2 and heat budgets of the open lattice."""
    w = W.cathode2d_200x40()
    m = L.Model(L.geometry_from_workload(w), L.Params.from_workload(w))
    s = m.run(m.initial_state(), 150)
    _check_2d(m, s, 3)


def test_current_density_budget_with_a_porosity_field_and_butler_volmer():
    """Per-cell porosity (the 4096x1024 recipe at 48x20) and the
    Butler-Volmer kinetics: the O2 budget still fixes the current density.
    The heat check needs a uniform CL heat capacity and is left to the
    layered case."""
    w = W.cathode2d_scaled(48, 20, precision=64, V_op=0.7)
    phi = torch.as_tensor(W.porosity_field(w))
    p = L.Params.from_workload(w)
    p.butler_volmer = True
    m = L.Model(L.geometry_from_workload(w), p, phi=phi)
    s = m.run(m.initial_state(), 100)
    _check_2d(m, s, 3, heat=False)


def test_pressure_driven_inlet_budget():
    """The pressure-driven inlet (Section 4's flow driving): the budget
    does not depend on how the inlet sets the flow."""
    w = W.cathode2d_200x40()
    w.update(nx=40, ny=12, ny_channel=6, ny_gdl=5, ny_cl=1, pressure_inlet=True, p_in=2e-3)
    m = L.Model(L.geometry_from_workload(w), L.Params.from_workload(w))
    s = m.run(m.initial_state(), 100)
    _check_2d(m, s, 3)


def test_steady_state_current_is_the_net_o2_inflow():
    """At steady state nothing accumulates: the O2 flowing in through the
    inlet column minus what leaves through the outlet column (advective and
    diffusive alike, as the lattice carries them) is what the CL consumes,
    and I = 4 F C_ref dx (in - out) / (dt nx) to 1e-6; likewise the heat
    leaving through the end columns is the reaction heat.  A 12x5 cathode
    (channel 2, GDL 2, CL 1 rows) with a fast-diffusing solid so that the
    slowest thermal mode has died out within 5000 steps."""
    g = L.Geometry(12, 5, 2, 2, 1)
    p = L.Params(V_op=0.6, T_in=353.0, Re=1.0, phi_gdl=0.6, Da_gdl=1e-3, D_f_lat=0.025, rhocp_s=0.06)
    m = L.Model(g, p)
    s = m.run(m.initial_state(), 5000)
    dx, dt = _scales(p, g.ny_gdl)
    o = m.observables(s)
    inj_c, sto_c, _, _ = _budget(m, s, slice(14, 19))
    inj_t, sto_t, _, _ = _budget(m, s, slice(9, 14))
    assert abs(sto_c) < 1e-6 * inj_c and abs(sto_t) < 1e-6 * abs(inj_t)
    I = 4.0 * p.faraday * p.C_ref * dx * inj_c / (dt * g.nx)
    assert abs(float(o["current_density"]) / I - 1.0) < 1e-6
    rhocp_cl = p.phi_gdl * p.rhocp_f + (1.0 - p.phi_gdl) * p.rhocp_s
    H = rhocp_cl * dx * (-inj_t) / (dt * g.nx)
    assert abs(float(o["heat_rate"]) / H - 1.0) < 1e-6
    assert float(o["current_density"]) > 0 and float(o["heat_rate"]) > 0


@pytest.mark.parametrize("shape", [(10, 4, 8, (3, 4, 1)), (7, 5, 6, (2, 2, 2))])
def test_3d_current_density_is_the_o2_budget(shape):
    """3D variant: I is a mean over the (x, y) membrane area, so
    I = 4 F C_ref dx consumed / (dt nx ny); heat likewise."""
    nx, ny, nz, layers = shape
    w = W.cathode3d_scaled(nx, ny, nz, precision=64, nz_channel=layers[0], nz_gdl=layers[1], nz_cl=layers[2],
                           Re=1.0, dp_lat=0.0, Da_gdl=1e-2, phi_gdl=0.6)
    p = L3.params_from_workload(w)
    m = L3.Model3D(L3.geometry_from_workload(w), p)
    s = m.run(m.initial_state(), 40)
    dx, dt = _scales(p, layers[1])
    four_f_cref = 4.0 * p.faraday * p.C_ref
    rhocp_cl = p.phi_gdl * p.rhocp_f + (1.0 - p.phi_gdl) * p.rhocp_s
    for _ in range(2):
        o = m.observables(s)
        inj_c, sto_c, _, err_c = _budget(m, s, slice(26, 33))
        inj_t, sto_t, s, err_t = _budget(m, s, slice(19, 26))
        I = four_f_cref * dx * (inj_c - sto_c) / (dt * nx * ny)
        H = rhocp_cl * dx * (sto_t - inj_t) / (dt * nx * ny)
        assert abs(float(o["current_density"]) / I - 1.0) < 1e-13 + err_c / (inj_c - sto_c)
        assert abs(float(o["heat_rate"]) / H - 1.0) < 1e-13 + err_t / (sto_t - inj_t)
