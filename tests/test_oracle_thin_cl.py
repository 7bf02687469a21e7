"""Pins of the oracle's thin-film catalyst layer (a reactive wall under the
GDL, the paper's CL of negligible thickness): the decay rate of a
diffusion / first-order surface-reaction problem against its closed-form
Robin eigenvalue (second-order convergence), exact O2 and heat budgets of
a closed box, and the geometry checks.  CPU only."""
import math

import pytest
import torch
from scipy.optimize import brentq

from oracle import lbm2d as L


def _robin_decay(H, Bi, D=0.1):
    """Lattice decay rate and the continuum rate D lambda^2 of the slowest
    mode of c_t = D c_yy on (0, H), no flux at 0, -D c_y = k c at H, with
    lambda H tan(lambda H) = Bi = k H / D.  Isothermal: V_op = U0 intercept
    makes eta + T dU0/dT = 0, so the film releases no heat (Eqs. 15-16)."""
    pr = L.Params(thin_cl=True, V_op=0.2329, D_f_lat=D, deff_ratio_gdl=1.0, phi_gdl=0.4, dx_cm=1e-3)
    m = L.Model(L.Geometry(3, H, 0, H, 0, periodic_x=True), pr)
    T = pr.T_in
    eta = pr.V_op - (pr.U0_slope * T + pr.U0_icept)
    # areal rate constant per unit a j0_ref of a film one lattice spacing thick
    per_aj0 = (math.exp(-pr.E_over_R * (1 / T - 1 / pr.T_arrh)) * m.dx
               * math.exp(-pr.alpha_c * pr.faraday * eta / (pr.R_gas * T)))
    k_lat = Bi * D / H  # wall flux per unit c per step, lattice units
    pr.aj0_ref = k_lat * 4 * pr.faraday * pr.C_ref * m.dx / (per_aj0 * m.dt)
    lam = brentq(lambda z: z * math.tan(z) - Bi, 1e-9, math.pi / 2 - 1e-9) / H
    n0, n1 = int(1.5 * H * H / D), int(0.75 * H * H / D)
    s = m.run(m.initial_state(), n0)
    c0 = float(m.fields(s)["c"].sum())
    s = m.run(s, n1)
    c1 = float(m.fields(s)["c"].sum())
    assert float(m.fields(s)["theta"].abs().max()) < 1e-12  # heat zero up to rounding
    return math.log(c0 / c1) / n1, D * lam * lam


@pytest.mark.parametrize("Bi", [1.0, 10.0])
def test_surface_reaction_decay_converges_to_the_robin_eigenvalue(Bi):
    e8 = _robin_decay(8, Bi)
    e16 = _robin_decay(16, Bi)
    err8, err16 = e8[0] / e8[1] - 1, e16[0] / e16[1] - 1
    print(f"Bi {Bi}: rel err H=8 {err8:.3e}, H=16 {err16:.3e}")
    assert abs(err8) < 1e-2
    assert 3.5 < err8 / err16 < 4.5  # second order in the lattice spacing


def test_closed_box_budgets_are_exact():
    # No inlet or outlet (periodic x), walls in y, the film under a porous
    # layer, reaction heat on: every step the O2 sum falls by exactly the
    # film's consumption and the temperature sum rises by its heat.
    g = L.Geometry(16, 9, 3, 6, 0, periodic_x=True)
    m = L.Model(g, L.Params(thin_cl=True, V_op=0.5, phi_gdl=0.5, Da_gdl=1e-2, dx_cm=2e-3))
    s = m.initial_state()
    o = m.observables(s)
    for _ in range(30):
        s = m.step(s)
        o1 = m.observables(s)
        assert abs(float(o["sum_c"] - o1["consumed_c"] - o1["sum_c"])) < 1e-12 * float(o["sum_c"])
        assert abs(float(o["sum_theta"] + o1["heat_added"] - o1["sum_theta"])) < 1e-12 * float(o1["sum_theta"])
        o = o1
    assert float(o["consumed_c"]) > 0 and float(o["sum_theta"]) > 0
    # the current is the film's consumption per area and time
    I = 4 * m.p.faraday * m.p.C_ref * m.dx * float(o["consumed_c"]) / (m.dt * g.nx)
    assert abs(float(o["current_density"]) / I - 1) < 1e-13


def test_thin_film_geometry_checks():
    with pytest.raises(ValueError):
        L.Model(L.Geometry(8, 6, 3, 2, 1), L.Params(thin_cl=True))
    with pytest.raises(ValueError):
        L.Model(L.Geometry(8, 6, 6, 0, 0), L.Params(thin_cl=True, dx_cm=1e-3))
    with pytest.raises(ValueError):
        L.Model(L.Geometry(8, 6, 3, 3, 0, periodic_x=True, periodic_y=True), L.Params(thin_cl=True))
