"""Pins of the oracle's porous energy equation with the heat-capacity ratio
sigma and of the physically signed reaction heat (model-fidelity variants
of Eqs. 10, 15 and 19).  CPU only."""
import math

import torch

from oracle import lbm2d as L

DT = torch.float64


def _materials(**kw):
    # a solid heat capacity and conductivity that keep sigma and the
    # relaxation times small enough for short runs
    return dict(rhocp_s=0.01, k_s=0.05, phi_gdl=0.4, dx_cm=2e-3, **kw)


def test_closed_box_conserves_energy_and_relaxes_to_the_discrete_steady_state():
    # Channel (sigma = 1) over a porous layer (sigma = 6.4), adiabatic walls,
    # periodic x, no flow, hot channel and cold GDL at t = 0.  The lattice
    # conserves sum(sigma theta) (energy / (rho c_p)_f) exactly; at rest it
    # settles where every node's moving populations, (4 + b) theta / 20, are
    # equal (equilibria that stream into themselves): theta_i = C / (4 + b_i)
    # with C fixed by the energy.
    m = L.Model(L.Geometry(3, 10, 4, 6, 0, periodic_x=True), L.Params(reaction=False, sigma_energy=True,
                                                                      **_materials()))
    assert float(m.sigma[0, 0]) == 1.0 and abs(float(m.sigma[-1, 0]) - 6.4) < 1e-12
    z = torch.zeros(10, 3, dtype=DT)
    th0 = torch.zeros(10, 3, dtype=DT)
    th0[:4] = 2.0
    s = m.equilibrium_state(z, z, z, th0, torch.ones(10, 3, dtype=DT))
    E0 = float((m.sigma * m.fields(s)["theta"]).sum())
    assert abs(E0 - 24.0) < 1e-13
    C = E0 / float((m.sigma / (4 + m.b_T)).sum())
    for _ in range(2):
        s = m.run(s, 4000)
        f = m.fields(s)
        assert abs(float((m.sigma * f["theta"]).sum()) / E0 - 1) < 1e-12
    assert float((f["theta"] - C / (4 + m.b_T)).abs().max()) / C < 1e-9


def test_sigma_diffusion_rate_is_the_effective_diffusivity():
    # Uniform porous box: theta = sin(k x) decays at k^2 k_eff / (rho c_p)_eff
    # (Eq. 19's alpha_eff) with sigma = (rho c_p)_eff / (rho c_p)_f and the
    # lattice carrying alpha_m = k_eff / (rho c_p)_f.
    nx = 32
    m = L.Model(L.Geometry(nx, 2, 0, 2, 0, periodic_x=True, periodic_y=True),
                L.Params(reaction=False, sigma_energy=True, **_materials()))
    p = m.p
    phi = p.phi_gdl
    k_eff = (p.k_f * phi + p.k_s * (1 - phi)) / 100.0
    a_eff = k_eff / (phi * p.rhocp_f + (1 - phi) * p.rhocp_s) * m.dt / m.dx ** 2
    k = 2 * math.pi / nx
    x = torch.arange(nx, dtype=DT).view(1, nx).expand(2, nx)
    z = torch.zeros(2, nx, dtype=DT)
    s = m.equilibrium_state(z, z, z, torch.sin(k * x), torch.ones(2, nx, dtype=DT))

    def amp(st):
        return float((m.fields(st)["theta"][0] * torch.sin(k * x[0])).sum() * 2 / nx)

    s = m.run(s, 50)
    a0 = amp(s)
    n = int(0.5 / (a_eff * k * k))
    s = m.run(s, n)
    rate = -math.log(amp(s) / a0) / n
    assert abs(rate / (a_eff * k * k) - 1) < 1e-5


def test_physically_signed_heat_special_cases():
    one = torch.ones(1, dtype=DT)
    g = L.Geometry(4, 1, 0, 0, 1, periodic_x=True, periodic_y=True)
    printed = L.Model(g, L.Params(dx_cm=1e-3))
    phys = L.Model(g, L.Params(dx_cm=1e-3, heat_physical=True))
    rc = printed.rhocp[0, :1]
    T = printed.p.T_in
    U0 = printed.p.U0_slope * T + printed.p.U0_icept
    # at zero overpotential only the entropic part is left, the same in both
    for m in (printed, phys):
        m.p.V_op = U0
    _, _, j0, q0, _ = printed.reaction(0 * one, one, rc)
    _, _, j1, q1, _ = phys.reaction(0 * one, one, rc)
    assert abs(float(q1) / float(q0) - 1) < 1e-12 and float(j0) == float(j1)
    # below the open-circuit voltage the physical heat exceeds the printed
    # one by twice the irreversible part |j| |eta|, and stays positive where
    # the printed heat changes sign (V < 0.2329 V)
    for V in (0.1, 0.2329, 0.5, 0.9):
        printed.p.V_op = phys.p.V_op = V
        _, _, j, qp, _ = printed.reaction(0 * one, one, rc)
        _, _, jj, qq, _ = phys.reaction(0 * one, one, rc)
        eta = V - U0
        assert float(qq) > 0 and float(j) == float(jj)
        assert abs(float(qq - qp) - 2 * float(j) * eta) < 1e-12 * abs(float(qq))
