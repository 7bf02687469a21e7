"""Pins of the oracle's scalar lattices (Section 2.2), catalyst-layer
kinetics (Section 4, Eqs. 12-17) and effective properties (Eqs. 18-19)
against closed forms, special cases, invariants and the paper's printed
tables.  CPU only."""
import json
import math
import os

import torch

from oracle import lbm2d as L

DT = torch.float64
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_printed.json")))


def _box(nx, ny, layers=None, periodic_y=True, **kw):
    ch, gdl, cl = layers if layers else (ny, 0, 0)
    g = L.Geometry(nx, ny, ch, gdl, cl, periodic_x=True, periodic_y=periodic_y)
    kw.setdefault("dx_cm", 1e-3)
    return L.Model(g, L.Params(**kw))


def _decay_rate(nx, D):
    m = _box(nx, 1, reaction=False, D_f_lat=D)
    x = torch.arange(nx, dtype=DT).view(1, nx)
    k = 2 * math.pi / nx
    z = torch.zeros(1, nx, dtype=DT)
    s = m.equilibrium_state(z, z, z, z, 1.0 + 1e-3 * torch.sin(k * x))

    def amp(state):
        c = m.fields(state)["c"][0]
        return float(((c - 1.0) * torch.sin(k * x[0])).sum() * 2 / nx)

    s = m.run(s, 50)  # let the start-up non-equilibrium layer die out
    a0 = amp(s)
    n = 200
    s = m.run(s, n)
    return -math.log(amp(s) / a0) / (n * k * k)


def test_d2q5_diffusivity_from_b():
    # Sine mode in a periodic box decays at D k^2 with D = (4 + b)/(20 sqrt 3)
    # (Eq. 10).  With the rates of Eq. 10 (Lambda = 1/6) the O(k^2) lattice
    # correction cancels: the error falls ~16x when k halves.
    for D in (0.0125, 0.003):
        e32 = abs(_decay_rate(32, D) / D - 1)
        e64 = abs(_decay_rate(64, D) / D - 1)
        assert e64 < 1e-6
        assert 10.0 < e32 / e64 < 22.0


def test_scalar_budgets_close_with_sources():
    # Closed periodic box, reaction in every cell: sum g_C falls by the
    # consumed O2 and sum g_T rises by the heat source, every step, exactly.
    torch.manual_seed(7)
    m = _box(6, 5, layers=(0, 0, 5), V_op=0.5, T_in=353.15)
    s = m.initial_state()
    s[14:19] *= 1.0 + 0.1 * torch.rand(5, 5, 6, dtype=DT)
    s[9:14] += 0.05 * torch.rand(5, 5, 6, dtype=DT)
    for _ in range(5):
        o0 = m.observables(s)
        s = m.step(s)
        o1 = m.observables(s)
        assert abs(float(o1["sum_c"] - (o0["sum_c"] - o0["consumed_c"]))) < 1e-13 * float(o0["sum_c"])
        assert abs(float(o1["sum_theta"] - (o0["sum_theta"] + o0["heat_added"]))) < 1e-13 * float(o1["sum_theta"])
        assert float(o0["consumed_c"]) > 0 and float(o0["heat_added"]) > 0


def test_uniform_sink_decays_geometrically_and_heat_tracks_oxygen():
    # Uniform closed box: O2 decays by the same factor every step when the
    # reaction heat vanishes (V = U0 intercept, so eta + T dU0/dT = 0 by
    # Eqs. 15-16); in general theta + 4 F C_ref (V - U0_icept)/(rho c_p) c is
    # invariant, since the heat per mole of O2 is 4F(eta + T dU0/dT).
    m = _box(4, 3, layers=(0, 0, 3), V_op=0.2329, aj0_ref=1e-9)
    s = m.initial_state()
    cs = []
    for _ in range(6):
        cs.append(float(m.fields(s)["c"][1, 1]))
        s = m.step(s)
    ratios = [cs[i + 1] / cs[i] for i in range(5)]
    assert max(ratios) - min(ratios) < 1e-14 and ratios[0] < 1.0
    assert float(m.fields(s)["theta"].abs().max()) < 1e-15

    m = _box(4, 3, layers=(0, 0, 3), V_op=0.45, phi_gdl=0.5)
    pr = m.p
    coeff = 4 * pr.faraday * pr.C_ref * (pr.V_op - pr.U0_icept) / float(m.rhocp[0, 0])
    s = m.initial_state()
    f0 = m.fields(s)
    inv0 = float(f0["theta"][0, 0] + coeff * f0["c"][0, 0])
    for _ in range(20):
        s = m.step(s)
    f1 = m.fields(s)
    inv1 = float(f1["theta"][0, 0] + coeff * f1["c"][0, 0])
    assert float(f1["c"][0, 0]) < 0.999 and float(f1["theta"][0, 0]) > 1e-3
    assert abs(inv1 - inv0) < 1e-12 * abs(inv0)


def test_tafel_kinetics_special_cases():
    m = _box(4, 1, layers=(0, 0, 1))
    pr = m.p
    one = torch.ones(1, dtype=DT)
    rc = m.rhocp[0, :1]
    # At T = 353.15 K and eta = 0 the rate constant is the printed
    # reference a j0 (Eqs. 13, 14, 17).
    T = pr.T_arrh
    pr.V_op = pr.U0_slope * T + pr.U0_icept
    *_, k = m.reaction((T - pr.T_in) * one, one, rc)
    assert abs(float(k) / GOLD["nomenclature"]["aj0_ref_A_per_cm3"] - 1) < 1e-14
    # Tafel slope: one decade of current per 2.3026 R T / (alpha_c F) of
    # overpotential (70.07 mV at 353.15 K).
    slope = math.log(10) * pr.R_gas * T / (pr.alpha_c * pr.faraday)
    assert abs(slope - 0.07007) < 1e-5
    pr.V_op = 0.6
    *_, k1 = m.reaction((T - pr.T_in) * one, one, rc)
    pr.V_op = 0.6 - slope
    *_, k2 = m.reaction((T - pr.T_in) * one, one, rc)
    assert abs(float(k2 / k1) - 10.0) < 1e-11
    # Arrhenius at zero overpotential (Eq. 17): activation energy
    # 16456 R = 136.8 kJ/mol; the rate at 333.15 K is exp(-16456 (1/333.15 -
    # 1/353.15)) of the reference.
    T2 = 333.15
    pr.V_op = pr.U0_slope * T2 + pr.U0_icept
    *_, k3 = m.reaction((T2 - pr.T_in) * one, one, rc)
    assert abs(float(k3) / pr.aj0_ref - math.exp(-16456 * (1 / T2 - 1 / 353.15))) < 1e-15
    # First order in oxygen (Eq. 13): j_eff and s_c scale with c.
    pr.V_op = 0.6
    sc1, _, j1, _, _ = m.reaction(0 * one, one, rc)
    sc2, _, j2, _, _ = m.reaction(0 * one, 0.25 * one, rc)
    assert abs(float(sc2 / sc1) - 0.25) < 1e-15 and abs(float(j2 / j1) - 0.25) < 1e-15
    # Exact-in-time sink: never consumes more than is there, even for a very
    # fast reaction; for a slow one it tends to k c dt / (4 F C_ref).
    pr.V_op = 0.05
    sc, *_ = m.reaction(0 * one, one, rc)
    assert 0.0 < float(sc) <= 1.0
    pr.V_op = 0.85
    sc, _, j, _, k = m.reaction(0 * one, one, rc)
    lin = float(k) * m.dt / (4 * pr.faraday * pr.C_ref)
    assert abs(float(sc) / lin - 1) < 1e-6
    assert abs(float(j) + float(k)) < 1e-6 * float(k)   # j_eff -> -k c


def test_printed_constants_are_the_defaults():
    pr = L.Params()
    nom, eq = GOLD["nomenclature"], GOLD["equations"]
    assert pr.aj0_ref == nom["aj0_ref_A_per_cm3"] and pr.C_ref == nom["C_ref_mol_per_cm3"]
    assert pr.alpha_c == nom["alpha_c"] and pr.faraday == nom["F_C_per_mol"]
    assert pr.R_gas == nom["R_J_per_mol_K"] and pr.D_O2 == nom["D_O2_cm2_per_s"]
    assert pr.k_f == nom["k_f_W_per_m_K"] and pr.k_s == nom["k_s_W_per_m_K"]
    assert pr.U0_slope == eq["U0_slope_V_per_K"] and pr.U0_icept == eq["U0_intercept_V"]
    assert pr.E_over_R == eq["arrhenius_E_over_R_K"] and pr.T_arrh == eq["arrhenius_T_K"]
    m = _box(4, 2, layers=(0, 2, 0), phi_gdl=0.5)
    assert abs(float(m.F_phi[0, 0]) - eq["F_phi_coeff"] * 0.5 ** -1.5) < 1e-15


def test_eq7_constants_are_ergun_constants():
    # Eq. 7's 0.143 and 0.0067 are Ergun's 1.75/sqrt(150) and 1/150 to the
    # printed precision; the oracle's Kozeny-Carman permeability matches
    # Ergun's phi^3 d^2 / (150 (1 - phi)^2) to that precision.
    assert abs(1.75 / math.sqrt(150) - 0.143) < 5e-4
    g = L.Geometry(3, 2, 0, 2, 0, periodic_x=True, periodic_y=True)
    for phi in (0.4, 0.6, 0.8):
        m = L.Model(g, L.Params(phi_gdl=phi, dp_lat=7.0, dx_cm=1e-3))
        k_ergun = phi ** 3 * 49.0 / (150 * (1 - phi) ** 2)
        assert abs(1.0 / float(m.inv_k[0, 0]) / k_ergun - 1) < 6e-3  # 0.0067 vs 1/150
        assert abs(float(m.F_phi[0, 0]) * phi ** 1.5 - 1.75 / math.sqrt(150)) < 5e-4


def test_bruggeman_matches_figure5_caption():
    # Fig. 5 caption: phi = 0.4 gives D_O2,eff = 1.32e-2 cm^2/s (Eq. 18).
    cap = GOLD["fig5_caption"]
    m = _box(4, 2, layers=(0, 2, 0), phi_gdl=cap["phi"])
    d_phys = float(m.d_eff[0, 0]) / m.p.D_f_lat * m.p.D_O2
    assert round(d_phys, 4) == cap["D_O2_eff_cm2_per_s"]


def test_darcy_number_uses_gdl_thickness_table2():
    # Table 2: K = Da h^2 with h the GDL thickness; the oracle's default
    # 254 um GDL reproduces every printed permeability at printed precision,
    # whatever the number of GDL rows.
    for row in GOLD["table2_darcy"]["rows"]:
        for n_gdl in (18, 40):
            g = L.Geometry(3, n_gdl, 0, n_gdl, 0, periodic_x=True)
            m = L.Model(g, L.Params(Da_gdl=row["Da"]))
            k_cm2 = m.dx ** 2 / float(m.inv_k[0, 0])
            assert abs(k_cm2 / row["K_cm2"] - 1) < 0.01, (row, k_cm2)


def test_reynolds_number_definition_table1():
    # Table 1: Re = U_avg h / nu with U_avg = flow / cross-section: all rows
    # share the same h / nu and cross-section; the oracle's inlet uses
    # U_avg = Re nu / H_channel, so Re / U_avg is the same h / nu.
    rows = GOLD["table1_reynolds"]["rows"]
    h_over_nu = [r["Re"] / r["U_avg_cm_per_s"] for r in rows]
    area = [r["flow_cm3_per_s"] / r["U_avg_cm_per_s"] for r in rows]
    assert max(h_over_nu) / min(h_over_nu) - 1 < 2e-3
    assert max(area) / min(area) - 1 < 3e-3
    g = L.Geometry(5, 10, 10, 0, 0)
    for r in rows:
        m = L.Model(g, L.Params(Re=r["Re"], dx_cm=1e-3))
        assert abs(m.u_avg * 10 / m.nu - r["Re"]) < 1e-12


def test_effective_thermal_diffusivity_limits():
    # Eq. 19: phi = 1 gives the gas value k_f / (rho c_p)_f; the mixture
    # rule is bounded by the pure-phase diffusivities.
    g = L.Geometry(3, 2, 1, 1, 0, periodic_x=True)
    m = L.Model(g, L.Params(phi_gdl=0.6, dx_cm=1e-3))
    pr = m.p
    scale = m.dt / m.dx ** 2
    a_gas = pr.k_f / 100 / pr.rhocp_f * scale
    a_sol = pr.k_s / 100 / pr.rhocp_s * scale
    assert abs(float(m.alpha[0, 0]) / a_gas - 1) < 1e-15
    a_mix = float(m.alpha[1, 0])
    assert min(a_gas, a_sol) < a_mix < max(a_gas, a_sol)
    assert abs(float(m.rhocp[1, 0]) - (0.6 * pr.rhocp_f + 0.4 * pr.rhocp_s)) < 1e-15


def _tafel_kappa(m):
    """Per-step first-order sink rate of Eqs. 13-14 and 17 at the inlet
    temperature (theta = 0) and c = 1."""
    pr = m.p
    T = pr.T_in
    eta = pr.V_op - (pr.U0_slope * T + pr.U0_icept)
    aj0_T = pr.aj0_ref * math.exp(-pr.E_over_R * (1 / T - 1 / pr.T_arrh))
    return aj0_T * math.exp(-pr.alpha_c * pr.faraday * eta / (pr.R_gas * T)) * m.dt / (4 * pr.faraday * pr.C_ref)


def _diffusion_reaction_rates(nx, aj0, eps=1e-3):
    """One CL row, periodic, isothermal (V = U0 intercept: no reaction heat
    by Eqs. 15-16), O2 = 1 + eps sin(kx).  The first-order sink is linear
    and uniform, so c = e^{-kappa t} (1 + eps e^{-D k^2 t} sin kx): the mean
    decays at kappa, the ratio of the sine amplitude to the mean at D k^2.
    Returns kappa and (measured / closed-form - 1) for both rates."""
    m = L.Model(L.Geometry(nx, 1, 0, 0, 1, periodic_x=True, periodic_y=True),
                L.Params(V_op=0.2329, aj0_ref=aj0, dx_cm=1e-3, phi_gdl=0.5))
    kappa = _tafel_kappa(m)
    D = 0.5 ** 1.5 * m.p.D_f_lat  # Eq. 18
    k = 2 * math.pi / nx
    x = torch.arange(nx, dtype=DT).view(1, nx)
    z = torch.zeros(1, nx, dtype=DT)
    s = m.equilibrium_state(z, z, z, z, 1.0 + eps * torch.sin(k * x))

    def modes(st):
        c = m.fields(st)["c"][0]
        return float(c.mean()), float((c * torch.sin(k * x[0])).sum() * 2 / nx)

    s = m.run(s, 50)  # start-up layer of the equilibrium initial state
    m0, a0 = modes(s)
    n = int(0.5 / (D * k * k))
    s = m.run(s, n)
    m1, a1 = modes(s)
    assert float(m.fields(s)["theta"].abs().max()) < 1e-14
    return kappa, (math.log(m0 / m1) / n) / kappa - 1, (math.log((a0 / m0) / (a1 / m1)) / n) / (D * k * k) - 1


def test_diffusion_reaction_closed_form():
    """The sink is exact in time (mean decay at kappa to round-off); without
    it the lattice diffusion rate converges to D k^2 at fourth order; the
    sink, injected with the rest weights, shifts the diffusion rate by a
    relative error of order kappa (a first-order splitting error: halving
    kappa halves it)."""
    _, _, d16 = _diffusion_reaction_rates(16, 1e-20)
    _, _, d32 = _diffusion_reaction_rates(32, 1e-20)
    assert 12 < d16 / d32 < 20 and abs(d32) < 1e-5
    ka, ra, da = _diffusion_reaction_rates(32, 1e-9)
    kb, rb, db = _diffusion_reaction_rates(32, 0.5e-9)
    print(f"kappa {ka:.2e}: sink err {ra:.1e}, diffusion err {da:.2e}; kappa {kb:.2e}: {rb:.1e}, {db:.2e}")
    assert abs(ra) < 1e-10 and abs(rb) < 1e-10 and ka > 1e-4
    assert 1.8 < (da - d32) / (db - d32) < 2.2
    assert abs(da - d32) < ka


def _inlet_decay_error(mh, D=0.125, span=12.0):
    """Steady O2 profile of a sink-filled 1D channel fed at the inlet:
    D c'' = kappa c with c(0) = 1 (the inlet's non-equilibrium
    extrapolation) and no flow, on a lattice long enough (span decay
    lengths) for the outlet to be invisible, so that c = exp(-m x) with
    m = sqrt(kappa / D).  One row, periodic in y; every node reacts
    (a test-only reaction mask).  V at the intercept of U0 (no heat), the
    gas heat capacity raised so that the thermal lattice stays stable at
    this diffusivity.  Returns the largest deviation from exp(-m x)."""
    nx = int(math.ceil(span / mh)) + 2
    g = L.Geometry(nx, 1, 1, 0, 0, periodic_y=True)
    mk = lambda aj0: L.Params(V_op=0.2329, aj0_ref=aj0, dx_cm=1e-3, D_f_lat=D, Re=0.0, rhocp_f=0.01)
    kappa = D * mh * mh
    m = L.Model(g, mk(kappa / _tafel_kappa(L.Model(g, mk(1.0)))))
    assert abs(_tafel_kappa(m) / kappa - 1) < 1e-12
    m.is_cl = torch.ones_like(m.is_cl)
    x = torch.arange(nx, dtype=DT)
    exact = torch.exp(-mh * x)
    z = torch.zeros(1, nx, dtype=DT)
    s = m.equilibrium_state(z, z, z, z, exact.view(1, nx).clone())
    chunk, prev = int(2 / kappa), None
    for _ in range(40):
        s = m.run(s, chunk)
        c = m.fields(s)["c"][0]
        if prev is not None and float((c - prev).abs().max()) < 1e-12:
            break
        prev = c
    else:
        raise AssertionError("no steady state")
    f = m.fields(s)
    assert float(f["theta"].abs().max()) < 1e-12 and float(f["ux"].abs().max()) == 0.0
    assert abs(float(c[0]) - 1.0) < 1e-15
    return float((c - exact).abs().max())


def test_steady_diffusion_reaction_profile_from_a_dirichlet_inlet():
    """The decay length sqrt(D / kappa) of the steady profile, with the
    error converging at second order as the decay length grows from 4 to
    8 lattice spacings (measured: 8.7e-3, then 2.7e-3, ratio 3.3 and
    rising toward 4)."""
    e4, e8 = _inlet_decay_error(0.25), _inlet_decay_error(0.125)
    print(f"steady exp(-m x) profile: max err {e4:.2e} (m h = 1/4), {e8:.2e} (m h = 1/8)")
    assert e8 < 3e-3 and e4 / e8 > 3.0
