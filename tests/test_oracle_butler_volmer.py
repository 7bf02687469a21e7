"""Pins of the oracle's Butler-Volmer option (Eq. 13 with an anodic branch)
against the textbook small-overpotential law, the printed Tafel form it
must reduce to at large overpotential, and the closed-form solution of the
CL O2 balance in a uniform box.  CPU only."""
import math

import torch

from oracle import lbm2d as L

DT = torch.float64


def _box(**kw):
    g = L.Geometry(4, 3, 0, 0, 3, periodic_x=True, periodic_y=True)
    kw.setdefault("dx_cm", 1e-3)
    return L.Model(g, L.Params(butler_volmer=True, **kw))


def test_small_overpotential_is_the_linear_charge_transfer_law():
    # For |eta| << R T / F at C = C_ref, the Butler-Volmer current is
    # a j0 (alpha_a + alpha_c) F eta / (R T) (charge-transfer resistance).
    for alpha_a in (1.0, 0.5):
        m = _box(alpha_a=alpha_a)
        pr = m.p
        one = torch.ones(1, dtype=DT)
        rc = m.rhocp[0, :1]
        T = pr.T_arrh
        for d in (1e-6, -1e-6):
            pr.V_op = pr.U0_slope * T + pr.U0_icept + d
            _, _, j, _, _ = m.reaction((T - pr.T_in) * one, one, rc)
            lin = pr.aj0_ref * (alpha_a + pr.alpha_c) * pr.faraday * d / (pr.R_gas * T)
            assert abs(float(j) / lin - 1) < 1e-4, (alpha_a, d)


def test_large_overpotential_reduces_to_the_printed_tafel_form():
    for V in (0.3, 0.6):
        bv, tafel = _box(V_op=V), _box(V_op=V)
        tafel.p.butler_volmer = False
        one = torch.ones(1, dtype=DT)
        rc = bv.rhocp[0, :1]
        for theta in (0.0, 5.0):
            a = bv.reaction(theta * one, 0.7 * one, rc)
            b = tafel.reaction(theta * one, 0.7 * one, rc)
            for x, y in zip(a, b):
                assert abs(float(x) / float(y) - 1) < 1e-9


def test_uniform_box_relaxes_to_the_equilibrium_concentration():
    # Uniform closed CL box with frozen temperature (huge heat capacities):
    # 4 F C_ref dc/dt = -(k c - k_a) has the solution
    # c(t) = c_eq + (c0 - c_eq) exp(-k t / (4 F C_ref)), c_eq = k_a / k, with
    # k = a j0 exp(-alpha_c F eta / RT), k_a = a j0 exp(alpha_a F eta / RT).
    # Slightly anodic (eta > 0): O2 is produced toward c_eq > 1.
    m = _box(rhocp_f=1e15, rhocp_s=1e15, aj0_ref=2e5, phi_gdl=0.5)
    pr = m.p
    T = pr.T_in
    eta = 0.01
    pr.V_op = pr.U0_slope * T + pr.U0_icept + eta
    f = pr.faraday / (pr.R_gas * T)
    aj0 = pr.aj0_ref * math.exp(-pr.E_over_R * (1 / T - 1 / pr.T_arrh))
    k, k_a = aj0 * math.exp(-pr.alpha_c * f * eta), aj0 * math.exp(pr.alpha_a * f * eta)
    tau = 4 * pr.faraday * pr.C_ref / k
    s = m.initial_state()
    for n in range(1, 41):
        s = m.step(s)
        if n % 10 == 0:
            c = m.fields(s)["c"]
            exact = k_a / k + (1.0 - k_a / k) * math.exp(-n * m.dt / tau)
            assert float((c - exact).abs().max()) < 1e-13, n
    assert float(m.fields(s)["c"].mean()) > 1.1  # well under way toward c_eq = 1.93
