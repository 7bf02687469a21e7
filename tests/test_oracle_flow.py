"""Pins of the oracle's flow lattice (Section 2.1) against closed-form flows
and exact invariants.  CPU only."""
import math

import torch

from oracle import lbm2d as L

DT = torch.float64


def _channel(nx, ny, **kw):
    g = L.Geometry(nx, ny, ny, 0, 0, periodic_x=True, periodic_y=kw.pop("periodic_y", False))
    return L.Model(g, L.Params(reaction=False, dx_cm=1e-3, **kw))


def test_poiseuille_exact_with_halfway_bounce_back():
    # Body-force-driven clear channel between half-way walls at y = -1/2 and
    # y = H - 1/2: the steady profile (a / 2 nu)(y + 1/2)(H - 1/2 - y) is
    # reproduced exactly by the MRT rates of Section 2.1 (Lambda = 3/16) up to
    # the model's O(u F) pressure source.  u is odd in a, so that remainder
    # is O(a^3): the error relative to u_max falls as a^2 and vanishes as
    # a -> 0, i.e. the O(a) solution is exact.
    H = 8
    errs = []
    for a in (1e-6, 1e-7):
        m = _channel(3, H, tau_f=0.8, body_force=(a, 0.0))
        s = m.run(m.initial_state(), 2500)
        y = torch.arange(H, dtype=DT)
        exact = a / (2 * m.nu) * (y + 0.5) * (H - 0.5 - y)
        u = m.fields(s)["ux"][:, 0]
        errs.append(float((u - exact).abs().max() / exact.max()))
    assert errs[1] < 1e-11
    assert 50.0 < errs[0] / errs[1] < 200.0


def test_darcy_forchheimer_slab_steady_state():
    # Uniform porous medium, fully periodic, body force a: the state stays
    # uniform and relaxes to (nu/K) u + (F_phi / sqrt K) u^2 = a (Eq. 7 with
    # F = 0); the quadratic gives u in closed form.
    g = L.Geometry(3, 3, 0, 3, 0, periodic_x=True, periodic_y=True)
    phi, Da, a = 0.6, 0.01, 2e-4
    m = L.Model(g, L.Params(reaction=False, dx_cm=1e-3, phi_gdl=phi, Da_gdl=Da, body_force=(a, 0.0)))
    K = Da * 3 ** 2
    Fphi = 0.143 * phi ** -1.5
    A, B = Fphi / math.sqrt(K), m.nu / K
    u_exact = (-B + math.sqrt(B * B + 4 * A * a)) / (2 * A)
    s = m.run(m.initial_state(), 600)
    u = m.fields(s)["ux"]
    assert float((u - u_exact).abs().max()) / u_exact < 1e-12
    # The transient is the scalar recursion v_{n+1} = v_n + F(u(v_n)) of
    # Eqs. 7-8 (momentum is not relaxed): check ten steps from rest.
    s = m.initial_state()
    v = 0.0
    l0 = 0.5 + phi * m.nu / K / 4
    l1 = phi * Fphi / math.sqrt(K) / 2
    for _ in range(10):
        V = v + phi * a / 2
        un = V / (l0 + math.sqrt(l0 * l0 + l1 * abs(V)))
        Fn = phi * a - phi * m.nu / K * un - phi * Fphi / math.sqrt(K) * abs(un) * un
        v = v + Fn
        s = m.step(s)
    vx = sum(L.E9[q][0] * s[q] for q in range(9))  # post-collision momentum
    assert abs(float(vx[1, 1]) - v) < 1e-17


def _brinkman_error(H):
    # Uniform porous channel, walls at -1/2 and H - 1/2, weak forcing
    # (Forchheimer term negligible): Brinkman solution
    # u = (a K / nu)[1 - cosh(r (y - c)) / cosh(r H / 2)], r = sqrt(phi / K).
    phi = 0.6
    rH = 4.0  # keep r H fixed while refining
    K = phi * (H / rH) ** 2
    a = 1e-8 * (8.0 / H) ** 2
    g = L.Geometry(3, H, 0, H, 0, periodic_x=True)
    m = L.Model(g, L.Params(reaction=False, dx_cm=1e-3, tau_f=0.8, phi_gdl=phi,
                            Da_gdl=K / H ** 2, body_force=(a, 0.0)))
    s = m.run(m.initial_state(), 60 * H)
    u = m.fields(s)["ux"][:, 0]
    y = torch.arange(H, dtype=DT)
    r = math.sqrt(phi / K)
    c = (H - 1) / 2
    exact = a * K / m.nu * (1 - torch.cosh(r * (y - c)) / math.cosh(r * H / 2))
    return float((u - exact).abs().max() / exact.max())


def test_brinkman_channel_second_order():
    e1, e2 = _brinkman_error(8), _brinkman_error(16)
    assert e2 < 1e-2
    order = math.log2(e1 / e2)
    assert 1.6 < order < 2.6, (e1, e2, order)


def test_moving_population_sum_conserved_in_clear_fluid():
    # With the density moment relaxed like e and zeta, collision in clear
    # fluid with no force conserves sum_{i>=1} f_i exactly at every node, and
    # streaming with bounce-back conserves it globally: the model's discrete
    # mass invariant.  Here a closed box with walls, an arbitrary state.
    g = L.Geometry(7, 6, 6, 0, 0, periodic_x=True)
    m = L.Model(g, L.Params(reaction=False, dx_cm=1e-3))
    torch.manual_seed(5)
    s = m.initial_state()
    s[1:9] += torch.rand(8, 6, 7, dtype=DT) * 1e-3
    x0 = float(m.stream(s)[1:9].sum())
    for _ in range(50):
        s = m.step(s)
    x1 = float(m.stream(s)[1:9].sum())
    assert abs(x1 - x0) / abs(x0) < 1e-13
    # Per node: collision alone keeps sum_{i>=1} f_i.
    pre = m.stream(s)
    post = m.collide(pre)
    assert torch.allclose(post[1:9].sum(0), pre[1:9].sum(0), atol=2e-15, rtol=0)


def test_porous_forcing_exchanges_pressure_with_drag_work():
    # In porous cells the moving-population sum changes by the forcing's
    # pressure source, (1 - s_e/2)(G1 - G2)/9 = (4/3)(1 - s/2) u.F / phi per
    # node, with s = 1/tau; nothing else changes it.
    g = L.Geometry(5, 4, 0, 4, 0, periodic_x=True, periodic_y=True)
    m = L.Model(g, L.Params(reaction=False, dx_cm=1e-3, phi_gdl=0.5, Da_gdl=0.05))
    torch.manual_seed(6)
    pre = m.initial_state()
    pre[1:9] += torch.rand(8, 4, 5, dtype=DT) * 1e-2
    post = m.collide(pre)
    ux, uy, _, Fx, Fy = m.flow_macros(pre[0:9], m.phi, m.l0, m.l1, m.inv_k, m.sqrt_inv_k, m.F_phi)
    s = 1 / m.p.tau_f
    expect = 4 / 3 * (1 - s / 2) * (ux * Fx + uy * Fy) / m.phi
    assert torch.allclose(post[1:9].sum(0) - pre[1:9].sum(0), expect, atol=2e-16, rtol=1e-9)
