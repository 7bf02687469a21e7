"""Pins of the 3D oracle (D3Q19 + 2 x D3Q7): the two-rate form it uses is
the paper's 2D MRT (checked on D2Q9 / D2Q5 against ``lbm2d``), its
equilibria have the textbook moments, and closed forms hold.  CPU only."""
import math

import torch

import workloads as W
from oracle import lbm2d as L
from oracle import lbm3d as L3

DT = torch.float64


def test_trt_form_equals_the_2d_mrt_collision():
    # The paper's D2Q9 MRT (with the s_0 reading) and D2Q5 MRT, written as
    # two-rate collisions on symmetric / antisymmetric parts in velocity
    # space, give the same post-collision populations as ``lbm2d``.
    g = L.Geometry(6, 5, 2, 2, 1, periodic_x=True)
    m = L.Model(g, L.Params(phi_gdl=0.55, Da_gdl=0.02, V_op=0.5, dx_cm=1e-3))
    pre = torch.from_numpy(W.random_populations(5, 6, 77))
    ref = m.collide(pre)
    f, gT, gC = pre[0:9], pre[9:14], pre[14:19]
    ux, uy, p, Fx, Fy = m.flow_macros(f, m.phi, m.l0, m.l1, m.inv_k, m.sqrt_inv_k, m.F_phi)
    feq = m.feq(p, ux, uy, m.phi)
    w = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4
    Fi = torch.stack([w[i] * (3 * (ex * Fx + ey * Fy) + 9 * (ex * ux + ey * uy) * (ex * Fx + ey * Fy) / m.phi
                              - 3 * (ux * Fx + uy * Fy) / m.phi) for i, (ex, ey) in enumerate(L.E9)])
    s_plus = 1 / m.p.tau_f
    s_minus = 8 * (2 - s_plus) / (8 - s_plus)
    f_trt = L3.collide_trt(f, feq, Fi, s_plus, s_minus, L.OPP9)
    assert float((f_trt - ref[0:9]).abs().max()) < 1e-15
    th, c = gT.sum(0), gC.sum(0)
    s_c, S_T, *_ = m.reaction(th, c, m.rhocp)
    z = torch.zeros_like(th)
    for g5, X, b, src, lo in ((gT, th, m.b_T, torch.where(m.is_cl, S_T, z), 9),
                              (gC, c, m.b_C, torch.where(m.is_cl, -s_c, z), 14)):
        geq = m.geq(X, ux, uy, b)
        post = L3.collide_trt(g5, geq, torch.zeros_like(g5), L3.S_EVEN_SCALAR, L3.S_ODD_SCALAR, L.OPP5)
        post = post + m.geq(src, z, z, b)
        assert float((post - ref[lo:lo + 5]).abs().max()) < 1e-15
    # and the D2Q5 rest weight (4 + b)/20 equals sqrt(3) alpha
    assert torch.allclose((4 + m.b_C) / 20, math.sqrt(3) * m.d_eff, atol=1e-16)


def _box3(nx=4, ny=3, nz=5, layers=(5, 0, 0), per=(True, True, True), **kw):
    g = L3.Geometry3D(nx, ny, nz, *layers, periodic_x=per[0], periodic_y=per[1], periodic_z=per[2])
    kw.setdefault("dx_cm", 1e-3)
    return L3.Model3D(g, L.Params(**kw))


def test_d3q19_equilibrium_and_forcing_moments():
    m = _box3()
    torch.manual_seed(8)
    n = 7
    p = torch.rand(n, dtype=DT) * 0.02
    u = [torch.rand(n, dtype=DT) * 0.1 - 0.05 for _ in range(3)]
    F = [torch.rand(n, dtype=DT) * 0.01 - 0.005 for _ in range(3)]
    phi = torch.rand(n, dtype=DT) * 0.6 + 0.4
    feq = m.feq(p, *u, phi)
    e = torch.tensor(L3.E19, dtype=DT)
    assert torch.allclose(feq.sum(0), torch.ones(n, dtype=DT), atol=1e-15)
    for a in range(3):
        assert torch.allclose((e[:, a:a + 1] * feq).sum(0), u[a], atol=1e-16)
        for b in range(3):
            pi = (e[:, a:a + 1] * e[:, b:b + 1] * feq).sum(0)
            assert torch.allclose(pi, phi * p * (a == b) + u[a] * u[b] / phi, atol=1e-16)
    # pressure recovery of the 3D equilibrium
    z = torch.zeros(n, dtype=DT)
    uu, pr, _ = m.flow_macros(feq, phi, 0.5 + z, z, z, z, 0.143 + z)
    assert torch.allclose(pr, p, atol=1e-16)
    Fi = m.forcing(*u, *F, phi)
    assert torch.allclose(Fi.sum(0), z, atol=1e-17)
    for a in range(3):
        assert torch.allclose((e[:, a:a + 1] * Fi).sum(0), F[a], atol=1e-17)
        for b in range(3):
            s = (e[:, a:a + 1] * e[:, b:b + 1] * Fi).sum(0)
            assert torch.allclose(s, (u[a] * F[b] + F[a] * u[b]) / phi, atol=1e-17)


def test_poiseuille_between_plates_3d():
    H, a = 8, 1e-7
    m = _box3(3, 3, H, layers=(H, 0, 0), per=(True, True, False), reaction=False, tau_f=1.0,
              body_force=(a, 0.0))
    s = m.run(m.initial_state(), 1500)
    u = m.fields(s)["ux"][:, 1, 1]
    z = torch.arange(H, dtype=DT)
    exact = a / (2 * m.nu) * (z + 0.5) * (H - 0.5 - z)
    assert float((u - exact).abs().max() / exact.max()) < 1e-11


def _decay3(n, D):
    m = _box3(n, 1, 1, layers=(1, 0, 0), reaction=False, D_f_lat=D)
    x = torch.arange(n, dtype=DT).view(1, 1, n)
    k = 2 * math.pi / n
    z = torch.zeros(1, 1, n, dtype=DT)
    s = m.equilibrium_state(z, (z, z, z), z, 1.0 + 1e-3 * torch.sin(k * x))

    def amp(st):
        c = m.fields(st)["c"][0, 0]
        return float(((c - 1.0) * torch.sin(k * x[0, 0])).sum() * 2 / n)

    s = m.run(s, 50)
    a0 = amp(s)
    s = m.run(s, 200)
    return -math.log(amp(s) / a0) / (200 * k * k)


def test_d3q7_diffusivity_from_rest_weight():
    D = 0.0125
    e32, e64 = abs(_decay3(32, D) / D - 1), abs(_decay3(64, D) / D - 1)
    assert e64 < 1e-6 and 10 < e32 / e64 < 22


def test_closed_box_budgets_3d():
    m = _box3(4, 3, 4, layers=(0, 0, 4), V_op=0.5, T_in=353.15)
    torch.manual_seed(9)
    s = m.initial_state()
    s[26:33] *= 1 + 0.1 * torch.rand(7, 4, 3, 4, dtype=DT)
    for _ in range(4):
        o0 = m.observables(s)
        s = m.step(s)
        o1 = m.observables(s)
        assert abs(float(o1["sum_c"] - (o0["sum_c"] - o0["consumed_c"]))) < 1e-13 * float(o0["sum_c"])
        assert abs(float(o1["sum_theta"] - (o0["sum_theta"] + o0["heat_added"]))) < 1e-13 * float(o1["sum_theta"])


def test_inlet_and_outlet_columns_3d():
    g = L3.Geometry3D(8, 5, 6, 3, 2, 1)
    m = L3.Model3D(g, L.Params(Re=2.0, c_in=0.9))
    torch.manual_seed(10)
    s = m.initial_state() + 0.002 * torch.rand(33, 6, 5, 8, dtype=DT)
    f = m.fields(s)
    assert torch.allclose(f["ux"][:3, :, 0], m.inlet_velocity(), atol=1e-16)
    assert float(f["uy"][:3, :, 0].abs().max()) < 1e-16 and float(f["uz"][:3, :, 0].abs().max()) < 1e-16
    assert float(f["theta"][:3, :, 0].abs().max()) < 1e-15
    assert torch.allclose(f["c"][:3, :, 0], torch.full((3, 5), 0.9, dtype=DT), atol=1e-15)
    assert float(f["p"][..., -1].abs().max()) < 1e-15
    # mean of the inlet profile over the continuous cross-section is U_avg
    H, ny = 3, 5
    mean_discrete = float(m.inlet_velocity().mean())
    assert abs(mean_discrete / (m.u_avg * (1 + 1 / (2 * H * H)) * (1 + 1 / (2 * ny * ny))) - 1) < 1e-14
