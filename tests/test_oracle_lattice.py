"""Pins of the oracle's lattice algebra (Section 2, Eqs. 2-10) against
closed forms and textbook special cases.  CPU only."""
import math

import pytest
import torch

from oracle import lbm2d as L

DT = torch.float64


def test_velocity_sets_match_transformation_rows():
    # Eq. 2 vs Eq. 3: the j_x and j_y rows of M are e_x and e_y of the
    # velocity set; Eq. 9 vs Eq. 10: rows 1 and 2 of N likewise.
    ex = torch.tensor([e[0] for e in L.E9], dtype=DT)
    ey = torch.tensor([e[1] for e in L.E9], dtype=DT)
    assert torch.equal(L.M9[3], ex) and torch.equal(L.M9[5], ey)
    assert torch.equal(L.N5[1], ex[:5]) and torch.equal(L.N5[2], ey[:5])
    assert L.E9 == [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
    assert L.OPP9 == [0, 3, 4, 1, 2, 7, 8, 5, 6] and L.OPP5 == [0, 3, 4, 1, 2]


def test_moment_matrices_orthogonal_and_inverse():
    mmt = L.M9 @ L.M9.T
    assert torch.equal(mmt, torch.diag(torch.tensor([9., 36, 36, 6, 12, 6, 12, 4, 4], dtype=DT)))
    nnt = L.N5 @ L.N5.T
    assert torch.equal(nnt, torch.diag(torch.tensor([5., 2, 2, 20, 4], dtype=DT)))
    assert torch.allclose(L.M9_INV @ L.M9, torch.eye(9, dtype=DT), atol=1e-15)
    assert torch.allclose(L.N5_INV @ L.N5, torch.eye(5, dtype=DT), atol=1e-15)


def test_relaxation_magic_combination():
    # s_q of Section 2.1 is the rate that makes (1/s_nu - 1/2)(1/s_q - 1/2) = 3/16.
    for tau in (0.55, 0.65, 0.8, 1.0, 1.7):
        S = L.relaxation_d2q9(tau)
        lam = (1 / S[7] - 0.5) * (1 / S[4] - 0.5)
        assert abs(float(lam) - 3 / 16) < 1e-15
        assert float(S[3]) == 0.0 and float(S[5]) == 0.0  # momentum is not relaxed
    # Eq. 10: the D2Q5 flux and energy rates give Lambda = 1/6.
    lam5 = (1 / L.Q5[1] - 0.5) * (1 / L.Q5[3] - 0.5)
    assert abs(float(lam5) - 1 / 6) < 1e-15


def _velocity_space_feq(p, ux, uy, phi):
    """Textbook incompressible porous equilibrium in velocity space
    (Guo-Zhao generalized model with the pressure weights lambda_i):
    f_i = lambda_i phi p + w_i rho0 [3 e.u + 4.5 (e.u)^2/phi - 1.5 u^2/phi],
    lambda = (-5/3, 1/3 x4, 1/12 x4), plus rho0 on the rest population."""
    w = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4
    lam = [-5 / 3] + [1 / 3] * 4 + [1 / 12] * 4
    out = []
    for i, (ex, ey) in enumerate(L.E9):
        eu = ex * ux + ey * uy
        s = w[i] * (3 * eu + 4.5 * eu * eu / phi - 1.5 * (ux * ux + uy * uy) / phi)
        out.append(lam[i] * phi * p + s + (1.0 if i == 0 else 0.0))
    return torch.stack(out)


def _model(nx=4, ny=3, **kw):
    g = L.Geometry(nx, ny, ny, 0, 0, periodic_x=True, periodic_y=True)
    return L.Model(g, L.Params(reaction=False, dx_cm=1e-3, **kw))


def test_equilibrium_moments_match_velocity_space_form():
    torch.manual_seed(1)
    p = torch.rand(7, dtype=DT) * 0.02 - 0.01
    ux = torch.rand(7, dtype=DT) * 0.1 - 0.05
    uy = torch.rand(7, dtype=DT) * 0.1 - 0.05
    phi = torch.rand(7, dtype=DT) * 0.6 + 0.4
    m = _model()
    fv = _velocity_space_feq(p, ux, uy, phi)
    assert torch.allclose(L.M9 @ fv, m.meq(p, ux, uy, phi), atol=1e-15)
    assert torch.allclose(m.feq(p, ux, uy, phi), fv, atol=1e-15)


def test_pressure_recovery_inverts_equilibrium():
    # Section 2.1 pressure relation applied to f_eq returns p (and u).
    torch.manual_seed(2)
    p = torch.rand(5, 1, dtype=DT) * 0.02 - 0.01
    ux = torch.rand(5, 1, dtype=DT) * 0.1 - 0.05
    uy = torch.rand(5, 1, dtype=DT) * 0.1 - 0.05
    m = _model()
    phi = torch.ones(5, 1, dtype=DT)
    f = m.feq(p, ux, uy, phi)
    z = torch.zeros_like(phi)
    u_x, u_y, pr, _, _ = m.flow_macros(f, phi, 0.5 + z, z, z, z, 0.143 + z)
    assert torch.allclose(pr, p, atol=1e-16) and torch.allclose(u_x, ux, atol=1e-16)
    assert torch.allclose(u_y, uy, atol=1e-16)


def test_forcing_equals_guo_forcing_in_moment_space():
    # The textbook Guo forcing for the porous model,
    # F_i = w_i rho0 [3 e.F + 9 (e.u)(e.F)/phi - 3 u.F/phi],
    # mapped by M, equals the oracle's moment-space forcing (Eq. 6 read with
    # the sign and index of G7, G8 fixed).
    torch.manual_seed(3)
    ux, uy, Fx, Fy = (torch.rand(6, dtype=DT) * 0.1 - 0.05 for _ in range(4))
    phi = torch.rand(6, dtype=DT) * 0.6 + 0.4
    w = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4
    Fi = torch.stack([w[i] * (3 * (ex * Fx + ey * Fy) + 9 * (ex * ux + ey * uy) * (ex * Fx + ey * Fy) / phi
                              - 3 * (ux * Fx + uy * Fy) / phi) for i, (ex, ey) in enumerate(L.E9)])
    G = L.Model.forcing_moments(ux, uy, Fx, Fy, phi)
    assert torch.allclose(L.M9 @ Fi, G, atol=1e-16)
    # G1..G6 are exactly as printed in Eq. 6.
    uF = ux * Fx + uy * Fy
    assert torch.allclose(G[1], 6 * uF / phi) and torch.allclose(G[2], -6 * uF / phi)
    assert torch.equal(G[3], Fx) and torch.equal(G[4], -Fx)
    assert torch.equal(G[5], Fy) and torch.equal(G[6], -Fy)


def test_velocity_recovery_solves_half_force_relation():
    # Eq. 8 closes u = v + (dt/2) F(u) with F of Eq. 7; check that implicit
    # relation on random velocities and porous media, including v = 0.
    torch.manual_seed(4)
    n = 64
    phi = torch.rand(n, dtype=DT) * 0.6 + 0.4
    inv_k = torch.rand(n, dtype=DT) * 5.0
    f = torch.rand(9, n, dtype=DT) * 0.02
    f[:, 0] = 0.0  # v = 0 exactly at one point
    m = _model(tau_f=0.7)
    sq = torch.sqrt(inv_k)
    Fphi = 0.143 * phi ** -1.5
    l0 = 0.5 + phi * m.nu * inv_k / 4
    l1 = phi * Fphi * sq / 2
    ux, uy, _, Fx, Fy = m.flow_macros(f, phi, l0, l1, inv_k, sq, Fphi)
    vx = sum(L.E9[q][0] * f[q] for q in range(9))
    vy = sum(L.E9[q][1] * f[q] for q in range(9))
    assert torch.allclose(ux, vx + Fx / 2, atol=1e-17, rtol=1e-14)
    assert torch.allclose(uy, vy + Fy / 2, atol=1e-17, rtol=1e-14)
    # Drag of Eq. 7 opposes the velocity; clear fluid (K^-1 = 0) has u = v.
    assert bool(((ux * Fx + uy * Fy) <= 0).all())
    z = torch.zeros(n, dtype=DT)
    ux0, uy0, _, Fx0, _ = m.flow_macros(f, torch.ones(n, dtype=DT), 0.5 + z, z, z, z, 0.143 + z)
    assert torch.equal(ux0, vx) and torch.equal(Fx0, z)


def test_scalar_equilibrium_moments_and_diffusivity_relation():
    # Eq. 10: g_eq = N^-1 (X, u_x X, u_y X, b X, 0); its zeroth moment is X,
    # its flux is u X, and its second moment sum e_x^2 g = (4 + b) X / 10.
    m = _model()
    X = torch.tensor([0.3, 1.0, 2.5], dtype=DT)
    ux = torch.tensor([0.01, -0.02, 0.0], dtype=DT)
    uy = torch.tensor([0.0, 0.03, -0.01], dtype=DT)
    b = torch.tensor([-3.5, -1.0, 0.9], dtype=DT)
    g = m.geq(X, ux, uy, b)
    assert torch.allclose(g.sum(0), X, atol=1e-16)
    assert torch.allclose(g[1] - g[3], ux * X, atol=1e-16)
    assert torch.allclose(g[1] + g[3], (4 + b) * X / 10, atol=1e-16)
    # b = 20 sqrt(3) alpha - 4 <=> alpha = (4 + b)/(20 sqrt(3)); with the flux
    # relaxation 6/(3+sqrt(3)) of Eq. 10, (1/q - 1/2)(4 + b)/10 = alpha.
    q1 = float(L.Q5[1])
    for alpha in (0.002, 0.0125, 0.06, 0.1443):
        b = 20 * math.sqrt(3) * alpha - 4
        assert abs((1 / q1 - 0.5) * (4 + b) / 10 - alpha) < 1e-16


def test_streaming_moves_each_population_along_its_velocity():
    # A single population placed at one node appears one link downstream
    # after streaming (periodic box), and bounces back into the opposite
    # population at the same node when the link crosses a wall.
    g = L.Geometry(6, 5, 5, 0, 0, periodic_x=True, periodic_y=False)
    m = L.Model(g, L.Params(reaction=False, dx_cm=1e-3))
    for q, (ex, ey) in enumerate(L.E9):
        post = torch.zeros(19, 5, 6, dtype=DT)
        post[q, 2, 3] = 1.0
        pre = m.stream(post)
        assert float(pre[q, 2 + ey, (3 + ex) % 6]) == 1.0 and float(pre.sum()) == 1.0
        wall = torch.zeros(19, 5, 6, dtype=DT)
        wall[q, 4, 3] = 1.0  # top row: links with ey = +1 leave the lattice
        pre = m.stream(wall)
        if ey == 1:
            assert float(pre[L.OPP9[q], 4, 3]) == 1.0
        else:
            assert float(pre[q, 4 + ey, (3 + ex) % 6]) == 1.0
    for q, (ex, ey) in enumerate(L.E5):
        post = torch.zeros(19, 5, 6, dtype=DT)
        post[14 + q, 0, 0] = 1.0  # bottom row, O2 lattice
        pre = m.stream(post)
        if ey == -1:
            assert float(pre[14 + L.OPP5[q], 0, 0]) == 1.0
        else:
            assert float(pre[14 + q, 0 + ey, (0 + ex) % 6]) == 1.0


def test_density_moment_relaxation_is_linearly_stable():
    # The reading of the density-moment rate: with it, a rest state is
    # linearly stable for every wave vector (von Neumann); with the printed
    # s_0 = 0 it is not.
    import numpy as np

    def worst(s0, tau=0.65):
        m = _model(nx=3, ny=1, tau_f=tau)
        m.S9 = m.S9.clone()
        m.S9[0] = s0
        base = m.initial_state()
        f0 = base[:9, 0, 0].clone()
        J = torch.zeros(9, 9, dtype=DT)
        for j in range(9):
            cols = []
            for h in (1e-7, -1e-7):
                st = base.clone()
                st[j, 0, :] += h
                cols.append(m.collide(st)[:9, 0, 0])
            J[:, j] = (cols[0] - cols[1]) / 2e-7
        w = 0.0
        for kx in np.linspace(-math.pi, math.pi, 17):
            for ky in np.linspace(-math.pi, math.pi, 17):
                Sh = np.diag([np.exp(-1j * (kx * ex + ky * ey)) for ex, ey in L.E9])
                w = max(w, float(np.abs(np.linalg.eigvals(Sh @ J.numpy())).max()))
        return w

    assert worst(1 / 0.65) < 1 + 1e-8
    assert worst(0.0) > 1.2
