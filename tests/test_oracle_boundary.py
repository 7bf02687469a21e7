"""Pins of the oracle's inlet, outlet and wall treatment (Section 4
boundary conditions) and of the open-domain O2 / heat balance.  CPU only."""
import torch

import workloads as W
from oracle import lbm2d as L

DT = torch.float64


def _cathode(nx=12, ny=10, layers=(5, 4, 1), seed=11, **kw):
    g = L.Geometry(nx, ny, *layers)
    prm = L.Params(**kw)
    m = L.Model(g, prm)
    s = torch.from_numpy(W.random_populations(ny, nx, seed))
    return m, s


def test_inlet_profile_mean_is_discrete_parabola_mean():
    # Mean over the H channel rows of 6 U (y+1/2)(H-1/2-y)/H^2 is U (1 + 1/(2 H^2)).
    g = L.Geometry(5, 13, 7, 5, 1)
    m = L.Model(g, L.Params(Re=20.0))
    u = m.inlet_velocity()
    H = 7
    assert abs(float(u.mean()) / (m.u_avg * (1 + 1 / (2 * H * H))) - 1) < 1e-14
    assert abs(m.u_avg * H / m.nu - 20.0) < 1e-12


def test_inlet_node_takes_inlet_velocity_temperature_and_oxygen():
    # After the non-equilibrium extrapolation the inlet nodes carry exactly
    # the Dirichlet data: u = u_in(y) (clear channel, K^-1 = 0), v = 0,
    # theta = 0, c = c_in; and the pressure extrapolated from column 1.
    m, s = _cathode(c_in=0.8)
    pre = m.pre_collision(s)
    f = m.fields(s)
    H = m.g.ny_channel
    assert torch.allclose(f["ux"][:H, 0], m.inlet_velocity(), atol=1e-16)
    assert float(f["uy"][:H, 0].abs().max()) < 1e-16
    assert float(f["theta"][:H, 0].abs().max()) < 1e-15
    assert torch.allclose(f["c"][:H, 0], torch.full((H,), 0.8, dtype=DT), atol=1e-15)
    assert torch.allclose(f["p"][:H, 0], f["p"][:H, 1], atol=1e-15)
    # Non-equilibrium parts are copied from column 1.
    neq0 = pre[0:9, :H, 0] - m.feq(f["p"][:H, 0], f["ux"][:H, 0], f["uy"][:H, 0], m.phi[:H, 0])
    neq1 = pre[0:9, :H, 1] - m.feq(f["p"][:H, 1], f["ux"][:H, 1], f["uy"][:H, 1], m.phi[:H, 1])
    assert torch.allclose(neq0, neq1, atol=1e-15)


def test_outlet_node_zero_pressure_and_zero_gradient_scalars():
    m, s = _cathode()
    pre = m.pre_collision(s)
    f = m.fields(s)
    nx = m.g.nx
    # Same porosity and permeability in the last two columns (layered input):
    # p = 0 and u = u(nx-2) exactly; scalars copied.
    assert float(f["p"][:, nx - 1].abs().max()) < 1e-15
    assert torch.allclose(f["ux"][:, nx - 1], f["ux"][:, nx - 2], atol=1e-16)
    assert torch.equal(pre[9:19, :, nx - 1], pre[9:19, :, nx - 2])


def test_walls_are_insulated_and_impermeable():
    # Non-inlet rows of column 0 stream their x-entering populations from the
    # wall at x = -1/2 (bounce-back): after streaming a state whose only
    # non-zero populations point at the wall, they come back reversed.
    m, _ = _cathode()
    s = torch.zeros(19, 10, 12, dtype=DT)
    s[3, 7, 0] = 1.0     # flow, e = (-1, 0) at a GDL row of column 0
    s[17, 7, 0] = 1.0    # O2, e = (-1, 0)
    s[4, 0, 5] = 1.0     # flow, e = (0, -1) at the channel-side wall row
    s[13, 9, 5] = 1.0    # temperature, e = (0, -1), away from the CL-side wall
    pre = m.stream(s)
    assert float(pre[1, 7, 0]) == 1.0 and float(pre[15, 7, 0]) == 1.0
    assert float(pre[2, 0, 5]) == 1.0
    assert float(pre[13, 8, 5]) == 1.0  # moved down one row, no wall crossed
    assert abs(float(pre.sum()) - 4.0) < 1e-15


def _plane_flux(post, x, q_plus, q_minus):
    """Net population crossing the plane between columns x and x+1."""
    return float(post[q_plus, :, x].sum() - post[q_minus, :, x + 1].sum())


def test_interior_oxygen_and_heat_budget_per_step():
    # For the interior columns 1..nx-2 of an open cathode, one step changes
    # the O2 content by (inflow across x = 1/2) - (outflow across
    # x = nx - 3/2) - (O2 consumed in interior CL cells), and the heat content
    # likewise with the reaction heat: walls carry no flux, streaming and
    # collision conserve the rest.  Exact for any state.
    m, s = _cathode(nx=14, ny=12, layers=(6, 4, 2), seed=12, V_op=0.45)
    nx = m.g.nx
    for _ in range(3):
        o = m.observables(s)
        pre0 = m.pre_collision(s)
        post = m.collide(pre0)
        pre1 = m.pre_collision(post)
        for base, src_key in ((14, "c"), (9, "T")):
            inside0 = float(pre0[base:base + 5, :, 1:nx - 1].sum())
            inside1 = float(pre1[base:base + 5, :, 1:nx - 1].sum())
            inflow = _plane_flux(post, 0, base + 1, base + 3)
            outflow = _plane_flux(post, nx - 2, base + 1, base + 3)
            theta = pre0[9:14].sum(0)
            c = pre0[14:19].sum(0)
            s_c, S_T, *_ = m.reaction(theta, c, m.rhocp)
            src = torch.where(m.is_cl, -s_c if src_key == "c" else S_T, torch.zeros_like(c))
            interior_src = float(src[:, 1:nx - 1].sum())
            lhs = inside1 - inside0
            rhs = inflow - outflow + interior_src
            assert abs(lhs - rhs) < 1e-13 * max(abs(inside0), 1.0), (src_key, lhs, rhs)
        s = post
    assert float(o["consumed_c"]) > 0


def test_cathode_trends_smoke():
    # Section 5 trends on a short run (not a parity check): a lower voltage or
    # a higher temperature gives a higher mean current density; the heat
    # rate is positive for voltages above the U0 intercept.
    def current(**kw):
        g = L.Geometry(30, 12, 6, 5, 1)
        m = L.Model(g, L.Params(phi_gdl=0.6, Da_gdl=1e-3, **kw))
        s = m.run(m.initial_state(), 60)
        return m.observables(s)

    base = current(V_op=0.6, T_in=353.0)
    assert float(current(V_op=0.5, T_in=353.0)["current_density"]) > float(base["current_density"])
    assert float(current(V_op=0.6, T_in=363.0)["current_density"]) > float(base["current_density"])
    assert float(base["heat_rate"]) > 0 and 0 < float(base["o2_utilisation"]) < 1


def test_outlet_link_carries_no_flux_at_rest_in_a_porosity_field():
    # Reading of the "fully developed" scalar outlet: the outlet node collides
    # the copied populations with column nx-2's scalar material, so a resting
    # state of uniform O2 and temperature rise exchanges nothing across the
    # last link even where the porosity (hence b) jumps between the two
    # columns; colliding with the node's own b would leak (4 + b) X / 20
    # differences through the outlet every step.
    w = W.cathode2d_scaled(12, 10, precision=64, phi_seed=5, Re=0.0)
    phi = torch.as_tensor(W.porosity_field(w))
    g = L.Geometry(12, 10, w["ny_channel"], w["ny_gdl"], w["ny_cl"])
    p = L.Params.from_workload(w)
    p.reaction = False
    m = L.Model(g, p, phi=phi)
    z = torch.zeros(10, 12, dtype=DT)
    pre = m.equilibrium_state(z, z, z, z + 0.3, z + 0.8)
    post = m.collide(m.open_boundaries(pre))
    nx = 12
    for base in (9, 14):
        flux = post[base + 1, :, nx - 2] - post[base + 3, :, nx - 1]
        assert float(flux.abs().max()) < 1e-16
    assert float((m.b_C[:, nx - 1] - m.b_C[:, nx - 2]).abs().max()) > 1e-2  # the jump is real
