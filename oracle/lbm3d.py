"""Plain FP64 oracle of the coupled step in three dimensions (D3Q19 + 2 x D3Q7).

TEST INFRASTRUCTURE ONLY (see the package docstring).  The paper is
two-dimensional; this extends its method to 3D with the same physics:

* Flow.  With the density moment relaxed at 1/tau (reading R0 of
  ``lbm2d``) the D2Q9 MRT of Section 2.1 relaxes every even moment at
  s+ = 1/tau and every non-conserved odd moment at s- = 8(2 - s+)/(8 - s+),
  and the rate of the momentum moment is immaterial (the half-force
  velocity of Eq. 8 makes m_j* = v + F for any rate).  It is therefore the
  two-relaxation-time collision f* = f - s+(f+ - f+eq) - s-(f- - f-eq)
  + (1 - s+/2) F+ + (1 - s-/2) F- on the symmetric / antisymmetric parts,
  with Guo's porous forcing F_i; ``collide_trt`` writes it for any lattice
  and a test checks it against ``lbm2d``'s MRT on D2Q9.  Here it runs on
  D3Q19 with the same two rates (Lambda = 3/16).
* Equilibrium.  The 3D form of the pressure-based porous equilibrium of
  Eq. 5: f0 = rho0 - 2 phi p - 0.5 |u|^2/phi, f_i = 3 w_i phi p
  + w_i [3 e.u + 4.5 (e.u)^2/phi - 1.5 |u|^2/phi]; then
  p = (sum_{i>=1} f_i - 0.5 |u|^2/phi) / (2 phi).  Eqs. 7-8 unchanged.
* Scalars.  The D2Q5 MRT of Eq. 10 is TRT with odd rate 6/(3+sqrt 3) and
  even rate 6/(3+2 sqrt 3); its b = 20 sqrt(3) alpha - 4 is the rest weight
  a = (4 + b)/20 = sqrt(3) alpha of each moving population.  On D3Q7 the
  same rates give g0 = X (1 - 6a), g_i = X (a + e.u/2), a = sqrt(3) alpha,
  diffusivity a / sqrt(3) (re-derived; pinned by a decay test).
* Geometry.  x from inlet to outlet, y across (walls at both ends), z
  through the layers: channel, GDL, CL (walls below the channel and below
  the CL).  Inlet: channel cells of x = 0, velocity
  36 U (y+1/2)(ny-1/2-y)(z+1/2)(H-1/2-z) / (ny^2 H^2) (mean U), Dirichlet
  scalars; outlet x = nx-1 as in 2D (reading R10 included).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch

from . import lbm2d as L

DT = torch.float64
RHO0 = 1.0


def d3q19():
    """Velocities (opposites adjacent: 1/2, 3/4, ...) and weights."""
    e = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
         (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
         (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]
    w = [1 / 3] + [1 / 18] * 6 + [1 / 36] * 12
    return e, w


E19, W19 = d3q19()
E7 = E19[:7]
OPP19 = [E19.index((-a, -b, -c)) for (a, b, c) in E19]
OPP7 = OPP19[:7]
_S3 = math.sqrt(3.0)
S_ODD_SCALAR = 6.0 / (3.0 + _S3)
S_EVEN_SCALAR = 6.0 / (3.0 + 2.0 * _S3)


def collide_trt(f, feq, F, s_plus, s_minus, opp):
    """Two-relaxation-time collision on populations [Q, ...] with forcing
    populations F (zeros for none)."""
    fo, eo, Fo = f[opp], feq[opp], F[opp]
    fp, fm = 0.5 * (f + fo), 0.5 * (f - fo)
    ep, em = 0.5 * (feq + eo), 0.5 * (feq - eo)
    Fp, Fm = 0.5 * (F + Fo), 0.5 * (F - Fo)
    return f - s_plus * (fp - ep) - s_minus * (fm - em) + (1.0 - s_plus / 2.0) * Fp + (1.0 - s_minus / 2.0) * Fm


@dataclass
class Geometry3D:
    nx: int
    ny: int
    nz: int
    nz_channel: int
    nz_gdl: int
    nz_cl: int
    periodic_x: bool = False
    periodic_y: bool = False
    periodic_z: bool = False

    def __post_init__(self):
        if self.nz_channel + self.nz_gdl + self.nz_cl != self.nz:
            raise ValueError("layers must sum to nz")


def _safe_sqrt(a):
    """sqrt with derivative 0 at a = 0; a complex argument (complex-step
    differentiation in the tests) is tested on its real part."""
    pos = (a.real if a.is_complex() else a) > 0
    return torch.where(pos, torch.sqrt(torch.where(pos, a, torch.ones_like(a))), torch.zeros_like(a))


class Model3D:
    """Coupled D3Q19 / 2 x D3Q7 model.  Arrays are [plane, nz, ny, nx]."""

    def __init__(self, geom: Geometry3D, prm: L.Params, phi=None, inv_k=None, d_eff=None):
        self.g, self.p = geom, prm
        nz, ny, nx = geom.nz, geom.ny, geom.nx
        shape = (nz, ny, nx)
        self.nu = (prm.tau_f - 0.5) / 3.0
        self.s_plus = 1.0 / prm.tau_f
        self.s_minus = 8.0 * (2.0 - self.s_plus) / (8.0 - self.s_plus)
        self.dx = prm.dx_cm if prm.dx_cm > 0 else prm.gdl_thickness_cm / geom.nz_gdl
        self.dt = prm.D_f_lat * self.dx ** 2 / prm.D_O2
        self.u_avg = prm.Re * self.nu / geom.nz_channel if geom.nz_channel > 0 else 0.0
        z = torch.arange(nz).view(nz, 1, 1).expand(shape)
        self.is_channel = z < geom.nz_channel
        self.is_cl = z >= geom.nz_channel + geom.nz_gdl
        porous = ~self.is_channel
        if phi is None:
            phi = torch.where(porous, torch.full(shape, prm.phi_gdl, dtype=DT), torch.ones(shape, dtype=DT))
        self.phi = phi
        if inv_k is None:
            if prm.dp_lat > 0:
                inv_k = (1.0 - phi) ** 2 / (0.0067 * phi ** 3 * prm.dp_lat ** 2)
            else:
                k_lat = prm.Da_gdl * geom.nz_gdl ** 2
                inv_k = torch.where(porous, torch.full(shape, 1.0 / k_lat if k_lat > 0 else 0.0, dtype=DT),
                                    torch.zeros(shape, dtype=DT))
        self.inv_k = inv_k
        if d_eff is None:
            if prm.deff_ratio_gdl > 0:
                d_eff = torch.where(porous, torch.full(shape, prm.deff_ratio_gdl * prm.D_f_lat, dtype=DT),
                                    torch.full(shape, prm.D_f_lat, dtype=DT))
            else:
                d_eff = phi ** 1.5 * prm.D_f_lat
        self.d_eff = d_eff
        self.rhocp = phi * prm.rhocp_f + (1.0 - phi) * prm.rhocp_s
        self.alpha = (prm.k_f * phi + prm.k_s * (1.0 - phi)) / 100.0 / self.rhocp * self.dt / self.dx ** 2
        self.a_T = _S3 * self.alpha      # rest weight of each moving D3Q7 population
        self.a_C = _S3 * self.d_eff
        # Outlet scalar material from column nx-2 (reading R10 of lbm2d).
        self.a_T_coll, self.a_C_coll, self.rhocp_coll = self.a_T, self.a_C, self.rhocp
        if not geom.periodic_x:
            last = lambda a: torch.cat([a[..., :-1], a[..., -2:-1]], dim=-1)
            self.a_T_coll, self.a_C_coll, self.rhocp_coll = last(self.a_T), last(self.a_C), last(self.rhocp)
        self.F_phi = 0.143 * phi ** (-1.5)
        self.sqrt_inv_k = _safe_sqrt(inv_k)
        self.l0 = 0.5 + phi * self.nu * inv_k / 4.0
        self.l1 = phi * self.F_phi * self.sqrt_inv_k / 2.0
        self._inside19 = [self._link_inside(e) for e in E19]

    def _link_inside(self, e):
        nz, ny, nx = self.g.nz, self.g.ny, self.g.nx
        ok = torch.ones((nz, ny, nx), dtype=torch.bool)
        for axis, (n, per, comp) in enumerate(((nz, self.g.periodic_z, e[2]), (ny, self.g.periodic_y, e[1]),
                                               (nx, self.g.periodic_x, e[0]))):
            if per or comp == 0:
                continue
            idx = torch.arange(n) - comp
            good = (idx >= 0) & (idx < n)
            view = [1, 1, 1]
            view[axis] = n
            ok &= good.view(view).expand(nz, ny, nx)
        return ok

    def inlet_velocity(self):
        H, ny = self.g.nz_channel, self.g.ny
        zc = torch.arange(H, dtype=DT).view(H, 1) + 0.5
        yc = torch.arange(ny, dtype=DT).view(1, ny) + 0.5
        return 36.0 * self.u_avg * yc * (ny - yc) * zc * (H - zc) / (ny ** 2 * H ** 2)

    # -------------------------------------------------------------- equilibria
    def feq(self, p, ux, uy, uz, phi):
        u2 = ux * ux + uy * uy + uz * uz
        out = []
        for i, (ex, ey, ez) in enumerate(E19):
            eu = ex * ux + ey * uy + ez * uz
            s = W19[i] * RHO0 * (3 * eu + 4.5 * eu * eu / phi - 1.5 * u2 / phi)
            if i == 0:
                out.append(RHO0 - 2.0 * phi * p + s)
            else:
                out.append(3.0 * W19[i] * phi * p + s)
        return torch.stack(out)

    @staticmethod
    def geq(X, ux, uy, uz, a):
        out = [X * (1.0 - 6.0 * a)]
        for (ex, ey, ez) in E7[1:]:
            out.append(X * (a + 0.5 * (ex * ux + ey * uy + ez * uz)))
        return torch.stack(out)

    def forcing(self, ux, uy, uz, Fx, Fy, Fz, phi):
        """Guo's forcing populations for the porous model."""
        uF = ux * Fx + uy * Fy + uz * Fz
        out = []
        for i, (ex, ey, ez) in enumerate(E19):
            eu = ex * ux + ey * uy + ez * uz
            eF = ex * Fx + ey * Fy + ez * Fz
            out.append(W19[i] * RHO0 * (3 * eF + 9 * eu * eF / phi - 3 * uF / phi))
        return torch.stack(out)

    # ----------------------------------------------------------------- macros
    def flow_macros(self, f, phi, l0, l1, inv_k, sqk, Fphi):
        ax, ay = self.p.body_force
        v = [sum(E19[q][d] * f[q] for q in range(19)) / RHO0 for d in range(3)]
        v[0] = v[0] + 0.5 * phi * ax
        v[1] = v[1] + 0.5 * phi * ay
        vmag = _safe_sqrt(v[0] ** 2 + v[1] ** 2 + v[2] ** 2)
        den = l0 + torch.sqrt(l0 * l0 + l1 * vmag)
        u = [vi / den for vi in v]
        u2 = u[0] ** 2 + u[1] ** 2 + u[2] ** 2
        drag = phi * self.nu * inv_k + phi * Fphi * sqk * _safe_sqrt(u2)
        F = [phi * ax - drag * u[0], phi * ay - drag * u[1], -drag * u[2]]
        p = (sum(f[q] for q in range(1, 19)) - 0.5 * RHO0 * u2 / phi) / (2.0 * phi)
        return u, p, F

    def _macros_cols(self, f, sl):
        return self.flow_macros(f, self.phi[..., sl], self.l0[..., sl], self.l1[..., sl], self.inv_k[..., sl],
                                self.sqrt_inv_k[..., sl], self.F_phi[..., sl])

    # -------------------------------------------------------------- streaming
    def stream(self, post):
        out = torch.empty_like(post)
        blocks = ((0, E19, OPP19, 19), (19, E7, OPP7, 7), (26, E7, OPP7, 7))
        for base, E, OPP, n in blocks:
            for q in range(n):
                ex, ey, ez = E[q]
                src = torch.roll(post[base + q], shifts=(ez, ey, ex), dims=(0, 1, 2))
                out[base + q] = torch.where(self._inside19[q], src, post[base + OPP[q]])
        return out

    def open_boundaries(self, pre):
        if self.g.periodic_x:
            return pre
        out = pre.clone()
        nx, H = self.g.nx, self.g.nz_channel
        if H > 0:
            s1 = slice(1, 2)
            f1 = pre[0:19, :H, :, 1:2]
            sub = lambda a: a[:H, :, 1:2]
            sub0 = lambda a: a[:H, :, 0:1]
            u1, p1, _ = self.flow_macros(f1, sub(self.phi), sub(self.l0), sub(self.l1), sub(self.inv_k),
                                         sub(self.sqrt_inv_k), sub(self.F_phi))
            uin = self.inlet_velocity().unsqueeze(-1)
            z0 = torch.zeros_like(uin)
            out[0:19, :H, :, 0:1] = (self.feq(p1, uin, z0, z0, sub0(self.phi)) + f1
                                     - self.feq(p1, u1[0], u1[1], u1[2], sub(self.phi)))
            gT1, gC1 = pre[19:26, :H, :, 1:2], pre[26:33, :H, :, 1:2]
            th1, c1 = gT1.sum(0), gC1.sum(0)
            out[19:26, :H, :, 0:1] = (self.geq(z0, uin, z0, z0, sub0(self.a_T)) + gT1
                                      - self.geq(th1, u1[0], u1[1], u1[2], sub(self.a_T)))
            cin = torch.full_like(uin, self.p.c_in)
            out[26:33, :H, :, 0:1] = (self.geq(cin, uin, z0, z0, sub0(self.a_C)) + gC1
                                      - self.geq(c1, u1[0], u1[1], u1[2], sub(self.a_C)))
        c2 = slice(nx - 2, nx - 1)
        f2 = pre[0:19, :, :, c2]
        u2, p2, _ = self._macros_cols(f2, c2)
        out[0:19, :, :, nx - 1:nx] = (self.feq(torch.zeros_like(p2), u2[0], u2[1], u2[2], self.phi[..., nx - 1:nx])
                                      + f2 - self.feq(p2, u2[0], u2[1], u2[2], self.phi[..., c2]))
        out[19:33, :, :, nx - 1:nx] = pre[19:33, :, :, c2]
        return out

    def pre_collision(self, post):
        return self.open_boundaries(self.stream(post))

    # -------------------------------------------------------------- collision
    def collide(self, pre):
        f, gT, gC = pre[0:19], pre[19:26], pre[26:33]
        u, p, F = self.flow_macros(f, self.phi, self.l0, self.l1, self.inv_k, self.sqrt_inv_k, self.F_phi)
        feq = self.feq(p, u[0], u[1], u[2], self.phi)
        Fi = self.forcing(u[0], u[1], u[2], F[0], F[1], F[2], self.phi)
        f_post = collide_trt(f, feq, Fi, self.s_plus, self.s_minus, OPP19)
        theta, c = gT.sum(0), gC.sum(0)
        zero = torch.zeros_like(theta)
        if self.p.reaction:
            s_c, S_T, *_ = L.catalyst_reaction(self.p, self.dt, theta, c, self.rhocp_coll)
            src_C = torch.where(self.is_cl, -s_c, zero)
            src_T = torch.where(self.is_cl, S_T, zero)
        else:
            src_C = src_T = zero
        out = [f_post]
        for g, X, a, src in ((gT, theta, self.a_T_coll, src_T), (gC, c, self.a_C_coll, src_C)):
            geq = self.geq(X, u[0], u[1], u[2], a)
            post = collide_trt(g, geq, torch.zeros_like(g), S_EVEN_SCALAR, S_ODD_SCALAR, OPP7)
            out.append(post + self.geq(src, zero, zero, zero, a))  # source with the rest weights
        return torch.cat(out)

    def step(self, post):
        return self.collide(self.pre_collision(post))

    def run(self, post, n):
        for _ in range(n):
            post = self.step(post)
        return post

    def equilibrium_state(self, p, u, theta, c):
        return torch.cat([self.feq(p, u[0], u[1], u[2], self.phi), self.geq(theta, u[0], u[1], u[2], self.a_T),
                          self.geq(c, u[0], u[1], u[2], self.a_C)])

    def initial_state(self):
        shape = (self.g.nz, self.g.ny, self.g.nx)
        z = torch.zeros(shape, dtype=DT)
        return self.equilibrium_state(z, (z, z, z), z, torch.full(shape, self.p.c_in, dtype=DT))

    def fields(self, post):
        pre = self.pre_collision(post)
        u, p, _ = self.flow_macros(pre[0:19], self.phi, self.l0, self.l1, self.inv_k, self.sqrt_inv_k, self.F_phi)
        theta = pre[19:26].sum(0)
        return dict(ux=u[0], uy=u[1], uz=u[2], p=p, theta=theta, T=self.p.T_in + theta, c=pre[26:33].sum(0))

    def observables(self, post):
        """As in 2D: i(x, y) = sum over CL layers of (-j_eff) dx; I = its mean."""
        pre = self.pre_collision(post)
        theta, c = pre[19:26].sum(0), pre[26:33].sum(0)
        s_c, S_T, j_eff, Q, _ = L.catalyst_reaction(self.p, self.dt, theta, c, self.rhocp_coll)
        zero = torch.zeros_like(theta)
        cl = self.is_cl if self.p.reaction else torch.zeros_like(self.is_cl)
        s_c, S_T = torch.where(cl, s_c, zero), torch.where(cl, S_T, zero)
        j_eff, Q = torch.where(cl, j_eff, zero), torch.where(cl, Q, zero)
        I = ((-j_eff).sum(0) * self.dx).mean()
        H = (Q.sum(0) * self.dx).mean()
        inflow = (self.inlet_velocity() * self.p.c_in).sum() if self.g.nz_channel > 0 else torch.zeros((), dtype=DT)
        util = s_c.sum() / inflow if float(inflow.real) > 0 else torch.zeros((), dtype=DT)
        return dict(current_density=I, power_density=self.p.V_op * I, heat_rate=H, o2_utilisation=util,
                    T_max=(self.p.T_in + theta).real.max(), sum_f=pre[0:19].sum(), sum_theta=theta.sum(),
                    sum_c=c.sum(), consumed_c=s_c.sum(), heat_added=S_T.sum())


def params_from_workload(w: dict) -> L.Params:
    """Oracle parameters of a 3D workload dictionary."""
    p = L.Params.from_workload({k: v for k, v in w.items() if k != "dp_over_hgdl"})
    if w.get("dp_lat", 0.0) > 0:
        p.dp_lat = float(w["dp_lat"])
    return p


def geometry_from_workload(w: dict, **flags) -> Geometry3D:
    return Geometry3D(w["nx"], w["ny"], w["nz"], w["nz_channel"], w["nz_gdl"], w["nz_cl"], **flags)
