// Discrete adjoint of the 3D step (reverse mode, written by hand).
//
// Same structure as the 2D adjoint: the step is S' = C(P(S)) with P the
// pull (a permutation with bounce-back) plus the inlet / outlet columns and
// C the per-node collision, so per node
//   mu_x   = (dC_x / d pre_x)^T lambda_x
//   mu_xp += (dB / d pre_xp)^T mu_b   for the boundary node b fed by xp
//   lambda_new[source of pull (x, q)] = mu_x[q].
// The collision is two-rate, so its transpose acts pair by pair on the
// symmetric / antisymmetric parts.
#pragma once

#include "lbm3d_device.hpp"
#include "lbm_adjoint.hpp"  // reaction_tape, ReactAdj

namespace lbm3 {

using lbm::ReactAdj;
using lbm::reaction_tape;

template <typename R>
struct MatAdj3 {
  R phi = R(0), invk = R(0), sqk = R(0), fphi = R(0), l0 = R(0), l1 = R(0), aT = R(0), aC = R(0), rhocp = R(0);
};

constexpr double kSqrt3 = 1.7320508075688772935;

// Chain the adjoints of the derived material quantities to (phi, 1/K, D).
template <typename R>
__device__ __forceinline__ void material_adj(const Consts3<R>& k, const Mat3<R>& m, const MatAdj3<R>& a, R& g_phi,
                                             R& g_invk, R& g_d) {
  const R phi = m.phi;
  const R iphi = R(1) / phi, irc = R(1) / m.rhocp;
  R lphi = a.phi, linvk = a.invk, lsqk = a.sqk, lfphi = a.fphi;
  lphi += a.l1 * m.fphi * m.sqk * R(0.5);  // l1 = phi fphi sqk / 2
  lfphi += a.l1 * phi * m.sqk * R(0.5);
  lsqk += a.l1 * phi * m.fphi * R(0.5);
  lphi += a.l0 * k.nu * m.invk * R(0.25);  // l0 = 1/2 + phi nu invk / 4
  linvk += a.l0 * phi * k.nu * R(0.25);
  lphi += lfphi * R(-1.5) * m.fphi * iphi;  // fphi = 0.143 phi^-1.5
  if (m.sqk > R(0)) linvk += lsqk * R(0.5) / m.sqk;  // 0 at invk = 0
  // aT = sqrt3 alpha, alpha = (k_f phi + k_s (1 - phi)) scale / rhocp (Eq. 19)
  const R alpha = (k.k_f * phi + k.k_s * (R(1) - phi)) * k.alpha_scale * irc;
  const R drc = k.rhocp_f - k.rhocp_s;
  const R lalpha = a.aT * R(kSqrt3);
  lphi += lalpha * ((k.k_f - k.k_s) * k.alpha_scale - alpha * drc) * irc;
  lphi += a.rhocp * drc;
  g_phi += lphi;
  g_invk += linvk;
  g_d += a.aC * R(kSqrt3);  // aC = sqrt3 D
}

// Forward intermediates of the flow macros, with the reciprocals the
// adjoint divides by (each taken once per node).
template <typename R>
struct MacroTape3 {
  R vx, vy, vz, vm, r, den, ux, uy, uz, um, drag, s, p, Fx, Fy, Fz;
  R iphi, iden, ir;  // 1 / phi, 1 / den, 1 / r
};

template <typename R>
__device__ __forceinline__ MacroTape3<R> flow_macros_tape(const R (&f)[33], const Mat3<R>& m, const Consts3<R>& k) {
  MacroTape3<R> t;
  t.vx = t.vy = t.vz = t.s = R(0);
#pragma unroll
  for (int q = 1; q < 19; ++q) {
    t.vx += R(EX[q]) * f[q];
    t.vy += R(EY[q]) * f[q];
    t.vz += R(EZ[q]) * f[q];
    t.s += f[q];
  }
  if (k.flags & F_BODY_FORCE) {
    t.vx += R(0.5) * m.phi * k.ax;
    t.vy += R(0.5) * m.phi * k.ay;
  }
  t.vm = sqrt(t.vx * t.vx + t.vy * t.vy + t.vz * t.vz);
  t.r = sqrt(m.l0 * m.l0 + m.l1 * t.vm);
  t.den = m.l0 + t.r;
  t.iden = R(1) / t.den;
  t.ir = R(1) / t.r;
  t.ux = t.vx * t.iden;
  t.uy = t.vy * t.iden;
  t.uz = t.vz * t.iden;
  const R u2 = t.ux * t.ux + t.uy * t.uy + t.uz * t.uz;
  t.um = sqrt(u2);
  t.drag = m.phi * (k.nu * m.invk + m.fphi * m.sqk * t.um);
  t.Fx = -t.drag * t.ux;
  t.Fy = -t.drag * t.uy;
  t.Fz = -t.drag * t.uz;
  if (k.flags & F_BODY_FORCE) {
    t.Fx += m.phi * k.ax;
    t.Fy += m.phi * k.ay;
  }
  t.iphi = R(1) / m.phi;
  t.p = (t.s - R(0.5) * u2 * t.iphi) * R(0.5) * t.iphi;
  return t;
}

// Adjoint of flow_macros: from the adjoints of (u, p, F) add the adjoints of
// the flow populations to lf[1..18] and of the material to ma.
template <typename R>
__device__ __forceinline__ void flow_macros_adj(const MacroTape3<R>& t, const Mat3<R>& m, const Consts3<R>& k, R lux,
                                                R luy, R luz, R lp, R lFx, R lFy, R lFz, R* lf, MatAdj3<R>& ma) {
  const R iphi = t.iphi;
  const R u2 = t.ux * t.ux + t.uy * t.uy + t.uz * t.uz;
  // p = 0.5 s iphi - 0.25 u2 iphi^2
  const R ls = R(0.5) * iphi * lp;
  R lu2 = R(-0.25) * iphi * iphi * lp;
  const R liphi = (R(0.5) * t.s - R(0.5) * u2 * iphi) * lp;
  if (k.flags & F_BODY_FORCE) ma.phi += k.ax * lFx + k.ay * lFy;
  const R ldrag = -(t.ux * lFx + t.uy * lFy + t.uz * lFz);
  lux += -t.drag * lFx;
  luy += -t.drag * lFy;
  luz += -t.drag * lFz;
  ma.phi += (k.nu * m.invk + m.fphi * m.sqk * t.um) * ldrag;
  ma.invk += m.phi * k.nu * ldrag;
  ma.fphi += m.phi * m.sqk * t.um * ldrag;
  ma.sqk += m.phi * m.fphi * t.um * ldrag;
  const R lum = m.phi * m.fphi * m.sqk * ldrag;
  if (t.um > R(0)) lu2 += lum * R(0.5) / t.um;
  lux += R(2) * t.ux * lu2;
  luy += R(2) * t.uy * lu2;
  luz += R(2) * t.uz * lu2;
  ma.phi += -iphi * iphi * liphi;
  R lvx = lux * t.iden, lvy = luy * t.iden, lvz = luz * t.iden;
  const R lden = -(t.ux * lux + t.uy * luy + t.uz * luz) * t.iden;
  const R ldr = lden * t.ir;
  ma.l0 += lden + ldr * m.l0;
  ma.l1 += ldr * t.vm * R(0.5);
  const R lvm = ldr * m.l1 * R(0.5);
  if (t.vm > R(0)) {
    const R q = lvm / t.vm;
    lvx += q * t.vx;
    lvy += q * t.vy;
    lvz += q * t.vz;
  }
  if (k.flags & F_BODY_FORCE) ma.phi += R(0.5) * (k.ax * lvx + k.ay * lvy);
#pragma unroll
  for (int q = 1; q < 19; ++q) lf[q] += R(EX[q]) * lvx + R(EY[q]) * lvy + R(EZ[q]) * lvz + ls;
}

// Adjoint of add_feq(p, u, phi, sgn, .) given L[0..18], the adjoint of its output.
template <typename R>
__device__ __forceinline__ void feq_adj(R p, R ux, R uy, R uz, R phi, R sgn, const R* L, R& lp, R& lux, R& luy,
                                        R& luz, R& lphi) {
  const R iphi = R(1) / phi;
  const R u2 = ux * ux + uy * uy + uz * uz;
  R ap = R(-2) * phi * L[0];
  R aphi = (R(-2) * p + R(0.5) * u2 * iphi * iphi) * L[0];
  R au2 = R(-0.5) * iphi * L[0];
  R ax = R(0), ay = R(0), az = R(0);
#pragma unroll
  for (int q = 1; q < 19; ++q) {
    const R w = weight<R>(q);
    const R eu = R(EX[q]) * ux + R(EY[q]) * uy + R(EZ[q]) * uz;
    ap += R(3) * w * phi * L[q];
    aphi += (R(3) * w * p - w * (R(4.5) * eu * eu - R(1.5) * u2) * iphi * iphi) * L[q];
    au2 += R(-1.5) * w * iphi * L[q];
    const R leu = w * (R(3) + R(9) * eu * iphi) * L[q];
    ax += R(EX[q]) * leu;
    ay += R(EY[q]) * leu;
    az += R(EZ[q]) * leu;
  }
  lp += sgn * ap;
  lphi += sgn * aphi;
  lux += sgn * (ax + R(2) * ux * au2);
  luy += sgn * (ay + R(2) * uy * au2);
  luz += sgn * (az + R(2) * uz * au2);
}

// Adjoint of add_geq(X, u, a, sgn, .) given L[0..6].
template <typename R>
__device__ __forceinline__ void geq_adj(R X, R ux, R uy, R uz, R a, R sgn, const R* L, R& lX, R& lux, R& luy,
                                        R& luz, R& la) {
  R sX = (R(1) - R(6) * a) * L[0];
  R sa = R(-6) * X * L[0];
  R ax = R(0), ay = R(0), az = R(0);
#pragma unroll
  for (int q = 1; q < 7; ++q) {
    const R eu = R(EX[19 + q]) * ux + R(EY[19 + q]) * uy + R(EZ[19 + q]) * uz;
    sX += (a + R(0.5) * eu) * L[q];
    sa += X * L[q];
    const R leu = R(0.5) * X * L[q];
    ax += R(EX[19 + q]) * leu;
    ay += R(EY[19 + q]) * leu;
    az += R(EZ[19 + q]) * leu;
  }
  lX += sgn * sX;
  la += sgn * sa;
  lux += sgn * ax;
  luy += sgn * ay;
  luz += sgn * az;
}

// Collision adjoint of one node.  In: pre-collision f, material, adjoint la
// of the post-collision populations.  Out: adjoint mu of the pre-collision
// populations; material adjoints accumulated in ma.
template <typename R>
__device__ __forceinline__ void collide_adj(const R (&f)[33], const Mat3<R>& mt, const Consts3<R>& k, bool cl,
                                            const R (&la)[33], R (&mu)[33], MatAdj3<R>& ma) {
  const MacroTape3<R> t = flow_macros_tape(f, mt, k);
  R lux = R(0), luy = R(0), luz = R(0);
#pragma unroll
  for (int i = 0; i < 33; ++i) mu[i] = R(0);

  // ---- scalars: two-rate D3Q7 collisions and the CL source ----
  R th = R(0), c = R(0);
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    th += f[19 + q];
    c += f[26 + q];
  }
  ReactAdj<R> rx{};
  if (cl) rx = reaction_tape(th, c, mt.rhocp, k);
  const R srcT = cl ? rx.S_T : R(0), srcC = cl ? -rx.s_c : R(0);
  const R qp = R(0.9282032302755092), qm = R(1.2679491924311228);
  R lX[2], lsrc[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const R* a = la + 19 + 7 * s;
    R* o = mu + 19 + 7 * s;
    const R X = s == 0 ? th : c;
    const R aw = s == 0 ? mt.aT : mt.aC;
    const R src = s == 0 ? srcT : srcC;
    // The forward sets the rest population to X + src minus the six moving
    // ones: its adjoint a[0] goes to X and src, and is taken off the moving.
    o[0] = R(0);
    R lx = a[0];
    R law = R(0);
    R ls = a[0];
#pragma unroll
    for (int pr = 0; pr < 3; ++pr) {
      const int i = 2 * pr + 1, j = i + 1;
      const R eu = R(EX[19 + i]) * t.ux + R(EY[19 + i]) * t.uy + R(EZ[19 + i]) * t.uz;
      const R ai = a[i] - a[0], aj = a[j] - a[0];
      const R lnp = ai + aj, lnm = ai - aj;
      o[i] = R(0.5) * (R(1) - qp) * lnp + R(0.5) * (R(1) - qm) * lnm;
      o[j] = R(0.5) * (R(1) - qp) * lnp - R(0.5) * (R(1) - qm) * lnm;
      lx += qp * aw * lnp + qm * R(0.5) * eu * lnm;
      law += (qp * X + src) * lnp;
      ls += aw * lnp;
      const R leu = qm * R(0.5) * X * lnm;
      lux += R(EX[19 + i]) * leu;
      luy += R(EY[19 + i]) * leu;
      luz += R(EZ[19 + i]) * leu;
    }
    lX[s] = lx;
    lsrc[s] = ls;
    if (s == 0) ma.aT += law; else ma.aC += law;
  }
  if (cl) {  // src_T = S_T(theta, c, rhocp), src_C = -s_c(theta, c)
    const R irc = R(1) / mt.rhocp;
    const R lsc = -lsrc[1] + k.four_f_cref * rx.ehs * irc * lsrc[0];
    ma.rhocp += -rx.S_T * irc * lsrc[0];
    lX[1] += rx.dsc_dc * lsc;
    lX[0] += rx.dsc_dth * lsc;
    if (k.flags & lbm::F_PHYSICAL_HEAT) lX[0] += k.four_f_cref * rx.s_c * R(2) * k.U0_slope * irc * lsrc[0];
  }
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    mu[19 + q] += lX[0];
    mu[26 + q] += lX[1];
  }

  // ---- flow: two-rate D3Q19 collision with porous forcing ----
  const R sp = k.s_plus, sm = k.s_minus;
  const R hp = R(1) - R(0.5) * sp, hm = R(1) - R(0.5) * sm;
  const R phi = mt.phi, iphi = t.iphi;
  const R u2 = t.ux * t.ux + t.uy * t.uy + t.uz * t.uz;
  const R uF = t.ux * t.Fx + t.uy * t.Fy + t.uz * t.Fz;
  R lp = R(0), lu2 = R(0), luF = R(0), liphi = R(0);
  R lFx = R(0), lFy = R(0), lFz = R(0);
  {  // rest: f0* = (1 - sp) f0 + sp eq0 + hp F0, eq0 = -2 phi p - u2/(2 phi), F0 = -uF / phi
    const R L0 = la[0];
    mu[0] += (R(1) - sp) * L0;
    const R le = sp * L0, lF = hp * L0;
    lp += R(-2) * phi * le;
    ma.phi += R(-2) * t.p * le;
    lu2 += R(-0.5) * iphi * le;
    liphi += R(-0.5) * u2 * le;
    luF += -iphi * lF;
    liphi += -uF * lF;
  }
#pragma unroll
  for (int pr = 0; pr < 9; ++pr) {
    const int i = 2 * pr + 1, j = i + 1;
    const R w = weight<R>(i);
    const R ex = R(EX[i]), ey = R(EY[i]), ez = R(EZ[i]);
    const R eu = ex * t.ux + ey * t.uy + ez * t.uz;
    const R eF = ex * t.Fx + ey * t.Fy + ez * t.Fz;
    const R lnp = la[i] + la[j], lnm = la[i] - la[j];
    mu[i] += R(0.5) * (R(1) - sp) * lnp + R(0.5) * (R(1) - sm) * lnm;
    mu[j] += R(0.5) * (R(1) - sp) * lnp - R(0.5) * (R(1) - sm) * lnm;
    const R leqe = sp * lnp, leqo = sm * lnm, lFe = hp * lnp, lFo = hm * lnm;
    // eq_even = 3 w phi p + w (4.5 eu^2 - 1.5 u2) / phi; eq_odd = 3 w eu
    lp += R(3) * w * phi * leqe;
    ma.phi += R(3) * w * t.p * leqe;
    R leu = R(9) * w * eu * iphi * leqe + R(3) * w * leqo;
    lu2 += R(-1.5) * w * iphi * leqe;
    liphi += w * (R(4.5) * eu * eu - R(1.5) * u2) * leqe;
    // F_even = w (9 eu eF - 3 uF) / phi; F_odd = 3 w eF
    leu += R(9) * w * eF * iphi * lFe;
    const R leF = R(9) * w * eu * iphi * lFe + R(3) * w * lFo;
    luF += R(-3) * w * iphi * lFe;
    liphi += w * (R(9) * eu * eF - R(3) * uF) * lFe;
    lux += ex * leu;
    luy += ey * leu;
    luz += ez * leu;
    lFx += ex * leF;
    lFy += ey * leF;
    lFz += ez * leF;
  }
  lux += t.Fx * luF + R(2) * t.ux * lu2;
  luy += t.Fy * luF + R(2) * t.uy * lu2;
  luz += t.Fz * luF + R(2) * t.uz * lu2;
  lFx += t.ux * luF;
  lFy += t.uy * luF;
  lFz += t.uz * luF;
  ma.phi += -iphi * iphi * liphi;
  flow_macros_adj(t, mt, k, lux, luy, luz, lp, lFx, lFy, lFz, mu, ma);
}

// Adjoint of the boundary-column extrapolation of node b fed by node xp.
// pre_xp: pulled populations of xp; mu_b: adjoint of the boundary node's
// pre-collision populations.  Adds to mu_xp and to the material adjoints of
// xp (maxp) and of b (mab).  ub: inlet velocity at b.
template <typename R>
__device__ __forceinline__ void boundary_adj(const R (&pre_xp)[33], const Mat3<R>& mxp, const Mat3<R>& mb,
                                             const Consts3<R>& k, bool inlet, R ub, const R (&mu_b)[33],
                                             R (&mu_xp)[33], MatAdj3<R>& maxp, MatAdj3<R>& mab) {
  const MacroTape3<R> t = flow_macros_tape(pre_xp, mxp, k);
#pragma unroll
  for (int i = 0; i < 33; ++i) mu_xp[i] += mu_b[i];  // identity part (outlet scalars: a copy)
  R lp1 = R(0), lux1 = R(0), luy1 = R(0), luz1 = R(0);
  R d0 = R(0), d1 = R(0), d2 = R(0), d3 = R(0);
  if (inlet) {  // + feq(p1, ub; phi_b)
    feq_adj(t.p, ub, R(0), R(0), mb.phi, R(1), mu_b, lp1, d0, d1, d2, mab.phi);
  } else {  // + feq(0, u1; phi_b)
    feq_adj(R(0), t.ux, t.uy, t.uz, mb.phi, R(1), mu_b, d3, lux1, luy1, luz1, mab.phi);
  }
  feq_adj(t.p, t.ux, t.uy, t.uz, mxp.phi, R(-1), mu_b, lp1, lux1, luy1, luz1, maxp.phi);  // - feq(p1, u1; phi_xp)
  if (inlet) {
    R th1 = R(0), c1 = R(0);
#pragma unroll
    for (int q = 0; q < 7; ++q) {
      th1 += pre_xp[19 + q];
      c1 += pre_xp[26 + q];
    }
    R lth1 = R(0), lc1 = R(0), dX = R(0);
    // + geq(0, ub; aT_b) is a constant; - geq(theta1, u1; aT_xp)
    geq_adj(th1, t.ux, t.uy, t.uz, mxp.aT, R(-1), mu_b + 19, lth1, lux1, luy1, luz1, maxp.aT);
    geq_adj(k.c_in, ub, R(0), R(0), mb.aC, R(1), mu_b + 26, dX, d0, d1, d2, mab.aC);  // + geq(c_in, ub; aC_b)
    geq_adj(c1, t.ux, t.uy, t.uz, mxp.aC, R(-1), mu_b + 26, lc1, lux1, luy1, luz1, maxp.aC);
#pragma unroll
    for (int q = 0; q < 7; ++q) {
      mu_xp[19 + q] += lth1;
      mu_xp[26 + q] += lc1;
    }
  }
  flow_macros_adj(t, mxp, k, lux1, luy1, luz1, lp1, R(0), R(0), R(0), mu_xp, maxp);
}

}  // namespace lbm3
