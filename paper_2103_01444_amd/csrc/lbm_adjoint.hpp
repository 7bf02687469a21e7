// Discrete adjoint of the coupled step (reverse mode, written by hand).
//
// The forward step is S' = C(P(S)): P pulls the populations (a permutation
// with half-way bounce-back) and applies the inlet / outlet extrapolation
// columns, C collides every node.  With lambda the adjoint of S', the
// adjoint of S is obtained per node x by
//   mu_x  = (dC_x / d pre_x)^T lambda_x                       (collision)
//   mu_xp += (dB / d pre_xp)^T mu_b     for the boundary node b fed by xp
//   lambda_new[source of pull (x, q)] = mu_x[q]                (push)
// Every element of the state is pulled by exactly one node, so the push
// writes every element of lambda_new once; boundary nodes, whose pulled
// values the forward step discards, write zeros.  Each node accumulates
// only its own gradient with respect to (porosity, 1/K, D_eff).
#pragma once

#include "lbm_device.hpp"

namespace lbm {

// EXT: the instances of the reverse step that also cover Boussinesq
// buoyancy, the energy equation with the heat-capacity ratio sigma and the
// pressure-driven inlet; the default instances leave their terms out (and
// their registers free).
template <typename R>
struct MatAdj {
  R phi = R(0), invk = R(0), sqk = R(0), fphi = R(0), l0 = R(0), l1 = R(0), bT = R(0), bC = R(0), rhocp = R(0);
  R sig = R(0);  // heat-capacity ratio (EXT only)
};

// Chain the adjoints of the derived material quantities to (phi, 1/K, D).
template <typename R, bool EXT = false>
__device__ __forceinline__ void material_adj(const Consts<R>& k, const Mat<R>& m, const MatAdj<R>& a, R& g_phi,
                                             R& g_invk, R& g_d) {
  const R phi = m.phi;
  const R iphi = R(1) / phi, irc = R(1) / m.rhocp;
  R lphi = a.phi, linvk = a.invk, lsqk = a.sqk, lfphi = a.fphi;
  // l1 = phi fphi sqk / 2
  lphi += a.l1 * m.fphi * m.sqk * R(0.5);
  lfphi += a.l1 * phi * m.sqk * R(0.5);
  lsqk += a.l1 * phi * m.fphi * R(0.5);
  // l0 = 1/2 + phi nu invk / 4
  lphi += a.l0 * k.nu * m.invk * R(0.25);
  linvk += a.l0 * phi * k.nu * R(0.25);
  // fphi = 0.143 phi^-1.5
  lphi += lfphi * R(-1.5) * m.fphi * iphi;
  // sqk = sqrt(invk); derivative taken as 0 at invk = 0 (clear fluid)
  if (m.sqk > R(0)) linvk += lsqk * R(0.5) / m.sqk;
  // rhocp = phi rhocp_f + (1 - phi) rhocp_s; alpha (Eq. 19) -> bT = 20 sqrt3 alpha - 4
  const R c20s3 = R(34.64101615137754587);
  const R alpha = (m.bT + R(4)) * R(0.028867513459481288225);  // 1 / (20 sqrt 3)
  const R drc = k.rhocp_f - k.rhocp_s;
  const R lalpha = a.bT * c20s3;
  if (EXT && (k.flags & F_SIGMA_ENERGY)) {
    // alpha = k_eff alpha_scale / rhocp_f, sigma = rhocp / rhocp_f
    lphi += lalpha * (k.k_f - k.k_s) * k.alpha_scale / k.rhocp_f;
    lphi += (a.rhocp + a.sig / k.rhocp_f) * drc;
  } else {
    lphi += lalpha * ((k.k_f - k.k_s) * k.alpha_scale - alpha * drc) * irc;
    lphi += a.rhocp * drc;
  }
  g_phi += lphi;
  g_invk += linvk;
  g_d += a.bC * c20s3;
}

// Adjoint of meq_shifted(p, ux, uy, phi) given the adjoint lm[1..8] of the
// moments; iphi = 1 / phi.
template <typename R>
__device__ __forceinline__ void meq_adj(R p, R ux, R uy, R phi, R iphi, const R (&lm)[9], R& lp, R& lux, R& luy,
                                        R& lphi) {
  const R u2 = ux * ux + uy * uy;
  lp += R(6) * phi * lm[1] - R(9) * phi * lm[2];
  lphi += R(6) * p * lm[1] - R(9) * p * lm[2] + (lm[2] - lm[1]) * R(3) * u2 * iphi * iphi -
          (ux * ux - uy * uy) * iphi * iphi * lm[7] - ux * uy * iphi * iphi * lm[8];
  const R a12 = R(6) * iphi * (lm[1] - lm[2]);
  lux += a12 * ux + lm[3] - lm[4] + R(2) * ux * iphi * lm[7] + uy * iphi * lm[8];
  luy += a12 * uy + lm[5] - lm[6] - R(2) * uy * iphi * lm[7] + ux * iphi * lm[8];
}

// Forward intermediates of flow_macros kept for its adjoint, with the
// reciprocals the adjoint divides by (each taken once per node).
template <typename R>
struct MacroTape {
  R vx, vy, vm, r, den, ux, uy, um, drag, s18, p, Fx, Fy;
  R iphi, iden, ir;  // 1 / phi, 1 / den, 1 / r
  R ax, ay, thb;     // acceleration, and the temperature rise buoyancy takes it from (EXT)
};

// The acceleration a of flow_macros is on when the test-mode body force is,
// or (EXT) Boussinesq buoyancy.
template <typename R, bool EXT>
__device__ __forceinline__ bool accelerated(const Consts<R>& k) {
  return (k.flags & F_BODY_FORCE) || (EXT && (k.flags & F_BUOYANCY));
}

template <typename R, bool EXT = false>
__device__ __forceinline__ MacroTape<R> flow_macros_tape(const R (&f)[19], const Mat<R>& m, const Consts<R>& k) {
  MacroTape<R> t;
  t.vx = f[1] - f[3] + f[5] - f[6] - f[7] + f[8];
  t.vy = f[2] - f[4] + f[5] + f[6] - f[7] - f[8];
  if constexpr (EXT) {
    t.ax = R(0);
    t.ay = R(0);
    t.thb = R(0);
    if (k.flags & F_BODY_FORCE) {
      t.ax = k.ax;
      t.ay = k.ay;
    }
    if (k.flags & F_BUOYANCY) {
      t.thb = theta_of(f + 9, m.sig, k);
      t.ax += k.bx * t.thb;
      t.ay += k.by * t.thb;
    }
    if (accelerated<R, EXT>(k)) {
      t.vx += R(0.5) * m.phi * t.ax;
      t.vy += R(0.5) * m.phi * t.ay;
    }
  } else if (k.flags & F_BODY_FORCE) {
    t.vx += R(0.5) * m.phi * k.ax;
    t.vy += R(0.5) * m.phi * k.ay;
  }
  t.vm = dsqrt(t.vx * t.vx + t.vy * t.vy);
  t.r = dsqrt(m.l0 * m.l0 + m.l1 * t.vm);
  t.den = m.l0 + t.r;
  t.iden = R(1) / t.den;
  t.ir = R(1) / t.r;
  t.ux = t.vx * t.iden;
  t.uy = t.vy * t.iden;
  const R u2 = t.ux * t.ux + t.uy * t.uy;
  t.um = dsqrt(u2);
  t.drag = m.phi * (k.nu * m.invk + m.fphi * m.sqk * t.um);
  t.Fx = -t.drag * t.ux;
  t.Fy = -t.drag * t.uy;
  if constexpr (EXT) {
    if (accelerated<R, EXT>(k)) {
      t.Fx += m.phi * t.ax;
      t.Fy += m.phi * t.ay;
    }
  } else if (k.flags & F_BODY_FORCE) {
    t.Fx += m.phi * k.ax;
    t.Fy += m.phi * k.ay;
  }
  t.s18 = f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
  t.iphi = R(1) / m.phi;
  t.p = R(0.6) * t.iphi * t.s18 - R(0.4) * u2 * t.iphi * t.iphi;
  return t;
}

// Adjoint of flow_macros: given the adjoints of (ux, uy, p, Fx, Fy), add the
// adjoints of the flow populations to lf[0..8] (with buoyancy also of the
// temperature populations, lf[9..13]) and of the material to ma.
template <typename R, bool EXT = false>
__device__ __forceinline__ void flow_macros_adj(const MacroTape<R>& t, const Mat<R>& m, const Consts<R>& k, R lux,
                                                R luy, R lp, R lFx, R lFy, R* lf, MatAdj<R>& ma) {
  const R iphi = t.iphi;
  const R u2 = t.ux * t.ux + t.uy * t.uy;
  // p = 0.6 iphi s18 - 0.4 u2 iphi^2
  const R ls18 = R(0.6) * iphi * lp;
  R lu2 = R(-0.4) * iphi * iphi * lp;
  R liphi = (R(0.6) * t.s18 - R(0.8) * u2 * iphi) * lp;
  // F = -drag u (+ phi a)
  R lax = R(0), lay = R(0);
  if constexpr (EXT) {
    if (accelerated<R, EXT>(k)) {
      ma.phi += t.ax * lFx + t.ay * lFy;
      lax += m.phi * lFx;
      lay += m.phi * lFy;
    }
  } else if (k.flags & F_BODY_FORCE) {
    ma.phi += k.ax * lFx + k.ay * lFy;
  }
  const R ldrag = -(t.ux * lFx + t.uy * lFy);
  lux += -t.drag * lFx;
  luy += -t.drag * lFy;
  // drag = phi (nu invk + fphi sqk um)
  ma.phi += (k.nu * m.invk + m.fphi * m.sqk * t.um) * ldrag;
  ma.invk += m.phi * k.nu * ldrag;
  ma.fphi += m.phi * m.sqk * t.um * ldrag;
  ma.sqk += m.phi * m.fphi * t.um * ldrag;
  const R lum = m.phi * m.fphi * m.sqk * ldrag;
  if (t.um > R(0)) lu2 += lum * R(0.5) / t.um;  // one division (vm, um > 0 only in moving cells)
  lux += R(2) * t.ux * lu2;
  luy += R(2) * t.uy * lu2;
  ma.phi += -iphi * iphi * liphi;
  // u = v / den, den = l0 + r, r = sqrt(l0^2 + l1 vm)
  R lvx = lux * t.iden, lvy = luy * t.iden;
  const R lden = -(t.ux * lux + t.uy * luy) * t.iden;
  const R ldr = lden * t.ir;
  ma.l0 += lden + ldr * m.l0;
  ma.l1 += ldr * t.vm * R(0.5);
  const R lvm = ldr * m.l1 * R(0.5);
  if (t.vm > R(0)) {
    const R q = lvm / t.vm;
    lvx += q * t.vx;
    lvy += q * t.vy;
  }
  if constexpr (EXT) {
    if (accelerated<R, EXT>(k)) {
      ma.phi += R(0.5) * (t.ax * lvx + t.ay * lvy);
      lax += R(0.5) * m.phi * lvx;
      lay += R(0.5) * m.phi * lvy;
    }
  } else if (k.flags & F_BODY_FORCE) {
    ma.phi += R(0.5) * (k.ax * lvx + k.ay * lvy);
  }
  if (EXT && (k.flags & F_BUOYANCY)) {  // a = ... + b theta, theta = sum g_T (/ sigma)
    R lth = k.bx * lax + k.by * lay;
    if (k.flags & F_SIGMA_ENERGY) {
      const R isg = R(1) / m.sig;
      ma.sig += -t.thb * isg * lth;
      lth *= isg;
    }
#pragma unroll
    for (int i = 9; i < 14; ++i) lf[i] += lth;
  }
  // v = sum e f, s18 = sum_{1..8} f
  lf[1] += lvx + ls18;
  lf[2] += lvy + ls18;
  lf[3] += -lvx + ls18;
  lf[4] += -lvy + ls18;
  lf[5] += lvx + lvy + ls18;
  lf[6] += -lvx + lvy + ls18;
  lf[7] += -lvx - lvy + ls18;
  lf[8] += lvx - lvy + ls18;
}

// (M^T y)_i = sum_k M[k][i] y_k: the columns of the Eq. 3 matrix (integer
// coefficients, additions only).
template <typename R>
__device__ __forceinline__ void mt_times(const R (&y)[9], R* out) {
  const R b14 = y[0] - y[1] - R(2) * y[2];
  const R b58 = y[0] + R(2) * y[1] + y[2];
  out[0] = y[0] - R(4) * y[1] + R(4) * y[2];
  out[1] = b14 + y[3] - R(2) * y[4] + y[7];
  out[2] = b14 + y[5] - R(2) * y[6] - y[7];
  out[3] = b14 - y[3] + R(2) * y[4] + y[7];
  out[4] = b14 - y[5] + R(2) * y[6] - y[7];
  out[5] = b58 + y[3] + y[4] + y[5] + y[6] + y[8];
  out[6] = b58 - y[3] - y[4] + y[5] + y[6] - y[8];
  out[7] = b58 - y[3] - y[4] - y[5] - y[6] + y[8];
  out[8] = b58 + y[3] + y[4] - y[5] - y[6] - y[8];
}

// 1 / diag(M M^T): M^{-T} a = (M a) / diag(M M^T).
template <typename R>
__device__ __forceinline__ R inv_mmt(int i) {
  constexpr double d[9] = {1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 6, 1.0 / 12, 1.0 / 6, 1.0 / 12, 0.25, 0.25};
  return R(d[i]);
}

template <typename R>
__device__ __forceinline__ void m_times(const R* a, R (&out)[9]) {
  R f[19];
#pragma unroll
  for (int i = 0; i < 9; ++i) f[i] = a[i];
  moments9(f, out);
}

// Adjoint of add_geq(X, ux, uy, b, sgn, g): given lg (adjoint of g) add the
// adjoints of X, ux, uy, b.
template <typename R>
__device__ __forceinline__ void geq_adj(R X, R ux, R uy, R b, R sgn, const R* lg, R& lX, R& lux, R& luy, R& lb) {
  const R n0 = (lg[0] + lg[1] + lg[2] + lg[3] + lg[4]) * R(0.2);
  const R n1 = (lg[1] - lg[3]) * R(0.5);
  const R n2 = (lg[2] - lg[4]) * R(0.5);
  const R n3 = (R(-4) * lg[0] + lg[1] + lg[2] + lg[3] + lg[4]) * R(0.05);
  lX += sgn * (n0 + ux * n1 + uy * n2 + b * n3);
  lux += sgn * X * n1;
  luy += sgn * X * n2;
  lb += sgn * X * n3;
}

// The same with the heat-capacity ratio of add_geq (rest moment sigma X,
// energy moment (b + 4 (1 - sigma)) X); also adds the adjoint of sigma.
template <typename R>
__device__ __forceinline__ void geq_adj_sig(R X, R ux, R uy, R b, R sig, R sgn, const R* lg, R& lX, R& lux, R& luy,
                                            R& lb, R& lsig) {
  const R n0 = (lg[0] + lg[1] + lg[2] + lg[3] + lg[4]) * R(0.2);
  const R n1 = (lg[1] - lg[3]) * R(0.5);
  const R n2 = (lg[2] - lg[4]) * R(0.5);
  const R n3 = (R(-4) * lg[0] + lg[1] + lg[2] + lg[3] + lg[4]) * R(0.05);
  lX += sgn * (sig * n0 + ux * n1 + uy * n2 + (b + R(4) * (R(1) - sig)) * n3);
  lux += sgn * X * n1;
  luy += sgn * X * n2;
  lb += sgn * X * n3;
  lsig += sgn * X * (n0 - R(4) * n3);
}

// Reaction sensitivities: ds_c/dc, ds_c/dtheta, and S_T's.
template <typename R>
struct ReactAdj {
  R s_c, S_T, ehs, dsc_dc, dsc_dth;
};

// Tape of the CL reaction (Eqs. 12-17 as the forward step computes them,
// Tafel or Butler-Volmer, printed or physical heat) and its derivatives:
// s_c = -(c - c_eq) expm1(-kappa), c_eq = exp(alpha_sum F eta / (R T)) with
// Butler-Volmer (0 with Tafel), S_T = 4 F C_ref s_c ehs / (rho c_p).  With
// the printed heat ehs = eta + T dU0/dT = V - U0(0) does not depend on T;
// with the physical heat ehs = -eta + T dU0/dT has dehs/dT = 2 dU0/dT, which
// the callers add to the temperature adjoint.

template <typename R, typename K>
__device__ __forceinline__ ReactAdj<R> reaction_tape(R theta, R c, R rhocp, const K& k) {
  const R T = k.T_in + theta;
  const R iT = R(1) / T;
  const R eta = k.V_op - (k.U0_slope * T + k.U0_icept);
  const R kappa = exp(k.ln_k0 - k.E_over_R * (iT - k.inv_T_arrh) - k.aF_over_R * eta * iT);
  const R em = expm1(-kappa);
  const R ceq = k.bv ? exp(k.aFsum_over_R * eta * iT) : R(0);
  ReactAdj<R> r;
  r.s_c = -(c - ceq) * em;
  r.ehs = ((k.flags & F_PHYSICAL_HEAT) ? -eta : eta) + T * k.U0_slope;
  r.S_T = k.four_f_cref * r.s_c * r.ehs / rhocp;
  // dE/dT of the exponent E = ln_k0 - E/R (1/T - 1/T0) - aF/R eta / T, with
  // deta/dT = -U0_slope; dc_eq/dT = -c_eq alpha_sum F/R (U0_slope / T + eta / T^2).
  const R dE = k.E_over_R * iT * iT + k.aF_over_R * k.U0_slope * iT + k.aF_over_R * eta * iT * iT;
  r.dsc_dc = -em;
  r.dsc_dth = (c - ceq) * (em + R(1)) * kappa * dE;
  if (k.bv) r.dsc_dth -= em * ceq * k.aFsum_over_R * (k.U0_slope * iT + eta * iT * iT);
  return r;
}

// Tape of the thin-film reaction (surface_reaction: the populations g_t, g_c
// that cross the reactive wall, wall values g / a with a = (4 + b) / 20)
// and its derivatives with respect to the wall temperature T, g_c and a_c.
template <typename R>
struct FilmTape {
  R a_t, T, s, S_T, ehs, em, ds_dT, ds_dac, dehs_dT;
};

template <typename R>
__device__ __forceinline__ FilmTape<R> film_tape(R g_t, R g_c, const Mat<R>& m, const Consts<R>& k) {
  FilmTape<R> f;
  f.a_t = (R(4) + m.bT) / R(20);
  const R a_c = (R(4) + m.bC) / R(20);
  f.T = k.T_in + g_t / f.a_t;
  const R iT = R(1) / f.T;
  const R eta = k.V_op - (k.U0_slope * f.T + k.U0_icept);
  const R kappa_a =
      exp(k.ln_k0 + k.ln_thin - k.E_over_R * (iT - k.inv_T_arrh) - k.aF_over_R * eta * iT) / a_c;
  const R ceq = k.bv ? exp(k.aFsum_over_R * eta * iT) : R(0);
  f.em = expm1(-kappa_a);
  f.s = -(g_c - a_c * ceq) * f.em;
  const bool phys = k.flags & F_PHYSICAL_HEAT;
  f.ehs = (phys ? -eta : eta) + f.T * k.U0_slope;
  f.S_T = k.four_f_cref * f.s * f.ehs / m.rhocp;
  // ds/dkappa = (g_c - a_c c_eq)(em + 1); dkappa/dT = kappa dE/dT as in the
  // volumetric tape; ds/dc_eq = a_c em with dc_eq/dT as there
  const R dE = k.E_over_R * iT * iT + k.aF_over_R * k.U0_slope * iT + k.aF_over_R * eta * iT * iT;
  const R ds_dk = (g_c - a_c * ceq) * (f.em + R(1));
  f.ds_dT = ds_dk * kappa_a * dE;
  if (k.bv) f.ds_dT -= a_c * f.em * ceq * k.aFsum_over_R * (k.U0_slope * iT + eta * iT * iT);
  f.ds_dac = -ds_dk * kappa_a / a_c + ceq * f.em;
  f.dehs_dT = phys ? R(2) * k.U0_slope : R(0);
  return f;
}

// Transpose of the film's update of the two populations, g_t += sigma S_T
// and g_c -= s: given the adjoints l13, l18 of the updated values, returns
// those of the incoming ones in place and adds the material adjoints.
// ls, le: adjoints of s and of the heat factor from other uses (the seed
// of J takes ls = its weight).
template <typename R>
__device__ __forceinline__ void film_adj(const FilmTape<R>& f, const Mat<R>& m, const Consts<R>& k, R ls, R& l13,
                                         R& l18, MatAdj<R>& ma) {
  const R sg = (k.flags & F_SIGMA_ENERGY) ? m.sig : R(1);
  const R irc = R(1) / m.rhocp;
  const R lST = sg * l13;
  if (k.flags & F_SIGMA_ENERGY) ma.sig += f.S_T * l13;
  ls += lST * k.four_f_cref * f.ehs * irc - l18;
  const R lehs = lST * k.four_f_cref * f.s * irc;
  ma.rhocp += -lST * f.S_T * irc;
  const R lT = ls * f.ds_dT + lehs * f.dehs_dT;
  l13 += lT / f.a_t;
  l18 += -ls * f.em;
  // T = T_in + g_t / a_t, a = (4 + b) / 20
  ma.bT += -lT * (f.T - k.T_in) / f.a_t * R(0.05);
  ma.bC += ls * f.ds_dac * R(0.05);
}

// Collision adjoint of one node.  In: pre-collision f, material, adjoint of
// the post-collision populations la.  Out: adjoint of the pre-collision
// populations mu; material adjoints accumulated in ma.
// With the heat-capacity ratio (EXT) the temperature lattice conserves
// sigma theta: theta = sum g_T / sigma, the rest moment takes sigma S_T, the
// energy moment relaxes with b_T + 4 (1 - sigma); the adjoint of theta is
// then divided by sigma onto the populations and its sigma part goes to ma.
template <typename R, bool EXT = false>
__device__ __forceinline__ void collide_adj(const R (&f)[19], const Mat<R>& mt, const Consts<R>& k, bool cl,
                                            const R (&la)[19], R (&mu)[19], MatAdj<R>& ma) {
  const MacroTape<R> t = flow_macros_tape<R, EXT>(f, mt, k);
  R lux = R(0), luy = R(0);
#pragma unroll
  for (int i = 0; i < 19; ++i) mu[i] = R(0);

  // ---- scalars (reverse of the D2Q5 collisions and the CL source) ----
  const bool sigma = EXT && (k.flags & F_SIGMA_ENERGY);
  const R thsum = f[9] + f[10] + f[11] + f[12] + f[13];
  const R th = sigma ? thsum / mt.sig : thsum;
  const R c = f[14] + f[15] + f[16] + f[17] + f[18];
  R ln0T = R(0);  // sigma: adjoint of the conserved temperature moment, apart from theta's
  ReactAdj<R> rx{};
  if (cl) rx = reaction_tape(th, c, mt.rhocp, k);
  const R srcT = cl ? rx.S_T : R(0), srcC = cl ? -rx.s_c : R(0);
  const R q1 = R(1.2679491924311228);
  const R q3 = R(0.9282032302755092);
  R lsrc[2], lX[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const R* a = la + 9 + 5 * s;
    const R* g = f + 9 + 5 * s;
    const R X = s == 0 ? th : c;
    const R b = s == 0 ? (sigma ? mt.bT + R(4) * (R(1) - mt.sig) : mt.bT) : mt.bC;
    const R src = s == 0 ? srcT : srcC;
    // g* = N^-1 n*: adjoint of n* is (N a) / (5, 2, 2, 20, 4)
    // Divided (not multiplied by fl(0.2)): the uniform component of the
    // adjoint is carried unchanged, without a relative 1.5e-8 gain per step.
    const R ln0 = (a[0] + a[1] + a[2] + a[3] + a[4]) / R(5);
    const R ln1 = (a[1] - a[3]) * R(0.5);
    const R ln2 = (a[2] - a[4]) * R(0.5);
    const R ln3 = (R(-4) * a[0] + a[1] + a[2] + a[3] + a[4]) * R(0.05);
    const R ln4 = (a[1] - a[2] + a[3] - a[4]) * R(0.25);
    const R lb = q3 * X * ln3 + src * ln3;
    if (sigma && s == 0) {  // n0 = sum g_T + sigma S_T; b = b_T + 4 (1 - sigma)
      ln0T = ln0;
      lX[s] = q1 * t.ux * ln1 + q1 * t.uy * ln2 + q3 * b * ln3;
      lsrc[s] = mt.sig * ln0 + b * ln3;
      ma.sig += src * ln0 - R(4) * lb;
    } else {
      lX[s] = ln0 + q1 * t.ux * ln1 + q1 * t.uy * ln2 + q3 * b * ln3;
      lsrc[s] = ln0 + b * ln3;
    }
    if (s == 0) ma.bT += lb; else ma.bC += lb;
    lux += q1 * X * ln1;
    luy += q1 * X * ln2;
    const R m1 = (R(1) - q1) * ln1, m2 = (R(1) - q1) * ln2, m3 = (R(1) - q3) * ln3, m4 = (R(1) - q3) * ln4;
    R* o = mu + 9 + 5 * s;
    o[0] = R(-4) * m3;
    o[1] = m1 + m3 + m4;
    o[2] = m2 + m3 - m4;
    o[3] = -m1 + m3 + m4;
    o[4] = -m2 + m3 - m4;
    (void)g;
  }
  if (cl) {
    // src_T = S_T(theta, c, rhocp), src_C = -s_c(theta, c)
    const R lST = lsrc[0], lSC = lsrc[1];
    const R irc = R(1) / mt.rhocp;
    const R lsc = -lSC + k.four_f_cref * rx.ehs * irc * lST;
    ma.rhocp += -rx.S_T * irc * lST;
    lX[1] += rx.dsc_dc * lsc;
    lX[0] += rx.dsc_dth * lsc;
    if (k.flags & F_PHYSICAL_HEAT) lX[0] += k.four_f_cref * rx.s_c * R(2) * k.U0_slope * irc * lST;
  }
  if (sigma) {  // theta = sum g_T / sigma
    const R isg = R(1) / mt.sig;
    ma.sig += -th * isg * lX[0];
    lX[0] = ln0T + lX[0] * isg;
  }
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    mu[9 + i] += lX[0];
    mu[14 + i] += lX[1];
  }

  // ---- flow (reverse of the MRT collision with porous forcing) ----
  // f* = M^-1 m*, m* = (1 - S) M f + S m_eq + (1 - S/2) G, M^-1 = M^T
  // diag(M M^T)^-1: the adjoint of m* is M la times the constants
  // 1 / diag(M M^T), and the part that goes back through M f is M^T of
  // (1 - S) times it (integer coefficients, no division).
  R lms[9];
  m_times(la, lms);
  const R se = k.s_e, sq = k.s_q;
  const R s[9] = {se, se, se, R(0), sq, R(0), sq, se, se};
  R lm[9], lme[9], lG[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    lms[i] *= inv_mmt<R>(i);
    lm[i] = (R(1) - s[i]) * lms[i];
    lme[i] = s[i] * lms[i];
    lG[i] = (R(1) - R(0.5) * s[i]) * lms[i];
  }
  lme[0] = R(0);  // the density-moment equilibrium is a constant
  const R iphi = t.iphi;
  const R uF = t.ux * t.Fx + t.uy * t.Fy;
  // G(u, F, phi)
  const R luF = R(6) * iphi * (lG[1] - lG[2]);
  R lFx = lG[3] - lG[4] + R(2) * t.ux * iphi * lG[7] + t.uy * iphi * lG[8] + t.ux * luF;
  R lFy = lG[5] - lG[6] - R(2) * t.uy * iphi * lG[7] + t.ux * iphi * lG[8] + t.uy * luF;
  lux += R(2) * t.Fx * iphi * lG[7] + t.Fy * iphi * lG[8] + t.Fx * luF;
  luy += R(-2) * t.Fy * iphi * lG[7] + t.Fx * iphi * lG[8] + t.Fy * luF;
  const R liphi_G = R(6) * uF * (lG[1] - lG[2]) + R(2) * (t.ux * t.Fx - t.uy * t.Fy) * lG[7] +
                    (t.ux * t.Fy + t.uy * t.Fx) * lG[8];
  ma.phi += -iphi * iphi * liphi_G;
  // meq(p, u, phi)
  R lp = R(0);
  meq_adj(t.p, t.ux, t.uy, mt.phi, iphi, lme, lp, lux, luy, ma.phi);
  // m = M f
  R lfm[9];
  mt_times(lm, lfm);
#pragma unroll
  for (int i = 0; i < 9; ++i) mu[i] += lfm[i];
  flow_macros_adj<R, EXT>(t, mt, k, lux, luy, lp, lFx, lFy, mu, ma);
}

// Adjoint of the boundary-column extrapolation of node b fed by node xp.
// pre_xp: pulled populations of xp; mu_b: adjoint of the boundary node's
// pre-collision populations.  Adds to mu_xp and to the material adjoints of
// xp (maxp) and of b (mab).
// EXT: also the pressure-driven inlet (p_in fixed, u taken from xp) and the
// heat-capacity ratio in the inlet's temperature extrapolation.
template <typename R, bool EXT = false>
__device__ __forceinline__ void boundary_adj(const R (&pre_xp)[19], const Mat<R>& mxp, const Mat<R>& mb,
                                             const Consts<R>& k, bool inlet, R ubx, R uby, const R (&mu_b)[19],
                                             R (&mu_xp)[19], MatAdj<R>& maxp, MatAdj<R>& mab) {
  const MacroTape<R> t = flow_macros_tape<R, EXT>(pre_xp, mxp, k);
  const bool pressure = EXT && inlet && (k.flags & F_PRESSURE_INLET);
#pragma unroll
  for (int i = 0; i < 19; ++i) mu_xp[i] += mu_b[i];  // identity part (scalars at the outlet: a copy)
  R ldm[9];
  m_times(mu_b, ldm);
#pragma unroll
  for (int i = 0; i < 9; ++i) ldm[i] *= inv_mmt<R>(i);
  ldm[0] = R(0);
  const R iphi_b = R(1) / mb.phi;
  R lp1 = R(0), lux1 = R(0), luy1 = R(0);
  // + meq(pb, ub; phi_b): inlet pb = p1 (ub fixed); outlet pb = p_out, ub = u1.
  R dumx = R(0), dumy = R(0);
  if (pressure) {  // pb = p_in, ub = u1
    R dp = R(0);
    meq_adj(k.p_in, t.ux, t.uy, mb.phi, iphi_b, ldm, dp, lux1, luy1, mab.phi);
  } else if (inlet) {
    meq_adj(t.p, ubx, uby, mb.phi, iphi_b, ldm, lp1, dumx, dumy, mab.phi);
  } else {
    R dp = R(0);
    meq_adj(k.p_out, t.ux, t.uy, mb.phi, iphi_b, ldm, dp, lux1, luy1, mab.phi);
  }
  // - meq(p1, u1; phi_xp)
  R nldm[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) nldm[i] = -ldm[i];
  meq_adj(t.p, t.ux, t.uy, mxp.phi, t.iphi, nldm, lp1, lux1, luy1, maxp.phi);
  if (inlet) {
    const bool sigma = EXT && (k.flags & F_SIGMA_ENERGY);
    const R th1sum = pre_xp[9] + pre_xp[10] + pre_xp[11] + pre_xp[12] + pre_xp[13];
    const R th1 = sigma ? th1sum / mxp.sig : th1sum;
    const R c1 = pre_xp[14] + pre_xp[15] + pre_xp[16] + pre_xp[17] + pre_xp[18];
    R lth1 = R(0), lc1 = R(0), dX = R(0);
    // + geq(0, ub; bT_b): no dependence.  - geq(theta1, u1; bT_xp)
    if (sigma) {
      geq_adj_sig(th1, t.ux, t.uy, mxp.bT, mxp.sig, R(-1), mu_b + 9, lth1, lux1, luy1, maxp.bT, maxp.sig);
      const R isg = R(1) / mxp.sig;  // theta1 = sum g_T / sigma
      maxp.sig += -th1 * isg * lth1;
      lth1 *= isg;
    } else {
      geq_adj(th1, t.ux, t.uy, mxp.bT, R(-1), mu_b + 9, lth1, lux1, luy1, maxp.bT);
    }
    // + geq(c_in, ub; bC_b): ub = u1 with the pressure-driven inlet
    if (pressure)
      geq_adj(k.c_in, t.ux, t.uy, mb.bC, R(1), mu_b + 14, dX, lux1, luy1, mab.bC);
    else
      geq_adj(k.c_in, ubx, uby, mb.bC, R(1), mu_b + 14, dX, dumx, dumy, mab.bC);
    // - geq(c1, u1; bC_xp)
    geq_adj(c1, t.ux, t.uy, mxp.bC, R(-1), mu_b + 14, lc1, lux1, luy1, maxp.bC);
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      mu_xp[9 + i] += lth1;
      mu_xp[14 + i] += lc1;
    }
  }
  flow_macros_adj<R, EXT>(t, mxp, k, lux1, luy1, lp1, R(0), R(0), mu_xp, maxp);
}

}  // namespace lbm
