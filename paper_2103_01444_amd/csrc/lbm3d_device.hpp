// Three-dimensional coupled update: D3Q19 flow + two D3Q7 scalar lattices.
//
// The paper's D2Q9 MRT (density moment relaxed at 1/tau) relaxes all even
// moments at s+ = 1/tau and all non-conserved odd moments at
// s- = 8(2 - s+)/(8 - s+); the momentum moment's rate is immaterial with the
// half-force velocity of Eq. 8.  It is a two-rate collision on the
// symmetric / antisymmetric parts of each opposite pair, and the 3D lattice
// keeps exactly those rates.  Likewise the D2Q5 MRT of Eq. 10 (odd rate
// 6/(3+sqrt3), even rate 6/(3+2sqrt3)); its b = 20 sqrt3 alpha - 4 is the
// rest weight a = sqrt3 alpha of each moving D3Q7 population.
//
// Storage: 33 planes (19 flow, 7 theta, 7 c), each [nz][ny][pitch], x
// fastest; the flow rest population is stored as f0 - rho0.  Planes come in
// opposite pairs (1,2), (3,4), ... so pair p holds planes 2p+1 and 2p+2.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_device.hpp"

namespace lbm3 {

using lbm::F_BODY_FORCE;
using lbm::F_NO_REACTION;
using lbm::F_PERIODIC_X;
using lbm::F_PERIODIC_Y;
using lbm::MAT_FULL;
using lbm::MAT_LAYERED;
using lbm::MAT_PHI;

constexpr uint32_t F_PERIODIC_Z = 16u;

// D3Q19 (planes 0-18), D3Q7 temperature (19-25), D3Q7 O2 (26-32).
constexpr int EX[33] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0,
                        0, 1, -1, 0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0};
constexpr int EY[33] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1,
                        0, 0, 0, 1, -1, 0, 0, 0, 0, 0, 1, -1, 0, 0};
constexpr int EZ[33] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1,
                        0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 0, 1, -1};
constexpr int OPP[33] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17,
                         19, 21, 20, 23, 22, 25, 24, 26, 28, 27, 30, 29, 32, 31};

template <typename R>
struct Consts3 {
  int32_t nx, ny, nz, pitch, nz_ch, z_cl0;
  uint32_t flags;
  int32_t plane;  // pitch * ny * nz elements
  int32_t ty;     // y rows per chunk of the launch order
  int32_t bv;     // nonzero: Butler-Volmer kinetics
  R s_plus, s_minus, nu, u_in_coef, ax, ay;
  R phi_gdl, invk_gdl, d_gdl, D_f, kc_inv, deff_ratio;
  R k_f, k_s, rhocp_f, rhocp_s, alpha_scale;
  R T_in, c_in, V_op, U0_slope, U0_icept, ln_k0, E_over_R, inv_T_arrh, aF_over_R, four_f_cref;
  R aFsum_over_R;  // (alpha_a + alpha_c) F / R, Butler-Volmer only
};

template <typename R>
struct Mat3 {
  R phi, invk, d, sqk, fphi, l0, l1, aT, aC, rhocp;
};

template <typename R, int MAT>
__device__ __forceinline__ Mat3<R> material(const Consts3<R>& k, const R* __restrict__ phi_f,
                                            const R* __restrict__ invk_f, const R* __restrict__ d_f, int x, int y,
                                            int z) {
  R phi, invk, d;
  const bool porous = z >= k.nz_ch;
  if constexpr (MAT == MAT_LAYERED) {
    phi = porous ? k.phi_gdl : R(1);
    invk = porous ? k.invk_gdl : R(0);
    d = porous ? k.d_gdl : k.D_f;
  } else {
    const int cell = (z * k.ny + y) * k.pitch + x;
    phi = phi_f[cell];
    if constexpr (MAT == MAT_PHI) {
      const R om = R(1) - phi;
      invk = om * om * k.kc_inv / (phi * phi * phi);
      d = (porous && k.deff_ratio > R(0)) ? k.deff_ratio * k.D_f : phi * sqrt(phi) * k.D_f;
    } else {
      invk = invk_f[cell];
      d = d_f[cell];
    }
  }
  Mat3<R> m;
  m.phi = phi;
  m.invk = invk;
  m.d = d;
  m.sqk = sqrt(invk);
  m.fphi = R(0.143) / (phi * sqrt(phi));
  m.l0 = R(0.5) + phi * k.nu * invk * R(0.25);
  m.l1 = phi * m.fphi * m.sqk * R(0.5);
  m.rhocp = phi * k.rhocp_f + (R(1) - phi) * k.rhocp_s;
  const R alpha = (k.k_f * phi + k.k_s * (R(1) - phi)) * k.alpha_scale / m.rhocp;
  const R s3 = R(1.7320508075688772935);
  m.aT = s3 * alpha;
  m.aC = s3 * d;
  return m;
}

// UNIFORM: a wavefront whose nodes all lie one node or more inside the
// lattice folds each population's plane and neighbour shift into a
// wave-uniform buffer base (scalar registers) and adds one shared 32-bit
// lane offset (used by the reverse step).
template <typename R, bool UNIFORM = false>
__device__ __forceinline__ void pull(const R* __restrict__ src, const Consts3<R>& k, int x, int y, int z,
                                     R (&f)[33]) {
  const int row = k.pitch * k.ny;
  if (UNIFORM && __all(x >= 1 && x <= k.nx - 2 && y >= 1 && y <= k.ny - 2 && z >= 1 && z <= k.nz - 2)) {
    const uint32_t ob = uint32_t(z * row + y * k.pitch + x) * uint32_t(sizeof(R));
#pragma unroll
    for (int q = 0; q < 33; ++q)
      f[q] = lbm::buffer_load<R, 2>(
          src + (int64_t(q) * k.plane - int64_t(EZ[q]) * row - int64_t(EY[q]) * k.pitch - EX[q]), ob);
    return;
  }
  const bool px = k.flags & F_PERIODIC_X, py = k.flags & F_PERIODIC_Y, pz = k.flags & F_PERIODIC_Z;
#pragma unroll
  for (int q = 0; q < 33; ++q) {
    int xs = x - EX[q], ys = y - EY[q], zs = z - EZ[q];
    if (px) xs = xs < 0 ? xs + k.nx : (xs >= k.nx ? xs - k.nx : xs);
    if (py) ys = ys < 0 ? ys + k.ny : (ys >= k.ny ? ys - k.ny : ys);
    if (pz) zs = zs < 0 ? zs + k.nz : (zs >= k.nz ? zs - k.nz : zs);
    const bool in = (unsigned)xs < (unsigned)k.nx && (unsigned)ys < (unsigned)k.ny && (unsigned)zs < (unsigned)k.nz;
    const int off = in ? (q * k.plane + zs * row + ys * k.pitch + xs) : (OPP[q] * k.plane + z * row + y * k.pitch + x);
    f[q] = __builtin_nontemporal_load(src + off);
  }
}

// Pull of the planes [Q0, Q1) only, into f[0 .. Q1 - Q0) (as pull).  A
// wavefront whose nodes all lie inside the lattice by one node or more
// loads through wave-uniform buffer bases (one 32-bit lane offset for all
// planes: no per-load 64-bit address registers).
template <typename R, int Q0, int Q1>
__device__ __forceinline__ void pull_range(const R* __restrict__ src, const Consts3<R>& k, int x, int y, int z,
                                           R* f) {
  const int row = k.pitch * k.ny;
  if (__all(x >= 1 && x <= k.nx - 2 && y >= 1 && y <= k.ny - 2 && z >= 1 && z <= k.nz - 2)) {
    const uint32_t ob = uint32_t(z * row + y * k.pitch + x) * uint32_t(sizeof(R));
#pragma unroll
    for (int q = Q0; q < Q1; ++q)
      f[q - Q0] = lbm::buffer_load<R, 2>(
          src + (int64_t(q) * k.plane - int64_t(EZ[q]) * row - int64_t(EY[q]) * k.pitch - EX[q]), ob);
    return;
  }
  const bool px = k.flags & F_PERIODIC_X, py = k.flags & F_PERIODIC_Y, pz = k.flags & F_PERIODIC_Z;
#pragma unroll
  for (int q = Q0; q < Q1; ++q) {
    int xs = x - EX[q], ys = y - EY[q], zs = z - EZ[q];
    if (px) xs = xs < 0 ? xs + k.nx : (xs >= k.nx ? xs - k.nx : xs);
    if (py) ys = ys < 0 ? ys + k.ny : (ys >= k.ny ? ys - k.ny : ys);
    if (pz) zs = zs < 0 ? zs + k.nz : (zs >= k.nz ? zs - k.nz : zs);
    const bool in = (unsigned)xs < (unsigned)k.nx && (unsigned)ys < (unsigned)k.ny && (unsigned)zs < (unsigned)k.nz;
    const int off = in ? (q * k.plane + zs * row + ys * k.pitch + xs) : (OPP[q] * k.plane + z * row + y * k.pitch + x);
    f[q - Q0] = __builtin_nontemporal_load(src + off);
  }
}

template <typename R>
struct Macro3 {
  R ux, uy, uz, p, Fx, Fy, Fz;
};

// Eq. 8 velocity, Eq. 7 drag, 3D pressure relation of the porous equilibrium.
template <typename R, int N>
__device__ __forceinline__ Macro3<R> flow_macros(const R (&f)[N], const Mat3<R>& m, const Consts3<R>& k) {
  static_assert(N >= 19, "the 19 flow populations come first");
  R vx = R(0), vy = R(0), vz = R(0), s = R(0);
#pragma unroll
  for (int q = 1; q < 19; ++q) {
    vx += R(EX[q]) * f[q];
    vy += R(EY[q]) * f[q];
    vz += R(EZ[q]) * f[q];
    s += f[q];
  }
  const bool body = k.flags & F_BODY_FORCE;
  if (body) {
    vx += R(0.5) * m.phi * k.ax;
    vy += R(0.5) * m.phi * k.ay;
  }
  const R vm = sqrt(vx * vx + vy * vy + vz * vz);
  const R den = m.l0 + sqrt(m.l0 * m.l0 + m.l1 * vm);
  Macro3<R> o;
  o.ux = vx / den;
  o.uy = vy / den;
  o.uz = vz / den;
  const R u2 = o.ux * o.ux + o.uy * o.uy + o.uz * o.uz;
  const R drag = m.phi * (k.nu * m.invk + m.fphi * m.sqk * sqrt(u2));
  o.Fx = -drag * o.ux;
  o.Fy = -drag * o.uy;
  o.Fz = -drag * o.uz;
  if (body) {
    o.Fx += m.phi * k.ax;
    o.Fy += m.phi * k.ay;
  }
  const R iphi = R(1) / m.phi;
  o.p = (s - R(0.5) * u2 * iphi) * R(0.5) * iphi;
  return o;
}

template <typename R>
__device__ __forceinline__ R weight(int q) {
  return q == 0 ? R(1.0 / 3.0) : (q < 7 ? R(1.0 / 18.0) : R(1.0 / 36.0));
}

// Add sgn * f_eq(p, u; phi) (shifted rest population) to f[0..18].
template <typename R>
__device__ __forceinline__ void add_feq(R p, R ux, R uy, R uz, R phi, R sgn, R* f) {
  const R iphi = R(1) / phi;
  const R u2 = ux * ux + uy * uy + uz * uz;
  f[0] += sgn * (R(-2) * phi * p - R(0.5) * u2 * iphi);
#pragma unroll
  for (int q = 1; q < 19; ++q) {
    const R w = weight<R>(q);
    const R eu = R(EX[q]) * ux + R(EY[q]) * uy + R(EZ[q]) * uz;
    f[q] += sgn * (R(3) * w * phi * p + w * (R(3) * eu + R(4.5) * eu * eu * iphi - R(1.5) * u2 * iphi));
  }
}

// Add sgn * g_eq(X, u; a) to g[0..6].
template <typename R>
__device__ __forceinline__ void add_geq(R X, R ux, R uy, R uz, R a, R sgn, R* g) {
  g[0] += sgn * X * (R(1) - R(6) * a);
#pragma unroll
  for (int q = 1; q < 7; ++q) {
    const R eu = R(EX[q]) * ux + R(EY[q]) * uy + R(EZ[q]) * uz;
    g[q] += sgn * X * (a + R(0.5) * eu);
  }
}

template <typename R>
__device__ __forceinline__ R inlet_velocity(const Consts3<R>& k, int y, int z) {
  const R yc = R(y) + R(0.5), zc = R(z) + R(0.5);
  return k.u_in_coef * yc * (R(k.ny) - yc) * zc * (R(k.nz_ch) - zc);
}

// Boundary columns (non-equilibrium extrapolation, as in 2D), flow part: the
// 19 flow populations f[0..18] of the column next to the boundary become
// the boundary node's; returns that column's macroscopic fields (the scalar
// part of the inlet needs them).
template <typename R, int N>
__device__ __forceinline__ Macro3<R> boundary_flow(R (&f)[N], const Consts3<R>& k, int y, int z, bool inlet,
                                                   const Mat3<R>& mp, const Mat3<R>& mb) {
  const Macro3<R> a = flow_macros(f, mp, k);
  if (inlet) {
    const R ub = inlet_velocity(k, y, z);
    add_feq(a.p, ub, R(0), R(0), mb.phi, R(1), f);
    add_feq(a.p, a.ux, a.uy, a.uz, mp.phi, R(-1), f);
  } else {
    add_feq(R(0), a.ux, a.uy, a.uz, mb.phi, R(1), f);
    add_feq(a.p, a.ux, a.uy, a.uz, mp.phi, R(-1), f);
  }
  return a;
}

// Scalar part of the inlet column: g[0..6] temperature rise, g[7..13] O2 of
// the column next to the inlet; a: that column's macroscopic fields.  (At
// the outlet the scalars are copies of that column.)
template <typename R>
__device__ __forceinline__ void boundary_scalars_inlet(R* g, const Consts3<R>& k, int y, int z, const Macro3<R>& a,
                                                       const Mat3<R>& mp, const Mat3<R>& mb) {
  const R ub = inlet_velocity(k, y, z);
  R th = R(0), c = R(0);
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    th += g[q];
    c += g[7 + q];
  }
  add_geq(R(0), ub, R(0), R(0), mb.aT, R(1), g);
  add_geq(th, a.ux, a.uy, a.uz, mp.aT, R(-1), g);
  add_geq(k.c_in, ub, R(0), R(0), mb.aC, R(1), g + 7);
  add_geq(c, a.ux, a.uy, a.uz, mp.aC, R(-1), g + 7);
}

template <typename R>
__device__ __forceinline__ void boundary_column(R (&f)[33], const Consts3<R>& k, int y, int z, bool inlet,
                                                const Mat3<R>& mp, const Mat3<R>& mb) {
  const Macro3<R> a = boundary_flow(f, k, y, z, inlet, mp, mb);
  if (inlet) boundary_scalars_inlet(f + 19, k, y, z, a, mp, mb);
}

template <typename R, int MAT>
__device__ __forceinline__ Mat3<R> pre_collision(const R* __restrict__ src, const Consts3<R>& k,
                                                 const R* __restrict__ phi_f, const R* __restrict__ invk_f,
                                                 const R* __restrict__ d_f, int x, int y, int z, R (&f)[33]) {
  const bool open = !(k.flags & F_PERIODIC_X);
  const bool inlet = open && x == 0 && z < k.nz_ch;
  const bool outlet = open && x == k.nx - 1;
  const int xp = inlet ? 1 : (outlet ? k.nx - 2 : x);
  pull(src, k, xp, y, z, f);
  const Mat3<R> mp = material<R, MAT>(k, phi_f, invk_f, d_f, xp, y, z);
  if (!(inlet || outlet)) return mp;
  Mat3<R> mb = material<R, MAT>(k, phi_f, invk_f, d_f, x, y, z);
  boundary_column(f, k, y, z, inlet, mp, mb);
  if (outlet) {  // scalar material of column nx-2 at the outlet (as in 2D)
    mb.aT = mp.aT;
    mb.aC = mp.aC;
    mb.rhocp = mp.rhocp;
  }
  return mb;
}

using lbm::reaction;  // the CL reaction of Eqs. 12-17 (shared with 2D)

// Two-rate collision of the 19 flow populations with Guo's porous forcing;
// a: the node's macroscopic fields.
template <typename R>
__device__ __forceinline__ void collide_flow(R* f, const Macro3<R>& a, const Mat3<R>& mt, const Consts3<R>& k) {
  const R iphi = R(1) / mt.phi;
  const R u2 = a.ux * a.ux + a.uy * a.uy + a.uz * a.uz;
  const R uF = a.ux * a.Fx + a.uy * a.Fy + a.uz * a.Fz;
  const R sp = k.s_plus, sm = k.s_minus;
  const R hp = R(1) - R(0.5) * sp, hm = R(1) - R(0.5) * sm;
  {  // rest population: even only
    const R eq0 = R(-2) * mt.phi * a.p - R(0.5) * u2 * iphi;
    const R F0 = R(1.0 / 3.0) * (R(-3) * uF * iphi);
    f[0] = f[0] - sp * (f[0] - eq0) + hp * F0;
  }
#pragma unroll
  for (int pr = 0; pr < 9; ++pr) {
    const int i = 2 * pr + 1, o = i + 1;
    const R w = weight<R>(i);
    const R eu = R(EX[i]) * a.ux + R(EY[i]) * a.uy + R(EZ[i]) * a.uz;
    const R eF = R(EX[i]) * a.Fx + R(EY[i]) * a.Fy + R(EZ[i]) * a.Fz;
    const R eq_even = R(3) * w * mt.phi * a.p + w * (R(4.5) * eu * eu * iphi - R(1.5) * u2 * iphi);
    const R eq_odd = R(3) * w * eu;
    const R F_even = w * (R(9) * eu * eF * iphi - R(3) * uF * iphi);
    const R F_odd = R(3) * w * eF;
    const R fp = R(0.5) * (f[i] + f[o]), fm = R(0.5) * (f[i] - f[o]);
    const R np = fp - sp * (fp - eq_even) + hp * F_even;
    const R nm = fm - sm * (fm - eq_odd) + hm * F_odd;
    f[i] = np + nm;
    f[o] = np - nm;
  }
}

// Two-rate collisions of the scalar lattices g[0..6] (temperature rise) and
// g[7..13] (O2) advected by (ux, uy, uz), with the CL source injected with
// the rest weights.
template <typename R>
__device__ __forceinline__ void collide_scalars(R* gs, R ux, R uy, R uz, const Mat3<R>& mt, const Consts3<R>& k,
                                                bool cl) {
  R srcT = R(0), srcC = R(0);
  R th = R(0), c = R(0);
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    th += gs[q];
    c += gs[7 + q];
  }
  if (cl) {
    const lbm::React<R> r = reaction(th, c, mt.rhocp, k);
    srcT = r.S_T;
    srcC = -r.s_c;
  }
  const R qp = R(0.9282032302755092);  // even rate 6 / (3 + 2 sqrt 3)
  const R qm = R(1.2679491924311228);  // odd rate 6 / (3 + sqrt 3)
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    R* g = gs + 7 * s;
    const R X = s == 0 ? th : c;
    const R aw = s == 0 ? mt.aT : mt.aC;
    const R src = s == 0 ? srcT : srcC;
    R moving = R(0);
#pragma unroll
    for (int pr = 0; pr < 3; ++pr) {
      const int i = 2 * pr + 1, o = i + 1;
      const R eu = R(EX[19 + i]) * ux + R(EY[19 + i]) * uy + R(EZ[19 + i]) * uz;
      const R gp = R(0.5) * (g[i] + g[o]), gm = R(0.5) * (g[i] - g[o]);
      const R np = gp - qp * (gp - X * aw) + src * aw;
      const R nm = gm - qm * (gm - R(0.5) * X * eu);
      g[i] = np + nm;
      g[o] = np - nm;
      moving += g[i] + g[o];
    }
    // Rest population from the conserved sum X + src (in exact arithmetic
    // equal to its own relaxation toward X (1 - 6a) plus src (1 - 6a)):
    // 1 - 6a and a are rounded once per material, the same way at every
    // step of every cell of that material, so the relaxation form would add
    // a fixed relative ~1e-7 of the scalar per step; this form conserves it.
    g[0] = (X + src) - moving;
  }
}

// Two-rate collision of every population of a node (flow with Guo's porous
// forcing; scalars with the CL source injected with the rest weights).
template <typename R>
__device__ __forceinline__ void collide(R (&f)[33], const Mat3<R>& mt, const Consts3<R>& k, bool cl) {
  const Macro3<R> a = flow_macros(f, mt, k);
  collide_flow(f, a, mt, k);
  collide_scalars(f + 19, a.ux, a.uy, a.uz, mt, k, cl);
}

// Store f[0 .. Q1 - Q0) into the planes [Q0, Q1) at element offset o, through
// wave-uniform buffer bases (the 33 planes hold fewer than 2^31 elements).
template <typename R, int Q0, int Q1>
__device__ __forceinline__ void store_range(R* __restrict__ dst, const Consts3<R>& k, int o, const R* f) {
  const uint32_t ob = uint32_t(o) * uint32_t(sizeof(R));
#pragma unroll
  for (int q = Q0; q < Q1; ++q) lbm::buffer_store(dst + int64_t(q) * k.plane, ob, f[q - Q0]);
}

// One time step of node (x, y, z) in two passes: the 19 flow populations
// (pull, boundary extrapolation, collision, store), then the 14 scalar ones
// with the node's velocity, so that at most 19 populations are held at once.
template <typename R, int MAT>
__device__ __forceinline__ void step_node(const R* __restrict__ src, R* __restrict__ dst, const R* __restrict__ phi_f,
                                          const R* __restrict__ invk_f, const R* __restrict__ d_f,
                                          const Consts3<R>& k, int x, int y, int z) {
  const bool open = !(k.flags & F_PERIODIC_X);
  const bool inlet = open && x == 0 && z < k.nz_ch;
  const bool outlet = open && x == k.nx - 1;
  const int xp = inlet ? 1 : (outlet ? k.nx - 2 : x);
  const Mat3<R> mp = material<R, MAT>(k, phi_f, invk_f, d_f, xp, y, z);
  Mat3<R> mt = mp;
  if (inlet || outlet) mt = material<R, MAT>(k, phi_f, invk_f, d_f, x, y, z);
  const int o = (z * k.ny + y) * k.pitch + x;
  Macro3<R> a, nb{};
  {
    R f[19];
    pull_range<R, 0, 19>(src, k, xp, y, z, f);
    if (inlet || outlet) nb = boundary_flow(f, k, y, z, inlet, mp, mt);
    a = flow_macros(f, mt, k);
    collide_flow(f, a, mt, k);
    store_range<R, 0, 19>(dst, k, o, f);
  }
  if (outlet) {  // scalar material of column nx-2 at the outlet
    mt.aT = mp.aT;
    mt.aC = mp.aC;
    mt.rhocp = mp.rhocp;
  }
  R g[14];
  pull_range<R, 19, 33>(src, k, xp, y, z, g);
  if (inlet) boundary_scalars_inlet(g, k, y, z, nb, mp, mt);
  collide_scalars(g, a.ux, a.uy, a.uz, mt, k, z >= k.z_cl0 && !(k.flags & F_NO_REACTION));
  store_range<R, 19, 33>(dst, k, o, g);
}

}  // namespace lbm3
