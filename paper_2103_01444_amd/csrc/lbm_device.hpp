// Device-side building blocks of the coupled D2Q9 / 2 x D2Q5 MRT update.
//
// Storage: 19 population planes (9 flow, 5 temperature rise, 5 O2), each a
// pitched [ny][pitch] array, x fastest.  The flow rest population is stored
// shifted, f0 - rho0, so that FP32 keeps the small pressure-carrying part of
// f0 at full relative precision; every moment below is taken of the shifted
// vector, and the shift cancels from all differences used by the scheme.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

enum MatMode : int { MAT_LAYERED = 0, MAT_PHI = 1, MAT_FULL = 2 };

constexpr uint32_t F_PERIODIC_X = 1u;
constexpr uint32_t F_PERIODIC_Y = 2u;
constexpr uint32_t F_BODY_FORCE = 4u;
constexpr uint32_t F_NO_REACTION = 8u;
constexpr uint32_t F_PRESSURE_INLET = 32u;
constexpr uint32_t F_THIN_CL = 64u;
constexpr uint32_t F_BUOYANCY = 128u;
constexpr uint32_t F_SIGMA_ENERGY = 256u;
constexpr uint32_t F_PHYSICAL_HEAT = 512u;

// Velocity sets of Eq. 2 (planes 0-8) and Eq. 9 (planes 9-13 and 14-18).
constexpr int EX[19] = {0, 1, 0, -1, 0, 1, -1, -1, 1, 0, 1, 0, -1, 0, 0, 1, 0, -1, 0};
constexpr int EY[19] = {0, 0, 1, 0, -1, 1, 1, -1, -1, 0, 0, 1, 0, -1, 0, 0, 1, 0, -1};
constexpr int OPP[19] = {0, 3, 4, 1, 2, 7, 8, 5, 6, 9, 12, 13, 10, 11, 14, 17, 18, 15, 16};

// Per-launch constants, in the kernel's arithmetic type R.
template <typename R>
struct Consts {
  // Population q of node (x, y) is element q * plane + y * pitch + x: planar
  // states have pitch = the padded row length and plane = pitch * ny (plus
  // padding); the batched pool is row-interleaved, plane = the row length
  // and pitch = 19 row lengths.  Per-cell fields use y * pitch + x and exist
  // only in the planar (single-lattice) layout.
  int32_t nx, ny, pitch, ny_ch, y_cl0;
  uint32_t flags;
  int32_t plane;        // stride between population q and q + 1
  int32_t bv;           // nonzero: Butler-Volmer kinetics (anodic branch), else the printed Tafel form
  // flow (Section 2.1)
  R s_e, s_q, nu;       // s_e: rate of rho, e, zeta, pxx, pxy; s_q: energy flux
  R u_in_coef;          // 6 U_avg / H_channel^2
  R ax, ay;             // body force (test mode)
  // materials (Eqs. 7, 18, 19)
  R phi_gdl, invk_gdl, d_gdl, D_f;
  R kc_inv;             // 1 / (0.0067 d_p^2)
  R deff_ratio;         // D_eff / D_f in porous layers; 0 = Bruggeman
  R k_f, k_s, rhocp_f, rhocp_s;
  R alpha_scale;        // lattice alpha = (k [W/(m K)] / 100) / (rho c_p) * dt / dx^2
  // reaction (Eqs. 13-17) and scalar boundary data
  R T_in, c_in, V_op, U0_slope, U0_icept;
  R ln_k0;              // ln(aj0_ref dt / (4 F C_ref))
  R E_over_R, inv_T_arrh, aF_over_R;
  R four_f_cref;        // 4 F C_ref, C / cm^3
  R p_in;               // inlet pressure of the pressure-driven mode
  R p_out;              // outlet pressure
  R aFsum_over_R;       // (alpha_a + alpha_c) F / R, Butler-Volmer only
  R ln_thin;            // ln(film thickness / dx), thin-film CL only
  R bx, by;             // buoyancy: acceleration per kelvin of temperature rise
};

template <typename R>
struct Mat {
  R phi, invk, sqk, fphi, l0, l1, bT, bC, rhocp;
  R sig;  // heat-capacity ratio (rho c_p)_eff / (rho c_p)_f with F_SIGMA_ENERGY, else 1
};

template <typename R>
__device__ __forceinline__ R dsqrt(R a) { return sqrt(a); }

// Porous-medium properties of one cell.  Layered: clear channel (phi = 1,
// 1/K = 0, D = D_f) above the porous rows.  Per-cell porosity: Kozeny-Carman
// permeability (Eq. 7) and Bruggeman or ratio diffusivity (Eq. 18).  Full:
// three given fields.  Thermal diffusivity from Eq. 19 in every mode.
template <typename R, int MAT>
__device__ __forceinline__ void base_fields(const Consts<R>& k, const R* __restrict__ phi_f,
                                            const R* __restrict__ invk_f, const R* __restrict__ d_f, int x, int y,
                                            R& phi, R& invk, R& d) {
  const bool porous = y >= k.ny_ch;
  if constexpr (MAT == MAT_LAYERED) {
    phi = porous ? k.phi_gdl : R(1);
    invk = porous ? k.invk_gdl : R(0);
    d = porous ? k.d_gdl : k.D_f;
  } else {
    const int cell = y * k.pitch + x;
    phi = phi_f[cell];
    if constexpr (MAT == MAT_PHI) {
      const R om = R(1) - phi;
      invk = om * om * k.kc_inv / (phi * phi * phi);
      d = (porous && k.deff_ratio > R(0)) ? k.deff_ratio * k.D_f : phi * dsqrt(phi) * k.D_f;
    } else {
      invk = invk_f[cell];
      d = d_f[cell];
    }
  }
}

template <typename R, int MAT>
__device__ __forceinline__ Mat<R> material(const Consts<R>& k, const R* __restrict__ phi_f,
                                           const R* __restrict__ invk_f,
                                           const R* __restrict__ d_f, int x, int y) {
  R phi, invk, d;
  base_fields<R, MAT>(k, phi_f, invk_f, d_f, x, y, phi, invk, d);
  Mat<R> m;
  m.phi = phi;
  m.invk = invk;
  m.sqk = dsqrt(invk);
  m.fphi = R(0.143) / (phi * dsqrt(phi));
  m.l0 = R(0.5) + phi * k.nu * invk * R(0.25);
  m.l1 = phi * m.fphi * m.sqk * R(0.5);
  m.rhocp = phi * k.rhocp_f + (R(1) - phi) * k.rhocp_s;
  // Eq. 19; with the heat-capacity ratio the lattice carries k_eff / (rho c_p)_f
  // and conserves sigma T
  const bool sigma = k.flags & F_SIGMA_ENERGY;
  const R alpha = (k.k_f * phi + k.k_s * (R(1) - phi)) * k.alpha_scale / (sigma ? k.rhocp_f : m.rhocp);
  m.sig = sigma ? m.rhocp / k.rhocp_f : R(1);
  const R c20s3 = R(34.64101615137754587);  // 20 sqrt(3)
  m.bT = c20s3 * alpha - R(4);
  m.bC = c20s3 * d - R(4);
  return m;
}

// Pull the 19 pre-collision populations of node (x, y) from the
// post-collision state: f_q(x) = f*_q(x - e_q), or f*_opp(q)(x) where the
// link crosses a wall (half-way bounce-back).  Every element of the state is
// read exactly once per step, so on a large lattice the loads carry the
// non-temporal hint (NT): measured on MI355X the 4096x1024 FP32 step drops
// from 118.6 us to 112.6 us with it (streamed lines stop displacing the
// x +- 1 neighbour lines that adjacent wavefronts still need from L2), and
// it is 9 % slower with plain loads in the final kernel (119.1 against
// 109.3 us on one GPU).  The batched sweep of many narrow lattices is the
// other way round: plain loads take it from 182.5 to 175.3 us per step.
//
// Wave-uniform addressing: a base address that is the same for every lane
// of the wavefront is held as a raw buffer resource in scalar registers and
// every lane adds one 32-bit byte offset, so a run of loads at one node (or
// at one neighbour shift) needs no per-lane address arithmetic.  The
// state holds fewer than 2^31 elements, so a node's byte offset inside a
// plane fits 32 bits.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const void* base) {
  // stride 0 (raw), the largest record count, the gfx9 dword-3 format word
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), short(0), -1, 0x00020000);
}

// aux: the instruction's cache-policy bits; 2 is the non-temporal hint.
template <typename R, int AUX>
__device__ __forceinline__ R buffer_load(const R* base, uint32_t byte_off) {
  if constexpr (sizeof(R) == 4) {
    return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b32(buffer_of(base), int(byte_off), 0, AUX));
  } else {
    return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b64(buffer_of(base), int(byte_off), 0, AUX));
  }
}

template <typename R>
__device__ __forceinline__ void buffer_store(R* base, uint32_t byte_off, R v) {
  if constexpr (sizeof(R) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), buffer_of(base), int(byte_off), 0, 0);
  } else {
    using U2 = uint32_t __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, v), buffer_of(base), int(byte_off), 0, 0);
  }
}

//
// UNIFORM: a wavefront whose nodes all lie one node or more inside the
// lattice (no wall link, no periodic wrap) folds each population's plane and
// neighbour shift into a wave-uniform base.  The reverse step, whose
// register-bound collision adjoint leaves little issue slack, gains from it
// (per reverse step of the 1024x256 adjoint 34.3 against 35.0 us, on another
// GPU 33.4 against 34.9 us); the forward kernels run 0.5-1.5 % slower with
// it (A/B on one GPU) and keep the per-lane form.
template <typename R, bool NT = true, bool UNIFORM = false>
__device__ __forceinline__ void pull(const R* __restrict__ src, const Consts<R>& k, int x, int y,
                                     R (&f)[19]) {
  if (UNIFORM && __all(x >= 1 && x <= k.nx - 2 && y >= 1 && y <= k.ny - 2)) {
    const uint32_t ob = uint32_t(y * k.pitch + x) * uint32_t(sizeof(R));
#pragma unroll
    for (int q = 0; q < 19; ++q) {
      f[q] = buffer_load<R, NT ? 2 : 0>(src + (int64_t(q) * k.plane - int64_t(EY[q]) * k.pitch - EX[q]), ob);
    }
    return;
  }
  const bool px = k.flags & F_PERIODIC_X;
  const bool py = k.flags & F_PERIODIC_Y;
#pragma unroll
  for (int q = 0; q < 19; ++q) {
    int xs = x - EX[q];
    int ys = y - EY[q];
    if (px) xs = xs < 0 ? xs + k.nx : (xs >= k.nx ? xs - k.nx : xs);
    if (py) ys = ys < 0 ? ys + k.ny : (ys >= k.ny ? ys - k.ny : ys);
    const bool in = (unsigned)xs < (unsigned)k.nx && (unsigned)ys < (unsigned)k.ny;
    const int off = in ? (q * k.plane + ys * k.pitch + xs) : (OPP[q] * k.plane + y * k.pitch + x);
    if constexpr (NT)
      f[q] = __builtin_nontemporal_load(src + off);
    else
      f[q] = src[off];
  }
}

// Temperature rise of a node from its five temperature populations g (their
// sum is sigma theta with the heat-capacity ratio, theta otherwise).
template <typename R, typename K>
__device__ __forceinline__ R theta_of(const R* g, R sig, const K& k) {
  const R s = g[0] + g[1] + g[2] + g[3] + g[4];
  return (k.flags & F_SIGMA_ENERGY) ? s / sig : s;
}

template <typename R>
struct Macro {
  R ux, uy, p, Fx, Fy;
};

// Eq. 8 velocity recovery, Eq. 7 drag, Section 2.1 pressure relation.  The
// acceleration a (test-mode body force and/or Boussinesq buoyancy b theta,
// theta from this node's temperature populations) enters as phi a in F and
// phi a / 2 in v.
template <typename R>
__device__ __forceinline__ Macro<R> flow_macros(const R (&f)[19], const Mat<R>& m, const Consts<R>& k) {
  R vx = f[1] - f[3] + f[5] - f[6] - f[7] + f[8];
  R vy = f[2] - f[4] + f[5] + f[6] - f[7] - f[8];
  const bool body = k.flags & (F_BODY_FORCE | F_BUOYANCY);
  R ax = R(0), ay = R(0);
  if (k.flags & F_BODY_FORCE) {
    ax = k.ax;
    ay = k.ay;
  }
  if (k.flags & F_BUOYANCY) {
    const R th = theta_of(f + 9, m.sig, k);
    ax += k.bx * th;
    ay += k.by * th;
  }
  if (body) {
    vx += R(0.5) * m.phi * ax;
    vy += R(0.5) * m.phi * ay;
  }
  const R vmag = dsqrt(vx * vx + vy * vy);
  const R den = m.l0 + dsqrt(m.l0 * m.l0 + m.l1 * vmag);
  Macro<R> o;
  o.ux = vx / den;
  o.uy = vy / den;
  const R u2 = o.ux * o.ux + o.uy * o.uy;
  const R drag = m.phi * (k.nu * m.invk + m.fphi * m.sqk * dsqrt(u2));
  o.Fx = -drag * o.ux;
  o.Fy = -drag * o.uy;
  if (body) {
    o.Fx += m.phi * ax;
    o.Fy += m.phi * ay;
  }
  const R s18 = f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
  const R iphi = R(1) / m.phi;
  o.p = R(0.6) * iphi * s18 - R(0.4) * u2 * iphi * iphi;
  return o;
}

// Eq. 5 equilibrium moments minus the rest-state moments (rho0, -4 rho0, 4 rho0, 0...).
template <typename R>
__device__ __forceinline__ void meq_shifted(R p, R ux, R uy, R phi, R (&me)[9]) {
  const R iphi = R(1) / phi;
  const R u2 = ux * ux + uy * uy;
  me[0] = R(0);
  me[1] = R(6) * phi * p + R(3) * u2 * iphi;
  me[2] = R(-9) * phi * p - R(3) * u2 * iphi;
  me[3] = ux;
  me[4] = -ux;
  me[5] = uy;
  me[6] = -uy;
  me[7] = (ux * ux - uy * uy) * iphi;
  me[8] = ux * uy * iphi;
}

// Eq. 3: m = M f.
template <typename R>
__device__ __forceinline__ void moments9(const R (&f)[19], R (&m)[9]) {
  const R a14 = f[1] + f[2] + f[3] + f[4];
  const R a58 = f[5] + f[6] + f[7] + f[8];
  m[0] = f[0] + a14 + a58;
  m[1] = R(-4) * f[0] - a14 + R(2) * a58;
  m[2] = R(4) * f[0] - R(2) * a14 + a58;
  const R jx = f[5] - f[6] - f[7] + f[8];
  const R jy = f[5] + f[6] - f[7] - f[8];
  m[3] = f[1] - f[3] + jx;
  m[4] = R(-2) * (f[1] - f[3]) + jx;
  m[5] = f[2] - f[4] + jy;
  m[6] = R(-2) * (f[2] - f[4]) + jy;
  m[7] = f[1] - f[2] + f[3] - f[4];
  m[8] = f[5] - f[6] + f[7] - f[8];
}

// f = M^-1 m = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4) m.
template <typename R>
__device__ __forceinline__ void inv_moments9(const R (&m)[9], R* f) {
  const R a0 = m[0] * R(1.0 / 9.0), a1 = m[1] * R(1.0 / 36.0), a2 = m[2] * R(1.0 / 36.0);
  const R a3 = m[3] * R(1.0 / 6.0), a4 = m[4] * R(1.0 / 12.0), a5 = m[5] * R(1.0 / 6.0);
  const R a6 = m[6] * R(1.0 / 12.0), a7 = m[7] * R(0.25), a8 = m[8] * R(0.25);
  const R b14 = a0 - a1 - R(2) * a2;
  const R b58 = a0 + R(2) * a1 + a2;
  f[0] = a0 - R(4) * a1 + R(4) * a2;
  f[1] = b14 + a3 - R(2) * a4 + a7;
  f[2] = b14 + a5 - R(2) * a6 - a7;
  f[3] = b14 - a3 + R(2) * a4 + a7;
  f[4] = b14 - a5 + R(2) * a6 - a7;
  f[5] = b58 + a3 + a4 + a5 + a6 + a8;
  f[6] = b58 - a3 - a4 + a5 + a6 - a8;
  f[7] = b58 - a3 - a4 - a5 - a6 + a8;
  f[8] = b58 + a3 + a4 - a5 - a6 - a8;
}

// Eq. 10 scalar equilibrium N^-1 (X, u_x X, u_y X, b X, 0), added with sign
// sgn; with the heat-capacity ratio sig: N^-1 (sig X, u_x X, u_y X,
// (b + 4 (1 - sig)) X, 0) (sig = 1 gives the printed form exactly).
template <typename R>
__device__ __forceinline__ void add_geq(R X, R ux, R uy, R b, R sgn, R* g, R sig = R(1)) {
  const R b0 = sig * X * R(0.2);
  const R b1 = R(0.5) * ux * X, b2 = R(0.5) * uy * X;
  const R b3 = (b + R(4) * (R(1) - sig)) * X * R(0.05);
  g[0] += sgn * (b0 - R(4) * b3);
  g[1] += sgn * (b0 + b1 + b3);
  g[2] += sgn * (b0 + b2 + b3);
  g[3] += sgn * (b0 - b1 + b3);
  g[4] += sgn * (b0 - b2 + b3);
}

// Pre-collision populations of node (x, y) including the boundary columns:
// inlet (x = 0, channel rows) and outlet (x = nx-1) by non-equilibrium
// extrapolation from columns 1 and nx-2 (Section 4 boundary conditions).
// Returns the node's own material.
template <typename R>
__device__ __forceinline__ void boundary_column(R (&f)[19], const Consts<R>& k, int y, bool inlet, const Mat<R>& mp,
                                                const Mat<R>& mb);
template <typename R>
__device__ __forceinline__ void outlet_scalar_material(Mat<R>& mb, const Mat<R>& mp);
template <typename R>
struct React;
template <typename R>
__device__ __forceinline__ React<R> surface_reaction(R g_t, R g_c, const Mat<R>& m, const Consts<R>& k);

// Thin-film CL (Section 1): on the row above the reactive wall, planes 13
// and 18 hold the bounced-back populations that crossed the wall; the
// surface reaction adds its heat (sigma theta with the heat-capacity ratio)
// and removes its O2.  mp: the material of the pulled column.
template <typename R>
__device__ __forceinline__ void thin_film(R (&f)[19], const Mat<R>& mp, const Consts<R>& k, int y) {
  if ((k.flags & F_THIN_CL) && !(k.flags & F_NO_REACTION) && y == k.ny - 1) {
    const React<R> r = surface_reaction(f[13], f[18], mp, k);
    f[13] += r.S_T * mp.sig;
    f[18] -= r.s_c;
  }
}

template <typename R, int MAT, bool NT = true, bool UNIFORM = false>
__device__ __forceinline__ Mat<R> pre_collision(const R* __restrict__ src, const Consts<R>& k,
                                                const R* __restrict__ phi_f,
                                                const R* __restrict__ invk_f,
                                                const R* __restrict__ d_f, int x, int y,
                                                R (&f)[19]) {
  const bool open = !(k.flags & F_PERIODIC_X);
  const bool inlet = open && x == 0 && y < k.ny_ch;
  const bool outlet = open && x == k.nx - 1;
  const int xp = inlet ? 1 : (outlet ? k.nx - 2 : x);
  pull<R, NT, UNIFORM>(src, k, xp, y, f);
  Mat<R> mp = material<R, MAT>(k, phi_f, invk_f, d_f, xp, y);
  thin_film(f, mp, k, y);
  if (!(inlet || outlet)) return mp;
  Mat<R> mb = material<R, MAT>(k, phi_f, invk_f, d_f, x, y);
  boundary_column(f, k, y, inlet, mp, mb);
  if (outlet) outlet_scalar_material(mb, mp);
  return mb;
}

// The outlet node collides its copied scalar populations with the scalar
// material (b_T, b_C, rho c_p) of column nx-2, so that the last two columns
// are one medium for temperature and O2: with its own b the equilibrium
// fluxes (4 + b) X / 20 across the last link differ and the outlet turns
// into a source or sink proportional to X (unbounded growth for porosity
// fields).  For layers uniform in x nothing changes.
template <typename R>
__device__ __forceinline__ void outlet_scalar_material(Mat<R>& mb, const Mat<R>& mp) {
  mb.bT = mp.bT;
  mb.bC = mp.bC;
  mb.rhocp = mp.rhocp;
  mb.sig = mp.sig;
}

// Inlet velocity of row y (parabolic over the channel rows).
template <typename R>
__device__ __forceinline__ R inlet_velocity(const Consts<R>& k, int y) {
  const R yc = R(y) + R(0.5);
  return k.u_in_coef * yc * (R(k.ny_ch) - yc);
}

// Turn the pulled populations f of the column next to a boundary node into
// the boundary node's pre-collision populations (inlet: velocity u_in(y)
// with the pressure of the neighbour, or in the pressure-driven mode the
// pressure p_in with the neighbour's velocity; Dirichlet theta = 0 and
// c = c_in; outlet: the outlet pressure p_out with the neighbour's velocity,
// scalars copied).
template <typename R>
__device__ __forceinline__ void boundary_column(R (&f)[19], const Consts<R>& k, int y, bool inlet, const Mat<R>& mp,
                                                const Mat<R>& mb) {
  const Macro<R> a = flow_macros(f, mp, k);
  R ubx, uby, pb;
  if (inlet && (k.flags & F_PRESSURE_INLET)) {
    ubx = a.ux;
    uby = a.uy;
    pb = k.p_in;
  } else if (inlet) {
    ubx = inlet_velocity(k, y);
    uby = R(0);
    pb = a.p;
  } else {
    ubx = a.ux;
    uby = a.uy;
    pb = k.p_out;
  }
  R m1[9], m2[9], dm[9], df[9];
  meq_shifted(pb, ubx, uby, mb.phi, m1);
  meq_shifted(a.p, a.ux, a.uy, mp.phi, m2);
#pragma unroll
  for (int i = 0; i < 9; ++i) dm[i] = m1[i] - m2[i];
  inv_moments9(dm, df);
#pragma unroll
  for (int i = 0; i < 9; ++i) f[i] += df[i];
  if (inlet) {
    const R th1 = theta_of(f + 9, mp.sig, k);
    const R c1 = f[14] + f[15] + f[16] + f[17] + f[18];
    add_geq(R(0), ubx, uby, mb.bT, R(1), f + 9, mb.sig);
    add_geq(th1, a.ux, a.uy, mp.bT, R(-1), f + 9, mp.sig);
    add_geq(k.c_in, ubx, uby, mb.bC, R(1), f + 14);
    add_geq(c1, a.ux, a.uy, mp.bC, R(-1), f + 14);
  }
}

template <typename R>
struct React {
  R s_c, S_T, ehs;  // O2 consumed, temperature source, eta + T dU0/dT
};

// CL oxygen reduction over one step (Eqs. 12-17), integrated exactly in time:
// kappa = a j0(T) exp(-alpha_c F eta / (R T)) dt / (4 F C_ref),
// s_c = c (1 - exp(-kappa)), heat source 4 F C_ref s_c (eta + T dU0/dT) / (rho c_p).
// Butler-Volmer (Eq. 13 with the anodic branch, O2 dependence on the
// cathodic branch only): c relaxes toward c_eq = exp((alpha_a + alpha_c) F
// eta / (R T)) instead of 0, s_c = (c - c_eq)(1 - exp(-kappa)).
// K: the launch constants (2D or 3D), which carry the same reaction fields.
template <typename R, typename K>
__device__ __forceinline__ React<R> reaction(R theta, R c, R rhocp, const K& k) {
  const R T = k.T_in + theta;
  const R iT = R(1) / T;
  const R eta = k.V_op - (k.U0_slope * T + k.U0_icept);
  const R kappa = exp(k.ln_k0 - k.E_over_R * (iT - k.inv_T_arrh) - k.aF_over_R * eta * iT);
  React<R> r;
  const R ceq = k.bv ? exp(k.aFsum_over_R * eta * iT) : R(0);
  r.s_c = -(c - ceq) * expm1(-kappa);
  // Eq. 15 as printed, or with the irreversible part |j| |eta| counted positive
  // (the sign goes on eta alone, so both forms are the same expression)
  const R e = (k.flags & F_PHYSICAL_HEAT) ? -eta : eta;
  r.ehs = e + T * k.U0_slope;
  r.S_T = k.four_f_cref * r.s_c * r.ehs / rhocp;
  return r;
}

// Thin-film CL (the CL of negligible thickness): the wall half a cell below
// the last row reacts with the Eq. 13 kinetics carried over a film of
// thickness delta, k_s = a j0(T) delta exp(-alpha_c F eta / (R T)).  The wall
// values come from the populations that cross it, c_w = g_c / a_c and
// theta_w = g_t / a_t, a = (4 + b) / 20 being the equilibrium weight of a
// moving population at zero wall-normal velocity.  Exactly in time for the
// incident population: s_c = (g_c - a_c c_eq)(1 - exp(-kappa_s / a_c)),
// kappa_s = k_s dt / (4 F C_ref dx); heat 4 F C_ref s_c (eta + T dU0/dT) / (rho c_p).
template <typename R>
__device__ __forceinline__ React<R> surface_reaction(R g_t, R g_c, const Mat<R>& m, const Consts<R>& k) {
  const R a_t = (R(4) + m.bT) / R(20);
  const R a_c = (R(4) + m.bC) / R(20);
  const R T = k.T_in + g_t / a_t;
  const R iT = R(1) / T;
  const R eta = k.V_op - (k.U0_slope * T + k.U0_icept);
  const R kappa_a =
      exp(k.ln_k0 + k.ln_thin - k.E_over_R * (iT - k.inv_T_arrh) - k.aF_over_R * eta * iT) / a_c;
  const R ceq = k.bv ? exp(k.aFsum_over_R * eta * iT) : R(0);
  React<R> r;
  r.s_c = -(g_c - a_c * ceq) * expm1(-kappa_a);
  const R e = (k.flags & F_PHYSICAL_HEAT) ? -eta : eta;
  r.ehs = e + T * k.U0_slope;
  r.S_T = k.four_f_cref * r.s_c * r.ehs / m.rhocp;
  return r;
}

// Collision of one node: D2Q9 MRT with porous forcing (Eqs. 1, 3-6), CL
// reaction, D2Q5 MRT for both scalars (Eq. 10) with the source injected as
// S (1, 0, 0, b, 0).  In: pre-collision f; out: post-collision f.
template <typename R>
__device__ __forceinline__ void collide(R (&f)[19], const Mat<R>& mt, const Consts<R>& k, bool cl) {
  const Macro<R> a = flow_macros(f, mt, k);
  R m[9], me[9];
  moments9(f, m);
  meq_shifted(a.p, a.ux, a.uy, mt.phi, me);
  const R iphi = R(1) / mt.phi;
  const R uF = a.ux * a.Fx + a.uy * a.Fy;
  const R se = k.s_e, sq = k.s_q;
  const R he = R(1) - R(0.5) * se, hq = R(1) - R(0.5) * sq;
  m[0] = m[0] - se * m[0];
  m[1] = m[1] - se * (m[1] - me[1]) + he * R(6) * uF * iphi;
  m[2] = m[2] - se * (m[2] - me[2]) - he * R(6) * uF * iphi;
  m[3] = m[3] + a.Fx;
  m[4] = m[4] - sq * (m[4] - me[4]) - hq * a.Fx;
  m[5] = m[5] + a.Fy;
  m[6] = m[6] - sq * (m[6] - me[6]) - hq * a.Fy;
  m[7] = m[7] - se * (m[7] - me[7]) + he * R(2) * (a.ux * a.Fx - a.uy * a.Fy) * iphi;
  m[8] = m[8] - se * (m[8] - me[8]) + he * (a.ux * a.Fy + a.uy * a.Fx) * iphi;
  inv_moments9(m, f);

  R srcT = R(0), srcC = R(0);
  const R thsum = f[9] + f[10] + f[11] + f[12] + f[13];  // sigma theta with the heat-capacity ratio
  const R th = (k.flags & F_SIGMA_ENERGY) ? thsum / mt.sig : thsum;
  const R c = f[14] + f[15] + f[16] + f[17] + f[18];
  if (cl) {
    const React<R> r = reaction(th, c, mt.rhocp, k);
    srcT = r.S_T;
    srcC = -r.s_c;
  }
  const R q1 = R(1.2679491924311228);  // 6 / (3 + sqrt 3)
  const R q3 = R(0.9282032302755092);  // 6 / (3 + 2 sqrt 3)
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    R* g = f + 9 + 5 * s;
    const R X = s == 0 ? th : c;
    const R sg = s == 0 ? mt.sig : R(1);
    const R b = s == 0 ? mt.bT + R(4) * (R(1) - sg) : mt.bC;  // b + 4 (1 - sigma): unchanged at sigma = 1
    const R src = s == 0 ? srcT : srcC;
    R n0 = s == 0 ? thsum : c;
    R n1 = g[1] - g[3];
    R n2 = g[2] - g[4];
    R n3 = R(-4) * g[0] + g[1] + g[2] + g[3] + g[4];
    R n4 = g[1] - g[2] + g[3] - g[4];
    n0 = n0 + sg * src;
    n1 = n1 - q1 * (n1 - a.ux * X);
    n2 = n2 - q1 * (n2 - a.uy * X);
    n3 = n3 - q3 * (n3 - b * X) + b * src;
    n4 = n4 - q3 * n4;
    const R b0 = n0 * R(0.2), b1 = n1 * R(0.5), b2 = n2 * R(0.5), b3 = n3 * R(0.05), b4 = n4 * R(0.25);
    g[1] = b0 + b1 + b3 + b4;
    g[2] = b0 + b2 + b3 - b4;
    g[3] = b0 - b1 + b3 + b4;
    g[4] = b0 - b2 + b3 - b4;
    // Rest population from the conserved moment (equal to b0 - 4 b3 in
    // exact arithmetic): 0.2 is not a binary fraction, and 5 * fl(0.2 n0)
    // would add a relative 7.5e-8 of the scalar to every node at every FP32
    // step, a systematic drift that the 1/5-free form does not have.
    g[0] = n0 - ((g[1] + g[3]) + (g[2] + g[4]));
  }
}

}  // namespace lbm
