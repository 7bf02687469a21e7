// Kernels of the 3D reverse sweep (three per-cell fields: porosity, 1/K, D_eff).
#pragma once

#include "lbm3d_adjoint.hpp"
#include "lbm3d_kernels.hpp"

namespace lbm3 {

// Adjoint of J = mean current density on the pre-collision populations: for
// CL nodes w dJ/dc and w dJ/dtheta on every scalar population.
template <typename R>
__device__ __forceinline__ void seed_mu(const R (&pre)[33], const Mat3<R>& mt, const Consts3<R>& k, bool cl, R w,
                                        R (&mu)[33]) {
#pragma unroll
  for (int i = 0; i < 33; ++i) mu[i] = R(0);
  if (!cl) return;
  R th = R(0), c = R(0);
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    th += pre[19 + q];
    c += pre[26 + q];
  }
  const ReactAdj<R> r = reaction_tape(th, c, mt.rhocp, k);
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    mu[19 + q] = w * r.dsc_dth;
    mu[26 + q] = w * r.dsc_dc;
  }
}

template <typename R, bool SEED>
__device__ __forceinline__ void node_mu(const R (&pre)[33], const Mat3<R>& mt, const Consts3<R>& k, bool cl,
                                        const R* __restrict__ lam_in, int o, R w, R (&mu)[33], MatAdj3<R>& ma) {
  if constexpr (SEED) {
    seed_mu(pre, mt, k, cl, w, mu);
  } else {
    R la[33];
#pragma unroll
    for (int q = 0; q < 33; ++q) la[q] = lbm::buffer_load<R, 0>(lam_in + int64_t(q) * k.plane, uint32_t(o) * uint32_t(sizeof(R)));
    collide_adj(pre, mt, k, cl, la, mu, ma);
  }
}

// Push: the adjoint of the pulled element (x - e_q, q), or of the
// bounced-back (x, opp q), is mu[q].  ADD: add to what is there.
template <typename R, bool ADD>
__device__ __forceinline__ void push(R* __restrict__ lam_out, const Consts3<R>& k, int x, int y, int z,
                                     const R (&mu)[33]) {
  const int rowp = k.pitch * k.ny;
  const int o = z * rowp + y * k.pitch + x;
  if (!ADD && __all(x >= 1 && x <= k.nx - 2 && y >= 1 && y <= k.ny - 2 && z >= 1 && z <= k.nz - 2)) {
    const uint32_t ob = uint32_t(o) * uint32_t(sizeof(R));
#pragma unroll
    for (int q = 0; q < 33; ++q)
      lbm::buffer_store(lam_out + (int64_t(q) * k.plane - int64_t(EZ[q]) * rowp - int64_t(EY[q]) * k.pitch - EX[q]),
                        ob, mu[q]);
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
    const int off = in ? (q * k.plane + zs * rowp + ys * k.pitch + xs) : (OPP[q] * k.plane + o);
    if constexpr (ADD) lam_out[off] += mu[q]; else lam_out[off] = mu[q];
  }
}

// One reverse step, interior pass: lam_out = (dS'/dS)^T lam_in at the state
// S without the boundary-column terms, gradients accumulated into grad
// (planes phi, 1/K, D_eff).  Boundary nodes push zeros (the values of their
// own pull are never read by the forward step) and leave their gradient to
// the boundary pass.  SEED: lam_out = w dJ/dS.
template <typename R, bool SEED>
__global__ __launch_bounds__(kBlock3) void k3_adj_step(const R* __restrict__ S, const R* __restrict__ lam_in,
                                                       R* __restrict__ lam_out, R* __restrict__ grad,
                                                       const R* __restrict__ phi_f, const R* __restrict__ invk_f,
                                                       const R* __restrict__ d_f, Consts3<R> k, R w) {
  int x, y, z;
  node_of(k, x, y, z);
  if (x >= k.nx) return;
  const bool open = !(k.flags & F_PERIODIC_X);
  const bool cl = !(k.flags & F_NO_REACTION) && z >= k.z_cl0;
  const bool boundary = open && ((x == 0 && z < k.nz_ch) || x == k.nx - 1);
  R mu[33];
  if (boundary) {
#pragma unroll
    for (int q = 0; q < 33; ++q) mu[q] = R(0);
  } else {
    const int o = (z * k.ny + y) * k.pitch + x;
    R p[33];
    pull<R, true>(S, k, x, y, z, p);
    const Mat3<R> mt = material<R, MAT_FULL>(k, phi_f, invk_f, d_f, x, y, z);
    MatAdj3<R> ma{};
    node_mu<R, SEED>(p, mt, k, cl, lam_in, o, w, mu, ma);
    R g0 = R(0), g1 = R(0), g2 = R(0);
    material_adj(k, mt, ma, g0, g1, g2);
    grad[o] += g0;
    grad[k.plane + o] += g1;
    grad[2 * k.plane + o] += g2;
  }
  push<R, false>(lam_out, k, x, y, z, mu);
}

// Values per boundary slot in the side buffer: the feeding column's share of
// the adjoint (33) and of its gradient (3).  Slots are [side][row], side 0
// the inlet node of the row, side 1 the outlet node; stored plane by plane.
constexpr int kSideVals = 36;

// One reverse step, boundary pass (open x only; reads what the interior
// pass reads, writes only the boundary nodes' gradient and the side buffer,
// so it may run concurrently with the interior pass): one thread per
// boundary node b fed by column xp computes b's collision adjoint on b's
// pre-collision populations and the transposed extrapolation.
template <typename R, bool SEED>
__global__ __launch_bounds__(64) void k3_adj_bnd(const R* __restrict__ S, const R* __restrict__ lam_in,
                                                 R* __restrict__ grad, R* __restrict__ side,
                                                 const R* __restrict__ phi_f, const R* __restrict__ invk_f,
                                                 const R* __restrict__ d_f, Consts3<R> k, R w) {
  // This pass runs beside the interior pass on the same CUs and is the
  // longer of the two: its waves take instruction-issue priority.
  __builtin_amdgcn_s_setprio(3);
  const int nrows = k.ny * k.nz;
  const int t = blockIdx.x * 64 + threadIdx.x;
  if (t >= 2 * nrows) return;
  const bool inlet = t < nrows;
  const int r = inlet ? t : t - nrows;
  const int z = r / k.ny, y = r - z * k.ny;
  if (inlet && z >= k.nz_ch) return;
  const bool cl = !(k.flags & F_NO_REACTION) && z >= k.z_cl0;
  const int xb = inlet ? 0 : k.nx - 1, xp = inlet ? 1 : k.nx - 2;
  const int row = (z * k.ny + y) * k.pitch;
  R p[33];
  pull(S, k, xp, y, z, p);
  const Mat3<R> mxp = material<R, MAT_FULL>(k, phi_f, invk_f, d_f, xp, y, z);
  Mat3<R> mb = material<R, MAT_FULL>(k, phi_f, invk_f, d_f, xb, y, z);
  if (!inlet) {  // the outlet node collides with column nx-2's scalar material
    mb.aT = mxp.aT;
    mb.aC = mxp.aC;
    mb.rhocp = mxp.rhocp;
  }
  MatAdj3<R> mab{}, maxp{};
  R mub[33];
  {
    R pre[33];
#pragma unroll
    for (int q = 0; q < 33; ++q) pre[q] = p[q];
    boundary_column(pre, k, y, z, inlet, mxp, mb);
    node_mu<R, SEED>(pre, mb, k, cl, lam_in, row + xb, w, mub, mab);
  }
  R dmu[33];
#pragma unroll
  for (int q = 0; q < 33; ++q) dmu[q] = R(0);
  boundary_adj(p, mxp, mb, k, inlet, inlet ? inlet_velocity(k, y, z) : R(0), mub, dmu, maxp, mab);
  if (!inlet) {
    maxp.aT += mab.aT;
    maxp.aC += mab.aC;
    maxp.rhocp += mab.rhocp;
    mab.aT = mab.aC = mab.rhocp = R(0);
  }
  R g0 = R(0), g1 = R(0), g2 = R(0);
  material_adj(k, mb, mab, g0, g1, g2);
  grad[row + xb] += g0;
  grad[k.plane + row + xb] += g1;
  grad[2 * k.plane + row + xb] += g2;
  g0 = g1 = g2 = R(0);
  material_adj(k, mxp, maxp, g0, g1, g2);
  const int slots = 2 * nrows;
#pragma unroll
  for (int q = 0; q < 33; ++q) side[q * slots + t] = dmu[q];
  side[33 * slots + t] = g0;
  side[34 * slots + t] = g1;
  side[35 * slots + t] = g2;
}

// One reverse step, apply pass (after both): one thread per (row,
// population) adds the inlet and the outlet slot to the elements the feeding
// columns pushed, and one thread per (row, gradient component) adds the
// gradient shares.  For nx > 3 the two targets of a thread differ (columns 1
// and nx - 2), so both are loaded before either is stored; for nx = 3, where
// both feed column 1, they are added one after the other.
template <typename R>
__device__ __forceinline__ int apply_target(const Consts3<R>& k, int q, int xp, int y, int z) {
  const bool py = k.flags & F_PERIODIC_Y, pz = k.flags & F_PERIODIC_Z;
  const int rowp = k.pitch * k.ny;
  const int xs = xp - EX[q];  // in [0, nx - 1]: x is open here
  int ys = y - EY[q], zs = z - EZ[q];
  if (py) ys = ys < 0 ? ys + k.ny : (ys >= k.ny ? ys - k.ny : ys);
  if (pz) zs = zs < 0 ? zs + k.nz : (zs >= k.nz ? zs - k.nz : zs);
  const bool in = (unsigned)ys < (unsigned)k.ny && (unsigned)zs < (unsigned)k.nz;
  return in ? (q * k.plane + zs * rowp + ys * k.pitch + xs) : (OPP[q] * k.plane + z * rowp + y * k.pitch + xp);
}

template <typename R>
__global__ __launch_bounds__(kBlock3) void k3_adj_apply(const R* __restrict__ side, R* __restrict__ lam_out,
                                                        R* __restrict__ grad, Consts3<R> k) {
  const int nrows = k.ny * k.nz;
  const int t = blockIdx.x * kBlock3 + threadIdx.x;
  if (t >= 36 * nrows) return;
  const int q = t / nrows, r = t - q * nrows;
  const int z = r / k.ny, y = r - z * k.ny;
  const int slots = 2 * nrows;
  const bool in_row = z < k.nz_ch;  // the row has an inlet node
  const R a_in = in_row ? side[q * slots + r] : R(0);
  const R a_out = side[q * slots + nrows + r];
  int o_in, o_out;
  R* base;
  if (q < 33) {
    base = lam_out;
    o_in = apply_target(k, q, 1, y, z);
    o_out = apply_target(k, q, k.nx - 2, y, z);
  } else {
    base = grad + int64_t(q - 33) * k.plane;
    const int rowp = k.pitch * k.ny;
    o_in = z * rowp + y * k.pitch + 1;
    o_out = z * rowp + y * k.pitch + k.nx - 2;
  }
  if (k.nx > 3 && in_row) {
    const R v_in = base[o_in], v_out = base[o_out];
    base[o_in] = v_in + a_in;
    base[o_out] = v_out + a_out;
  } else {
    if (in_row) base[o_in] += a_in;
    base[o_out] += a_out;
  }
}

// Gradient through the initial state: the O2 equilibrium at rest depends on
// a_C = sqrt(3) D (g0 = c_in (1 - 6 a_C), g_i = c_in a_C).
template <typename R>
__global__ __launch_bounds__(kBlock3) void k3_adj_init(const R* __restrict__ lam0, R* __restrict__ grad,
                                                       Consts3<R> k) {
  const int x = blockIdx.x * kBlock3 + threadIdx.x;
  const int y = blockIdx.y, z = blockIdx.z;
  if (x >= k.nx) return;
  const int o = (z * k.ny + y) * k.pitch + x;
  R l16 = R(0);
#pragma unroll
  for (int q = 27; q < 33; ++q) l16 += lam0[q * k.plane + o];
  grad[2 * k.plane + o] += R(kSqrt3) * k.c_in * (R(-6) * lam0[26 * k.plane + o] + l16);
}

template <typename R>
__global__ __launch_bounds__(kBlock3) void k3_fill(R* __restrict__ dst, int64_t n, R v) {
  const int64_t i = blockIdx.x * int64_t(kBlock3) + threadIdx.x;
  if (i < n) dst[i] = v;
}

// Pitched plane -> dense [nz][ny][nx] caller array.
template <typename R>
__global__ __launch_bounds__(kBlock3) void k3_unpitch(const R* __restrict__ src, R* __restrict__ dst, int nx, int ny,
                                                      int pitch) {
  const int x = blockIdx.x * kBlock3 + threadIdx.x;
  const int y = blockIdx.y, z = blockIdx.z;
  if (x >= nx) return;
  dst[(size_t(z) * ny + y) * nx + x] = src[(z * ny + y) * pitch + x];
}

}  // namespace lbm3
