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
    for (int q = 0; q < 33; ++q) la[q] = lam_in[q * k.plane + o];
    collide_adj(pre, mt, k, cl, la, mu, ma);
  }
}

// One reverse step: lam_out = (dS'/dS)^T lam_in at the state S, gradients
// accumulated into grad (planes phi, 1/K, D_eff).  SEED: lam_out = w dJ/dS.
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
  const bool inlet = open && x == 0 && z < k.nz_ch;
  const bool outlet = open && x == k.nx - 1;
  const int xp = inlet ? 1 : (outlet ? k.nx - 2 : x);
  const int row = (z * k.ny + y) * k.pitch;
  const int o = row + x;

  R p[33];
  pull(S, k, xp, y, z, p);
  const Mat3<R> mxp = material<R, MAT_FULL>(k, phi_f, invk_f, d_f, xp, y, z);
  MatAdj3<R> ma{};
  R mu[33];
  if (inlet || outlet) {
    // Boundary node: its collision adjoint and the material part of its
    // extrapolation; the values of its own pull are never read.
    Mat3<R> mb = material<R, MAT_FULL>(k, phi_f, invk_f, d_f, x, y, z);
    R pre[33];
#pragma unroll
    for (int q = 0; q < 33; ++q) pre[q] = p[q];
    boundary_column(pre, k, y, z, inlet, mxp, mb);
    if (outlet) {
      mb.aT = mxp.aT;
      mb.aC = mxp.aC;
      mb.rhocp = mxp.rhocp;
    }
    node_mu<R, SEED>(pre, mb, k, cl, lam_in, o, w, mu, ma);
    R dmu[33];
#pragma unroll
    for (int q = 0; q < 33; ++q) dmu[q] = R(0);
    MatAdj3<R> dmaxp{};
    boundary_adj(p, mxp, mb, k, inlet, inlet ? inlet_velocity(k, y, z) : R(0), mu, dmu, dmaxp, ma);
    if (outlet) {  // the outlet's scalar material is column nx-2's: that thread takes these terms
      ma.aT = R(0);
      ma.aC = R(0);
      ma.rhocp = R(0);
    }
    R g0 = R(0), g1 = R(0), g2 = R(0);
    material_adj(k, mb, ma, g0, g1, g2);
    grad[o] += g0;
    grad[k.plane + o] += g1;
    grad[2 * k.plane + o] += g2;
#pragma unroll
    for (int q = 0; q < 33; ++q) mu[q] = R(0);
  } else {
    node_mu<R, SEED>(p, mxp, k, cl, lam_in, o, w, mu, ma);
    // A column feeding a boundary node adds that node's adjoint through the
    // extrapolation (recomputed here: every thread writes only its own data).
    const bool feeds_inlet = open && x == 1 && z < k.nz_ch;
    const bool feeds_outlet = open && x == k.nx - 2;
    if (feeds_inlet || feeds_outlet) {
      const int xb = feeds_inlet ? 0 : k.nx - 1;
      Mat3<R> mb = material<R, MAT_FULL>(k, phi_f, invk_f, d_f, xb, y, z);
      R pre[33];
#pragma unroll
      for (int q = 0; q < 33; ++q) pre[q] = p[q];
      boundary_column(pre, k, y, z, feeds_inlet, mxp, mb);
      if (feeds_outlet) {
        mb.aT = mxp.aT;
        mb.aC = mxp.aC;
        mb.rhocp = mxp.rhocp;
      }
      R mub[33];
      MatAdj3<R> dmab{};
      node_mu<R, SEED>(pre, mb, k, cl, lam_in, row + xb, w, mub, dmab);
      if (feeds_outlet) {  // the outlet node collides with this column's scalar material
        ma.aT += dmab.aT;
        ma.aC += dmab.aC;
        ma.rhocp += dmab.rhocp;
      }
      MatAdj3<R> dmab2{};
      boundary_adj(p, mxp, mb, k, feeds_inlet, feeds_inlet ? inlet_velocity(k, y, z) : R(0), mub, mu, ma, dmab2);
    }
    R g0 = R(0), g1 = R(0), g2 = R(0);
    material_adj(k, mxp, ma, g0, g1, g2);
    grad[o] += g0;
    grad[k.plane + o] += g1;
    grad[2 * k.plane + o] += g2;
  }
  // Push: the adjoint of the pulled element (x - e_q, q), or of the
  // bounced-back (x, opp q), is mu[q].
  const bool px = k.flags & F_PERIODIC_X, py = k.flags & F_PERIODIC_Y, pz = k.flags & F_PERIODIC_Z;
  const int rowp = k.pitch * k.ny;
#pragma unroll
  for (int q = 0; q < 33; ++q) {
    int xs = x - EX[q], ys = y - EY[q], zs = z - EZ[q];
    if (px) xs = xs < 0 ? xs + k.nx : (xs >= k.nx ? xs - k.nx : xs);
    if (py) ys = ys < 0 ? ys + k.ny : (ys >= k.ny ? ys - k.ny : ys);
    if (pz) zs = zs < 0 ? zs + k.nz : (zs >= k.nz ? zs - k.nz : zs);
    const bool in = (unsigned)xs < (unsigned)k.nx && (unsigned)ys < (unsigned)k.ny && (unsigned)zs < (unsigned)k.nz;
    const int off = in ? (q * k.plane + zs * rowp + ys * k.pitch + xs) : (OPP[q] * k.plane + o);
    lam_out[off] = mu[q];
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
