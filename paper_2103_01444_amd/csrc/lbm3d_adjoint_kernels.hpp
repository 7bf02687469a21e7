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

// Shares of the boundary columns left for the next reverse step (open x).
// The boundary pass of a step computes, for the column xp_s feeding each
// boundary node (s = 0: column 1, inlet rows; s = 1: column nx - 2, every
// row), the share of the adjoint of every element that column pulled, and
// of the column's gradient.  The 33 shares of node (xp_s - 1 + dx, row) are
// contiguous (padded to kPendQ) at pend[((s * nrows + row) * 3 + dx) *
// kPendQ], so that a node near a boundary takes them in a few 16-byte
// loads; the gradient shares c of row `row` at pend[kPendLam * nrows +
// (s * nrows + row) * 4 + c].  Each element receives at most one share (a
// link of the column either crosses a wall or it does not), so the
// boundary pass writes them and every node adds its own when it loads its
// adjoint in the next step; the last step's are added by an apply pass.
// Slots that never receive a share hold zero.
constexpr int kPendQ = 36;
constexpr int kPendLam = 2 * 3 * kPendQ;
constexpr int kPendVals = kPendLam + 2 * 4;

__device__ __forceinline__ int pend_slot(int nrows, int s, int q, int dx, int row) {
  return ((s * nrows + row) * 3 + dx) * kPendQ + q;
}
__device__ __forceinline__ int pend_grad(int nrows, int s, int c, int row) {
  return kPendLam * nrows + (s * nrows + row) * 4 + c;
}

template <typename R>
struct Vec16;  // 16 bytes of R
template <>
struct Vec16<float> {
  using T = float __attribute__((ext_vector_type(4)));
  static constexpr int n = 4;
};
template <>
struct Vec16<double> {
  using T = double __attribute__((ext_vector_type(2)));
  static constexpr int n = 2;
};

// Add the shares of node (x, row) to the adjoint la it loaded (a node near
// both ends when nx <= 5 takes both sides').
template <typename R>
__device__ __forceinline__ void add_pending(R (&la)[33], const Consts3<R>& k, const R* __restrict__ pend, int x,
                                            int row) {
  const int nrows = k.ny * k.nz;
  constexpr int n = Vec16<R>::n;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int dx = x - (s == 0 ? 0 : k.nx - 3);
    if ((unsigned)dx <= 2u) {
      const auto* v = reinterpret_cast<const typename Vec16<R>::T*>(pend + pend_slot(nrows, s, 0, dx, row));
#pragma unroll
      for (int i = 0; i < (33 + n - 1) / n; ++i) {
        const typename Vec16<R>::T w = v[i];
#pragma unroll
        for (int j = 0; j < n; ++j)
          if (i * n + j < 33) la[i * n + j] += w[j];
      }
    }
  }
}

// The gradient shares of the feeding column at node (x, row).
template <typename R>
__device__ __forceinline__ void add_pending_grad(R& g0, R& g1, R& g2, const Consts3<R>& k, const R* __restrict__ pend,
                                                 int x, int row) {
  const int nrows = k.ny * k.nz;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    if (x == (s == 0 ? 1 : k.nx - 2)) {
      g0 += pend[pend_grad(nrows, s, 0, row)];
      g1 += pend[pend_grad(nrows, s, 1, row)];
      g2 += pend[pend_grad(nrows, s, 2, row)];
    }
  }
}

template <typename R, bool SEED>
__device__ __forceinline__ void node_mu(const R (&pre)[33], const Mat3<R>& mt, const Consts3<R>& k, bool cl,
                                        const R* __restrict__ lam_in, const R* __restrict__ pend, int o, int x,
                                        int row, R w, R (&mu)[33], MatAdj3<R>& ma) {
  if constexpr (SEED) {
    seed_mu(pre, mt, k, cl, w, mu);
  } else {
    R la[33];
#pragma unroll
    for (int q = 0; q < 33; ++q) la[q] = lbm::buffer_load<R, 0>(lam_in + int64_t(q) * k.plane, uint32_t(o) * uint32_t(sizeof(R)));
    if (pend) add_pending(la, k, pend, x, row);
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
                                                       const R* __restrict__ pend,
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
    node_mu<R, SEED>(p, mt, k, cl, lam_in, pend, o, x, z * k.ny + y, w, mu, ma);
    R g0 = R(0), g1 = R(0), g2 = R(0);
    material_adj(k, mt, ma, g0, g1, g2);
    if (pend) add_pending_grad(g0, g1, g2, k, pend, x, z * k.ny + y);
    grad[o] += g0;
    grad[k.plane + o] += g1;
    grad[2 * k.plane + o] += g2;
  }
  push<R, false>(lam_out, k, x, y, z, mu);
}

// One reverse step, boundary pass (open x only; reads what the interior
// pass reads, writes only the boundary nodes' gradient and the shares
// pend_out, so it may run concurrently with the interior pass): one thread
// per boundary node b fed by column xp computes b's collision adjoint on b's
// pre-collision populations and the transposed extrapolation.  pend_in: the
// previous step's shares (null for the first).
template <typename R, bool SEED>
__global__ __launch_bounds__(64) void k3_adj_bnd(const R* __restrict__ S, const R* __restrict__ lam_in,
                                                 R* __restrict__ grad, const R* __restrict__ pend_in,
                                                 R* __restrict__ pend_out,
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
    node_mu<R, SEED>(pre, mb, k, cl, lam_in, pend_in, row + xb, xb, r, w, mub, mab);
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
  // The share of element (q, xp - e_q) of the column's pull, or across a
  // wall of (opp q, xp) (as the pull reads them).
  const int s = inlet ? 0 : 1;
  const bool py = k.flags & F_PERIODIC_Y, pz = k.flags & F_PERIODIC_Z;
#pragma unroll
  for (int q = 0; q < 33; ++q) {
    int ys = y - EY[q], zs = z - EZ[q];
    if (py) ys = ys < 0 ? ys + k.ny : (ys >= k.ny ? ys - k.ny : ys);
    if (pz) zs = zs < 0 ? zs + k.nz : (zs >= k.nz ? zs - k.nz : zs);
    const bool in = (unsigned)ys < (unsigned)k.ny && (unsigned)zs < (unsigned)k.nz;
    const int slot = in ? pend_slot(nrows, s, q, 1 - EX[q], zs * k.ny + ys) : pend_slot(nrows, s, OPP[q], 1, r);
    pend_out[slot] = dmu[q];
  }
  pend_out[pend_grad(nrows, s, 0, r)] = g0;
  pend_out[pend_grad(nrows, s, 1, r)] = g1;
  pend_out[pend_grad(nrows, s, 2, r)] = g2;
}

// After the last reverse step: its boundary shares added to the adjoint of
// the initial state and to the gradient.  One thread per (population or the
// gradient slot, row) adds both sides in turn (for nx <= 5 they reach the
// same nodes).
template <typename R>
__global__ __launch_bounds__(kBlock3) void k3_adj_apply(const R* __restrict__ pend, R* __restrict__ lam,
                                                        R* __restrict__ grad, Consts3<R> k) {
  const int nrows = k.ny * k.nz;
  const int t = blockIdx.x * kBlock3 + threadIdx.x;
  if (t >= 34 * nrows) return;
  const int q = t / nrows, row = t - q * nrows;
  const int z = row / k.ny, y = row - z * k.ny;
  const int o = z * k.pitch * k.ny + y * k.pitch;
  for (int s = 0; s < 2; ++s) {
    const int x0 = s == 0 ? 0 : k.nx - 3;
    if (q < 33) {
      for (int dx = 0; dx < 3; ++dx) lam[q * k.plane + o + x0 + dx] += pend[pend_slot(nrows, s, q, dx, row)];
    } else {
      for (int c = 0; c < 3; ++c) grad[c * k.plane + o + x0 + 1] += pend[pend_grad(nrows, s, c, row)];
    }
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
