// Kernels of the reverse sweep (three per-cell fields: porosity, 1/K, D_eff).
#pragma once

#include "lbm_adjoint.hpp"
#include "lbm_kernels2d.hpp"

namespace lbm {

// Adjoint of the observable J = mean current density on the pre-collision
// populations: for CL nodes dJ/dc and dJ/dtheta on every scalar population.
// With the heat-capacity ratio (EXT) theta = sum g_T / sigma.
template <typename R, bool EXT>
__device__ __forceinline__ void seed_mu(const R (&pre)[19], const Mat<R>& mt, const Consts<R>& k, bool cl, R w,
                                        R (&mu)[19], MatAdj<R>& ma) {
#pragma unroll
  for (int i = 0; i < 19; ++i) mu[i] = R(0);
  if (!cl) return;
  const bool sigma = EXT && (k.flags & F_SIGMA_ENERGY);
  const R thsum = pre[9] + pre[10] + pre[11] + pre[12] + pre[13];
  const R th = sigma ? thsum / mt.sig : thsum;
  const R c = pre[14] + pre[15] + pre[16] + pre[17] + pre[18];
  const ReactAdj<R> r = reaction_tape(th, c, mt.rhocp, k);
  R lth = w * r.dsc_dth;
  if (sigma) {
    const R isg = R(1) / mt.sig;
    ma.sig += -th * isg * lth;
    lth *= isg;
  }
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    mu[9 + i] = lth;
    mu[14 + i] = w * r.dsc_dc;
  }
}

// a += (first ? b1 : b2), field by field (selecting values, not objects,
// keeps both operands in registers).
template <typename R>
__device__ __forceinline__ void add_mat_adj(MatAdj<R>& a, bool first, const MatAdj<R>& b1, const MatAdj<R>& b2) {
  a.phi += first ? b1.phi : b2.phi;
  a.invk += first ? b1.invk : b2.invk;
  a.sqk += first ? b1.sqk : b2.sqk;
  a.fphi += first ? b1.fphi : b2.fphi;
  a.l0 += first ? b1.l0 : b2.l0;
  a.l1 += first ? b1.l1 : b2.l1;
  a.bT += first ? b1.bT : b2.bT;
  a.bC += first ? b1.bC : b2.bC;
  a.rhocp += first ? b1.rhocp : b2.rhocp;
  a.sig += first ? b1.sig : b2.sig;
}

template <typename R>
__device__ __forceinline__ void load_node(const R* __restrict__ a, const Consts<R>& k, int x, int y, R (&v)[19]) {
  const uint32_t ob = uint32_t(y * k.pitch + x) * uint32_t(sizeof(R));
#pragma unroll
  for (int q = 0; q < 19; ++q) v[q] = buffer_load<R, 0>(a + int64_t(q) * k.plane, ob);
}

// Adjoint of node b's collision (or of J when SEED) given b's pre-collision populations.
template <typename R, bool SEED, bool EXT>
__device__ __forceinline__ void node_mu(const R (&pre)[19], const Mat<R>& mt, const Consts<R>& k, bool cl,
                                        const R* __restrict__ lam_in, int x, int y, R w, R (&mu)[19],
                                        MatAdj<R>& ma) {
  if constexpr (SEED) {
    seed_mu<R, EXT>(pre, mt, k, cl, w, mu, ma);
  } else {
    R la[19];
    load_node(lam_in, k, x, y, la);
    collide_adj<R, EXT>(pre, mt, k, cl, la, mu, ma);
  }
}

// One reverse step: lam_out = (dS'/dS)^T lam_in at the state S, gradients
// accumulated into grad (planes phi, 1/K, D_eff).  SEED: lam_out = dJ/dS
// (times w = dJ dx / nx * 4 F C_ref / dt), no lam_in.
// The first and last wavefront of a row carry the boundary nodes and the
// columns feeding them, whose chain is the longest.  A boundary lane runs
// its own collision adjoint in the common pass of the wavefront (on its
// extrapolated populations) and the feeding lane reads it across lanes, so
// that wavefront pays one collision adjoint plus the transposed
// extrapolation.  Per reverse step of the 1024x256 adjoint: 28.5 us at four
// waves per SIMD (128 VGPRs, 64 bytes spilled per lane), 29.7-30.1 us at
// three; 29.3-29.9 us when the feeding lane recomputed the boundary node's
// collision adjoint, 34.4 us when the boundary and feeding lanes took
// separate divergent passes.
// Registers: the instances are held to four waves per SIMD (the default
// FP32 one at 128 VGPRs with 64 bytes per lane spilled), except the FP32
// instances with the model options (EXT), which are left to the registers
// they need (162 VGPRs, three waves per SIMD, no spill).  Compiled for four
// waves, that instance spilled 100 bytes per lane and its gradients with the
// thin-film CL and Butler-Volmer kinetics varied from run to run on
// identical inputs (some runs NaN); unspilled it gives the same bits in
// every run.  The FP64 EXT instances stay at four waves: left free, the
// compiler moved part of their state into accumulation registers and their
// gradients departed from the oracle by 1e-6 to 2e-5, while at four waves
// (scratch spills) they match it within 1e-12 in every run.
template <typename R, bool SEED, bool EXT = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(EXT && sizeof(R) == 4 ? 1 : 4))) void k_adj_step(const R* __restrict__ S, const R* __restrict__ lam_in,
                                                     R* __restrict__ lam_out, R* __restrict__ grad,
                                                     const R* __restrict__ phi_f, const R* __restrict__ invk_f,
                                                     const R* __restrict__ d_f, Consts<R> k, R w) {
  int bx, by;
  xcd_tile(gridDim.x, gridDim.y, bx, by);
  const int x = bx * kBlock + threadIdx.x;
  const int y = by;
  if (x >= k.nx) return;
  const bool open = !(k.flags & F_PERIODIC_X);
  const bool react = !(k.flags & F_NO_REACTION);
  const bool cl = react && y >= k.y_cl0;
  const bool inlet = open && x == 0 && y < k.ny_ch;
  const bool outlet = open && x == k.nx - 1;
  const int xp = inlet ? 1 : (outlet ? k.nx - 2 : x);

  R p[19];
  pull<R, true, true>(S, k, xp, y, p);
  const Mat<R> mxp = material<R, MAT_FULL>(k, phi_f, invk_f, d_f, xp, y);
  // Thin-film CL (EXT): the bottom row's wall-crossing populations react as
  // the forward pull left them (column nx - 2's film for the outlet).
  const bool film = EXT && (k.flags & F_THIN_CL) && react && y == k.ny - 1;
  FilmTape<R> ft{};
  if (film) {
    ft = film_tape(p[13], p[18], mxp, k);
    p[13] += ft.S_T * mxp.sig;
    p[18] -= ft.s;
  }
  MatAdj<R> ma{};
  R mu[19];
  const int o = y * k.pitch + x;
  const bool bnode = inlet || outlet;

  // One collision adjoint per lane: its own node's, for an inlet / outlet
  // node on the populations extrapolated from the column next to it.
  {
    Mat<R> mc = mxp;
    if (bnode) {
      mc = material<R, MAT_FULL>(k, phi_f, invk_f, d_f, x, y);
      boundary_column(p, k, y, inlet, mxp, mc);
      if (outlet) outlet_scalar_material(mc, mxp);
    }
    node_mu<R, SEED, EXT>(p, mc, k, cl, lam_in, x, y, w, mu, ma);
  }
  if (bnode) {  // the column's own populations again
    pull<R, true, false>(S, k, xp, y, p);
    if (film) {
      p[13] += ft.S_T * mxp.sig;
      p[18] -= ft.s;
    }
  }

  // Transpose of the extrapolation of a boundary node from the column next
  // to it: the boundary node needs it for its own material, the feeding
  // column for its populations and material.  Both lanes pulled that
  // column; the feeding lane takes the boundary node's collision adjoint
  // from its lane by a cross-lane read, and the two run the block together.
  if (open && y < k.ny_ch && x < 64) {  // the wavefront holding x = 0 and 1
    R mub[19];
#pragma unroll
    for (int q = 0; q < 19; ++q) mub[q] = __shfl(mu[q], 0, 64);
    if (x <= 1) {
      const Mat<R> mb = material<R, MAT_FULL>(k, phi_f, invk_f, d_f, 0, y);
      MatAdj<R> axp{}, ab{};
      boundary_adj<R, EXT>(p, mxp, mb, k, true, inlet_velocity(k, y), R(0), mub, mu, axp, ab);
      add_mat_adj(ma, x == 0, ab, axp);
    }
  }
  if (open) {
    const int xo = k.nx - 1;
    if ((xo & 63) != 0) {  // x = nx - 2 and nx - 1 in one wavefront
      if ((x & ~63) == (xo & ~63)) {
        const int src = xo & 63;
        R mub[19];
#pragma unroll
        for (int q = 0; q < 19; ++q) mub[q] = __shfl(mu[q], src, 64);
        const R sbT = __shfl(ma.bT, src, 64), sbC = __shfl(ma.bC, src, 64), src_p = __shfl(ma.rhocp, src, 64);
        const R ssg = EXT ? __shfl(ma.sig, src, 64) : R(0);
        if (x >= xo - 1) {
          Mat<R> mb = material<R, MAT_FULL>(k, phi_f, invk_f, d_f, xo, y);
          outlet_scalar_material(mb, mxp);
          if (!outlet) {  // the outlet node collides with column nx - 2's scalar material
            ma.bT += sbT;
            ma.bC += sbC;
            ma.rhocp += src_p;
            if (EXT) ma.sig += ssg;
          }
          MatAdj<R> axp{}, ab{};
          boundary_adj<R, EXT>(p, mxp, mb, k, false, R(0), R(0), mub, mu, axp, ab);
          add_mat_adj(ma, outlet, ab, axp);
        }
      }
    } else if (x >= xo - 1) {  // the pair straddles two wavefronts: each lane on its own
      Mat<R> mb = material<R, MAT_FULL>(k, phi_f, invk_f, d_f, xo, y);
      R mub[19];
      if (outlet) {
#pragma unroll
        for (int q = 0; q < 19; ++q) mub[q] = mu[q];
        outlet_scalar_material(mb, mxp);
      } else {
        R pre[19];
#pragma unroll
        for (int q = 0; q < 19; ++q) pre[q] = p[q];
        boundary_column(pre, k, y, false, mxp, mb);
        outlet_scalar_material(mb, mxp);
        MatAdj<R> mab{};
        node_mu<R, SEED, EXT>(pre, mb, k, cl, lam_in, xo, y, w, mub, mab);
        ma.bT += mab.bT;
        ma.bC += mab.bC;
        ma.rhocp += mab.rhocp;
        if (EXT) ma.sig += mab.sig;
      }
      MatAdj<R> axp{}, ab{};
      boundary_adj<R, EXT>(p, mxp, mb, k, false, R(0), R(0), mub, mu, axp, ab);
      add_mat_adj(ma, outlet, ab, axp);
    }
  }
  // Transpose of the film's update in the column that pulled it (the
  // outlet's copy came back through the boundary transpose above); the seed
  // adds J's dependence on the film, which counts column nx - 2 twice (the
  // outlet carries its film).
  if (film && !bnode) {
    const R ls = SEED ? ((open && x == k.nx - 2) ? R(2) * w : w) : R(0);
    film_adj(ft, mxp, k, ls, mu[13], mu[18], ma);
  }
  if (outlet) {  // its scalar material terms belong to column nx - 2
    ma.bT = R(0);
    ma.bC = R(0);
    ma.rhocp = R(0);
    ma.sig = R(0);
  }
  if (bnode) {  // its pulled sources were never read: their adjoint is 0
#pragma unroll
    for (int q = 0; q < 19; ++q) mu[q] = R(0);
  }
  // The gradient of this node's own material (a boundary node's is read
  // again; its scalar-material terms are zero, so the outlet's copy of
  // column nx - 2's scalar material does not enter).
  R g0 = R(0), g1 = R(0), g2 = R(0);
  material_adj<R, EXT>(k, bnode ? material<R, MAT_FULL>(k, phi_f, invk_f, d_f, x, y) : mxp, ma, g0, g1, g2);
  grad[o] += g0;
  grad[k.plane + o] += g1;
  grad[2 * k.plane + o] += g2;
  // Push: the adjoint of the pulled element (x - e_q, q) (or of the
  // bounced-back (x, opp q)) is mu[q].  Interior wavefronts store through
  // wave-uniform bases, as the pull loads (30.0 -> 29.2 us per reverse step
  // together with the buffer loads of lambda; at four waves per SIMD the
  // same forms had cost more in spilled registers than they saved).
  if (__all(x >= 1 && x <= k.nx - 2 && y >= 1 && y <= k.ny - 2)) {
    const uint32_t ob = uint32_t(o) * uint32_t(sizeof(R));
#pragma unroll
    for (int q = 0; q < 19; ++q)
      buffer_store(lam_out + (int64_t(q) * k.plane - int64_t(EY[q]) * k.pitch - EX[q]), ob, mu[q]);
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
    lam_out[off] = mu[q];
  }
}

// Gradient through the initial state: the O2 equilibrium at rest depends on
// b_C = 20 sqrt(3) D - 4 (Eq. 10).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_adj_init(const R* __restrict__ lam0, R* __restrict__ grad, Consts<R> k) {
  const int x = blockIdx.x * kBlock + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= k.nx) return;
  const int o = y * k.pitch + x;
  const R l0 = lam0[14 * k.plane + o];
  const R l14 = lam0[15 * k.plane + o] + lam0[16 * k.plane + o] + lam0[17 * k.plane + o] + lam0[18 * k.plane + o];
  grad[2 * k.plane + o] += R(34.64101615137754587) * k.c_in * (-l0 * R(0.2) + l14 * R(0.05));
}

// Pitched plane -> dense [ny][nx] caller array.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_unpitch(const R* __restrict__ src, R* __restrict__ dst, int nx, int pitch) {
  const int x = blockIdx.x * kBlock + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= nx) return;
  dst[(size_t)y * nx + x] = src[y * pitch + x];
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_fill(R* __restrict__ dst, int64_t n, R v) {
  const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i < n) dst[i] = v;
}

}  // namespace lbm
