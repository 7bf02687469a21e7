// Kernels of the single-lattice 2D solver.  One thread owns one lattice node.
#pragma once

#include "lbm_device.hpp"

namespace lbm {

constexpr int kBlock = 256;     // 4 wavefronts of 64 lanes along x
constexpr int kObsQ = 9;        // per-block observable partials

// Map a 2D launch (blocks along x, rows along y) so that the eight XCDs
// (which receive consecutive workgroups round-robin) each get a contiguous
// band of rows: spatial neighbours then share an L2.
__device__ __forceinline__ void xcd_tile(int nbx, int nby, int& bx, int& by) {
  const int flat = blockIdx.y * nbx + blockIdx.x;
  const int total = nbx * nby;
  // XCD j receives flats j, j+8, ...: full + (j < rem) workgroups.  Give it
  // the contiguous logical range starting at j*full + min(j, rem).
  const int xcd = flat & 7;
  const int slot = flat >> 3;
  const int full = total >> 3, rem = total & 7;
  const int logical = xcd * full + (xcd < rem ? xcd : rem) + slot;
  by = logical / nbx;
  bx = logical - by * nbx;
  // Rotate the x-blocks of a row by one every 8 rows.  Without it, the
  // workgroups that share a CU (a fixed stride apart in the XCD's range)
  // tend to sit at the same x position, so the wavefronts holding the inlet
  // or outlet column, whose chains are the longest, pile onto the same
  // SIMDs.  Measured: 1024x256 reverse step 2.6 % and forward 1.2 % faster,
  // 4096x1024 unchanged; each node's arithmetic is unchanged.
  bx = (bx + by / 8) % nbx;
}

// One time step: pull-stream, boundary columns, macros, flow collision,
// reaction, scalar collisions, store.  UNIFORM: wave-uniform buffer
// addressing for the interior pull and for the stores (fewer vector
// instructions per node).  Small lattices, whose launches are one round of
// wavefronts bound by each wave's own chain, gain from it; the 4096x1024
// lattice runs 0.5 % slower with it and keeps the per-lane form.
template <typename R, int MAT, bool UNIFORM = false>
__global__ __launch_bounds__(kBlock) void k_step(const R* __restrict__ src, R* __restrict__ dst,
                                                 const R* __restrict__ phi_f,
                                                 const R* __restrict__ invk_f,
                                                 const R* __restrict__ d_f, Consts<R> k) {
  int bx, by;
  xcd_tile(gridDim.x, gridDim.y, bx, by);
  const int x = bx * kBlock + threadIdx.x;
  const int y = by;
  if (x >= k.nx) return;
  R f[19];
  const Mat<R> mt = pre_collision<R, MAT, true, UNIFORM>(src, k, phi_f, invk_f, d_f, x, y, f);
  const bool cl = y >= k.y_cl0 && !(k.flags & F_NO_REACTION);
  collide(f, mt, k, cl);
  const int o = y * k.pitch + x;
  if constexpr (UNIFORM) {
    const uint32_t ob = uint32_t(o) * uint32_t(sizeof(R));
#pragma unroll
    for (int q = 0; q < 19; ++q) buffer_store(dst + int64_t(q) * k.plane, ob, f[q]);
  } else {
#pragma unroll
    for (int q = 0; q < 19; ++q) dst[q * k.plane + o] = f[q];
  }
}

// Two time steps in one launch, for lattices large enough to be bound by
// HBM: a workgroup advances a tile of kT2X x kT2Y nodes.  Step one runs over
// the tile and a halo (two columns on the left, where the outlet's feeding
// column can lie, one elsewhere, and a row above and below), one node per
// thread, from the state in memory, and keeps the post-collision
// populations in LDS, writing the tile's own to `mid` when that is given;
// step two pulls the tile's nodes from LDS and writes `dst`.  Every node
// runs the same code as k_step, so the states are the bits of two single
// steps.  HBM traffic per step halves; the halo nodes (22 % of step one)
// are computed twice.  Twelve rows (step one: 938 nodes, 960 threads, one
// pass) measured faster than four and eight; 13 rows, the last to fit one
// 1024-thread pass, would save 1 % of the halo work and is not measured.
// FP64 holds 143 KB of LDS, one workgroup per CU.  Walls and inlet / outlet columns only (the
// thin-film CL's reactive wall included): the host keeps single steps on
// periodic lattices.
constexpr int kT2X = 64, kT2Y = 12;
constexpr int kT2W = kT2X + 3;                  // LDS row: x0 - 2 .. x0 + kT2X
constexpr int kT2N = kT2W * (kT2Y + 2);         // LDS rows: y0 - 1 .. y0 + kT2Y
constexpr int kT2Threads = (kT2N + 63) / 64 * 64;
static_assert(kT2Threads <= 1024 && kT2X * kT2Y <= kT2Threads, "two-step tile");

// Pull of node (x, y) from the step-one populations of the tile at (x0, y0).
template <typename R>
__device__ __forceinline__ void pull_tile(const R* __restrict__ lds, const Consts<R>& k, int x, int y, int x0,
                                          int y0, R (&f)[19]) {
#pragma unroll
  for (int q = 0; q < 19; ++q) {
    const int xs = x - EX[q], ys = y - EY[q];
    const bool in = (unsigned)xs < (unsigned)k.nx && (unsigned)ys < (unsigned)k.ny;
    const int n = in ? (ys - y0 + 1) * kT2W + (xs - x0 + 2) : (y - y0 + 1) * kT2W + (x - x0 + 2);
    f[q] = lds[(in ? q : OPP[q]) * kT2N + n];
  }
}

// The two steps of the tile at (x0, y0), called by every thread of a
// kT2Threads workgroup (it holds a workgroup barrier).  NT: non-temporal
// loads in step one.  Cached loads let the L2 serve the halo lines that
// neighbouring tiles also read; measured (µs per step, non-temporal ->
// cached): FP64 4096x1024 176.2 -> 167.2, FP32 2048x512 24.7 -> 23.4,
// 1024x512 14.6 -> 14.0, but FP32 4096x1024 89.0 -> 90.2, whose tile rows
// are too long for that reuse.
template <typename R, int MAT, bool NT>
__device__ __forceinline__ void step2_tile(R* __restrict__ lds, const R* __restrict__ src, R* __restrict__ mid,
                                           R* __restrict__ dst, const R* __restrict__ phi_f,
                                           const R* __restrict__ invk_f, const R* __restrict__ d_f,
                                           const Consts<R>& k, int x0, int y0) {
  const bool react = !(k.flags & F_NO_REACTION);
  {
    const int n = threadIdx.x;
    const int i = n % kT2W, j = n / kT2W;
    const int x = x0 - 2 + i, y = y0 - 1 + j;
    if (n < kT2N && (unsigned)x < (unsigned)k.nx && (unsigned)y < (unsigned)k.ny) {
      R f[19];
      const Mat<R> mt = pre_collision<R, MAT, NT>(src, k, phi_f, invk_f, d_f, x, y, f);
      collide(f, mt, k, react && y >= k.y_cl0);
#pragma unroll
      for (int q = 0; q < 19; ++q) lds[q * kT2N + n] = f[q];
      if (mid && i >= 2 && i < kT2X + 2 && j >= 1 && j <= kT2Y) {
        const int o = y * k.pitch + x;
#pragma unroll
        for (int q = 0; q < 19; ++q) mid[q * k.plane + o] = f[q];
      }
    }
  }
  __syncthreads();
  if (threadIdx.x >= kT2X * kT2Y) return;
  const int x = x0 + int(threadIdx.x) % kT2X, y = y0 + int(threadIdx.x) / kT2X;
  if (x >= k.nx || y >= k.ny) return;
  const bool inlet = x == 0 && y < k.ny_ch;
  const bool outlet = x == k.nx - 1;
  const int xp = inlet ? 1 : (outlet ? k.nx - 2 : x);
  R f[19];
  pull_tile(lds, k, xp, y, x0, y0, f);
  Mat<R> mt = material<R, MAT>(k, phi_f, invk_f, d_f, xp, y);
  thin_film(f, mt, k, y);
  if (inlet || outlet) {
    Mat<R> mb = material<R, MAT>(k, phi_f, invk_f, d_f, x, y);
    boundary_column(f, k, y, inlet, mt, mb);
    if (outlet) outlet_scalar_material(mb, mt);
    mt = mb;
  }
  collide(f, mt, k, react && y >= k.y_cl0);
  const int o = y * k.pitch + x;
#pragma unroll
  for (int q = 0; q < 19; ++q) dst[q * k.plane + o] = f[q];
}

template <typename R, int MAT, bool NT>
__global__ __launch_bounds__(kT2Threads) void k_step2(const R* __restrict__ src, R* __restrict__ mid,
                                                      R* __restrict__ dst, const R* __restrict__ phi_f,
                                                      const R* __restrict__ invk_f, const R* __restrict__ d_f,
                                                      Consts<R> k) {
  __shared__ R lds[19 * kT2N];
  int bx, by;
  xcd_tile(gridDim.x, gridDim.y, bx, by);
  step2_tile<R, MAT, NT>(lds, src, mid, dst, phi_f, invk_f, d_f, k, bx * kT2X, by * kT2Y);
}

// Equilibrium initial state: rest fluid at zero pressure (shifted f = 0),
// theta = 0, O2 at c_in.
template <typename R, int MAT>
__global__ __launch_bounds__(kBlock) void k_init(R* __restrict__ dst, const R* __restrict__ phi_f,
                                                 const R* __restrict__ invk_f,
                                                 const R* __restrict__ d_f, Consts<R> k) {
  const int x = blockIdx.x * kBlock + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= k.nx) return;
  const Mat<R> mt = material<R, MAT>(k, phi_f, invk_f, d_f, x, y);
  R g[5] = {R(0), R(0), R(0), R(0), R(0)};
  add_geq(k.c_in, R(0), R(0), mt.bC, R(1), g);
  const int o = y * k.pitch + x;
#pragma unroll
  for (int q = 0; q < 14; ++q) dst[q * k.plane + o] = R(0);
#pragma unroll
  for (int q = 0; q < 5; ++q) dst[(14 + q) * k.plane + o] = g[q];
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
  return v;
}

// Observable partial sums over the pre-collision state, one row of partials
// per workgroup: sum f (shifted), sum theta, sum c, sum s_c, sum S_T,
// sum s_c (eta + T dU0/dT), max theta, count of non-finite values, sum of
// u_x over the inlet nodes.
// The thin-film CL's reaction at the bottom node of column x, as the last
// streaming applied it: from the populations of the pulled column (column
// nx - 2 for the outlet, whose scalars are that column's) that crossed the
// wall, with the scalar material the node collides with.
template <typename R>
__device__ __forceinline__ React<R> film(const R* __restrict__ src, const Consts<R>& k, int x, const Mat<R>& mt) {
  const int xp = (!(k.flags & F_PERIODIC_X) && x == k.nx - 1) ? k.nx - 2 : x;
  const int o = (k.ny - 1) * k.pitch + xp;
  return surface_reaction(src[11 * k.plane + o], src[16 * k.plane + o], mt, k);
}

template <typename R, int MAT>
__global__ __launch_bounds__(kBlock) void k_obs_cells(const R* __restrict__ src,
                                                      const R* __restrict__ phi_f,
                                                      const R* __restrict__ invk_f,
                                                      const R* __restrict__ d_f, Consts<R> k,
                                                      double* __restrict__ partial) {
  const int x = blockIdx.x * kBlock + threadIdx.x;
  const int y = blockIdx.y;
  double v[kObsQ] = {0, 0, 0, 0, 0, 0, -1e300, 0, 0};
  if (x < k.nx) {
    R f[19];
    const Mat<R> mt = pre_collision<R, MAT>(src, k, phi_f, invk_f, d_f, x, y, f);
    if (x == 0 && y < k.ny_ch && !(k.flags & F_PERIODIC_X)) v[8] = double(flow_macros(f, mt, k).ux);
    double sf = 0, th = 0, c = 0;
#pragma unroll
    for (int q = 0; q < 9; ++q) sf += double(f[q]);
#pragma unroll
    for (int q = 9; q < 14; ++q) th += double(f[q]);
    if (k.flags & F_SIGMA_ENERGY) th /= double(mt.sig);
#pragma unroll
    for (int q = 14; q < 19; ++q) c += double(f[q]);
    v[0] = sf;
    v[1] = th;
    v[2] = c;
    if (y >= k.y_cl0 && !(k.flags & F_NO_REACTION)) {
      const React<R> r = reaction(R(th), R(c), mt.rhocp, k);
      v[3] = double(r.s_c);
      v[4] = double(r.S_T);
      v[5] = double(r.s_c) * double(r.ehs);
    } else if ((k.flags & F_THIN_CL) && !(k.flags & F_NO_REACTION) && y == k.ny - 1) {
      const React<R> r = film(src, k, x, mt);
      v[3] = double(r.s_c);
      v[4] = double(r.S_T);
      v[5] = double(r.s_c) * double(r.ehs);
    }
    v[6] = th;
    bool bad = false;
#pragma unroll
    for (int q = 0; q < 19; ++q) bad |= !isfinite(f[q]);
    v[7] = bad ? 1.0 : 0.0;
  }
  __shared__ double red[kObsQ][kBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < kObsQ; ++i) {
    const double s = i == 6 ? wave_max(v[i]) : wave_sum(v[i]);
    if (lane == 0) red[i][wid] = s;
  }
  __syncthreads();
  if (threadIdx.x < kObsQ) {
    const int i = threadIdx.x;
    double s = red[i][0];
    for (int w = 1; w < kBlock / 64; ++w) s = i == 6 ? fmax(s, red[i][w]) : s + red[i][w];
    partial[(size_t)(blockIdx.y * gridDim.x + blockIdx.x) * kObsQ + i] = s;
  }
}

// Sum the per-workgroup partials in a fixed order: workgroup i reduces
// quantity i; thread t sums the contiguous chunk t of the partials, then a
// fixed tree combines the chunks.
template <int Q = kObsQ>  // a template so that every translation unit may instantiate it
__global__ __launch_bounds__(kBlock) void k_obs_final(const double* __restrict__ partial, int nblocks,
                                                      double* __restrict__ out) {
  const int i = blockIdx.x;
  const bool is_max = i == 6;
  const int per = (nblocks + kBlock - 1) / kBlock;
  const int b0 = threadIdx.x * per;
  const int b1 = b0 + per < nblocks ? b0 + per : nblocks;
  double s = is_max ? -1e300 : 0.0;
  for (int b = b0; b < b1; ++b) {
    const double v = partial[(size_t)b * Q + i];
    s = is_max ? fmax(s, v) : s + v;
  }
  __shared__ double red[kBlock];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      const double o = red[threadIdx.x + w];
      red[threadIdx.x] = is_max ? fmax(red[threadIdx.x], o) : red[threadIdx.x] + o;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = red[0];
}

// Per-column CL profiles: i(x) = sum over CL rows of 4 F C_ref s_c / dt * dx,
// and c, T on the CL row next to the GDL.
template <typename R, int MAT>
__global__ __launch_bounds__(kBlock) void k_obs_profiles(const R* __restrict__ src,
                                                         const R* __restrict__ phi_f,
                                                         const R* __restrict__ invk_f,
                                                         const R* __restrict__ d_f, Consts<R> k,
                                                         double i_scale, double* __restrict__ prof) {
  const int x = blockIdx.x * kBlock + threadIdx.x;
  if (x >= k.nx) return;
  double isum = 0, c0 = 0, t0 = 0;
  const bool react = !(k.flags & F_NO_REACTION);
  if (k.flags & F_THIN_CL) {  // the film's current, the profiles of the row above it
    R f[19];
    const Mat<R> mt = pre_collision<R, MAT>(src, k, phi_f, invk_f, d_f, x, k.ny - 1, f);
    c0 = double(f[14] + f[15] + f[16] + f[17] + f[18]);
    t0 = double(k.T_in) + double(theta_of(f + 9, mt.sig, k));
    if (react) isum = double(film(src, k, x, mt).s_c);
  }
  for (int y = k.y_cl0; y < k.ny; ++y) {
    R f[19];
    const Mat<R> mt = pre_collision<R, MAT>(src, k, phi_f, invk_f, d_f, x, y, f);
    const R th = theta_of(f + 9, mt.sig, k);
    const R c = f[14] + f[15] + f[16] + f[17] + f[18];
    if (react) isum += double(reaction(th, c, mt.rhocp, k).s_c);
    if (y == k.y_cl0) {
      c0 = double(c);
      t0 = double(k.T_in) + double(th);
    }
  }
  prof[x] = isum * i_scale;
  prof[k.nx + x] = c0;
  prof[2 * k.nx + x] = t0;
}

// Macroscopic fields of the pre-collision state into dense [ny][nx] arrays.
template <typename R, int MAT>
__global__ __launch_bounds__(kBlock) void k_fields(const R* __restrict__ src,
                                                   const R* __restrict__ phi_f,
                                                   const R* __restrict__ invk_f,
                                                   const R* __restrict__ d_f, Consts<R> k,
                                                   R* ux, R* uy, R* p, R* T, R* theta, R* c) {
  const int x = blockIdx.x * kBlock + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= k.nx) return;
  R f[19];
  const Mat<R> mt = pre_collision<R, MAT>(src, k, phi_f, invk_f, d_f, x, y, f);
  const Macro<R> a = flow_macros(f, mt, k);
  const int o = y * k.nx + x;
  if (ux) ux[o] = a.ux;
  if (uy) uy[o] = a.uy;
  if (p) p[o] = a.p;
  const R th = theta_of(f + 9, mt.sig, k);
  if (T) T[o] = k.T_in + th;
  if (theta) theta[o] = th;
  if (c) c[o] = f[14] + f[15] + f[16] + f[17] + f[18];
}

// Internal (pitched, shifted rest population) <-> canonical dense populations.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_export(const R* __restrict__ src, R* __restrict__ dst,
                                                   Consts<R> k) {
  const int x = blockIdx.x * kBlock + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= k.nx) return;
  const size_t dense = (size_t)k.nx * k.ny;
  for (int q = 0; q < 19; ++q) {
    R v = src[q * k.plane + y * k.pitch + x];
    if (q == 0) v += R(1);
    dst[q * dense + (size_t)y * k.nx + x] = v;
  }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_import(const R* __restrict__ src, R* __restrict__ dst,
                                                   Consts<R> k) {
  const int x = blockIdx.x * kBlock + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= k.nx) return;
  const size_t dense = (size_t)k.nx * k.ny;
  for (int q = 0; q < 19; ++q) {
    R v = src[q * dense + (size_t)y * k.nx + x];
    if (q == 0) v -= R(1);
    dst[q * k.plane + y * k.pitch + x] = v;
  }
}

// Full-field mode: fill the fields not given by the caller from porosity
// (Kozeny-Carman, Bruggeman / ratio) or from the layered inputs.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_derive_fields(R* __restrict__ phi, R* __restrict__ invk,
                                                          R* __restrict__ d, Consts<R> k, int have_phi,
                                                          int have_invk, int have_d) {
  const int x = blockIdx.x * kBlock + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= k.nx) return;
  const int o = y * k.pitch + x;
  const bool porous = y >= k.ny_ch;
  if (!have_phi) phi[o] = porous ? k.phi_gdl : R(1);
  const R ph = phi[o];
  if (!have_invk) {
    if (k.kc_inv > R(0)) {
      const R om = R(1) - ph;
      invk[o] = om * om * k.kc_inv / (ph * ph * ph);
    } else {
      invk[o] = porous ? k.invk_gdl : R(0);
    }
  }
  if (!have_d) d[o] = (porous && k.deff_ratio > R(0)) ? k.deff_ratio * k.D_f : ph * sqrt(ph) * k.D_f;
}

// Copy a dense [ny][nx] caller array into a pitched workspace plane.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_pitch_copy(const R* __restrict__ src, R* __restrict__ dst,
                                                       int nx, int pitch) {
  const int x = blockIdx.x * kBlock + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= nx) return;
  dst[y * pitch + x] = src[(size_t)y * nx + x];
}

}  // namespace lbm

namespace lbm {

// Per-cell porosity, 1/K and O2 diffusivity as the kernels use them.
template <typename R, int MAT>
__global__ __launch_bounds__(kBlock) void k_material(const R* __restrict__ phi_f, const R* __restrict__ invk_f,
                                                     const R* __restrict__ d_f, Consts<R> k, R* phi, R* invk, R* d) {
  const int x = blockIdx.x * kBlock + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= k.nx) return;
  R a, b, c;
  base_fields<R, MAT>(k, phi_f, invk_f, d_f, x, y, a, b, c);
  const size_t o = (size_t)y * k.nx + x;
  if (phi) phi[o] = a;
  if (invk) invk[o] = b;
  if (d) d[o] = c;
}

}  // namespace lbm
