// Kernels of the 3D solver.  One thread owns one lattice node; a workgroup
// covers kBlock3 consecutive nodes of one (y, z) row.
#pragma once

#include "lbm3d_device.hpp"
#include "lbm_kernels2d.hpp"  // wave reductions and the fixed-order final reduction

namespace lbm3 {

constexpr int kBlock3 = 256;
constexpr int kObsQ3 = 9;

// Row order of the launch.  Rows (y, z) are visited in chunks of `ty`
// consecutive y: all z of the first chunk, then all z of the next, so the
// rows a z-neighbour pull touches were loaded ty rows earlier (not ny).  The
// eight XCDs receive consecutive workgroups round-robin; each gets one
// contiguous range of this order, so z- and y-neighbours share an L2.
__device__ __forceinline__ void row_of(int flat, int total, int nbx, int ny, int nz, int ty, int& bx, int& y,
                                       int& z) {
  const int xcd = flat & 7;
  const int slot = flat >> 3;
  const int full = total >> 3, rem = total & 7;
  const int logical = xcd * full + (xcd < rem ? xcd : rem) + slot;
  const int row = logical / nbx;
  bx = logical - row * nbx;
  const int per_chunk = ty * nz;
  const int chunk = row / per_chunk;
  const int y0 = chunk * ty;
  const int h = (ny - y0) < ty ? (ny - y0) : ty;  // the last chunk may be short
  const int r = row - chunk * per_chunk;
  z = r / h;
  y = y0 + (r - z * h);
}

template <typename R>
__device__ __forceinline__ void node_of(const Consts3<R>& k, int& x, int& y, int& z) {
  const int nbx = (k.nx + kBlock3 - 1) / kBlock3;
  int bx;
  row_of(blockIdx.x, gridDim.x, nbx, k.ny, k.nz, k.ty, bx, y, z);
  x = bx * kBlock3 + threadIdx.x;
}

// Waves per SIMD the FP32 step is compiled for: the flow and scalar passes
// of step_node and the wave-uniform loads and stores keep it at 63 VGPRs (8
// waves) with no spill, where the single-pass form needed 89 (5 waves).
// The FP64 instance is left unconstrained.
template <typename R>
struct StepWaves3 {
  static constexpr int value = sizeof(R) == 4 ? 8 : 1;
};

template <typename R, int MAT>
__global__ __launch_bounds__(kBlock3) __attribute__((amdgpu_waves_per_eu(StepWaves3<R>::value)))
void k3_step(const R* __restrict__ src, R* __restrict__ dst, const R* __restrict__ phi_f,
             const R* __restrict__ invk_f, const R* __restrict__ d_f, Consts3<R> k) {
  int x, y, z;
  node_of(k, x, y, z);
  if (x >= k.nx) return;
  step_node<R, MAT>(src, dst, phi_f, invk_f, d_f, k, x, y, z);
}

// Rest fluid at zero pressure (shifted f = 0), theta = 0, O2 at c_in.
template <typename R, int MAT>
__global__ __launch_bounds__(kBlock3) void k3_init(R* __restrict__ dst, const R* __restrict__ phi_f,
                                                   const R* __restrict__ invk_f, const R* __restrict__ d_f,
                                                   Consts3<R> k) {
  const int x = blockIdx.x * kBlock3 + threadIdx.x;
  const int y = blockIdx.y, z = blockIdx.z;
  if (x >= k.nx) return;
  const Mat3<R> mt = material<R, MAT>(k, phi_f, invk_f, d_f, x, y, z);
  R g[7] = {R(0), R(0), R(0), R(0), R(0), R(0), R(0)};
  add_geq(k.c_in, R(0), R(0), R(0), mt.aC, R(1), g);
  const int o = (z * k.ny + y) * k.pitch + x;
#pragma unroll
  for (int q = 0; q < 26; ++q) dst[q * k.plane + o] = R(0);
#pragma unroll
  for (int q = 0; q < 7; ++q) dst[(26 + q) * k.plane + o] = g[q];
}

// Per-workgroup observable partials of the pre-collision state: sum f
// (shifted), sum theta, sum c, sum s_c, sum S_T, sum s_c (eta + T dU0/dT),
// max theta, count of non-finite populations, sum of u_x over the inlet nodes.
template <typename R, int MAT>
__global__ __launch_bounds__(kBlock3) void k3_obs_cells(const R* __restrict__ src, const R* __restrict__ phi_f,
                                                        const R* __restrict__ invk_f, const R* __restrict__ d_f,
                                                        Consts3<R> k, double* __restrict__ partial) {
  const int x = blockIdx.x * kBlock3 + threadIdx.x;
  const int y = blockIdx.y, z = blockIdx.z;
  double v[kObsQ3] = {0, 0, 0, 0, 0, 0, -1e300, 0, 0};
  if (x < k.nx) {
    R f[33];
    const Mat3<R> mt = pre_collision<R, MAT>(src, k, phi_f, invk_f, d_f, x, y, z, f);
    if (x == 0 && z < k.nz_ch && !(k.flags & F_PERIODIC_X)) v[8] = double(flow_macros(f, mt, k).ux);
    double sf = 0, th = 0, c = 0;
#pragma unroll
    for (int q = 0; q < 19; ++q) sf += double(f[q]);
#pragma unroll
    for (int q = 19; q < 26; ++q) th += double(f[q]);
#pragma unroll
    for (int q = 26; q < 33; ++q) c += double(f[q]);
    v[0] = sf;
    v[1] = th;
    v[2] = c;
    if (z >= k.z_cl0 && !(k.flags & F_NO_REACTION)) {
      const lbm::React<R> r = reaction(R(th), R(c), mt.rhocp, k);
      v[3] = double(r.s_c);
      v[4] = double(r.S_T);
      v[5] = double(r.s_c) * double(r.ehs);
    }
    v[6] = th;
    bool bad = false;
#pragma unroll
    for (int q = 0; q < 33; ++q) bad |= !isfinite(f[q]);
    v[7] = bad ? 1.0 : 0.0;
  }
  __shared__ double red[kObsQ3][kBlock3 / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < kObsQ3; ++i) {
    const double s = i == 6 ? lbm::wave_max(v[i]) : lbm::wave_sum(v[i]);
    if (lane == 0) red[i][wid] = s;
  }
  __syncthreads();
  if (threadIdx.x < kObsQ3) {
    const int i = threadIdx.x;
    double s = red[i][0];
    for (int w = 1; w < kBlock3 / 64; ++w) s = i == 6 ? fmax(s, red[i][w]) : s + red[i][w];
    const size_t b = (size_t(blockIdx.z) * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    partial[b * kObsQ3 + i] = s;
  }
}

// Macroscopic fields of the pre-collision state into dense [nz][ny][nx].
template <typename R, int MAT>
__global__ __launch_bounds__(kBlock3) void k3_fields(const R* __restrict__ src, const R* __restrict__ phi_f,
                                                     const R* __restrict__ invk_f, const R* __restrict__ d_f,
                                                     Consts3<R> k, R* ux, R* uy, R* uz, R* p, R* T, R* theta, R* c) {
  const int x = blockIdx.x * kBlock3 + threadIdx.x;
  const int y = blockIdx.y, z = blockIdx.z;
  if (x >= k.nx) return;
  R f[33];
  const Mat3<R> mt = pre_collision<R, MAT>(src, k, phi_f, invk_f, d_f, x, y, z, f);
  const Macro3<R> a = flow_macros(f, mt, k);
  const size_t o = (size_t(z) * k.ny + y) * k.nx + x;
  if (ux) ux[o] = a.ux;
  if (uy) uy[o] = a.uy;
  if (uz) uz[o] = a.uz;
  if (p) p[o] = a.p;
  R th = R(0), cc = R(0);
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    th += f[19 + q];
    cc += f[26 + q];
  }
  if (T) T[o] = k.T_in + th;
  if (theta) theta[o] = th;
  if (c) c[o] = cc;
}

// Internal (pitched, shifted rest population) <-> canonical dense planes.
template <typename R>
__global__ __launch_bounds__(kBlock3) void k3_export(const R* __restrict__ src, R* __restrict__ dst, Consts3<R> k) {
  const int x = blockIdx.x * kBlock3 + threadIdx.x;
  const int y = blockIdx.y, z = blockIdx.z;
  if (x >= k.nx) return;
  const size_t dense = size_t(k.nx) * k.ny * k.nz;
  const size_t od = (size_t(z) * k.ny + y) * k.nx + x;
  const int oi = (z * k.ny + y) * k.pitch + x;
  for (int q = 0; q < 33; ++q) {
    R v = src[q * k.plane + oi];
    if (q == 0) v += R(1);
    dst[q * dense + od] = v;
  }
}

template <typename R>
__global__ __launch_bounds__(kBlock3) void k3_import(const R* __restrict__ src, R* __restrict__ dst, Consts3<R> k) {
  const int x = blockIdx.x * kBlock3 + threadIdx.x;
  const int y = blockIdx.y, z = blockIdx.z;
  if (x >= k.nx) return;
  const size_t dense = size_t(k.nx) * k.ny * k.nz;
  const size_t od = (size_t(z) * k.ny + y) * k.nx + x;
  const int oi = (z * k.ny + y) * k.pitch + x;
  for (int q = 0; q < 33; ++q) {
    R v = src[q * dense + od];
    if (q == 0) v -= R(1);
    dst[q * k.plane + oi] = v;
  }
}

// Full-field mode: fill the fields the caller did not give.
template <typename R>
__global__ __launch_bounds__(kBlock3) void k3_derive_fields(R* __restrict__ phi, R* __restrict__ invk,
                                                            R* __restrict__ d, Consts3<R> k, int have_phi,
                                                            int have_invk, int have_d) {
  const int x = blockIdx.x * kBlock3 + threadIdx.x;
  const int y = blockIdx.y, z = blockIdx.z;
  if (x >= k.nx) return;
  const int o = (z * k.ny + y) * k.pitch + x;
  const bool porous = z >= k.nz_ch;
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

template <typename R>
__global__ __launch_bounds__(kBlock3) void k3_pitch_copy(const R* __restrict__ src, R* __restrict__ dst, int nx,
                                                         int ny, int pitch) {
  const int x = blockIdx.x * kBlock3 + threadIdx.x;
  const int y = blockIdx.y, z = blockIdx.z;
  if (x >= nx) return;
  dst[(z * ny + y) * pitch + x] = src[(size_t(z) * ny + y) * nx + x];
}

// Per-cell porosity, 1/K and O2 diffusivity as the update uses them.
template <typename R, int MAT>
__global__ __launch_bounds__(kBlock3) void k3_material(const R* __restrict__ phi_f, const R* __restrict__ invk_f,
                                                       const R* __restrict__ d_f, Consts3<R> k, R* phi, R* invk,
                                                       R* d) {
  const int x = blockIdx.x * kBlock3 + threadIdx.x;
  const int y = blockIdx.y, z = blockIdx.z;
  if (x >= k.nx) return;
  const Mat3<R> m = material<R, MAT>(k, phi_f, invk_f, d_f, x, y, z);
  const size_t o = (size_t(z) * k.ny + y) * k.nx + x;
  if (phi) phi[o] = m.phi;
  if (invk) invk[o] = m.invk;
  if (d) d[o] = m.d;
}

}  // namespace lbm3
