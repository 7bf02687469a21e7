// Batched parameter sweep: many independent layered cathode lattices of
// uneven sizes advanced together.  The lattices live in one pool; a flat
// list of equal-shape tiles (case, x0, y0) covers all of them.  Two launch
// forms share the per-tile body:
//   k_batch_step        one workgroup per tile, one launch per time step;
//   k_batch_persistent  one cooperative launch for many steps: each
//                       workgroup owns a contiguous chunk of tiles and the
//                       grid synchronizes between steps (a barrier whose
//                       wait is bounded: a grid that is not co-resident
//                       fails the launch instead of hanging it).
#pragma once

#include "lbm_kernels2d.hpp"

namespace lbm {

template <typename R>
struct BatchCase {
  Consts<R> k;
  int64_t off[2];  // element offsets of the two state buffers in the pool
};

struct Tile {
  int32_t c, x0, y0, pad;
};

// Per-cell fields of a batch whose cases carry them (MAT_FULL): rows 19, 20
// and 21 of every lattice row of the case's first state buffer hold
// porosity, 1/K and D_eff, so that they share the populations' row
// interleave (element y * pitch + x of the planes at 19, 20, 21 rows).
constexpr int kFieldRow = 19;

// Advance cell i (row-major inside the tile) of a tile.  UNIFORM: wave-
// uniform buffer addressing for the interior pull and the stores (batches
// of few nodes, whose launches are one round of wavefronts).  MAT: the
// material of every case, MAT_LAYERED or MAT_FULL (fields at `fields`).
template <typename R, int MAT, bool UNIFORM = false>
__device__ __forceinline__ void batch_cell(const R* __restrict__ src, R* __restrict__ dst, const Consts<R>& k,
                                           const R* __restrict__ fields, const Tile& t, int i, int tx) {
  const int y = t.y0 + i / tx;
  const int x = t.x0 + i % tx;
  if (x >= k.nx || y >= k.ny) return;
  R f[19];
  const R* invk_f = MAT == MAT_LAYERED ? nullptr : fields + k.plane;
  const R* d_f = MAT == MAT_LAYERED ? nullptr : fields + 2 * k.plane;
  const Mat<R> mt = pre_collision<R, MAT, false, UNIFORM>(src, k, fields, invk_f, d_f, x, y, f);
  collide(f, mt, k, y >= k.y_cl0 && !(k.flags & F_NO_REACTION));
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

// Advance the cells of one tile (tx x ty cells).  ONE: the tile has exactly
// one cell per thread (tx ty = kBlock); without the cell loop the kernel
// needs 59 instead of 76 VGPRs (8 instead of 6 waves per SIMD in FP32).
template <typename R, int MAT, bool ONE, bool UNIFORM = false>
__device__ __forceinline__ void batch_tile(R* __restrict__ pool, const BatchCase<R>* __restrict__ cases,
                                           const Tile& t, int parity, int tx, int ty) {
  const Consts<R> k = cases[t.c].k;
  const int64_t o_src = cases[t.c].off[parity], o_dst = cases[t.c].off[parity ^ 1];
  const R* src = pool + o_src;
  R* dst = pool + o_dst;
  const R* fields = MAT == MAT_LAYERED ? nullptr : pool + cases[t.c].off[0] + int64_t(kFieldRow) * k.plane;
  if constexpr (ONE) {
    batch_cell<R, MAT, UNIFORM>(src, dst, k, fields, t, threadIdx.x, tx);
  } else {
    const int n = tx * ty;
    for (int i = threadIdx.x; i < n; i += blockDim.x) batch_cell<R, MAT, UNIFORM>(src, dst, k, fields, t, i, tx);
  }
}

// Logical index of this workgroup such that each XCD (workgroups are dealt
// to the 8 XCDs round-robin) owns a contiguous range of logical indices.
__device__ __forceinline__ int xcd_logical(int flat, int total) {
  const int xcd = flat & 7, slot = flat >> 3;
  const int full = total >> 3, rem = total & 7;
  return xcd * full + (xcd < rem ? xcd : rem) + slot;
}

// BS: workgroup size.  Tiles of exactly BS cells (64, 128 or 256) run one
// cell per thread; other tiles loop over their cells with 256 threads.
template <typename R, int MAT, bool ONE, bool UNIFORM, int BS = kBlock>
__global__ __launch_bounds__(BS) void k_batch_step(R* __restrict__ pool, const BatchCase<R>* __restrict__ cases,
                                                   const Tile* __restrict__ tiles, int ntiles, int parity, int tx,
                                                   int ty) {
  const int t = xcd_logical(blockIdx.x, gridDim.x);
  if (t >= ntiles) return;
  batch_tile<R, MAT, ONE, UNIFORM>(pool, cases, tiles[t], parity, tx, ty);
}

// Two steps per launch: one kT2Threads workgroup per tile of kT2X x kT2Y
// nodes (the tile list of that shape), the body of k_step2 on the tile's
// case.  Cases with periodic axes are not scheduled so.
template <typename R, int MAT>
__global__ __launch_bounds__(kT2Threads) void k_batch_step2(R* __restrict__ pool,
                                                            const BatchCase<R>* __restrict__ cases,
                                                            const Tile* __restrict__ tiles, int ntiles, int parity) {
  __shared__ R lds[19 * kT2N];
  const int t = xcd_logical(blockIdx.x, gridDim.x);
  if (t >= ntiles) return;  // the whole workgroup: no thread reaches the barrier
  const Tile tl = tiles[t];
  const Consts<R> k = cases[tl.c].k;
  const R* src = pool + cases[tl.c].off[parity];
  R* dst = pool + cases[tl.c].off[parity ^ 1];
  const R* fields = MAT == MAT_LAYERED ? nullptr : pool + cases[tl.c].off[0] + int64_t(kFieldRow) * k.plane;
  const R* invk_f = MAT == MAT_LAYERED ? nullptr : fields + k.plane;
  const R* d_f = MAT == MAT_LAYERED ? nullptr : fields + 2 * k.plane;
  step2_tile<R, MAT, false>(lds, src, nullptr, dst, fields, invk_f, d_f, k, tl.x0, tl.y0);
}

// Waves per SIMD the persistent kernel is compiled for (at least): the
// compiler keeps both its vector and its scalar registers within what that
// many waves can hold, so a grid of that many 256-lane workgroups per CU
// (four waves, one per SIMD) is co-resident.  The scalar registers matter:
// at 106 of them (112 allocated of 800 per SIMD) only 7 waves fit, however
// few vector registers the kernel uses.
template <typename R>
struct PersistentWaves;
template <>
struct PersistentWaves<float> {
  static constexpr int value = 6;
};
template <>
struct PersistentWaves<double> {
  static constexpr int value = 2;
};

// Grid-wide barrier of the persistent kernel, in two levels.  The
// workgroups form 8 groups (blockIdx.x mod 8, the XCD the dispatcher deals
// them to); each arrival adds to its group's count, and the group's last
// arrival of a step adds to the global count, which the waiters read:
// count[64 (1 + g)] holds group g's arrivals since the launch, count[0] the
// groups' (all cleared before the launch, 256 bytes apart).  Step s ends
// when count[0] reaches (s + 1) times the number of groups.  One count for
// every workgroup cost 125 us per step for the barrier alone on MI355X (1536
// workgroups), two levels 25 us.  A wait longer than `limit` wall-clock
// ticks (seconds, where a step takes micro- to milliseconds) means
// workgroups that never started: the waiter sets `failed`, and every
// workgroup that sees it leaves the kernel.
constexpr int kBarrierWords = 9;  // the global count and 8 group counts
struct GridBarrier {
  unsigned int* count;
  int* failed;
  long long limit;
};

// Only the arriving thread fences.  Every wavefront first waits for its
// stores of the step to complete into the XCD's L2 and meets the others at
// the workgroup barrier; the arriving thread's release fence at device scope
// then writes that L2 back, and its acquire fence after the wait invalidates
// this CU's L1 and the L2's stale lines before the second workgroup barrier
// lets the other threads load.  On gfx950 each device-scope fence is an L2
// write-back or invalidate of the whole XCD; fencing in every wavefront
// multiplied them by four and invalidated lines that workgroups still inside
// the step were reading.
__device__ __forceinline__ bool grid_barrier(const GridBarrier& gb, unsigned int step) {
  __shared__ int ok;
  // every wavefront's stores acknowledged by the L2 (s_waitcnt vmcnt(0);
  // expcnt and lgkmcnt left at their maxima) before the arriving thread's
  // write-back
  __builtin_amdgcn_s_waitcnt(0x0F70);
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // the workgroup's stores of the step, visible at device scope
    const unsigned groups = gridDim.x < 8u ? gridDim.x : 8u;
    const unsigned g = blockIdx.x & 7u;
    const unsigned members = gridDim.x / 8u + (g < gridDim.x % 8u ? 1u : 0u);
    const unsigned before =
        __hip_atomic_fetch_add(gb.count + 64 * (1 + g), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (before + 1u == step * members) {  // the group's last arrival: its members' releases, passed on
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
      __hip_atomic_fetch_add(gb.count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const unsigned target = step * groups;
    const long long t0 = wall_clock64();
    int good = 1;
    while (__hip_atomic_load(gb.count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(gb.failed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
          wall_clock64() - t0 > gb.limit) {
        __hip_atomic_store(gb.failed, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        good = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(4);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the other workgroups' stores, seen by this workgroup's loads
    ok = good;
  }
  __syncthreads();
  return ok != 0;
}

__global__ void k_clear_barrier(unsigned int* count, int* failed, int clear_failed) {
  if (threadIdx.x < kBarrierWords) count[64 * threadIdx.x] = 0u;
  if (threadIdx.x == 0 && clear_failed) *failed = 0;
}

// The persistent form keeps the cell loop for every tile shape.
template <typename R, int MAT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(PersistentWaves<R>::value)))
void k_batch_persistent(R* __restrict__ pool, const BatchCase<R>* __restrict__ cases,
                        const Tile* __restrict__ tiles, int ntiles, int nsteps, int parity0, int tx, int ty,
                        GridBarrier gb) {
  const int lb = xcd_logical(blockIdx.x, gridDim.x);
  const int t0 = int((int64_t(lb) * ntiles) / gridDim.x);
  const int t1 = int((int64_t(lb + 1) * ntiles) / gridDim.x);
  for (int s = 0; s < nsteps; ++s) {
    const int parity = (parity0 + s) & 1;
    for (int t = t0; t < t1; ++t) batch_tile<R, MAT, false>(pool, cases, tiles[t], parity, tx, ty);
    if (!grid_barrier(gb, unsigned(s + 1))) return;
  }
}

}  // namespace lbm
