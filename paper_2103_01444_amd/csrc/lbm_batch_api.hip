// Host side of the batched sweep (lbm_batch_* in include/lbm_pem.h).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <new>
#include <string>
#include <vector>

#include "lbm_batch.hpp"
#include "lbm_host.hpp"
#include "lbm_pem.h"

using namespace lbm;

namespace {

constexpr size_t kAlign = 256;
constexpr int kMinTileCells = 64;  // smallest tile the schedule accepts (sizes the tile table)
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct BatchLayout {
  std::vector<int64_t> state_off[2];  // element offsets per case
  int64_t pool_elems = 0;
  size_t off_pool = 0, off_backup = 0, off_cases = 0, off_tiles = 0, off_partial = 0, off_prof = 0, off_out = 0;
  size_t off_sync = 0;  // the persistent kernel's barrier: its counts (256 B apart), then the failure flag
  size_t total = 0;
  int max_tiles = 0;
  int max_obs_blocks = 0;
  int max_nx = 0;
  size_t esize = 4;
  int rows = 19;        // rows per lattice row of a state buffer: 19 populations (+ 3 field rows)
  bool fields = false;  // the cases carry per-cell fields (LBM_CELL_FIELDS)
};

bool batch_geometry_ok(const lbm_geometry* g, int n) {
  if (!g || n < 1) return false;
  for (int i = 0; i < n; ++i) {
    if (!geometry_ok(&g[i])) return false;
    if (g[i].precision != g[0].precision) return false;
    if ((g[i].flags & LBM_CELL_FIELDS) != (g[0].flags & LBM_CELL_FIELDS)) return false;
    if ((g[i].flags & LBM_CELL_FIELDS) && (int64_t(pitch_of(g[i].nx)) * g[i].ny * 22 >= (int64_t(1) << 31)))
      return false;  // 32-bit element offsets with the field rows
  }
  return true;
}

BatchLayout make_batch_layout(const lbm_geometry* g, int n) {
  BatchLayout L;
  L.esize = g[0].precision == 64 ? 8 : 4;
  L.fields = (g[0].flags & LBM_CELL_FIELDS) != 0;
  L.rows = L.fields ? kFieldRow + 3 : 19;
  int64_t e = 0;
  L.state_off[0].resize(n);
  L.state_off[1].resize(n);
  for (int i = 0; i < n; ++i) {
    const int64_t plane = plane_elems(int64_t(pitch_of(g[i].nx)) * g[i].ny);
    for (int s = 0; s < 2; ++s) {
      L.state_off[s][i] = e;
      e += (L.rows * plane + 63) / 64 * 64;  // 256-byte aligned per buffer
    }
    L.max_tiles += int((int64_t(pitch_of(g[i].nx)) * g[i].ny + kMinTileCells - 1) / kMinTileCells);
    L.max_obs_blocks = std::max(L.max_obs_blocks, ((g[i].nx + kBlock - 1) / kBlock) * g[i].ny);
    L.max_nx = std::max(L.max_nx, g[i].nx);
  }
  L.pool_elems = e;
  size_t o = 0;
  L.off_pool = o;
  o += align_up(size_t(e) * L.esize);
  L.off_backup = o;  // one state per case, for autotuning trials
  o += align_up(size_t(e) * L.esize / 2 + size_t(n) * 256);  // half the pool: one of the two buffers
  L.off_cases = o;
  o += align_up(size_t(n) * (L.esize == 8 ? sizeof(BatchCase<double>) : sizeof(BatchCase<float>)));
  L.off_tiles = o;
  o += align_up(size_t(L.max_tiles) * sizeof(Tile));
  L.off_partial = o;
  o += align_up(size_t(L.max_obs_blocks) * kObsQ * sizeof(double));
  L.off_prof = o;
  o += align_up(size_t(3) * L.max_nx * sizeof(double));
  L.off_out = o;
  o += align_up(16 * sizeof(double));
  L.off_sync = o;
  o += align_up(size_t(kBarrierWords + 1) * 256);
  L.total = o;
  return L;
}

}  // namespace

struct lbm_batch {
  int n = 0;
  std::vector<lbm_geometry> g;
  std::vector<lbm_params> p;
  std::vector<Derived> d;
  std::vector<Consts<float>> kf;
  std::vector<Consts<double>> kd;
  BatchLayout L;
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  int parity = 0;  // state buffer index holding the current state
  int64_t step = 0;
  lbm_schedule sched{256, 1, 0, 0};
  int ntiles = 0;
  int persistent_grid = 0;
  long long barrier_limit = 0;  // wall-clock ticks a persistent barrier waits at most
  int wall_khz = 0;             // the device wall clock's rate
  int64_t cells = 0;  // lattice nodes over all cases
  std::string err;

  template <typename R>
  R* pool() { return reinterpret_cast<R*>(ws + L.off_pool); }
  template <typename R>
  BatchCase<R>* cases() { return reinterpret_cast<BatchCase<R>*>(ws + L.off_cases); }
  // porosity row of case i (1/K and D_eff one and two row lengths further)
  template <typename R>
  R* field_rows(int i) { return pool<R>() + L.state_off[0][i] + int64_t(kFieldRow) * pitch_of(g[i].nx); }
  // elements of one state buffer of case i
  size_t state_elems(int i) const { return size_t(L.rows) * plane_elems(int64_t(pitch_of(g[i].nx)) * g[i].ny); }
  Tile* tiles() { return reinterpret_cast<Tile*>(ws + L.off_tiles); }
  double* partial() { return reinterpret_cast<double*>(ws + L.off_partial); }
  double* prof() { return reinterpret_cast<double*>(ws + L.off_prof); }
  double* out() { return reinterpret_cast<double*>(ws + L.off_out); }
  unsigned int* barrier_count() { return reinterpret_cast<unsigned int*>(ws + L.off_sync); }
  int* barrier_failed() { return reinterpret_cast<int*>(ws + L.off_sync + size_t(kBarrierWords) * 256); }
};

namespace {

lbm_status bfail(lbm_batch* b, lbm_status s, const std::string& m) {
  if (b) b->err = m;
  return s;
}

template <typename R>
const Consts<R>& bconsts(const lbm_batch* b, int i);
template <>
const Consts<float>& bconsts<float>(const lbm_batch* b, int i) { return b->kf[i]; }
template <>
const Consts<double>& bconsts<double>(const lbm_batch* b, int i) { return b->kd[i]; }

// Fill the field rows of case i that were not given (have_* = 0) from its
// layers and porosity, as lbm_set_params does for a context with
// independent_fields = 1.
template <typename R>
lbm_status derive_case_fields(lbm_batch* b, int i, int have_phi, int have_invk, int have_d) {
  R* f = b->field_rows<R>(i);
  const int64_t L = pitch_of(b->g[i].nx);
  const dim3 grid((b->g[i].nx + kBlock - 1) / kBlock, b->g[i].ny);
  hipLaunchKernelGGL(k_derive_fields<R>, grid, dim3(kBlock), 0, b->stream, f, f + L, f + 2 * L, bconsts<R>(b, i),
                     have_phi, have_invk, have_d);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? LBM_OK : bfail(b, LBM_ERR_DEVICE, std::string("field derivation: ") + hipGetErrorString(e));
}

// Smallest and largest value of a dense device array of n elements (lo =
// -1e300 if any is not finite).  Synchronous.
template <typename R>
bool device_range(hipStream_t stream, const void* dev, size_t n, double& lo, double& hi) {
  std::vector<R> h(n);
  if (hipMemcpyAsync(h.data(), dev, n * sizeof(R), hipMemcpyDeviceToHost, stream) != hipSuccess) return false;
  if (hipStreamSynchronize(stream) != hipSuccess) return false;
  for (size_t j = 0; j < n; ++j) {
    const double v = double(h[j]);
    if (!std::isfinite(v)) {
      lo = -1e300;
      return true;
    }
    lo = std::min(lo, v);
    hi = std::max(hi, v);
  }
  return true;
}

// Per-cell fields of case i: the given arrays are checked as lbm_set_params
// checks them, copied into the case's field rows, and the missing ones
// derived.
template <typename R>
lbm_status set_fields_t(lbm_batch* b, int i, const void* phi, const void* inv_k, const void* d_eff) {
  const lbm_geometry& g = b->g[i];
  const lbm_params& p = b->p[i];
  const Derived& dv = b->d[i];
  const size_t n = size_t(g.nx) * g.ny;
  const std::string which = "case " + std::to_string(i) + ": ";
  double phi_lo = p.phi_gdl, phi_hi = 1.0, d_lo = std::min(dv.d_gdl, p.D_f_lat), d_hi = std::max(dv.d_gdl, p.D_f_lat);
  double k_lo = dv.invk_gdl, k_hi = dv.invk_gdl;
  if (phi && !device_range<R>(b->stream, phi, n, phi_lo, phi_hi))
    return bfail(b, LBM_ERR_DEVICE, which + "reading porosity failed");
  if (inv_k && !device_range<R>(b->stream, inv_k, n, k_lo, k_hi))
    return bfail(b, LBM_ERR_DEVICE, which + "reading 1/K failed");
  if (d_eff) {
    if (!device_range<R>(b->stream, d_eff, n, d_lo, d_hi)) return bfail(b, LBM_ERR_DEVICE, which + "reading D_eff failed");
  } else if (phi) {
    const double dl = p.deff_ratio_gdl > 0 ? p.deff_ratio_gdl * p.D_f_lat : std::pow(phi_lo, 1.5) * p.D_f_lat;
    d_lo = std::min(dl, p.D_f_lat);
  }
  if (!(phi_lo > 0) || phi_hi > 1.0) return bfail(b, LBM_ERR_UNSTABLE_PARAMS, which + "porosity outside (0, 1]");
  if (!(k_lo >= 0)) return bfail(b, LBM_ERR_UNSTABLE_PARAMS, which + "negative or non-finite 1/K");
  if (!(d_lo > 0) || d_hi > kMaxDiff)
    return bfail(b, LBM_ERR_UNSTABLE_PARAMS, which + "O2 diffusivity outside (0, 1/(4 sqrt 3)]");
  const double a1 = alpha_lat(p, phi_lo, dv.alpha_scale), a2 = alpha_lat(p, phi_hi, dv.alpha_scale);
  const double a3 = alpha_lat(p, 1.0, dv.alpha_scale);
  if (std::max({a1, a2, a3}) > kMaxDiff || !(std::min({a1, a2, a3}) > 0))
    return bfail(b, LBM_ERR_UNSTABLE_PARAMS, which + "thermal diffusivity outside (0, 1/(4 sqrt 3)]");
  R* f = b->field_rows<R>(i);
  const int64_t L = pitch_of(g.nx);
  const int pitch = bconsts<R>(b, i).pitch;
  const dim3 grid((g.nx + kBlock - 1) / kBlock, g.ny);
  const void* src[3] = {phi, inv_k, d_eff};
  for (int c = 0; c < 3; ++c)
    if (src[c])
      hipLaunchKernelGGL(k_pitch_copy<R>, grid, dim3(kBlock), 0, b->stream, static_cast<const R*>(src[c]),
                         f + c * L, g.nx, pitch);
  if (lbm_status st = derive_case_fields<R>(b, i, phi ? 1 : 0, inv_k ? 1 : 0, d_eff ? 1 : 0); st != LBM_OK) return st;
  if (hipStreamSynchronize(b->stream) != hipSuccess) return bfail(b, LBM_ERR_DEVICE, which + "field copy failed");
  return LBM_OK;
}

template <typename R>
lbm_status upload_cases(lbm_batch* b) {
  std::vector<BatchCase<R>> h(b->n);
  for (int i = 0; i < b->n; ++i) {
    h[i].k = bconsts<R>(b, i);
    h[i].off[0] = b->L.state_off[0][i];
    h[i].off[1] = b->L.state_off[1][i];
  }
  if (hipMemcpyAsync(b->cases<R>(), h.data(), h.size() * sizeof(BatchCase<R>), hipMemcpyHostToDevice, b->stream) !=
      hipSuccess)
    return bfail(b, LBM_ERR_DEVICE, "case table upload failed");
  if (hipStreamSynchronize(b->stream) != hipSuccess) return bfail(b, LBM_ERR_DEVICE, "case table sync failed");
  return LBM_OK;
}

// Build the tile list for a tile shape; cases in order, rows then columns.
lbm_status build_tiles(lbm_batch* b, int tx, int ty) {
  std::vector<Tile> t;
  for (int i = 0; i < b->n; ++i)
    for (int y0 = 0; y0 < b->g[i].ny; y0 += ty)
      for (int x0 = 0; x0 < b->g[i].nx; x0 += tx) t.push_back({i, x0, y0, 0});
  if (int(t.size()) > b->L.max_tiles) return bfail(b, LBM_ERR_INVALID_ARG, "tile too small");
  if (hipMemcpyAsync(b->tiles(), t.data(), t.size() * sizeof(Tile), hipMemcpyHostToDevice, b->stream) != hipSuccess)
    return bfail(b, LBM_ERR_DEVICE, "tile table upload failed");
  if (hipStreamSynchronize(b->stream) != hipSuccess) return bfail(b, LBM_ERR_DEVICE, "tile table sync failed");
  b->ntiles = int(t.size());
  return LBM_OK;
}

// Workgroups of the persistent kernel's grid: every one must be resident at
// once for its grid barrier.  Per CU that is the smaller of the runtime's
// occupancy query and the derivation from the kernel's resources: a
// 256-lane workgroup is four waves, one per SIMD, so workgroups per CU =
// waves per SIMD; the vector registers (hipFuncGetAttributes, allocated in
// groups of 8 from 512 per SIMD) allow 512 / alloc waves, the scalar ones
// are within what the PersistentWaves the kernel is compiled for allow
// (the compiler's guarantee), and the kernel uses no LDS beyond a word.
// With LBM_LOG set, both figures go to stderr.
template <typename R, int MAT>
lbm_status persistent_grid(lbm_batch* b, int* grid_out) {
  const void* fn = reinterpret_cast<const void*>(&k_batch_persistent<R, MAT>);
  int dev = 0, ncu = 0, query = 0;
  hipFuncAttributes a{};
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&query, fn, kBlock, 0) != hipSuccess ||
      hipFuncGetAttributes(&a, fn) != hipSuccess)
    return bfail(b, LBM_ERR_DEVICE, "occupancy of the persistent kernel unavailable");
  const int vgpr_alloc = std::max(8, (a.numRegs + 7) / 8 * 8);
  const int by_vgpr = std::min(8, 512 / vgpr_alloc);
  const int derived = std::min(by_vgpr, PersistentWaves<R>::value);
  const int per_cu = std::min(query, derived);
  if (std::getenv("LBM_LOG"))
    std::fprintf(stderr,
                 "lbm: persistent kernel (%s): occupancy query %d workgroups/CU; derived %d (VGPRs %d -> %d waves, "
                 "compiled for >= %d); grid %d CUs x %d\n",
                 sizeof(R) == 8 ? "fp64" : "fp32", query, derived, a.numRegs, by_vgpr, PersistentWaves<R>::value,
                 ncu, per_cu);
  if (per_cu < 1) return bfail(b, LBM_ERR_DEVICE, "no co-resident grid for the persistent kernel");
  *grid_out = std::min(ncu * per_cu, b->ntiles);
  return LBM_OK;
}

// The persistent kernel's barrier gave up (workgroups that never started):
// sticky until lbm_batch_init_equilibrium, reported by every synchronising
// call.
lbm_status barrier_status(lbm_batch* b) {
  int failed = 0;
  if (hipMemcpyAsync(&failed, b->barrier_failed(), sizeof(int), hipMemcpyDeviceToHost, b->stream) != hipSuccess ||
      hipStreamSynchronize(b->stream) != hipSuccess)
    return bfail(b, LBM_ERR_DEVICE, "reading the persistent barrier flag failed");
  if (failed)
    return bfail(b, LBM_ERR_DEVICE,
                 "persistent launch: the grid barrier timed out (workgroups not co-resident); the state is invalid");
  return LBM_OK;
}

template <typename R, int MAT>
lbm_status launch_steps_mat(lbm_batch* b, int64_t nsteps) {
  R* pool = b->pool<R>();
  const BatchCase<R>* cases = b->cases<R>();
  const Tile* tiles = b->tiles();
  const int tx = b->sched.tile_x, ty = b->sched.tile_y;
  if (b->sched.persistent) {
    int grid = b->persistent_grid;
    int64_t left = nsteps;
    GridBarrier gb{b->barrier_count(), b->barrier_failed(), b->barrier_limit};
    while (left > 0) {
      int chunk = int(std::min<int64_t>(left, 1 << 20));  // (chunk) x (grid) arrivals fit the 32-bit count
      int ntiles = b->ntiles, par = b->parity;
      hipLaunchKernelGGL(k_clear_barrier, dim3(1), dim3(64), 0, b->stream, gb.count, gb.failed, 0);
      void* args[] = {&pool, &cases, &tiles, &ntiles, &chunk, &par, const_cast<int*>(&tx), const_cast<int*>(&ty),
                      &gb};
      const hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_batch_persistent<R, MAT>),
                                                      dim3(grid), dim3(kBlock), args, 0, b->stream);
      if (e != hipSuccess) return bfail(b, LBM_ERR_DEVICE, std::string("cooperative launch: ") + hipGetErrorString(e));
      b->parity = (b->parity + chunk) & 1;
      left -= chunk;
    }
  } else {
    // workgroups of 64 or 128 threads: one cell of the tile (of that many
    // cells) per thread; of 256: one cell per thread for tiles of 256 cells,
    // a cell loop otherwise.  Batches of few nodes (one round of wavefronts
    // per launch) take the wave-uniform addressing form.
    const int cells = tx * ty;
    const int bs = b->sched.block == 64 || b->sched.block == 128 ? b->sched.block : kBlock;
    const bool uniform = b->cells < (int64_t(1) << 20);
    const dim3 grid(b->ntiles);
    int64_t s = 0;
    if (b->sched.block == kT2Threads) {  // two steps per launch; an odd count ends with one step
      for (; s + 2 <= nsteps; s += 2) {
        hipLaunchKernelGGL((k_batch_step2<R, MAT>), grid, dim3(kT2Threads), 0, b->stream, pool, cases, tiles,
                           b->ntiles, b->parity);
        b->parity ^= 1;
      }
    }
    for (; s < nsteps; ++s) {
      if (bs == 64) {
        if (uniform)
          hipLaunchKernelGGL((k_batch_step<R, MAT, true, true, 64>), grid, dim3(64), 0, b->stream, pool, cases, tiles,
                             b->ntiles, b->parity, tx, ty);
        else
          hipLaunchKernelGGL((k_batch_step<R, MAT, true, false, 64>), grid, dim3(64), 0, b->stream, pool, cases, tiles,
                             b->ntiles, b->parity, tx, ty);
      } else if (bs == 128) {
        if (uniform)
          hipLaunchKernelGGL((k_batch_step<R, MAT, true, true, 128>), grid, dim3(128), 0, b->stream, pool, cases, tiles,
                             b->ntiles, b->parity, tx, ty);
        else
          hipLaunchKernelGGL((k_batch_step<R, MAT, true, false, 128>), grid, dim3(128), 0, b->stream, pool, cases, tiles,
                             b->ntiles, b->parity, tx, ty);
      } else if (cells == kBlock) {
        if (uniform)
          hipLaunchKernelGGL((k_batch_step<R, MAT, true, true>), grid, dim3(kBlock), 0, b->stream, pool, cases, tiles,
                             b->ntiles, b->parity, tx, ty);
        else
          hipLaunchKernelGGL((k_batch_step<R, MAT, true, false>), grid, dim3(kBlock), 0, b->stream, pool, cases, tiles,
                             b->ntiles, b->parity, tx, ty);
      } else if (uniform) {
        hipLaunchKernelGGL((k_batch_step<R, MAT, false, true>), grid, dim3(kBlock), 0, b->stream, pool, cases, tiles,
                           b->ntiles, b->parity, tx, ty);
      } else {
        hipLaunchKernelGGL((k_batch_step<R, MAT, false, false>), grid, dim3(kBlock), 0, b->stream, pool, cases, tiles,
                           b->ntiles, b->parity, tx, ty);
      }
      b->parity ^= 1;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return bfail(b, LBM_ERR_DEVICE, std::string("batch step: ") + hipGetErrorString(e));
  }
  b->step += nsteps;
  return LBM_OK;
}

template <typename R>
lbm_status launch_steps(lbm_batch* b, int64_t nsteps) {
  return b->L.fields ? launch_steps_mat<R, MAT_FULL>(b, nsteps) : launch_steps_mat<R, MAT_LAYERED>(b, nsteps);
}

template <typename R>
lbm_status set_schedule_t(lbm_batch* b, const lbm_schedule& s) {
  if (s.tile_x < 1 || s.tile_y < 1 || s.tile_x * s.tile_y < kMinTileCells || s.tile_x * s.tile_y > 1 << 16)
    return bfail(b, LBM_ERR_INVALID_ARG, "tile shape out of range");
  if (!(s.block == 0 || s.block == kBlock ||
        ((s.block == 64 || s.block == 128) && s.tile_x * s.tile_y == s.block && !s.persistent) ||
        (s.block == kT2Threads && s.tile_x == kT2X && s.tile_y == kT2Y && !s.persistent)))
    return bfail(b, LBM_ERR_INVALID_ARG,
                 "workgroup size: 0 or 256, 64 / 128 for a per-step tile of as many cells, or 960 for the "
                 "two-step form of 64 x 12 tiles");
  if (s.block == kT2Threads)
    for (int i = 0; i < b->n; ++i)
      if (b->g[i].flags & (LBM_PERIODIC_X | LBM_PERIODIC_Y))
        return bfail(b, LBM_ERR_INVALID_ARG, "the two-step form needs walls and inlet / outlet columns (no periodic axis)");
  b->sched = s;
  if (lbm_status st = build_tiles(b, s.tile_x, s.tile_y); st != LBM_OK) return st;
  if (s.persistent)
    return b->L.fields ? persistent_grid<R, MAT_FULL>(b, &b->persistent_grid)
                       : persistent_grid<R, MAT_LAYERED>(b, &b->persistent_grid);
  return LBM_OK;
}

template <typename R>
lbm_status init_t(lbm_batch* b) {
  for (int i = 0; i < b->n; ++i) {
    const dim3 grid((b->g[i].nx + kBlock - 1) / kBlock, b->g[i].ny);
    R* dst = b->pool<R>() + b->L.state_off[0][i];
    if (b->L.fields) {
      const R* f = b->field_rows<R>(i);
      const int64_t L = pitch_of(b->g[i].nx);
      hipLaunchKernelGGL((k_init<R, MAT_FULL>), grid, dim3(kBlock), 0, b->stream, dst, f, f + L, f + 2 * L,
                         bconsts<R>(b, i));
    } else {
      hipLaunchKernelGGL((k_init<R, MAT_LAYERED>), grid, dim3(kBlock), 0, b->stream, dst, nullptr, nullptr, nullptr,
                         bconsts<R>(b, i));
    }
  }
  hipLaunchKernelGGL(k_clear_barrier, dim3(1), dim3(64), 0, b->stream, b->barrier_count(), b->barrier_failed(), 1);
  b->parity = 0;
  b->step = 0;
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? LBM_OK : bfail(b, LBM_ERR_DEVICE, std::string("batch init: ") + hipGetErrorString(e));
}

template <typename R>
lbm_status observables_t(lbm_batch* b, lbm_obs* out) {
  if (lbm_status st = barrier_status(b); st != LBM_OK) return st;
  for (int i = 0; i < b->n; ++i) {
    const lbm_geometry& g = b->g[i];
    const lbm_params& p = b->p[i];
    const Consts<R>& k = bconsts<R>(b, i);
    const R* src = b->pool<R>() + b->L.state_off[b->parity][i];
    const dim3 grid((g.nx + kBlock - 1) / kBlock, g.ny);
    if (b->L.fields) {
      const R* f = b->field_rows<R>(i);
      hipLaunchKernelGGL((k_obs_cells<R, MAT_FULL>), grid, dim3(kBlock), 0, b->stream, src, f, f + k.plane,
                         f + 2 * k.plane, k, b->partial());
    } else {
      hipLaunchKernelGGL((k_obs_cells<R, MAT_LAYERED>), grid, dim3(kBlock), 0, b->stream, src, nullptr, nullptr,
                         nullptr, k, b->partial());
    }
    hipLaunchKernelGGL(k_obs_final<kObsQ>, dim3(kObsQ), dim3(kBlock), 0, b->stream, b->partial(),
                       int(grid.x * grid.y), b->out());
    double h[kObsQ];
    if (hipMemcpyAsync(h, b->out(), sizeof(h), hipMemcpyDeviceToHost, b->stream) != hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess)
      return bfail(b, LBM_ERR_DEVICE, "batch observables failed");
    const double i_scale = 4.0 * p.faraday * p.C_ref / b->d[i].dt * b->d[i].dx;
    lbm_obs r{};
    r.step = b->step;
    r.current_density = h[3] * i_scale / g.nx;
    r.power_density = p.V_op * r.current_density;
    r.heat_rate = h[5] * i_scale / g.nx;
    r.inlet_flux = h[8];
    const double inflow = (g.flags & LBM_PRESSURE_INLET) ? h[8] * p.c_in : b->d[i].inflow;
    r.o2_utilisation = inflow > 0 ? h[3] / inflow : 0.0;
    r.T_max = p.T_in_K + h[6];
    r.sum_f = h[0] + double(g.nx) * g.ny;
    r.sum_theta = h[1];
    r.sum_c = h[2];
    r.consumed_c = h[3];
    r.heat_added = h[4];
    out[i] = r;
    if (!std::isfinite(r.current_density) || !std::isfinite(r.sum_f) || h[7] > 0)
      return bfail(b, LBM_ERR_NONFINITE, "non-finite observable in case " + std::to_string(i));
  }
  return LBM_OK;
}

template <typename R>
lbm_status autotune_t(lbm_batch* b, int trial_steps, lbm_schedule* best, double* best_ms) {
  // Save the current state of every case, time each candidate from it, restore.
  const size_t bytes = size_t(b->L.pool_elems) * sizeof(R);
  char* pool = reinterpret_cast<char*>(b->pool<R>());
  char* backup = b->ws + b->L.off_backup;
  // The backup region holds one buffer per case: copy the current buffer of each case.
  std::vector<size_t> boff(b->n);
  size_t o = 0;
  for (int i = 0; i < b->n; ++i) {
    const size_t sz = b->state_elems(i) * sizeof(R);
    boff[i] = o;
    if (hipMemcpyAsync(backup + o, pool + b->L.state_off[b->parity][i] * sizeof(R), sz, hipMemcpyDeviceToDevice,
                       b->stream) != hipSuccess)
      return bfail(b, LBM_ERR_DEVICE, "autotune backup failed");
    o += align_up(sz);
  }
  (void)bytes;
  const int parity0 = b->parity;
  const int64_t step0 = b->step;
  const lbm_schedule keep = b->sched;
  static const int shapes[][2] = {{64, 1}, {128, 1}, {256, 1}, {512, 1}, {1024, 1}, {64, 2}, {64, 4}, {32, 4},
                                  {128, 2}, {256, 2}, {256, 4}, {512, 2}, {128, 8}, {64, 16}};
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return bfail(b, LBM_ERR_DEVICE, "autotune events failed");
  double best_t = 1e300;
  lbm_schedule best_s = keep;
  lbm_status st = LBM_OK;
  std::vector<lbm_schedule> cand;
  for (int persistent = 0; persistent < 2; ++persistent)
    for (const auto& sh : shapes) {
      cand.push_back({sh[0], sh[1], persistent, 0});
      const int cells = sh[0] * sh[1];
      if (!persistent && (cells == 64 || cells == 128)) cand.push_back({sh[0], sh[1], 0, cells});
    }
  cand.push_back({kT2X, kT2Y, 0, kT2Threads});
  for (const lbm_schedule& s : cand) {
    const int persistent = s.persistent;
    if (set_schedule_t<R>(b, s) != LBM_OK) continue;  // shape not usable here
    st = launch_steps<R>(b, 2);                        // warm up
    if (st != LBM_OK) break;
    (void)hipEventRecord(e0, b->stream);
    st = launch_steps<R>(b, trial_steps);
    if (st != LBM_OK) break;
    (void)hipEventRecord(e1, b->stream);
    if (hipEventSynchronize(e1) != hipSuccess) {
      st = bfail(b, LBM_ERR_DEVICE, "autotune trial failed");
      break;
    }
    if (persistent && barrier_status(b) != LBM_OK) {  // not co-resident: the schedule is unusable
      hipLaunchKernelGGL(k_clear_barrier, dim3(1), dim3(64), 0, b->stream, b->barrier_count(),
                         b->barrier_failed(), 1);
      b->err.clear();
      continue;
    }
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    const double per = double(ms) / trial_steps;
    if (per < best_t) {
      best_t = per;
      best_s = s;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // Restore the saved state into the original buffers.
  for (int i = 0; i < b->n; ++i) {
    const size_t sz = b->state_elems(i) * sizeof(R);
    if (hipMemcpyAsync(pool + b->L.state_off[parity0][i] * sizeof(R), backup + boff[i], sz, hipMemcpyDeviceToDevice,
                       b->stream) != hipSuccess)
      return bfail(b, LBM_ERR_DEVICE, "autotune restore failed");
  }
  b->parity = parity0;
  b->step = step0;
  if (st != LBM_OK) return st;
  if (lbm_status s2 = set_schedule_t<R>(b, best_s); s2 != LBM_OK) return s2;
  if (best) *best = best_s;
  if (best_ms) *best_ms = best_t;
  return hipStreamSynchronize(b->stream) == hipSuccess ? LBM_OK : bfail(b, LBM_ERR_DEVICE, "autotune sync failed");
}

// Tuner cache file: a JSON object with one schedule per line,
//   "gfx950|fp32|256x64,512x128": {"tile_x": 128, "tile_y": 1, "persistent": 0, "block": 0, "ms_per_step": 0.158}
// keyed by the GPU architecture, the precision and the case lattice sizes in
// case order.
std::string tune_key(const lbm_batch* b) {
  std::string arch = "unknown";
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
  }
  std::string k = arch + "|fp" + std::to_string(b->g[0].precision) + "|";
  for (int i = 0; i < b->n; ++i) k += (i ? "," : "") + std::to_string(b->g[i].nx) + "x" + std::to_string(b->g[i].ny);
  return k;
}

struct CacheEntry {
  std::string key;
  lbm_schedule s{};
  double ms = 0;
};

// Entries of a cache file; false if the file exists and holds anything else
// than the braces and entry lines (it is then neither used nor rewritten).
bool read_cache(const char* path, std::vector<CacheEntry>& out) {
  std::ifstream f(path);
  if (!f) return true;  // no file yet
  std::string line;
  while (std::getline(f, line)) {
    const size_t a = line.find_first_not_of(" \t\r");
    if (a == std::string::npos) continue;
    const std::string t = line.substr(a);
    if (t == "{" || t == "}") continue;
    if (t[0] != '"') return false;
    const size_t q = t.find('"', 1);
    if (q == std::string::npos) return false;
    CacheEntry e;
    e.key = t.substr(1, q - 1);
    if (std::sscanf(t.c_str() + q + 1,
                    ": {\"tile_x\": %d, \"tile_y\": %d, \"persistent\": %d, \"block\": %d, \"ms_per_step\": %lf}",
                    &e.s.tile_x, &e.s.tile_y, &e.s.persistent, &e.s.block, &e.ms) != 5)
      return false;
    out.push_back(e);
  }
  return true;
}

bool write_cache(const char* path, const std::vector<CacheEntry>& entries) {
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp, std::ios::trunc);
    if (!f) return false;
    f << "{\n";
    for (size_t i = 0; i < entries.size(); ++i) {
      const CacheEntry& e = entries[i];
      char buf[256];
      std::snprintf(buf, sizeof(buf),
                    ": {\"tile_x\": %d, \"tile_y\": %d, \"persistent\": %d, \"block\": %d, \"ms_per_step\": %.6g}",
                    e.s.tile_x, e.s.tile_y, e.s.persistent, e.s.block, e.ms);
      f << '"' << e.key << '"' << buf << (i + 1 < entries.size() ? ",\n" : "\n");
    }
    f << "}\n";
    if (!f) return false;
  }
  return std::rename(tmp.c_str(), path) == 0;
}

}  // namespace

extern "C" {

size_t lbm_batch_workspace_bytes(const lbm_geometry* g, int32_t ncases) {
  if (!batch_geometry_ok(g, ncases)) return 0;
  return make_batch_layout(g, ncases).total;
}

lbm_status lbm_batch_create(const lbm_geometry* g, const lbm_params* p, int32_t ncases, void* dev_ws,
                            size_t ws_bytes, void* hip_stream, lbm_batch** out) {
  if (!out) return LBM_ERR_INVALID_ARG;
  *out = nullptr;
  if (!batch_geometry_ok(g, ncases) || !p || !dev_ws) return LBM_ERR_INVALID_ARG;
  const BatchLayout L = make_batch_layout(g, ncases);
  if (ws_bytes < L.total || reinterpret_cast<uintptr_t>(dev_ws) % kAlign != 0) return LBM_ERR_INVALID_ARG;
  lbm_batch* b = new (std::nothrow) lbm_batch();
  if (!b) return LBM_ERR_INVALID_ARG;
  b->n = ncases;
  b->g.assign(g, g + ncases);
  b->p.assign(p, p + ncases);
  b->d.resize(ncases);
  b->kf.resize(ncases);
  b->kd.resize(ncases);
  b->L = L;
  b->ws = static_cast<char*>(dev_ws);
  b->stream = static_cast<hipStream_t>(hip_stream);
  for (int i = 0; i < ncases; ++i) b->cells += int64_t(g[i].nx) * g[i].ny;
  *out = b;
  for (int i = 0; i < ncases; ++i) {
    std::string msg;
    if (lbm_status st = derive(g[i], p[i], b->d[i], msg); st != LBM_OK)
      return bfail(b, st, "case " + std::to_string(i) + ": " + msg);
    fill_consts(b->kf[i], g[i], p[i], b->d[i], pitch_of(g[i].nx));
    fill_consts(b->kd[i], g[i], p[i], b->d[i], pitch_of(g[i].nx));
    // Row-interleaved state: the 19 population rows of lattice row y are
    // contiguous (element q * plane + y * pitch + x with plane = the row
    // length and pitch = 19 row lengths, 22 with the three field rows), so
    // that a tile's loads and stores stay within a few DRAM pages instead of
    // 19 planes apart.  64-case sweep: 174.5 -> 157.7 us per step.
    b->kf[i].plane = b->kd[i].plane = pitch_of(g[i].nx);
    b->kf[i].pitch = b->kd[i].pitch = b->L.rows * pitch_of(g[i].nx);
  }
  int dev = 0, wall_khz = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || wall_khz <= 0)
    return bfail(b, LBM_ERR_DEVICE, "device wall-clock rate unavailable");
  b->wall_khz = wall_khz;
  b->barrier_limit = 4000LL * wall_khz;  // 4 s
  const bool dbl = g[0].precision == 64;
  if (lbm_status st = dbl ? upload_cases<double>(b) : upload_cases<float>(b); st != LBM_OK) return st;
  if (b->L.fields)
    for (int i = 0; i < ncases; ++i)
      if (lbm_status st = dbl ? derive_case_fields<double>(b, i, 0, 0, 0) : derive_case_fields<float>(b, i, 0, 0, 0);
          st != LBM_OK)
        return st;
  hipLaunchKernelGGL(k_clear_barrier, dim3(1), dim3(64), 0, b->stream, b->barrier_count(), b->barrier_failed(), 1);
  lbm_schedule s{256, 1, 0, 0};
  return dbl ? set_schedule_t<double>(b, s) : set_schedule_t<float>(b, s);
}

lbm_status lbm_batch_init_equilibrium(lbm_batch* b) {
  if (!b) return LBM_ERR_INVALID_ARG;
  return b->g[0].precision == 64 ? init_t<double>(b) : init_t<float>(b);
}

lbm_status lbm_batch_set_schedule(lbm_batch* b, const lbm_schedule* s) {
  if (!b || !s) return LBM_ERR_INVALID_ARG;
  return b->g[0].precision == 64 ? set_schedule_t<double>(b, *s) : set_schedule_t<float>(b, *s);
}

lbm_status lbm_batch_get_schedule(const lbm_batch* b, lbm_schedule* s) {
  if (!b || !s) return LBM_ERR_INVALID_ARG;
  *s = b->sched;
  return LBM_OK;
}

lbm_status lbm_batch_autotune(lbm_batch* b, int32_t trial_steps, lbm_schedule* best, double* best_ms_per_step) {
  const TraceRange range("lbm_batch_autotune");
  if (!b || trial_steps < 1) return LBM_ERR_INVALID_ARG;
  return b->g[0].precision == 64 ? autotune_t<double>(b, trial_steps, best, best_ms_per_step)
                                 : autotune_t<float>(b, trial_steps, best, best_ms_per_step);
}

lbm_status lbm_batch_set_fields(lbm_batch* b, int32_t i, const void* phi, const void* inv_k, const void* d_eff) {
  if (!b || i < 0 || i >= b->n) return LBM_ERR_INVALID_ARG;
  if (!b->L.fields) return bfail(b, LBM_ERR_STATE, "the batch's cases do not carry LBM_CELL_FIELDS");
  return b->g[0].precision == 64 ? set_fields_t<double>(b, i, phi, inv_k, d_eff)
                                 : set_fields_t<float>(b, i, phi, inv_k, d_eff);
}

lbm_status lbm_batch_set_barrier_timeout(lbm_batch* b, double seconds) {
  if (!b || !(seconds >= 0.0) || seconds > 3600.0) return LBM_ERR_INVALID_ARG;
  b->barrier_limit = static_cast<long long>(seconds * 1000.0 * double(b->wall_khz));
  return LBM_OK;
}

lbm_status lbm_batch_autotune_cached(lbm_batch* b, int32_t trial_steps, const char* cache_path, lbm_schedule* best,
                                     double* best_ms_per_step, int32_t* from_cache) {
  const TraceRange range("lbm_batch_autotune_cached");
  if (!b || trial_steps < 1) return LBM_ERR_INVALID_ARG;
  if (from_cache) *from_cache = 0;
  if (!cache_path) return lbm_batch_autotune(b, trial_steps, best, best_ms_per_step);
  const std::string key = tune_key(b);
  std::vector<CacheEntry> entries;
  const bool usable = read_cache(cache_path, entries);
  if (usable)
    for (const CacheEntry& e : entries)
      if (e.key == key) {
        const bool dbl = b->g[0].precision == 64;
        if (lbm_status st = dbl ? set_schedule_t<double>(b, e.s) : set_schedule_t<float>(b, e.s); st != LBM_OK)
          break;  // not usable here: tune again
        if (best) *best = e.s;
        if (best_ms_per_step) *best_ms_per_step = e.ms;
        if (from_cache) *from_cache = 1;
        return LBM_OK;
      }
  lbm_schedule s{};
  double ms = 0;
  if (lbm_status st = lbm_batch_autotune(b, trial_steps, &s, &ms); st != LBM_OK) return st;
  if (best) *best = s;
  if (best_ms_per_step) *best_ms_per_step = ms;
  if (!usable) {
    b->err = std::string("tune cache ") + cache_path + " is not in the library's format: not rewritten";
    return LBM_OK;
  }
  bool found = false;
  for (CacheEntry& e : entries)
    if (e.key == key) {
      e.s = s;
      e.ms = ms;
      found = true;
    }
  if (!found) entries.push_back({key, s, ms});
  if (!write_cache(cache_path, entries)) b->err = std::string("tune cache ") + cache_path + " could not be written";
  return LBM_OK;
}

lbm_status lbm_batch_step(lbm_batch* b, int64_t nsteps) {
  const TraceRange range("lbm_batch_step");
  if (!b || nsteps < 0) return LBM_ERR_INVALID_ARG;
  return b->g[0].precision == 64 ? launch_steps<double>(b, nsteps) : launch_steps<float>(b, nsteps);
}

lbm_status lbm_batch_observables(lbm_batch* b, lbm_obs* out) {
  const TraceRange range("lbm_batch_observables");
  if (!b || !out) return LBM_ERR_INVALID_ARG;
  return b->g[0].precision == 64 ? observables_t<double>(b, out) : observables_t<float>(b, out);
}

lbm_status lbm_batch_get_populations(lbm_batch* b, int32_t i, void* dst) {
  if (!b || !dst || i < 0 || i >= b->n) return LBM_ERR_INVALID_ARG;
  const dim3 grid((b->g[i].nx + kBlock - 1) / kBlock, b->g[i].ny);
  if (b->g[0].precision == 64)
    hipLaunchKernelGGL(k_export<double>, grid, dim3(kBlock), 0, b->stream,
                       b->pool<double>() + b->L.state_off[b->parity][i], static_cast<double*>(dst), b->kd[i]);
  else
    hipLaunchKernelGGL(k_export<float>, grid, dim3(kBlock), 0, b->stream,
                       b->pool<float>() + b->L.state_off[b->parity][i], static_cast<float*>(dst), b->kf[i]);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? LBM_OK : bfail(b, LBM_ERR_DEVICE, std::string("get_populations: ") + hipGetErrorString(e));
}

int64_t lbm_batch_step_count(const lbm_batch* b) { return b ? b->step : -1; }

lbm_status lbm_batch_synchronize(lbm_batch* b) {
  if (!b) return LBM_ERR_INVALID_ARG;
  const hipError_t e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bfail(b, LBM_ERR_DEVICE, std::string("synchronize: ") + hipGetErrorString(e));
  return barrier_status(b);
}

void lbm_batch_destroy(lbm_batch* b) { delete b; }

const char* lbm_batch_last_error(const lbm_batch* b) { return b ? b->err.c_str() : "null batch"; }

}  // extern "C"
