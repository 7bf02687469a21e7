// Host side of the C ABI declared in include/lbm_pem.h: context, parameter
// derivation and validation, launches.  No device memory is allocated here;
// everything lives in the caller's workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lbm_host.hpp"
#include "lbm_kernels2d.hpp"
#include "lbm_pem.h"

using namespace lbm;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  int pitch = 0;
  int64_t plane = 0;  // elements
  size_t esize = 0;
  size_t off_state[2] = {0, 0};
  size_t off_mat = 0;
  size_t off_partial = 0;
  size_t off_prof = 0;
  size_t off_out = 0;
  size_t total = 0;
  int nblocks_obs = 0;
};

Layout make_layout(const lbm_geometry* g) {
  Layout L;
  L.esize = g->precision == 64 ? 8 : 4;
  L.pitch = (g->nx + 63) / 64 * 64;
  L.plane = lbm::plane_elems(int64_t(L.pitch) * g->ny);
  const size_t state = align_up(size_t(19) * L.plane * L.esize);
  L.nblocks_obs = ((g->nx + kBlock - 1) / kBlock) * g->ny;
  size_t o = 0;
  L.off_state[0] = o;
  o += state;
  L.off_state[1] = o;
  o += state;
  L.off_mat = o;
  o += align_up(size_t(3) * L.plane * L.esize);
  L.off_partial = o;
  o += align_up(size_t(L.nblocks_obs) * kObsQ * sizeof(double));
  L.off_prof = o;
  o += align_up(size_t(3) * g->nx * sizeof(double));
  L.off_out = o;
  o += align_up(16 * sizeof(double));
  L.total = o;
  return L;
}

}  // namespace

struct lbm_ctx {
  lbm_geometry g{};
  lbm_params p{};
  Layout L;
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  int device = 0;
  int cur = 0;            // index of the state buffer holding the current state
  int64_t step = 0;
  bool params_set = false;
  int mat = MAT_LAYERED;
  Consts<float> kf{};
  Consts<double> kd{};
  Derived d;
  std::string err;
  // checkpointed forward run held for lbm_backward
  char* adj_ws = nullptr;
  int64_t adj_nsteps = 0;
  int32_t adj_every = 0;
  int64_t adj_step = -1;
  bool adj_ready = false;
  bool adj_last_resident = false;  // replay buffer 0 holds the last segment's states
  // second stream and events of the reverse sweep: the replay of the next
  // segment runs there while the current one is swept
  hipStream_t aux = nullptr;
  hipEvent_t ev_in = nullptr, ev_rep[2] = {nullptr, nullptr}, ev_rev[2] = {nullptr, nullptr};

  void* state(int i) { return ws + L.off_state[i]; }
  void* mat_plane(int i) { return ws + L.off_mat + size_t(i) * L.plane * L.esize; }
  double* partial() { return reinterpret_cast<double*>(ws + L.off_partial); }
  double* prof() { return reinterpret_cast<double*>(ws + L.off_prof); }
  double* out() { return reinterpret_cast<double*>(ws + L.off_out); }
};

namespace {

lbm_status fail(lbm_ctx* c, lbm_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

lbm_status check_launch(lbm_ctx* c, const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, LBM_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return LBM_OK;
}

template <typename R>
bool host_range(lbm_ctx* c, const void* dev, double& lo, double& hi) {
  const size_t n = size_t(c->g.nx) * c->g.ny;
  std::vector<R> h(n);
  if (hipMemcpyAsync(h.data(), dev, n * sizeof(R), hipMemcpyDeviceToHost, c->stream) != hipSuccess) return false;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return false;
  lo = 1e300;
  hi = -1e300;
  for (size_t i = 0; i < n; ++i) {
    const double v = double(h[i]);
    if (!std::isfinite(v)) {
      lo = -1e300;
      return true;
    }
    lo = std::min(lo, v);
    hi = std::max(hi, v);
  }
  return true;
}

template <typename R>
hipError_t launch_pitch_copy(lbm_ctx* c, const void* src, void* dst) {
  const dim3 grid((c->g.nx + kBlock - 1) / kBlock, c->g.ny);
  hipLaunchKernelGGL(k_pitch_copy<R>, grid, dim3(kBlock), 0, c->stream, static_cast<const R*>(src),
                     static_cast<R*>(dst), c->g.nx, c->L.pitch);
  return hipGetLastError();
}

template <typename R>
const Consts<R>& consts(const lbm_ctx* c);
template <>
const Consts<float>& consts<float>(const lbm_ctx* c) { return c->kf; }
template <>
const Consts<double>& consts<double>(const lbm_ctx* c) { return c->kd; }

template <typename R>
struct MatPtrs {
  const R *phi, *invk, *d;
};
template <typename R>
MatPtrs<R> mat_ptrs(lbm_ctx* c) {
  return {static_cast<const R*>(c->mat_plane(0)), static_cast<const R*>(c->mat_plane(1)),
          static_cast<const R*>(c->mat_plane(2))};
}

// Lattices below this many nodes take the wave-uniform addressing form of
// the step (their launches are bound by each wavefront's own chain).
constexpr int64_t kUniformMaxCells = int64_t(1) << 20;

template <typename R, int MAT>
void launch_step_kernel(lbm_ctx* c, const R* src, R* dst, const MatPtrs<R>& m, const Consts<R>& k,
                        hipStream_t stream) {
  const dim3 grid((c->g.nx + kBlock - 1) / kBlock, c->g.ny);
  if (int64_t(c->g.nx) * c->g.ny < kUniformMaxCells)
    hipLaunchKernelGGL((k_step<R, MAT, true>), grid, dim3(kBlock), 0, stream, src, dst, m.phi, m.invk, m.d, k);
  else
    hipLaunchKernelGGL((k_step<R, MAT, false>), grid, dim3(kBlock), 0, stream, src, dst, m.phi, m.invk, m.d, k);
}

// Lattices of at least kTwoStepMinCells nodes with walls and inlet / outlet
// columns advance two steps per launch (k_step2: the same states, bit for
// bit, as two single steps).  Measured per step against single steps,
// 4096x1024: FP32 99.6 -> 89.6 us, FP64 247.6 -> 177.7 us; 1024x512 5 %
// faster in both precisions.  Smaller lattices, whose launches are bound by
// each wavefront's own chain rather than by HBM, run slower in pairs
// (1024x256 FP32 8.9 -> 12.5 us) and keep single steps.
constexpr int64_t kTwoStepMinCells = int64_t(1) << 19;
// FP32 lattices of at least this many nodes take non-temporal loads in
// step one (k_step2's NT), the others cached loads.
constexpr int64_t kTwoStepStreamCells = int64_t(1) << 22;
bool two_step_form_applies(const lbm_ctx* c) {
  return !(c->g.flags & (LBM_PERIODIC_X | LBM_PERIODIC_Y));
}
bool two_steps_per_launch(const lbm_ctx* c) {
  return int64_t(c->g.nx) * c->g.ny >= kTwoStepMinCells && two_step_form_applies(c);
}

// Two steps src -> (mid) -> dst; mid may be null (the middle state is not
// stored).
template <typename R, int MAT>
void launch_step_pair(lbm_ctx* c, const R* src, R* mid, R* dst, const MatPtrs<R>& m, const Consts<R>& k,
                      hipStream_t stream) {
  const dim3 grid((c->g.nx + kT2X - 1) / kT2X, (c->g.ny + kT2Y - 1) / kT2Y);
  if (sizeof(R) == 4 && int64_t(c->g.nx) * c->g.ny >= kTwoStepStreamCells)
    hipLaunchKernelGGL((k_step2<R, MAT, true>), grid, dim3(kT2Threads), 0, stream, src, mid, dst, m.phi, m.invk, m.d,
                       k);
  else
    hipLaunchKernelGGL((k_step2<R, MAT, false>), grid, dim3(kT2Threads), 0, stream, src, mid, dst, m.phi, m.invk,
                       m.d, k);
}

template <typename R, int MAT>
void launch_step_mat(lbm_ctx* c, int64_t n) {
  const MatPtrs<R> m = mat_ptrs<R>(c);
  const Consts<R> k = consts<R>(c);
  if (two_steps_per_launch(c)) {
    for (; n >= 2; n -= 2) {
      launch_step_pair<R, MAT>(c, static_cast<const R*>(c->state(c->cur)), nullptr,
                               static_cast<R*>(c->state(c->cur ^ 1)), m, k, c->stream);
      c->cur ^= 1;
    }
  }
  for (int64_t i = 0; i < n; ++i) {
    launch_step_kernel<R, MAT>(c, static_cast<const R*>(c->state(c->cur)), static_cast<R*>(c->state(c->cur ^ 1)), m,
                               k, c->stream);
    c->cur ^= 1;
  }
}

template <typename R>
void launch_step(lbm_ctx* c, int64_t n) {
  switch (c->mat) {
    case MAT_LAYERED: launch_step_mat<R, MAT_LAYERED>(c, n); break;
    case MAT_PHI: launch_step_mat<R, MAT_PHI>(c, n); break;
    default: launch_step_mat<R, MAT_FULL>(c, n); break;
  }
}

template <typename R, int MAT>
void launch_init_mat(lbm_ctx* c) {
  const MatPtrs<R> m = mat_ptrs<R>(c);
  const dim3 grid((c->g.nx + kBlock - 1) / kBlock, c->g.ny);
  hipLaunchKernelGGL((k_init<R, MAT>), grid, dim3(kBlock), 0, c->stream,
                     static_cast<R*>(c->state(c->cur)), m.phi, m.invk, m.d, consts<R>(c));
}

template <typename R>
void launch_init(lbm_ctx* c) {
  switch (c->mat) {
    case MAT_LAYERED: launch_init_mat<R, MAT_LAYERED>(c); break;
    case MAT_PHI: launch_init_mat<R, MAT_PHI>(c); break;
    default: launch_init_mat<R, MAT_FULL>(c); break;
  }
}

// Where the observable reduction keeps its intermediate results: the
// per-workgroup partial sums (nblocks_obs x kObsQ), the reduced values
// (kObsQ) and the three CL profiles (3 nx).  Every element is written
// before it is read, so the buffers need no clearing.
struct ObsBuffers {
  double* partial;
  double* out;
  double* prof;
};

template <typename R, int MAT>
void launch_obs_mat(lbm_ctx* c, double i_scale, const ObsBuffers& b) {
  const MatPtrs<R> m = mat_ptrs<R>(c);
  const R* src = static_cast<const R*>(c->state(c->cur));
  const dim3 grid((c->g.nx + kBlock - 1) / kBlock, c->g.ny);
  hipLaunchKernelGGL((k_obs_cells<R, MAT>), grid, dim3(kBlock), 0, c->stream, src, m.phi, m.invk, m.d,
                     consts<R>(c), b.partial);
  hipLaunchKernelGGL(k_obs_final<kObsQ>, dim3(kObsQ), dim3(kBlock), 0, c->stream, b.partial, c->L.nblocks_obs, b.out);
  const dim3 pgrid((c->g.nx + kBlock - 1) / kBlock);
  hipLaunchKernelGGL((k_obs_profiles<R, MAT>), pgrid, dim3(kBlock), 0, c->stream, src, m.phi, m.invk, m.d,
                     consts<R>(c), i_scale, b.prof);
}

template <typename R>
void launch_obs(lbm_ctx* c, double i_scale, const ObsBuffers& b) {
  switch (c->mat) {
    case MAT_LAYERED: launch_obs_mat<R, MAT_LAYERED>(c, i_scale, b); break;
    case MAT_PHI: launch_obs_mat<R, MAT_PHI>(c, i_scale, b); break;
    default: launch_obs_mat<R, MAT_FULL>(c, i_scale, b); break;
  }
}

template <typename R, int MAT>
void launch_fields_mat(lbm_ctx* c, void* ux, void* uy, void* p, void* T, void* th, void* cc) {
  const MatPtrs<R> m = mat_ptrs<R>(c);
  const dim3 grid((c->g.nx + kBlock - 1) / kBlock, c->g.ny);
  hipLaunchKernelGGL((k_fields<R, MAT>), grid, dim3(kBlock), 0, c->stream,
                     static_cast<const R*>(c->state(c->cur)), m.phi, m.invk, m.d, consts<R>(c),
                     static_cast<R*>(ux), static_cast<R*>(uy), static_cast<R*>(p), static_cast<R*>(T),
                     static_cast<R*>(th), static_cast<R*>(cc));
}

template <typename R>
void launch_fields(lbm_ctx* c, void* ux, void* uy, void* p, void* T, void* th, void* cc) {
  switch (c->mat) {
    case MAT_LAYERED: launch_fields_mat<R, MAT_LAYERED>(c, ux, uy, p, T, th, cc); break;
    case MAT_PHI: launch_fields_mat<R, MAT_PHI>(c, ux, uy, p, T, th, cc); break;
    default: launch_fields_mat<R, MAT_FULL>(c, ux, uy, p, T, th, cc); break;
  }
}

template <typename R>
lbm_status set_params_t(lbm_ctx* c, const lbm_params* p, const void* phi, const void* inv_k,
                        const void* d_eff) {
  const lbm_geometry& g = c->g;
  c->p = *p;
  std::string msg;
  if (lbm_status st = derive(g, *p, c->d, msg); st != LBM_OK) return fail(c, st, msg);
  const double invk_gdl = c->d.invk_gdl, d_gdl = c->d.d_gdl, alpha_scale = c->d.alpha_scale;
  fill_consts(c->kf, g, *p, c->d, c->L.pitch);
  fill_consts(c->kd, g, *p, c->d, c->L.pitch);

  // Material mode and per-cell arrays.
  const bool any = phi || inv_k || d_eff;
  if (!any && !p->independent_fields) {
    c->mat = MAT_LAYERED;
  } else if (phi && !inv_k && !d_eff && p->dp_lat > 0 && !p->independent_fields) {
    c->mat = MAT_PHI;
  } else {
    c->mat = MAT_FULL;
  }
  if (phi && launch_pitch_copy<R>(c, phi, c->mat_plane(0)) != hipSuccess)
    return fail(c, LBM_ERR_DEVICE, "copy of porosity failed");
  if (c->mat == MAT_FULL) {
    if (inv_k && launch_pitch_copy<R>(c, inv_k, c->mat_plane(1)) != hipSuccess)
      return fail(c, LBM_ERR_DEVICE, "copy of 1/K failed");
    if (d_eff && launch_pitch_copy<R>(c, d_eff, c->mat_plane(2)) != hipSuccess)
      return fail(c, LBM_ERR_DEVICE, "copy of D_eff failed");
    const dim3 grid((g.nx + kBlock - 1) / kBlock, g.ny);
    hipLaunchKernelGGL(k_derive_fields<R>, grid, dim3(kBlock), 0, c->stream, static_cast<R*>(c->mat_plane(0)),
                       static_cast<R*>(c->mat_plane(1)), static_cast<R*>(c->mat_plane(2)), consts<R>(c),
                       phi ? 1 : 0, inv_k ? 1 : 0, d_eff ? 1 : 0);
    if (hipGetLastError() != hipSuccess) return fail(c, LBM_ERR_DEVICE, "field derivation failed");
  }

  // Validation of porosity, permeability and both diffusivities.
  double phi_lo = p->phi_gdl, phi_hi = 1.0, d_lo = std::min(d_gdl, p->D_f_lat), d_hi = std::max(d_gdl, p->D_f_lat);
  double k_lo = invk_gdl;
  if (phi) {
    if (!host_range<R>(c, phi, phi_lo, phi_hi)) return fail(c, LBM_ERR_DEVICE, "reading porosity failed");
  }
  if (inv_k) {
    double hi;
    if (!host_range<R>(c, inv_k, k_lo, hi)) return fail(c, LBM_ERR_DEVICE, "reading 1/K failed");
  }
  if (d_eff) {
    if (!host_range<R>(c, d_eff, d_lo, d_hi)) return fail(c, LBM_ERR_DEVICE, "reading D_eff failed");
  } else if (phi) {
    const double dl = p->deff_ratio_gdl > 0 ? p->deff_ratio_gdl * p->D_f_lat : std::pow(phi_lo, 1.5) * p->D_f_lat;
    d_lo = std::min(dl, p->D_f_lat);
  }
  if (!(phi_lo > 0) || phi_hi > 1.0) return fail(c, LBM_ERR_UNSTABLE_PARAMS, "porosity outside (0, 1]");
  if (!(k_lo >= 0)) return fail(c, LBM_ERR_UNSTABLE_PARAMS, "negative or non-finite 1/K");
  if (!(d_lo > 0) || d_hi > kMaxDiff) return fail(c, LBM_ERR_UNSTABLE_PARAMS, "O2 diffusivity outside (0, 1/(4 sqrt 3)]");
  // Eq. 19 is monotone in porosity: check the extremes of the range and the gas.
  const double a1 = alpha_lat(*p, phi_lo, alpha_scale), a2 = alpha_lat(*p, phi_hi, alpha_scale);
  const double a3 = alpha_lat(*p, 1.0, alpha_scale);
  if (std::max({a1, a2, a3}) > kMaxDiff || !(std::min({a1, a2, a3}) > 0))
    return fail(c, LBM_ERR_UNSTABLE_PARAMS, "thermal diffusivity outside (0, 1/(4 sqrt 3)]");
  if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c, LBM_ERR_DEVICE, "set_params sync failed");
  c->params_set = true;
  return LBM_OK;
}

template <typename R>
lbm_status observables_t(lbm_ctx* c, lbm_obs* o, double* pi, double* pc, double* pT, const ObsBuffers& b) {
  const lbm_params& p = c->p;
  const double four_fc = 4.0 * p.faraday * p.C_ref;
  const double i_scale = four_fc / c->d.dt * c->d.dx;  // i(x) = sum_CL (4 F C_ref s_c / dt) dx
  launch_obs<R>(c, i_scale, b);
  if (lbm_status s = check_launch(c, "observables"); s != LBM_OK) return s;
  double h[kObsQ];
  if (hipMemcpyAsync(h, b.out, sizeof(h), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
    return fail(c, LBM_ERR_DEVICE, "observable copy failed");
  const size_t nx = size_t(c->g.nx);
  double* const dst[3] = {pi, pc, pT};
  for (int i = 0; i < 3; ++i)
    if (dst[i] && hipMemcpyAsync(dst[i], b.prof + i * nx, nx * sizeof(double), hipMemcpyDeviceToHost,
                                 c->stream) != hipSuccess)
      return fail(c, LBM_ERR_DEVICE, "profile copy failed");
  if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c, LBM_ERR_DEVICE, "observables sync failed");
  const double ncell = double(c->g.nx) * c->g.ny;
  lbm_obs r{};
  r.step = c->step;
  const double sum_sc = h[3];
  r.current_density = sum_sc * i_scale / c->g.nx;
  r.power_density = p.V_op * r.current_density;
  r.heat_rate = h[5] * i_scale / c->g.nx;
  r.inlet_flux = h[8];
  const double inflow = (c->g.flags & LBM_PRESSURE_INLET) ? h[8] * p.c_in : c->d.inflow;
  r.o2_utilisation = inflow > 0 ? sum_sc / inflow : 0.0;
  r.T_max = p.T_in_K + h[6];
  r.sum_f = h[0] + ncell;  // the rest population is stored as f0 - rho0
  r.sum_theta = h[1];
  r.sum_c = h[2];
  r.consumed_c = sum_sc;
  r.heat_added = h[4];
  if (o) *o = r;
  const double vals[] = {r.current_density, r.heat_rate, r.T_max, r.sum_f, r.sum_theta, r.sum_c, r.heat_added};
  for (double v : vals)
    if (!std::isfinite(v)) return fail(c, LBM_ERR_NONFINITE, "non-finite observable");
  if (h[7] > 0) return fail(c, LBM_ERR_NONFINITE, "non-finite populations");
  return LBM_OK;
}

// The observable reduction's scratch for lbm_observables_noalloc, for callers
// that cannot allocate device memory: the per-workgroup partial sums, the
// reduced values and the CL profiles (ObsBuffers) of one call.  Each GPU
// holds its own copy until the process ends; every call on a GPU reuses it,
// so calls that overlap on one GPU race.
constexpr size_t kNoAllocScratchDoubles = size_t(1) << 19;  // 4 MiB
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_addr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

namespace {

// Scratch doubles one lbm_observables_noalloc call needs (ObsBuffers).
size_t noalloc_scratch_doubles(const lbm_ctx* c) {
  return size_t(c->L.nblocks_obs) * kObsQ + kObsQ + 3 * size_t(c->g.nx);
}

// Device address of `scratch` on the context's GPU, resolved once per device
// with that device current (in host code the array's name is not a device
// address).
lbm_status scratch_for_device(lbm_ctx* c, double** out) {
  if (c->device < 0 || c->device >= kMaxDevices) return fail(c, LBM_ERR_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_addr[c->device]) {
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) return fail(c, LBM_ERR_DEVICE, "hipGetDevice failed");
    if (prev != c->device && hipSetDevice(c->device) != hipSuccess)
      return fail(c, LBM_ERR_DEVICE, "hipSetDevice failed");
    void* addr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
    if (prev != c->device) (void)hipSetDevice(prev);
    if (e != hipSuccess || !addr)
      return fail(c, LBM_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
    g_scratch_addr[c->device] = static_cast<double*>(addr);
  }
  *out = g_scratch_addr[c->device];
  return LBM_OK;
}

}  // namespace

extern "C" {

void lbm_default_params(lbm_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->tau_f = 0.65;
  p->D_f_lat = 0.0125;
  p->Re = 10.0;
  p->T_in_K = 353.0;
  p->c_in = 1.0;
  p->V_op = 0.6;
  p->phi_gdl = 0.4;
  p->Da_gdl = 1e-3;
  p->deff_ratio_gdl = 0.0;
  p->dp_lat = 0.0;
  p->gdl_thickness_cm = 0.0254;
  p->dx_cm = 0.0;
  p->D_O2_cm2s = 5.2197e-2;
  p->aj0_ref = 1.0e-4;
  p->C_ref = 17.808e-6;
  p->alpha_c = 1.0;
  p->faraday = 96487.0;
  p->R_gas = 8.314;
  p->E_over_R = 16456.0;
  p->T_arrh = 353.15;
  p->U0_slope = 0.0025;
  p->U0_icept = 0.2329;
  p->k_f = 0.026;
  p->k_s = 1.5;
  p->rhocp_f = 1.0e-3;
  p->rhocp_s = 1.6;
  p->kinetics = LBM_KINETICS_TAFEL;
  p->alpha_a = 1.0;
}

size_t lbm_workspace_bytes(const lbm_geometry* g) {
  if (!geometry_ok(g)) return 0;
  return make_layout(g).total;
}

lbm_status lbm_create(const lbm_geometry* g, void* dev_ws, size_t ws_bytes, void* hip_stream, lbm_ctx** out) {
  if (!out) return LBM_ERR_INVALID_ARG;
  *out = nullptr;
  if (!geometry_ok(g) || !dev_ws) return LBM_ERR_INVALID_ARG;
  const Layout L = make_layout(g);
  if (ws_bytes < L.total || (reinterpret_cast<uintptr_t>(dev_ws) % kAlign) != 0) return LBM_ERR_INVALID_ARG;
  lbm_ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) return LBM_ERR_INVALID_ARG;
  c->g = *g;
  c->L = L;
  c->ws = static_cast<char*>(dev_ws);
  c->stream = static_cast<hipStream_t>(hip_stream);
  (void)hipGetDevice(&c->device);
  *out = c;
  return LBM_OK;
}

lbm_status lbm_set_params(lbm_ctx* c, const lbm_params* p, const void* phi, const void* inv_k, const void* d_eff) {
  if (!c || !p) return LBM_ERR_INVALID_ARG;
  c->params_set = false;
  c->adj_ready = false;
  return c->g.precision == 64 ? set_params_t<double>(c, p, phi, inv_k, d_eff)
                              : set_params_t<float>(c, p, phi, inv_k, d_eff);
}

lbm_status lbm_init_equilibrium(lbm_ctx* c) {
  if (!c) return LBM_ERR_INVALID_ARG;
  if (!c->params_set) return fail(c, LBM_ERR_STATE, "lbm_set_params first");
  c->adj_ready = false;
  c->cur = 0;
  c->step = 0;
  if (c->g.precision == 64) launch_init<double>(c); else launch_init<float>(c);
  return check_launch(c, "init");
}

lbm_status lbm_step(lbm_ctx* c, int64_t n) {
  const TraceRange range("lbm_step");
  if (!c || n < 0) return LBM_ERR_INVALID_ARG;
  if (!c->params_set) return fail(c, LBM_ERR_STATE, "lbm_set_params first");
  if (c->g.precision == 64) launch_step<double>(c, n); else launch_step<float>(c, n);
  c->step += n;
  return check_launch(c, "step");
}

lbm_status lbm_observables(lbm_ctx* c, lbm_obs* out, double* pi, double* pc, double* pT) {
  const TraceRange range("lbm_observables");
  if (!c) return LBM_ERR_INVALID_ARG;
  if (!c->params_set) return fail(c, LBM_ERR_STATE, "lbm_set_params first");
  const ObsBuffers b{c->partial(), c->out(), c->prof()};
  return c->g.precision == 64 ? observables_t<double>(c, out, pi, pc, pT, b)
                              : observables_t<float>(c, out, pi, pc, pT, b);
}

lbm_status lbm_observables_noalloc(lbm_ctx* c, lbm_obs* out, double* pi, double* pc, double* pT) {
  if (!c) return LBM_ERR_INVALID_ARG;
  if (!c->params_set) return fail(c, LBM_ERR_STATE, "lbm_set_params first");
  const size_t need = noalloc_scratch_doubles(c);
  if (need > kNoAllocScratchDoubles)
    return fail(c, LBM_ERR_INVALID_ARG,
                "lattice too large for the static observable scratch: needs " + std::to_string(need * 8) +
                    " bytes, the maximum is " + std::to_string(kNoAllocScratchDoubles * 8));
  double* base = nullptr;
  if (lbm_status s = scratch_for_device(c, &base); s != LBM_OK) return s;
  const size_t n_part = size_t(c->L.nblocks_obs) * kObsQ;
  const ObsBuffers b{base, base + n_part, base + n_part + kObsQ};
  return c->g.precision == 64 ? observables_t<double>(c, out, pi, pc, pT, b)
                              : observables_t<float>(c, out, pi, pc, pT, b);
}

lbm_status lbm_get_fields(lbm_ctx* c, void* ux, void* uy, void* p, void* T, void* th, void* cc) {
  if (!c) return LBM_ERR_INVALID_ARG;
  if (!c->params_set) return fail(c, LBM_ERR_STATE, "lbm_set_params first");
  if (c->g.precision == 64) launch_fields<double>(c, ux, uy, p, T, th, cc);
  else launch_fields<float>(c, ux, uy, p, T, th, cc);
  return check_launch(c, "fields");
}

lbm_status lbm_get_material(lbm_ctx* c, void* phi, void* inv_k, void* d_eff) {
  if (!c) return LBM_ERR_INVALID_ARG;
  if (!c->params_set) return fail(c, LBM_ERR_STATE, "lbm_set_params first");
  const dim3 grid((c->g.nx + kBlock - 1) / kBlock, c->g.ny);
  if (c->g.precision == 64) {
    const MatPtrs<double> m = mat_ptrs<double>(c);
    auto* a = static_cast<double*>(phi);
    auto* b = static_cast<double*>(inv_k);
    auto* d = static_cast<double*>(d_eff);
    switch (c->mat) {
      case MAT_LAYERED: hipLaunchKernelGGL((k_material<double, MAT_LAYERED>), grid, dim3(kBlock), 0, c->stream, m.phi, m.invk, m.d, c->kd, a, b, d); break;
      case MAT_PHI: hipLaunchKernelGGL((k_material<double, MAT_PHI>), grid, dim3(kBlock), 0, c->stream, m.phi, m.invk, m.d, c->kd, a, b, d); break;
      default: hipLaunchKernelGGL((k_material<double, MAT_FULL>), grid, dim3(kBlock), 0, c->stream, m.phi, m.invk, m.d, c->kd, a, b, d); break;
    }
  } else {
    const MatPtrs<float> m = mat_ptrs<float>(c);
    auto* a = static_cast<float*>(phi);
    auto* b = static_cast<float*>(inv_k);
    auto* d = static_cast<float*>(d_eff);
    switch (c->mat) {
      case MAT_LAYERED: hipLaunchKernelGGL((k_material<float, MAT_LAYERED>), grid, dim3(kBlock), 0, c->stream, m.phi, m.invk, m.d, c->kf, a, b, d); break;
      case MAT_PHI: hipLaunchKernelGGL((k_material<float, MAT_PHI>), grid, dim3(kBlock), 0, c->stream, m.phi, m.invk, m.d, c->kf, a, b, d); break;
      default: hipLaunchKernelGGL((k_material<float, MAT_FULL>), grid, dim3(kBlock), 0, c->stream, m.phi, m.invk, m.d, c->kf, a, b, d); break;
    }
  }
  return check_launch(c, "get_material");
}

lbm_status lbm_get_populations(lbm_ctx* c, void* dst) {
  if (!c || !dst) return LBM_ERR_INVALID_ARG;
  if (!c->params_set) return fail(c, LBM_ERR_STATE, "lbm_set_params first");
  const dim3 grid((c->g.nx + kBlock - 1) / kBlock, c->g.ny);
  if (c->g.precision == 64)
    hipLaunchKernelGGL(k_export<double>, grid, dim3(kBlock), 0, c->stream,
                       static_cast<const double*>(c->state(c->cur)), static_cast<double*>(dst), c->kd);
  else
    hipLaunchKernelGGL(k_export<float>, grid, dim3(kBlock), 0, c->stream,
                       static_cast<const float*>(c->state(c->cur)), static_cast<float*>(dst), c->kf);
  return check_launch(c, "get_populations");
}

lbm_status lbm_set_populations(lbm_ctx* c, const void* src, int64_t step) {
  if (!c || !src) return LBM_ERR_INVALID_ARG;
  if (!c->params_set) return fail(c, LBM_ERR_STATE, "lbm_set_params first");
  const dim3 grid((c->g.nx + kBlock - 1) / kBlock, c->g.ny);
  if (c->g.precision == 64)
    hipLaunchKernelGGL(k_import<double>, grid, dim3(kBlock), 0, c->stream, static_cast<const double*>(src),
                       static_cast<double*>(c->state(c->cur)), c->kd);
  else
    hipLaunchKernelGGL(k_import<float>, grid, dim3(kBlock), 0, c->stream, static_cast<const float*>(src),
                       static_cast<float*>(c->state(c->cur)), c->kf);
  c->step = step;
  c->adj_ready = false;
  return check_launch(c, "set_populations");
}

size_t lbm_state_bytes(const lbm_ctx* c) {
  if (!c) return 0;
  return size_t(19) * c->L.plane * c->L.esize;
}

lbm_status lbm_save_state(lbm_ctx* c, void* dst, int64_t* step_out) {
  if (!c || !dst) return LBM_ERR_INVALID_ARG;
  if (hipMemcpyAsync(dst, c->state(c->cur), lbm_state_bytes(c), hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
    return fail(c, LBM_ERR_DEVICE, "save_state copy failed");
  if (step_out) *step_out = c->step;
  return LBM_OK;
}

lbm_status lbm_load_state(lbm_ctx* c, const void* src, int64_t step) {
  if (!c || !src) return LBM_ERR_INVALID_ARG;
  if (hipMemcpyAsync(c->state(c->cur), src, lbm_state_bytes(c), hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
    return fail(c, LBM_ERR_DEVICE, "load_state copy failed");
  c->step = step;
  c->adj_ready = false;
  return LBM_OK;
}

int64_t lbm_step_count(const lbm_ctx* c) { return c ? c->step : -1; }

lbm_status lbm_synchronize(lbm_ctx* c) {
  if (!c) return LBM_ERR_INVALID_ARG;
  const hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail(c, LBM_ERR_DEVICE, std::string("synchronize: ") + hipGetErrorString(e));
  return LBM_OK;
}

void lbm_destroy(lbm_ctx* c) {
  if (!c) return;
  if (c->aux) {
    (void)hipStreamSynchronize(c->aux);
    (void)hipStreamDestroy(c->aux);
  }
  for (hipEvent_t e : {c->ev_in, c->ev_rep[0], c->ev_rep[1], c->ev_rev[0], c->ev_rev[1]})
    if (e) (void)hipEventDestroy(e);
  delete c;
}

const char* lbm_status_string(lbm_status s) {
  switch (s) {
    case LBM_OK: return "ok";
    case LBM_ERR_INVALID_ARG: return "invalid argument";
    case LBM_ERR_UNSTABLE_PARAMS: return "parameters outside the stable range";
    case LBM_ERR_DEVICE: return "device error";
    case LBM_ERR_NONFINITE: return "non-finite result";
    case LBM_ERR_STATE: return "call out of order";
  }
  return "unknown status";
}

const char* lbm_last_error(const lbm_ctx* c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"

// ---------------------------------------------------------------------------
// Checkpointed forward run and discrete adjoint (lbm_forward_checkpointed,
// lbm_backward).
// ---------------------------------------------------------------------------
#include "lbm_adjoint_kernels.hpp"

namespace {

struct AdjLayout {
  size_t state = 0;  // aligned bytes of one state
  int nck = 0;
  size_t off_ck = 0, off_replay = 0, off_lam = 0, off_grad = 0, total = 0;
};

AdjLayout adj_layout(const lbm_ctx* c, int64_t nsteps, int32_t every) {
  AdjLayout A;
  A.state = align_up(size_t(19) * c->L.plane * c->L.esize);
  A.nck = int((nsteps + every - 1) / every);
  size_t o = 0;
  A.off_ck = o;
  o += size_t(A.nck) * A.state;
  A.off_replay = o;  // two replay buffers (the next segment is replayed while one is swept)
  o += size_t(2) * size_t(std::min<int64_t>(every, nsteps)) * A.state;
  A.off_lam = o;
  o += 2 * A.state;
  A.off_grad = o;
  o += align_up(size_t(3) * c->L.plane * c->L.esize);
  A.total = o;
  return A;
}

// Steps from state(0) to state(n) of a chain of states, storing each: a
// pair per launch where the lattice allows it, single steps otherwise.
// overlapped: the chain runs beside other work (the adjoint's replay, on
// the second stream during a reverse sweep), where pairs pay at any size:
// they store three states per two steps instead of four, and the latency
// of a launch is hidden (1024x256 FP32 adjoint 10.28 -> 10.55 GLUPS, the
// same gradient bits; run alone, pairs at that size are slower).
template <typename R, typename Slot>
void launch_step_chain(lbm_ctx* c, Slot state, int n, hipStream_t stream, bool overlapped) {
  const MatPtrs<R> m = mat_ptrs<R>(c);
  const Consts<R> k = consts<R>(c);
  int j = 1;
  if (overlapped ? two_step_form_applies(c) : two_steps_per_launch(c))
    for (; j + 1 <= n; j += 2)
      launch_step_pair<R, MAT_FULL>(c, static_cast<const R*>(state(j - 1)), static_cast<R*>(state(j)),
                                    static_cast<R*>(state(j + 1)), m, k, stream);
  for (; j <= n; ++j)
    launch_step_kernel<R, MAT_FULL>(c, static_cast<const R*>(state(j - 1)), static_cast<R*>(state(j)), m, k, stream);
}

// The last segment of the checkpointed forward run steps through replay
// buffer 0 (the same kernel as lbm_step, so the same states), where the
// first reverse sweep reads them: lbm_backward need not replay it.
template <typename R>
lbm_status forward_last_segment(lbm_ctx* c, const AdjLayout& A, int64_t n) {
  char* buf = c->adj_ws + A.off_replay;
  const size_t sb = size_t(19) * c->L.plane * c->L.esize;
  if (hipMemcpyAsync(buf, c->state(c->cur), sb, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
    return fail(c, LBM_ERR_DEVICE, "replay buffer copy failed");
  void* last = c->state(c->cur ^ 1);
  launch_step_chain<R>(c, [&](int64_t j) -> void* { return j < n ? buf + size_t(j) * A.state : last; }, int(n),
                       c->stream, false);
  c->cur ^= 1;
  c->step += n;
  return check_launch(c, "forward_checkpointed");
}

template <typename R>
lbm_status backward_t(lbm_ctx* c, double dJ, void* g_invk, void* g_phi, void* g_d) {
  const AdjLayout A = adj_layout(c, c->adj_nsteps, c->adj_every);
  char* ws = c->adj_ws;
  const MatPtrs<R> m = mat_ptrs<R>(c);
  const Consts<R> k = consts<R>(c);
  const dim3 grid((c->g.nx + kBlock - 1) / kBlock, c->g.ny);
  R* grad = reinterpret_cast<R*>(ws + A.off_grad);
  R* lam[2] = {reinterpret_cast<R*>(ws + A.off_lam), reinterpret_cast<R*>(ws + A.off_lam + A.state)};
  const int64_t ngrad = int64_t(3) * c->L.plane;
  hipLaunchKernelGGL(k_fill<R>, dim3(unsigned((ngrad + kBlock - 1) / kBlock)), dim3(kBlock), 0, c->stream, grad,
                     ngrad, R(0));
  // Seed: adjoint of J = current density on the final state.
  const lbm_params& p = c->p;
  const double w = dJ * c->d.dx / c->g.nx * 4.0 * p.faraday * p.C_ref / c->d.dt;
  // Buoyancy, the heat-capacity ratio, the pressure-driven inlet and the
  // thin-film CL take the reverse-step instances that carry their terms.
  const bool ext = c->g.flags & (LBM_BUOYANCY | LBM_SIGMA_ENERGY | LBM_PRESSURE_INLET | LBM_THIN_CL);
  const R* S_final = static_cast<const R*>(c->state(c->cur));
  if (ext)
    hipLaunchKernelGGL((k_adj_step<R, true, true>), grid, dim3(kBlock), 0, c->stream, S_final,
                       static_cast<const R*>(nullptr), lam[0], grad, m.phi, m.invk, m.d, k, R(w));
  else
    hipLaunchKernelGGL((k_adj_step<R, true>), grid, dim3(kBlock), 0, c->stream, S_final,
                       static_cast<const R*>(nullptr), lam[0], grad, m.phi, m.invk, m.d, k, R(w));
  // Segments are swept from the last to the first.  Segment s - 1 is
  // replayed from its checkpoint into one replay buffer on the second
  // stream while segment s is swept in reverse from the other on the
  // context stream: a replay waits for the sweep that last used its buffer,
  // a sweep waits for the replay of its segment.
  if (!c->aux) {
    if (hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) != hipSuccess) {
      c->aux = nullptr;
      return fail(c, LBM_ERR_DEVICE, "second stream creation failed");
    }
    for (hipEvent_t* e : {&c->ev_in, &c->ev_rep[0], &c->ev_rep[1], &c->ev_rev[0], &c->ev_rev[1]})
      if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess)
        return fail(c, LBM_ERR_DEVICE, "event creation failed");
  }
  const size_t rbuf = size_t(std::min<int64_t>(c->adj_every, c->adj_nsteps)) * A.state;
  bool used[2] = {false, false};
  if (hipEventRecord(c->ev_in, c->stream) != hipSuccess || hipStreamWaitEvent(c->aux, c->ev_in, 0) != hipSuccess)
    return fail(c, LBM_ERR_DEVICE, "replay ordering failed");
  auto seg_len = [&](int seg) {
    return int(std::min<int64_t>(c->adj_every, c->adj_nsteps - int64_t(seg) * c->adj_every));
  };
  auto replay = [&](int seg, int b) -> lbm_status {
    char* buf = ws + A.off_replay + size_t(b) * rbuf;
    if (used[b] && hipStreamWaitEvent(c->aux, c->ev_rev[b], 0) != hipSuccess)
      return fail(c, LBM_ERR_DEVICE, "replay ordering failed");
    if (hipMemcpyAsync(buf, ws + A.off_ck + size_t(seg) * A.state, A.state, hipMemcpyDeviceToDevice, c->aux) !=
        hipSuccess)
      return fail(c, LBM_ERR_DEVICE, "replay restore failed");
    launch_step_chain<R>(c, [&](int j) -> void* { return buf + size_t(j) * A.state; }, seg_len(seg) - 1, c->aux,
                         true);
    if (hipEventRecord(c->ev_rep[b], c->aux) != hipSuccess) return fail(c, LBM_ERR_DEVICE, "replay event failed");
    return LBM_OK;
  };
  if (c->adj_last_resident) {  // written on this stream by the forward run
    if (hipEventRecord(c->ev_rep[0], c->stream) != hipSuccess) return fail(c, LBM_ERR_DEVICE, "replay event failed");
  } else if (lbm_status st = replay(A.nck - 1, 0); st != LBM_OK) {
    return st;
  }
  c->adj_last_resident = false;  // the sweep below reuses buffer 0
  int cur = 0;
  for (int seg = A.nck - 1; seg >= 0; --seg) {
    const int b = (A.nck - 1 - seg) & 1;
    if (seg > 0)
      if (lbm_status st = replay(seg - 1, b ^ 1); st != LBM_OK) return st;
    if (hipStreamWaitEvent(c->stream, c->ev_rep[b], 0) != hipSuccess)
      return fail(c, LBM_ERR_DEVICE, "replay join failed");
    const char* buf = ws + A.off_replay + size_t(b) * rbuf;
    for (int j = seg_len(seg) - 1; j >= 0; --j) {
      const R* S = reinterpret_cast<const R*>(buf + size_t(j) * A.state);
      if (ext)
        hipLaunchKernelGGL((k_adj_step<R, false, true>), grid, dim3(kBlock), 0, c->stream, S, lam[cur],
                           lam[cur ^ 1], grad, m.phi, m.invk, m.d, k, R(0));
      else
        hipLaunchKernelGGL((k_adj_step<R, false>), grid, dim3(kBlock), 0, c->stream, S, lam[cur], lam[cur ^ 1], grad,
                           m.phi, m.invk, m.d, k, R(0));
      cur ^= 1;
    }
    if (hipEventRecord(c->ev_rev[b], c->stream) != hipSuccess) return fail(c, LBM_ERR_DEVICE, "sweep event failed");
    used[b] = true;
  }
  hipLaunchKernelGGL(k_adj_init<R>, grid, dim3(kBlock), 0, c->stream, lam[cur], grad, k);
  void* outs[3] = {g_phi, g_invk, g_d};
  for (int i = 0; i < 3; ++i)
    if (outs[i])
      hipLaunchKernelGGL(k_unpitch<R>, grid, dim3(kBlock), 0, c->stream, grad + size_t(i) * c->L.plane,
                         static_cast<R*>(outs[i]), c->g.nx, c->L.pitch);
  if (lbm_status s = check_launch(c, "backward"); s != LBM_OK) return s;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c, LBM_ERR_DEVICE, "backward sync failed");
  return LBM_OK;
}

}  // namespace

extern "C" {

size_t lbm_adjoint_workspace_bytes(const lbm_ctx* c, int64_t nsteps, int32_t every) {
  if (!c || nsteps < 1 || every < 1) return 0;
  return adj_layout(c, nsteps, every).total;
}

lbm_status lbm_forward_checkpointed(lbm_ctx* c, int64_t nsteps, int32_t every, void* dev_ws, size_t ws_bytes,
                                    double* J_out) {
  const TraceRange range("lbm_forward_checkpointed");
  if (!c || nsteps < 1 || every < 1 || !dev_ws) return LBM_ERR_INVALID_ARG;
  if (!c->params_set) return fail(c, LBM_ERR_STATE, "lbm_set_params first");
  if (c->mat != MAT_FULL)
    return fail(c, LBM_ERR_STATE, "the adjoint needs the three per-cell fields (independent_fields or all arrays)");
  const AdjLayout A = adj_layout(c, nsteps, every);
  if (ws_bytes < A.total || reinterpret_cast<uintptr_t>(dev_ws) % kAlign != 0)
    return fail(c, LBM_ERR_INVALID_ARG, "adjoint workspace too small or misaligned");
  c->adj_ready = false;
  if (lbm_status s = lbm_init_equilibrium(c); s != LBM_OK) return s;
  c->adj_ws = static_cast<char*>(dev_ws);
  c->adj_nsteps = nsteps;
  c->adj_every = every;
  const size_t sb = size_t(19) * c->L.plane * c->L.esize;
  for (int seg = 0; seg < A.nck; ++seg) {
    if (hipMemcpyAsync(c->adj_ws + A.off_ck + size_t(seg) * A.state, c->state(c->cur), sb, hipMemcpyDeviceToDevice,
                       c->stream) != hipSuccess)
      return fail(c, LBM_ERR_DEVICE, "checkpoint copy failed");
    const int64_t n = std::min<int64_t>(every, nsteps - int64_t(seg) * every);
    if (seg == A.nck - 1) {
      const lbm_status s = c->g.precision == 64 ? forward_last_segment<double>(c, A, n)
                                                : forward_last_segment<float>(c, A, n);
      if (s != LBM_OK) return s;
    } else if (lbm_status s = lbm_step(c, n); s != LBM_OK) {
      return s;
    }
  }
  c->adj_last_resident = true;
  lbm_obs o{};
  if (lbm_status s = lbm_observables(c, &o, nullptr, nullptr, nullptr); s != LBM_OK) return s;
  if (J_out) *J_out = o.current_density;
  c->adj_step = c->step;
  c->adj_ready = true;
  return LBM_OK;
}

lbm_status lbm_backward(lbm_ctx* c, double dJ, void* grad_inv_k, void* grad_phi, void* grad_d_eff) {
  const TraceRange range("lbm_backward");
  if (!c) return LBM_ERR_INVALID_ARG;
  if (!c->adj_ready || c->adj_step != c->step)
    return fail(c, LBM_ERR_STATE, "lbm_backward needs a preceding lbm_forward_checkpointed on the same state");
  return c->g.precision == 64 ? backward_t<double>(c, dJ, grad_inv_k, grad_phi, grad_d_eff)
                              : backward_t<float>(c, dJ, grad_inv_k, grad_phi, grad_d_eff);
}

}  // extern "C"
