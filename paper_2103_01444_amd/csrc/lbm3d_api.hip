// Host side of the 3D part of the C ABI (lbm3d_*): context, parameters,
// launches.  As in 2D, all device memory is the caller's workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lbm3d_kernels.hpp"
#include "lbm_host.hpp"
#include "lbm_pem.h"

using namespace lbm3;

namespace {

constexpr size_t kAlign3 = 256;
size_t align3(size_t v) { return (v + kAlign3 - 1) / kAlign3 * kAlign3; }
constexpr int kChunkY = 64;  // y rows per chunk of the step's launch order (fastest of 1..128 at 256x128x64)

struct Layout3 {
  int pitch = 0;
  int64_t plane = 0;  // elements per population plane
  size_t esize = 0;
  size_t state = 0;   // aligned bytes of one 33-plane state
  size_t off_state[2] = {0, 0};
  size_t off_mat = 0, off_partial = 0, off_out = 0, total = 0;
  int nbx = 0;
  int nblocks_obs = 0;
};

bool geometry3_ok(const lbm3d_geometry* g) {
  if (!g) return false;
  if (g->nx < 3 || g->ny < 1 || g->nz < 1 || g->ny > 65535 || g->nz > 65535) return false;
  if (g->nz_channel < 0 || g->nz_gdl < 0 || g->nz_cl < 0) return false;
  if (g->nz_channel + g->nz_gdl + g->nz_cl != g->nz) return false;
  if (g->precision != 32 && g->precision != 64) return false;
  if (g->flags & ~(LBM_PERIODIC_X | LBM_PERIODIC_Y | LBM_PERIODIC_Z | LBM_BODY_FORCE | LBM_NO_REACTION |
                   LBM_PHYSICAL_HEAT))
    return false;
  const int64_t pitch = (int64_t(g->nx) + 63) / 64 * 64;
  if (lbm::plane_elems(pitch * g->ny * g->nz) * 33 >= (int64_t(1) << 31)) return false;  // 32-bit element offsets
  return true;
}

Layout3 make_layout3(const lbm3d_geometry* g) {
  Layout3 L;
  L.esize = g->precision == 64 ? 8 : 4;
  L.pitch = (g->nx + 63) / 64 * 64;
  L.plane = lbm::plane_elems(int64_t(L.pitch) * g->ny * g->nz);
  L.state = align3(size_t(33) * L.plane * L.esize);
  L.nbx = (g->nx + kBlock3 - 1) / kBlock3;
  L.nblocks_obs = L.nbx * g->ny * g->nz;
  size_t o = 0;
  L.off_state[0] = o;
  o += L.state;
  L.off_state[1] = o;
  o += L.state;
  L.off_mat = o;
  o += align3(size_t(3) * L.plane * L.esize);
  L.off_partial = o;
  o += align3(size_t(L.nblocks_obs) * kObsQ3 * sizeof(double));
  L.off_out = o;
  o += align3(16 * sizeof(double));
  L.total = o;
  return L;
}

// The 2D derivation applied to the through-plane (z) layering.
lbm_geometry as_layers(const lbm3d_geometry& g) {
  lbm_geometry l{};
  l.nx = g.nx;
  l.ny = g.nz;
  l.ny_channel = g.nz_channel;
  l.ny_gdl = g.nz_gdl;
  l.ny_cl = g.nz_cl;
  l.precision = g.precision;
  l.flags = g.flags & (LBM_PERIODIC_X | LBM_BODY_FORCE | LBM_NO_REACTION);
  return l;
}

}  // namespace

struct lbm3d_ctx {
  lbm3d_geometry g{};
  lbm_params p{};
  Layout3 L;
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  int cur = 0;
  int64_t step = 0;
  bool params_set = false;
  int mat = MAT_LAYERED;
  Consts3<float> kf{};
  Consts3<double> kd{};
  lbm::Derived d;
  std::string err;
  // checkpointed forward run held for lbm3d_backward
  char* adj_ws = nullptr;
  int64_t adj_nsteps = 0;
  int32_t adj_every = 0;
  int64_t adj_step = -1;
  bool adj_ready = false;
  // second stream for the boundary pass of the reverse sweep, and its events
  hipStream_t aux = nullptr;
  hipEvent_t ev_in = nullptr, ev_bnd = nullptr;

  void* state(int i) { return ws + L.off_state[i]; }
  void* mat_plane(int i) { return ws + L.off_mat + size_t(i) * L.plane * L.esize; }
  double* partial() { return reinterpret_cast<double*>(ws + L.off_partial); }
  double* out() { return reinterpret_cast<double*>(ws + L.off_out); }
  dim3 grid3() const { return dim3(L.nbx, g.ny, g.nz); }
};

namespace {

lbm_status fail3(lbm3d_ctx* c, lbm_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

lbm_status check3(lbm3d_ctx* c, const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail3(c, LBM_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return LBM_OK;
}

template <typename R>
void fill_consts3(Consts3<R>& k, const lbm3d_geometry& g, const lbm_params& p, const lbm::Derived& d, int pitch) {
  lbm::Consts<R> k2{};
  lbm::fill_consts(k2, as_layers(g), p, d, pitch);
  k.nx = g.nx;
  k.ny = g.ny;
  k.nz = g.nz;
  k.pitch = pitch;
  k.nz_ch = g.nz_channel;
  k.z_cl0 = g.nz_channel + g.nz_gdl;
  k.flags = g.flags;
  k.plane = int32_t(lbm::plane_elems(int64_t(pitch) * g.ny * g.nz));
  k.ty = std::min(kChunkY, g.ny);
  k.bv = k2.bv;
  k.s_plus = k2.s_e;
  k.s_minus = k2.s_q;
  k.nu = k2.nu;
  const double H = g.nz_channel, W = g.ny;
  k.u_in_coef = g.nz_channel > 0 ? R(36.0 * d.u_avg / (W * W * H * H)) : R(0);
  k.ax = k2.ax;
  k.ay = k2.ay;
  k.phi_gdl = k2.phi_gdl;
  k.invk_gdl = k2.invk_gdl;
  k.d_gdl = k2.d_gdl;
  k.D_f = k2.D_f;
  k.kc_inv = k2.kc_inv;
  k.deff_ratio = k2.deff_ratio;
  k.k_f = k2.k_f;
  k.k_s = k2.k_s;
  k.rhocp_f = k2.rhocp_f;
  k.rhocp_s = k2.rhocp_s;
  k.alpha_scale = k2.alpha_scale;
  k.T_in = k2.T_in;
  k.c_in = k2.c_in;
  k.V_op = k2.V_op;
  k.U0_slope = k2.U0_slope;
  k.U0_icept = k2.U0_icept;
  k.ln_k0 = k2.ln_k0;
  k.E_over_R = k2.E_over_R;
  k.inv_T_arrh = k2.inv_T_arrh;
  k.aF_over_R = k2.aF_over_R;
  k.four_f_cref = k2.four_f_cref;
  k.aFsum_over_R = k2.aFsum_over_R;
}

template <typename R>
const Consts3<R>& consts3(const lbm3d_ctx* c);
template <>
const Consts3<float>& consts3<float>(const lbm3d_ctx* c) { return c->kf; }
template <>
const Consts3<double>& consts3<double>(const lbm3d_ctx* c) { return c->kd; }

template <typename R>
struct Mat3Ptrs {
  const R *phi, *invk, *d;
};
template <typename R>
Mat3Ptrs<R> mat3_ptrs(lbm3d_ctx* c) {
  return {static_cast<const R*>(c->mat_plane(0)), static_cast<const R*>(c->mat_plane(1)),
          static_cast<const R*>(c->mat_plane(2))};
}

template <typename R>
bool host_range3(lbm3d_ctx* c, const void* dev, double& lo, double& hi) {
  const size_t n = size_t(c->g.nx) * c->g.ny * c->g.nz;
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

// One kernel template per material mode; F is called with the mode as a
// compile-time constant.
template <typename F>
void by_mat(int mat, F&& f) {
  switch (mat) {
    case MAT_LAYERED: f(std::integral_constant<int, MAT_LAYERED>{}); break;
    case MAT_PHI: f(std::integral_constant<int, MAT_PHI>{}); break;
    default: f(std::integral_constant<int, MAT_FULL>{}); break;
  }
}

template <typename R>
void launch_step3(lbm3d_ctx* c, int64_t n) {
  const Mat3Ptrs<R> m = mat3_ptrs<R>(c);
  const Consts3<R> k = consts3<R>(c);
  const dim3 grid(unsigned(c->L.nblocks_obs));
  by_mat(c->mat, [&](auto mode) {
    constexpr int MAT = decltype(mode)::value;
    for (int64_t i = 0; i < n; ++i) {
      const R* src = static_cast<const R*>(c->state(c->cur));
      R* dst = static_cast<R*>(c->state(c->cur ^ 1));
      hipLaunchKernelGGL((k3_step<R, MAT>), grid, dim3(kBlock3), 0, c->stream, src, dst, m.phi, m.invk, m.d, k);
      c->cur ^= 1;
    }
  });
}

template <typename R>
lbm_status set_params3_t(lbm3d_ctx* c, const lbm_params* p, const void* phi, const void* inv_k, const void* d_eff) {
  const lbm3d_geometry& g = c->g;
  if (p->p_outlet != 0.0) return fail3(c, LBM_ERR_INVALID_ARG, "the 3D variant's outlet pressure is 0 (p_outlet)");
  c->p = *p;
  std::string msg;
  const lbm_geometry lg = as_layers(g);
  if (lbm_status st = lbm::derive(lg, *p, c->d, msg); st != LBM_OK) return fail3(c, st, msg);
  // Peak of the product inlet profile is 2.25 U_avg (1.5 per direction).
  if (!(g.flags & LBM_PERIODIC_X) && 2.25 * std::fabs(c->d.u_avg) > 0.1)
    return fail3(c, LBM_ERR_UNSTABLE_PARAMS, "inlet peak velocity above 0.1");
  c->d.inflow = 0;
  if (!(g.flags & LBM_PERIODIC_X) && g.nz_channel > 0) {
    const double H = g.nz_channel, W = g.ny;
    const double coef = 36.0 * c->d.u_avg / (W * W * H * H);
    for (int z = 0; z < g.nz_channel; ++z)
      for (int y = 0; y < g.ny; ++y) {
        const double zc = z + 0.5, yc = y + 0.5;
        c->d.inflow += coef * yc * (W - yc) * zc * (H - zc) * p->c_in;
      }
  }
  fill_consts3(c->kf, g, *p, c->d, c->L.pitch);
  fill_consts3(c->kd, g, *p, c->d, c->L.pitch);

  const bool any = phi || inv_k || d_eff;
  if (!any && !p->independent_fields) {
    c->mat = MAT_LAYERED;
  } else if (phi && !inv_k && !d_eff && p->dp_lat > 0 && !p->independent_fields) {
    c->mat = MAT_PHI;
  } else {
    c->mat = MAT_FULL;
  }
  const dim3 grid = c->grid3();
  auto copy = [&](const void* src, int plane) {
    hipLaunchKernelGGL(k3_pitch_copy<R>, grid, dim3(kBlock3), 0, c->stream, static_cast<const R*>(src),
                       static_cast<R*>(c->mat_plane(plane)), g.nx, g.ny, c->L.pitch);
    return hipGetLastError() == hipSuccess;
  };
  if (phi && !copy(phi, 0)) return fail3(c, LBM_ERR_DEVICE, "copy of porosity failed");
  if (c->mat == MAT_FULL) {
    if (inv_k && !copy(inv_k, 1)) return fail3(c, LBM_ERR_DEVICE, "copy of 1/K failed");
    if (d_eff && !copy(d_eff, 2)) return fail3(c, LBM_ERR_DEVICE, "copy of D_eff failed");
    hipLaunchKernelGGL(k3_derive_fields<R>, grid, dim3(kBlock3), 0, c->stream, static_cast<R*>(c->mat_plane(0)),
                       static_cast<R*>(c->mat_plane(1)), static_cast<R*>(c->mat_plane(2)), consts3<R>(c),
                       phi ? 1 : 0, inv_k ? 1 : 0, d_eff ? 1 : 0);
    if (hipGetLastError() != hipSuccess) return fail3(c, LBM_ERR_DEVICE, "field derivation failed");
  }
  double phi_lo = p->phi_gdl, phi_hi = 1.0;
  double d_lo = std::min(c->d.d_gdl, p->D_f_lat), d_hi = std::max(c->d.d_gdl, p->D_f_lat);
  double k_lo = c->d.invk_gdl;
  if (phi && !host_range3<R>(c, phi, phi_lo, phi_hi)) return fail3(c, LBM_ERR_DEVICE, "reading porosity failed");
  if (inv_k) {
    double hi;
    if (!host_range3<R>(c, inv_k, k_lo, hi)) return fail3(c, LBM_ERR_DEVICE, "reading 1/K failed");
  }
  if (d_eff) {
    if (!host_range3<R>(c, d_eff, d_lo, d_hi)) return fail3(c, LBM_ERR_DEVICE, "reading D_eff failed");
  } else if (phi) {
    const double dl = p->deff_ratio_gdl > 0 ? p->deff_ratio_gdl * p->D_f_lat : std::pow(phi_lo, 1.5) * p->D_f_lat;
    d_lo = std::min(dl, p->D_f_lat);
  }
  if (!(phi_lo > 0) || phi_hi > 1.0) return fail3(c, LBM_ERR_UNSTABLE_PARAMS, "porosity outside (0, 1]");
  if (!(k_lo >= 0)) return fail3(c, LBM_ERR_UNSTABLE_PARAMS, "negative or non-finite 1/K");
  if (!(d_lo > 0) || d_hi > lbm::kMaxDiff)
    return fail3(c, LBM_ERR_UNSTABLE_PARAMS, "O2 diffusivity outside (0, 1/(4 sqrt 3)]");
  const double as = c->d.alpha_scale;
  const double a1 = lbm::alpha_lat(*p, phi_lo, as), a2 = lbm::alpha_lat(*p, phi_hi, as), a3 = lbm::alpha_lat(*p, 1.0, as);
  if (std::max({a1, a2, a3}) > lbm::kMaxDiff || !(std::min({a1, a2, a3}) > 0))
    return fail3(c, LBM_ERR_UNSTABLE_PARAMS, "thermal diffusivity outside (0, 1/(4 sqrt 3)]");
  if (hipStreamSynchronize(c->stream) != hipSuccess) return fail3(c, LBM_ERR_DEVICE, "set_params sync failed");
  c->params_set = true;
  return LBM_OK;
}

template <typename R>
lbm_status observables3_t(lbm3d_ctx* c, lbm_obs* o) {
  const lbm_params& p = c->p;
  const Mat3Ptrs<R> m = mat3_ptrs<R>(c);
  const R* src = static_cast<const R*>(c->state(c->cur));
  by_mat(c->mat, [&](auto mode) {
    constexpr int MAT = decltype(mode)::value;
    hipLaunchKernelGGL((k3_obs_cells<R, MAT>), c->grid3(), dim3(kBlock3), 0, c->stream, src, m.phi, m.invk, m.d,
                       consts3<R>(c), c->partial());
  });
  hipLaunchKernelGGL(lbm::k_obs_final<kObsQ3>, dim3(kObsQ3), dim3(lbm::kBlock), 0, c->stream, c->partial(),
                     c->L.nblocks_obs, c->out());
  if (lbm_status s = check3(c, "observables"); s != LBM_OK) return s;
  double h[kObsQ3];
  if (hipMemcpyAsync(h, c->out(), sizeof(h), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
    return fail3(c, LBM_ERR_DEVICE, "observable copy failed");
  if (hipStreamSynchronize(c->stream) != hipSuccess) return fail3(c, LBM_ERR_DEVICE, "observables sync failed");
  // i(x, y) = sum over CL layers of 4 F C_ref s_c / dt * dx; reported: its mean over (x, y).
  const double i_scale = 4.0 * p.faraday * p.C_ref / c->d.dt * c->d.dx;
  const double ncol = double(c->g.nx) * c->g.ny;
  lbm_obs r{};
  r.step = c->step;
  r.current_density = h[3] * i_scale / ncol;
  r.power_density = p.V_op * r.current_density;
  r.heat_rate = h[5] * i_scale / ncol;
  r.o2_utilisation = c->d.inflow > 0 ? h[3] / c->d.inflow : 0.0;
  r.inlet_flux = h[8];
  r.T_max = p.T_in_K + h[6];
  r.sum_f = h[0] + ncol * c->g.nz;  // the rest population is stored as f0 - rho0
  r.sum_theta = h[1];
  r.sum_c = h[2];
  r.consumed_c = h[3];
  r.heat_added = h[4];
  if (o) *o = r;
  const double vals[] = {r.current_density, r.heat_rate, r.T_max, r.sum_f, r.sum_theta, r.sum_c, r.heat_added};
  for (double v : vals)
    if (!std::isfinite(v)) return fail3(c, LBM_ERR_NONFINITE, "non-finite observable");
  if (h[7] > 0) return fail3(c, LBM_ERR_NONFINITE, "non-finite populations");
  return LBM_OK;
}

}  // namespace

extern "C" {

size_t lbm3d_workspace_bytes(const lbm3d_geometry* g) {
  if (!geometry3_ok(g)) return 0;
  return make_layout3(g).total;
}

lbm_status lbm3d_create(const lbm3d_geometry* g, void* dev_ws, size_t ws_bytes, void* hip_stream, lbm3d_ctx** out) {
  if (!out) return LBM_ERR_INVALID_ARG;
  *out = nullptr;
  if (!geometry3_ok(g) || !dev_ws) return LBM_ERR_INVALID_ARG;
  const Layout3 L = make_layout3(g);
  if (ws_bytes < L.total || (reinterpret_cast<uintptr_t>(dev_ws) % kAlign3) != 0) return LBM_ERR_INVALID_ARG;
  lbm3d_ctx* c = new (std::nothrow) lbm3d_ctx();
  if (!c) return LBM_ERR_INVALID_ARG;
  c->g = *g;
  c->L = L;
  c->ws = static_cast<char*>(dev_ws);
  c->stream = static_cast<hipStream_t>(hip_stream);
  *out = c;
  return LBM_OK;
}

lbm_status lbm3d_set_params(lbm3d_ctx* c, const lbm_params* p, const void* phi, const void* inv_k, const void* d_eff) {
  if (!c || !p) return LBM_ERR_INVALID_ARG;
  c->params_set = false;
  c->adj_ready = false;
  return c->g.precision == 64 ? set_params3_t<double>(c, p, phi, inv_k, d_eff)
                              : set_params3_t<float>(c, p, phi, inv_k, d_eff);
}

lbm_status lbm3d_init_equilibrium(lbm3d_ctx* c) {
  if (!c) return LBM_ERR_INVALID_ARG;
  if (!c->params_set) return fail3(c, LBM_ERR_STATE, "lbm3d_set_params first");
  c->adj_ready = false;
  c->cur = 0;
  c->step = 0;
  auto run = [&](auto tag) {
    using R = decltype(tag);
    const Mat3Ptrs<R> m = mat3_ptrs<R>(c);
    by_mat(c->mat, [&](auto mode) {
      constexpr int MAT = decltype(mode)::value;
      hipLaunchKernelGGL((k3_init<R, MAT>), c->grid3(), dim3(kBlock3), 0, c->stream, static_cast<R*>(c->state(0)),
                         m.phi, m.invk, m.d, consts3<R>(c));
    });
  };
  if (c->g.precision == 64) run(double{}); else run(float{});
  return check3(c, "init");
}

lbm_status lbm3d_step(lbm3d_ctx* c, int64_t n) {
  const lbm::TraceRange range("lbm3d_step");
  if (!c || n < 0) return LBM_ERR_INVALID_ARG;
  if (!c->params_set) return fail3(c, LBM_ERR_STATE, "lbm3d_set_params first");
  if (c->g.precision == 64) launch_step3<double>(c, n); else launch_step3<float>(c, n);
  c->step += n;
  return check3(c, "step");
}

lbm_status lbm3d_observables(lbm3d_ctx* c, lbm_obs* out) {
  const lbm::TraceRange range("lbm3d_observables");
  if (!c) return LBM_ERR_INVALID_ARG;
  if (!c->params_set) return fail3(c, LBM_ERR_STATE, "lbm3d_set_params first");
  return c->g.precision == 64 ? observables3_t<double>(c, out) : observables3_t<float>(c, out);
}

lbm_status lbm3d_get_fields(lbm3d_ctx* c, void* ux, void* uy, void* uz, void* p, void* T, void* th, void* cc) {
  if (!c) return LBM_ERR_INVALID_ARG;
  if (!c->params_set) return fail3(c, LBM_ERR_STATE, "lbm3d_set_params first");
  auto run = [&](auto tag) {
    using R = decltype(tag);
    const Mat3Ptrs<R> m = mat3_ptrs<R>(c);
    by_mat(c->mat, [&](auto mode) {
      constexpr int MAT = decltype(mode)::value;
      hipLaunchKernelGGL((k3_fields<R, MAT>), c->grid3(), dim3(kBlock3), 0, c->stream,
                         static_cast<const R*>(c->state(c->cur)), m.phi, m.invk, m.d, consts3<R>(c),
                         static_cast<R*>(ux), static_cast<R*>(uy), static_cast<R*>(uz), static_cast<R*>(p),
                         static_cast<R*>(T), static_cast<R*>(th), static_cast<R*>(cc));
    });
  };
  if (c->g.precision == 64) run(double{}); else run(float{});
  return check3(c, "fields");
}

lbm_status lbm3d_get_material(lbm3d_ctx* c, void* phi, void* inv_k, void* d_eff) {
  if (!c) return LBM_ERR_INVALID_ARG;
  if (!c->params_set) return fail3(c, LBM_ERR_STATE, "lbm3d_set_params first");
  auto run = [&](auto tag) {
    using R = decltype(tag);
    const Mat3Ptrs<R> m = mat3_ptrs<R>(c);
    by_mat(c->mat, [&](auto mode) {
      constexpr int MAT = decltype(mode)::value;
      hipLaunchKernelGGL((k3_material<R, MAT>), c->grid3(), dim3(kBlock3), 0, c->stream, m.phi, m.invk, m.d,
                         consts3<R>(c), static_cast<R*>(phi), static_cast<R*>(inv_k), static_cast<R*>(d_eff));
    });
  };
  if (c->g.precision == 64) run(double{}); else run(float{});
  return check3(c, "get_material");
}

lbm_status lbm3d_get_populations(lbm3d_ctx* c, void* dst) {
  if (!c || !dst) return LBM_ERR_INVALID_ARG;
  if (!c->params_set) return fail3(c, LBM_ERR_STATE, "lbm3d_set_params first");
  if (c->g.precision == 64)
    hipLaunchKernelGGL(k3_export<double>, c->grid3(), dim3(kBlock3), 0, c->stream,
                       static_cast<const double*>(c->state(c->cur)), static_cast<double*>(dst), c->kd);
  else
    hipLaunchKernelGGL(k3_export<float>, c->grid3(), dim3(kBlock3), 0, c->stream,
                       static_cast<const float*>(c->state(c->cur)), static_cast<float*>(dst), c->kf);
  return check3(c, "get_populations");
}

lbm_status lbm3d_set_populations(lbm3d_ctx* c, const void* src, int64_t step) {
  if (!c || !src) return LBM_ERR_INVALID_ARG;
  if (!c->params_set) return fail3(c, LBM_ERR_STATE, "lbm3d_set_params first");
  if (c->g.precision == 64)
    hipLaunchKernelGGL(k3_import<double>, c->grid3(), dim3(kBlock3), 0, c->stream, static_cast<const double*>(src),
                       static_cast<double*>(c->state(c->cur)), c->kd);
  else
    hipLaunchKernelGGL(k3_import<float>, c->grid3(), dim3(kBlock3), 0, c->stream, static_cast<const float*>(src),
                       static_cast<float*>(c->state(c->cur)), c->kf);
  c->step = step;
  c->adj_ready = false;
  return check3(c, "set_populations");
}

int64_t lbm3d_step_count(const lbm3d_ctx* c) { return c ? c->step : -1; }

lbm_status lbm3d_synchronize(lbm3d_ctx* c) {
  if (!c) return LBM_ERR_INVALID_ARG;
  const hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail3(c, LBM_ERR_DEVICE, std::string("synchronize: ") + hipGetErrorString(e));
  return LBM_OK;
}

void lbm3d_destroy(lbm3d_ctx* c) {
  if (!c) return;
  if (c->aux) {
    (void)hipStreamSynchronize(c->aux);
    (void)hipStreamDestroy(c->aux);
  }
  if (c->ev_in) (void)hipEventDestroy(c->ev_in);
  if (c->ev_bnd) (void)hipEventDestroy(c->ev_bnd);
  delete c;
}

const char* lbm3d_last_error(const lbm3d_ctx* c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"

// ---------------------------------------------------------------------------
// Checkpointed forward run and discrete adjoint (lbm3d_forward_checkpointed,
// lbm3d_backward).
// ---------------------------------------------------------------------------
#include "lbm3d_adjoint_kernels.hpp"

namespace {

struct AdjLayout3 {
  size_t state = 0;
  int nck = 0;
  size_t off_ck = 0, off_replay = 0, off_lam = 0, off_grad = 0, off_pend = 0, total = 0;
};

AdjLayout3 adj_layout3(const lbm3d_ctx* c, int64_t nsteps, int32_t every) {
  AdjLayout3 A;
  A.state = c->L.state;
  A.nck = int((nsteps + every - 1) / every);
  size_t o = 0;
  A.off_ck = o;
  o += size_t(A.nck) * A.state;
  A.off_replay = o;
  o += size_t(every) * A.state;
  A.off_lam = o;
  o += 2 * A.state;
  A.off_grad = o;
  o += align3(size_t(3) * c->L.plane * c->L.esize);
  A.off_pend = o;  // two buffers of boundary shares (written by one step, added by the next)
  o += 2 * align3(size_t(kPendVals) * c->g.ny * c->g.nz * c->L.esize);
  A.total = o;
  return A;
}

// One reverse step: interior pass on the context stream and, for an open
// channel, the boundary pass on the second stream at the same time (both
// wait for what precedes on the context stream); the context stream then
// waits for the boundary pass, whose shares pend_out the next step adds.
template <typename R, bool SEED>
lbm_status reverse_step3(lbm3d_ctx* c, const R* S, const R* lam_in, R* lam_out, R* grad, const R* pend_in,
                         R* pend_out, R w) {
  const Mat3Ptrs<R> m = mat3_ptrs<R>(c);
  const Consts3<R>& k = consts3<R>(c);
  const bool open = !(c->g.flags & LBM_PERIODIC_X);
  const int nrows = c->g.ny * c->g.nz;
  if (open) {
    if (hipEventRecord(c->ev_in, c->stream) != hipSuccess || hipStreamWaitEvent(c->aux, c->ev_in, 0) != hipSuccess)
      return fail3(c, LBM_ERR_DEVICE, "boundary pass ordering failed");
    hipLaunchKernelGGL((k3_adj_bnd<R, SEED>), dim3(unsigned((2 * nrows + 63) / 64)), dim3(64), 0, c->aux, S, lam_in,
                       grad, pend_in, pend_out, m.phi, m.invk, m.d, k, w);
    if (hipEventRecord(c->ev_bnd, c->aux) != hipSuccess) return fail3(c, LBM_ERR_DEVICE, "boundary pass event failed");
  }
  hipLaunchKernelGGL((k3_adj_step<R, SEED>), dim3(unsigned(c->L.nblocks_obs)), dim3(kBlock3), 0, c->stream, S, lam_in,
                     lam_out, grad, open ? pend_in : nullptr, m.phi, m.invk, m.d, k, w);
  if (open && hipStreamWaitEvent(c->stream, c->ev_bnd, 0) != hipSuccess)
    return fail3(c, LBM_ERR_DEVICE, "boundary pass join failed");
  return LBM_OK;
}

template <typename R>
lbm_status backward3_t(lbm3d_ctx* c, double dJ, void* g_invk, void* g_phi, void* g_d) {
  const AdjLayout3 A = adj_layout3(c, c->adj_nsteps, c->adj_every);
  char* ws = c->adj_ws;
  const Mat3Ptrs<R> m = mat3_ptrs<R>(c);
  const Consts3<R> k = consts3<R>(c);
  const dim3 grid(unsigned(c->L.nblocks_obs));
  R* grad = reinterpret_cast<R*>(ws + A.off_grad);
  const bool open = !(c->g.flags & LBM_PERIODIC_X);
  const int64_t npend = int64_t(kPendVals) * c->g.ny * c->g.nz;
  R* pend[2] = {reinterpret_cast<R*>(ws + A.off_pend),
                reinterpret_cast<R*>(ws + A.off_pend + align3(size_t(npend) * c->L.esize))};
  R* lam[2] = {reinterpret_cast<R*>(ws + A.off_lam), reinterpret_cast<R*>(ws + A.off_lam + A.state)};
  if (!c->aux) {
    if (hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) != hipSuccess) {
      c->aux = nullptr;
      return fail3(c, LBM_ERR_DEVICE, "second stream creation failed");
    }
    if (hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_bnd, hipEventDisableTiming) != hipSuccess)
      return fail3(c, LBM_ERR_DEVICE, "event creation failed");
  }
  const int64_t ngrad = int64_t(3) * c->L.plane;
  hipLaunchKernelGGL(k3_fill<R>, dim3(unsigned((ngrad + kBlock3 - 1) / kBlock3)), dim3(kBlock3), 0, c->stream, grad,
                     ngrad, R(0));
  if (open)  // shares never written (rows without an inlet, ...) stay zero
    for (R* b : pend)
      hipLaunchKernelGGL(k3_fill<R>, dim3(unsigned((npend + kBlock3 - 1) / kBlock3)), dim3(kBlock3), 0, c->stream, b,
                         npend, R(0));
  // Seed: adjoint of J = mean over (x, y) of sum_CL 4 F C_ref s_c / dt * dx.
  const lbm_params& p = c->p;
  const double w = dJ * c->d.dx / (double(c->g.nx) * c->g.ny) * 4.0 * p.faraday * p.C_ref / c->d.dt;
  if (lbm_status st = reverse_step3<R, true>(c, static_cast<const R*>(c->state(c->cur)), nullptr, lam[0], grad,
                                             nullptr, pend[0], R(w));
      st != LBM_OK)
    return st;
  int cur = 0, pc = 0;  // pend[pc]: the shares the next reverse step adds
  for (int seg = A.nck - 1; seg >= 0; --seg) {
    const int64_t start = int64_t(seg) * c->adj_every;
    const int len = int(std::min<int64_t>(c->adj_every, c->adj_nsteps - start));
    char* replay = ws + A.off_replay;
    if (hipMemcpyAsync(replay, ws + A.off_ck + size_t(seg) * A.state, A.state, hipMemcpyDeviceToDevice,
                       c->stream) != hipSuccess)
      return fail3(c, LBM_ERR_DEVICE, "replay restore failed");
    for (int j = 1; j < len; ++j)
      hipLaunchKernelGGL((k3_step<R, MAT_FULL>), grid, dim3(kBlock3), 0, c->stream,
                         reinterpret_cast<const R*>(replay + size_t(j - 1) * A.state),
                         reinterpret_cast<R*>(replay + size_t(j) * A.state), m.phi, m.invk, m.d, k);
    for (int j = len - 1; j >= 0; --j) {
      if (lbm_status st = reverse_step3<R, false>(c, reinterpret_cast<const R*>(replay + size_t(j) * A.state),
                                                  lam[cur], lam[cur ^ 1], grad, pend[pc], pend[pc ^ 1], R(0));
          st != LBM_OK)
        return st;
      cur ^= 1;
      pc ^= 1;
    }
  }
  if (open)  // the last reverse step's boundary shares
    hipLaunchKernelGGL(k3_adj_apply<R>, dim3(unsigned((34 * int64_t(c->g.ny) * c->g.nz + kBlock3 - 1) / kBlock3)),
                       dim3(kBlock3), 0, c->stream, pend[pc], lam[cur], grad, k);
  hipLaunchKernelGGL(k3_adj_init<R>, c->grid3(), dim3(kBlock3), 0, c->stream, lam[cur], grad, k);
  void* outs[3] = {g_phi, g_invk, g_d};
  for (int i = 0; i < 3; ++i)
    if (outs[i])
      hipLaunchKernelGGL(k3_unpitch<R>, c->grid3(), dim3(kBlock3), 0, c->stream, grad + size_t(i) * c->L.plane,
                         static_cast<R*>(outs[i]), c->g.nx, c->g.ny, c->L.pitch);
  if (lbm_status s = check3(c, "backward"); s != LBM_OK) return s;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return fail3(c, LBM_ERR_DEVICE, "backward sync failed");
  return LBM_OK;
}

}  // namespace

extern "C" {

size_t lbm3d_adjoint_workspace_bytes(const lbm3d_ctx* c, int64_t nsteps, int32_t every) {
  if (!c || nsteps < 1 || every < 1) return 0;
  return adj_layout3(c, nsteps, every).total;
}

lbm_status lbm3d_forward_checkpointed(lbm3d_ctx* c, int64_t nsteps, int32_t every, void* dev_ws, size_t ws_bytes,
                                      double* J_out) {
  const lbm::TraceRange range("lbm3d_forward_checkpointed");
  if (!c || nsteps < 1 || every < 1 || !dev_ws) return LBM_ERR_INVALID_ARG;
  if (!c->params_set) return fail3(c, LBM_ERR_STATE, "lbm3d_set_params first");
  if (c->mat != MAT_FULL)
    return fail3(c, LBM_ERR_STATE, "the adjoint needs the three per-cell fields (independent_fields or all arrays)");
  const AdjLayout3 A = adj_layout3(c, nsteps, every);
  if (ws_bytes < A.total || reinterpret_cast<uintptr_t>(dev_ws) % kAlign3 != 0)
    return fail3(c, LBM_ERR_INVALID_ARG, "adjoint workspace too small or misaligned");
  c->adj_ready = false;
  if (lbm_status s = lbm3d_init_equilibrium(c); s != LBM_OK) return s;
  c->adj_ws = static_cast<char*>(dev_ws);
  c->adj_nsteps = nsteps;
  c->adj_every = every;
  const size_t sb = size_t(33) * c->L.plane * c->L.esize;
  for (int seg = 0; seg < A.nck; ++seg) {
    if (hipMemcpyAsync(c->adj_ws + A.off_ck + size_t(seg) * A.state, c->state(c->cur), sb, hipMemcpyDeviceToDevice,
                       c->stream) != hipSuccess)
      return fail3(c, LBM_ERR_DEVICE, "checkpoint copy failed");
    const int64_t n = std::min<int64_t>(every, nsteps - int64_t(seg) * every);
    if (lbm_status s = lbm3d_step(c, n); s != LBM_OK) return s;
  }
  lbm_obs o{};
  if (lbm_status s = lbm3d_observables(c, &o); s != LBM_OK) return s;
  if (J_out) *J_out = o.current_density;
  c->adj_step = c->step;
  c->adj_ready = true;
  return LBM_OK;
}

lbm_status lbm3d_backward(lbm3d_ctx* c, double dJ, void* grad_inv_k, void* grad_phi, void* grad_d_eff) {
  const lbm::TraceRange range("lbm3d_backward");
  if (!c) return LBM_ERR_INVALID_ARG;
  if (!c->adj_ready || c->adj_step != c->step)
    return fail3(c, LBM_ERR_STATE, "lbm3d_backward needs a preceding lbm3d_forward_checkpointed on the same state");
  return c->g.precision == 64 ? backward3_t<double>(c, dJ, grad_inv_k, grad_phi, grad_d_eff)
                              : backward3_t<float>(c, dJ, grad_inv_k, grad_phi, grad_d_eff);
}

}  // extern "C"
