// Host-side parameter derivation shared by the single-lattice and batched APIs.
#pragma once

#include <algorithm>
#include <cmath>
#include <string>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "lbm_device.hpp"
#include "lbm_pem.h"

namespace lbm {

// A named range in profiler traces (roctx; rocprofv3 --marker-trace) over
// one library call, for the calls that launch the hot path's kernels.
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

constexpr double kMaxDiff = 0.14433756729740643;  // 1/(4 sqrt 3): b <= 1 keeps g0_eq >= 0

// Elements of one population plane: the pitched cells, plus 320 elements
// on planes of 2^20 cells or more, so that the stride between the planes a
// node reads at once is not a large power of two (4096x1024 FP32: 16 MiB +
// 1280 B).  With 16 MiB strides the 19 streams of a wavefront fall on the
// same HBM channels: measured on MI355X the 4096x1024 step takes 103.6 us
// unpadded and 100.1 us padded (99.97 with 64 elements, 100.3 with 1024),
// the 256x128x64 3D step 102.3 and 99.6 us, with identical results; the
// 1024x256 adjoint (2^18 cells per plane) is 2.7 % slower padded, so small
// planes stay unpadded.
constexpr int64_t kPlanePad = 320;
constexpr int64_t kPadMinCells = int64_t(1) << 20;
inline int64_t plane_elems(int64_t pitched_cells) {
  return pitched_cells >= kPadMinCells ? pitched_cells + kPlanePad : pitched_cells;
}

// Scalars derived from (geometry, params).
struct Derived {
  double nu = 0, dx = 0, dt = 0, u_avg = 0, invk_gdl = 0, d_gdl = 0, alpha_scale = 0, ln_k0 = 0;
  double inflow = 0;  // O2 advected in per step over the inlet rows
};

inline bool geometry_ok(const lbm_geometry* g) {
  if (!g) return false;
  if (g->nx < 3 || g->ny < 1 || g->ny > 65535) return false;  // rows map to gridDim.y
  if (g->ny_channel < 0 || g->ny_gdl < 0 || g->ny_cl < 0) return false;
  if (g->ny_channel + g->ny_gdl + g->ny_cl != g->ny) return false;
  if (g->precision != 32 && g->precision != 64) return false;
  if (g->flags & ~(LBM_PERIODIC_X | LBM_PERIODIC_Y | LBM_BODY_FORCE | LBM_NO_REACTION | LBM_PRESSURE_INLET |
                   LBM_THIN_CL | LBM_BUOYANCY | LBM_SIGMA_ENERGY | LBM_PHYSICAL_HEAT | LBM_CELL_FIELDS))
    return false;
  if ((g->flags & LBM_THIN_CL) && (g->ny_cl != 0 || g->ny_gdl < 1 || (g->flags & LBM_PERIODIC_Y)))
    return false;  // the film lies under the GDL, at a wall
  const int64_t pitch = (int64_t(g->nx) + 63) / 64 * 64;
  if (plane_elems(pitch * g->ny) * 19 >= (int64_t(1) << 31)) return false;  // 32-bit element offsets
  return true;
}

inline int pitch_of(int nx) { return (nx + 63) / 64 * 64; }

// Lattice thermal diffusivity of Eq. 19 at porosity phi.
inline double alpha_lat(const lbm_params& p, double phi, double alpha_scale) {
  const double rc = phi * p.rhocp_f + (1.0 - phi) * p.rhocp_s;
  return (p.k_f * phi + p.k_s * (1.0 - phi)) * alpha_scale / rc;
}

// Derive the lattice constants and check the scalar inputs (and, for the
// layered inputs, the porous-layer diffusivities).  Per-cell arrays are
// checked by the caller.
inline lbm_status derive(const lbm_geometry& g, const lbm_params& p, Derived& d, std::string& err) {
  if (p.dx_cm > 0) {
    d.dx = p.dx_cm;
  } else if (g.ny_gdl > 0 && p.gdl_thickness_cm > 0) {
    d.dx = p.gdl_thickness_cm / g.ny_gdl;
  } else {
    err = "lattice spacing undefined: give dx_cm or a GDL with gdl_thickness_cm";
    return LBM_ERR_INVALID_ARG;
  }
  if (!(p.D_O2_cm2s > 0) || !(p.tau_f > 0.5)) {
    err = "need tau_f > 0.5 and D_O2_cm2s > 0";
    return LBM_ERR_UNSTABLE_PARAMS;
  }
  if (!(p.D_f_lat > 0) || p.D_f_lat > kMaxDiff) {
    err = "D_f_lat outside (0, 1/(4 sqrt 3)]";
    return LBM_ERR_UNSTABLE_PARAMS;
  }
  if (!(p.phi_gdl > 0) || p.phi_gdl > 1) {
    err = "phi_gdl outside (0, 1]";
    return LBM_ERR_UNSTABLE_PARAMS;
  }
  if (p.Da_gdl < 0 || p.deff_ratio_gdl < 0 || p.dp_lat < 0) {
    err = "negative Da_gdl, deff_ratio_gdl or dp_lat";
    return LBM_ERR_INVALID_ARG;
  }
  if (!(p.T_in_K > 0) || !(p.rhocp_f > 0) || !(p.rhocp_s > 0) || !(p.C_ref > 0) || !(p.faraday > 0) ||
      !(p.R_gas > 0) || !(p.aj0_ref > 0) || !(p.T_arrh > 0)) {
    err = "non-positive temperature, heat capacity or reaction constant";
    return LBM_ERR_INVALID_ARG;
  }
  d.dt = p.D_f_lat * d.dx * d.dx / p.D_O2_cm2s;
  d.nu = (p.tau_f - 0.5) / 3.0;
  const bool pressure = g.flags & LBM_PRESSURE_INLET;
  d.u_avg = (g.ny_channel > 0 && !pressure) ? p.Re * d.nu / g.ny_channel : 0.0;
  if (!(g.flags & LBM_PERIODIC_X) && 1.5 * std::fabs(d.u_avg) > 0.1) {
    err = "inlet peak velocity above 0.1";
    return LBM_ERR_UNSTABLE_PARAMS;
  }
  if (p.kinetics != LBM_KINETICS_TAFEL && p.kinetics != LBM_KINETICS_BUTLER_VOLMER) {
    err = "kinetics must be LBM_KINETICS_TAFEL or LBM_KINETICS_BUTLER_VOLMER";
    return LBM_ERR_INVALID_ARG;
  }
  if (p.kinetics == LBM_KINETICS_BUTLER_VOLMER && !(p.alpha_a >= 0 && std::isfinite(p.alpha_a))) {
    err = "alpha_a must be finite and non-negative";
    return LBM_ERR_INVALID_ARG;
  }
  if (!std::isfinite(p.buoyancy_x) || !std::isfinite(p.buoyancy_y)) {
    err = "buoyancy is not finite";
    return LBM_ERR_INVALID_ARG;
  }
  if (!std::isfinite(p.thin_cl_cm)) {
    err = "thin_cl_cm is not finite";
    return LBM_ERR_INVALID_ARG;
  }
  if (!std::isfinite(p.p_outlet)) {
    err = "p_outlet is not finite";
    return LBM_ERR_INVALID_ARG;
  }
  if (pressure && !(g.flags & LBM_PERIODIC_X)) {
    // plane Poiseuille estimate of the channel's peak velocity
    const double H = g.ny_channel;
    const double umax = std::fabs(p.p_inlet - p.p_outlet) / (g.nx - 1) * H * H / (8.0 * d.nu);
    if (!std::isfinite(p.p_inlet) || umax > 0.1) {
      err = "inlet pressure drives a channel peak velocity above 0.1";
      return LBM_ERR_UNSTABLE_PARAMS;
    }
  }
  if (p.dp_lat > 0) {  // Kozeny-Carman (Eq. 7) at the layered porosity
    const double ph = p.phi_gdl, om = 1.0 - ph;
    d.invk_gdl = om * om / (0.0067 * ph * ph * ph * p.dp_lat * p.dp_lat);
  } else {  // Darcy number K / h^2, h = GDL thickness
    d.invk_gdl = (p.Da_gdl > 0 && g.ny_gdl > 0) ? 1.0 / (p.Da_gdl * double(g.ny_gdl) * g.ny_gdl) : 0.0;
  }
  d.d_gdl = p.deff_ratio_gdl > 0 ? p.deff_ratio_gdl * p.D_f_lat : std::pow(p.phi_gdl, 1.5) * p.D_f_lat;
  if (d.d_gdl > kMaxDiff) {
    err = "O2 diffusivity outside (0, 1/(4 sqrt 3)]";
    return LBM_ERR_UNSTABLE_PARAMS;
  }
  d.alpha_scale = d.dt / (d.dx * d.dx) / 100.0;
  const double a1 = alpha_lat(p, p.phi_gdl, d.alpha_scale), a2 = alpha_lat(p, 1.0, d.alpha_scale);
  if (std::max(a1, a2) > kMaxDiff || !(std::min(a1, a2) > 0)) {
    err = "thermal diffusivity outside (0, 1/(4 sqrt 3)]";
    return LBM_ERR_UNSTABLE_PARAMS;
  }
  d.ln_k0 = std::log(p.aj0_ref * d.dt / (4.0 * p.faraday * p.C_ref));
  d.inflow = 0;
  if (!(g.flags & LBM_PERIODIC_X) && g.ny_channel > 0) {
    const double coef = 6.0 * d.u_avg / (double(g.ny_channel) * g.ny_channel);
    for (int y = 0; y < g.ny_channel; ++y) {
      const double yc = y + 0.5;
      d.inflow += coef * yc * (g.ny_channel - yc) * p.c_in;
    }
  }
  return LBM_OK;
}

template <typename R>
void fill_consts(Consts<R>& k, const lbm_geometry& g, const lbm_params& p, const Derived& d, int pitch) {
  k.nx = g.nx;
  k.ny = g.ny;
  k.pitch = pitch;
  k.ny_ch = g.ny_channel;
  k.y_cl0 = g.ny_channel + g.ny_gdl;
  k.flags = g.flags;
  k.plane = int32_t(plane_elems(int64_t(pitch) * g.ny));
  k.bv = p.kinetics == LBM_KINETICS_BUTLER_VOLMER;
  const double se = 1.0 / p.tau_f;
  k.s_e = R(se);
  k.s_q = R(8.0 * (2.0 - se) / (8.0 - se));
  k.nu = R(d.nu);
  k.u_in_coef = g.ny_channel > 0 ? R(6.0 * d.u_avg / (double(g.ny_channel) * g.ny_channel)) : R(0);
  k.ax = R(p.body_force_x);
  k.ay = R(p.body_force_y);
  k.phi_gdl = R(p.phi_gdl);
  k.invk_gdl = R(d.invk_gdl);
  k.d_gdl = R(d.d_gdl);
  k.D_f = R(p.D_f_lat);
  k.kc_inv = p.dp_lat > 0 ? R(1.0 / (0.0067 * p.dp_lat * p.dp_lat)) : R(0);
  k.deff_ratio = R(p.deff_ratio_gdl);
  k.k_f = R(p.k_f);
  k.k_s = R(p.k_s);
  k.rhocp_f = R(p.rhocp_f);
  k.rhocp_s = R(p.rhocp_s);
  k.alpha_scale = R(d.alpha_scale);
  k.T_in = R(p.T_in_K);
  k.c_in = R(p.c_in);
  k.V_op = R(p.V_op);
  k.U0_slope = R(p.U0_slope);
  k.U0_icept = R(p.U0_icept);
  k.ln_k0 = R(d.ln_k0);
  k.E_over_R = R(p.E_over_R);
  k.inv_T_arrh = R(1.0 / p.T_arrh);
  k.aF_over_R = R(p.alpha_c * p.faraday / p.R_gas);
  k.four_f_cref = R(4.0 * p.faraday * p.C_ref);
  k.p_in = R(p.p_inlet);
  k.p_out = R(p.p_outlet);
  k.aFsum_over_R = R((p.alpha_a + p.alpha_c) * p.faraday / p.R_gas);
  k.ln_thin = R(std::log((p.thin_cl_cm > 0 ? p.thin_cl_cm : d.dx) / d.dx));
  k.bx = R(p.buoyancy_x);
  k.by = R(p.buoyancy_y);
}

}  // namespace lbm
