// Host-side checks of the C ABI, built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code (tests/test_host_sanitizers.py):
// every call that needs no GPU (defaults, status strings, geometry
// validation and workspace sizes over a seeded sweep of valid and invalid
// geometries, argument and parameter checks) and the error paths of the
// calls that do, with no device present.  Prints "host checks: ok" and
// exits 0 when every check holds.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>

#include "lbm_pem.h"

static int failures = 0;
#define CHECK(c)                                                              \
  do {                                                                        \
    if (!(c)) {                                                               \
      std::fprintf(stderr, "check failed, line %d: %s\n", __LINE__, #c);      \
      ++failures;                                                             \
    }                                                                         \
  } while (0)

// Address of a pretend device workspace: aligned, never dereferenced by the
// host code (only HIP calls would touch it, and they fail without a device).
static void* fake_ws() { return reinterpret_cast<void*>(uintptr_t(1) << 40); }

static lbm_geometry geom2d(int nx, int ny, int prec, uint32_t flags) {
  const int ch = ny / 2, cl = ny >= 20 ? ny / 20 : (ny >= 3 ? 1 : 0);
  return lbm_geometry{nx, ny, ch, ny - ch - cl, cl, prec, flags};
}

static void sweep_2d(std::mt19937_64& rng) {
  const int nxs[] = {-1, 0, 2, 3, 63, 64, 65, 200, 1000, 4096, 65536, 1 << 20};
  const int nys[] = {-3, 0, 1, 2, 3, 40, 1024, 65535, 65536};
  const int precs[] = {16, 32, 64};
  const uint32_t flag_sets[] = {0u, LBM_PERIODIC_X, LBM_PERIODIC_Y, LBM_THIN_CL, LBM_PRESSURE_INLET | LBM_BUOYANCY,
                                LBM_CELL_FIELDS, 2048u, 0xffffffffu};
  for (int nx : nxs)
    for (int ny : nys)
      for (int prec : precs)
        for (uint32_t f : flag_sets) {
          const lbm_geometry g = geom2d(nx, ny, prec, f);
          const size_t n = lbm_workspace_bytes(&g);
          if (n > 0) {
            const size_t pitch = size_t((nx + 63) / 64 * 64);
            CHECK(n >= 2 * 19 * pitch * size_t(ny) * size_t(prec / 8));
            CHECK(prec == 32 || prec == 64);
          }
        }
  // random layer splits, including ones that do not add up
  std::uniform_int_distribution<int> d(-2, 300);
  for (int t = 0; t < 2000; ++t) {
    lbm_geometry g{d(rng), d(rng), d(rng), d(rng), d(rng), (t & 1) ? 32 : 64, uint32_t(rng() & 0x7ff)};
    const size_t n = lbm_workspace_bytes(&g);
    if (n > 0) CHECK(g.ny_channel + g.ny_gdl + g.ny_cl == g.ny && g.nx >= 3);
  }
}

static void sweep_batch(std::mt19937_64& rng) {
  std::uniform_int_distribution<int> pick(0, 2), ncase(1, 12);
  const int nxs[] = {256, 512, 1024}, nys[] = {64, 128, 256};
  for (int t = 0; t < 300; ++t) {
    const int n = ncase(rng);
    lbm_geometry g[12];
    const uint32_t f = (t % 3 == 0) ? LBM_CELL_FIELDS : 0u;
    for (int i = 0; i < n; ++i) g[i] = geom2d(nxs[pick(rng)], nys[pick(rng)], (t % 5 == 0) ? 64 : 32, f);
    const size_t size = lbm_batch_workspace_bytes(g, n);
    CHECK(size > 0);
    if (f) {
      for (int i = 0; i < n; ++i) g[i].flags = 0;
      CHECK(lbm_batch_workspace_bytes(g, n) < size);
      if (n > 1) {
        g[n - 1].flags = LBM_CELL_FIELDS;  // mixed
        CHECK(lbm_batch_workspace_bytes(g, n) == 0);
      }
    }
    if (n > 1) {
      g[0].precision = g[0].precision == 32 ? 64 : 32;  // mixed precisions
      for (int i = 1; i < n; ++i) g[i].flags = g[0].flags;
      CHECK(lbm_batch_workspace_bytes(g, n) == 0);
    }
  }
  CHECK(lbm_batch_workspace_bytes(nullptr, 3) == 0);
  lbm_geometry one = geom2d(200, 40, 32, 0);
  CHECK(lbm_batch_workspace_bytes(&one, 0) == 0);
}

static void sweep_3d() {
  const int ns[] = {-1, 0, 1, 2, 3, 8, 64, 256, 65535, 65536};
  for (int nx : ns)
    for (int ny : ns)
      for (int nz : ns) {
        const int ch = nz / 2, cl = nz > 2 ? 1 : 0;
        lbm3d_geometry g{nx, ny, nz, ch, nz - ch - cl, cl, 32, 0};
        (void)lbm3d_workspace_bytes(&g);
      }
  lbm3d_geometry g{256, 128, 64, 32, 28, 4, 32, 0};
  CHECK(lbm3d_workspace_bytes(&g) > 0);
  CHECK(lbm3d_workspace_bytes(nullptr) == 0);
}

static void null_and_order_checks() {
  lbm_params p;
  lbm_default_params(&p);
  CHECK(p.tau_f > 0.5);
  for (int s = 0; s <= 6; ++s) CHECK(lbm_status_string(lbm_status(s)) != nullptr);
  CHECK(lbm_last_error(nullptr) != nullptr && lbm_batch_last_error(nullptr) != nullptr &&
        lbm3d_last_error(nullptr) != nullptr);
  lbm_obs o;
  CHECK(lbm_create(nullptr, fake_ws(), 1u << 30, nullptr, nullptr) == LBM_ERR_INVALID_ARG);
  CHECK(lbm_set_params(nullptr, &p, nullptr, nullptr, nullptr) == LBM_ERR_INVALID_ARG);
  CHECK(lbm_step(nullptr, 1) == LBM_ERR_INVALID_ARG);
  CHECK(lbm_observables(nullptr, &o, nullptr, nullptr, nullptr) == LBM_ERR_INVALID_ARG);
  CHECK(lbm_observables_noalloc(nullptr, &o, nullptr, nullptr, nullptr) == LBM_ERR_INVALID_ARG);
  CHECK(lbm_backward(nullptr, 1.0, nullptr, nullptr, nullptr) == LBM_ERR_INVALID_ARG);
  CHECK(lbm_step_count(nullptr) < 0);
  lbm_destroy(nullptr);
  CHECK(lbm_batch_step(nullptr, 1) == LBM_ERR_INVALID_ARG);
  CHECK(lbm_batch_set_fields(nullptr, 0, nullptr, nullptr, nullptr) == LBM_ERR_INVALID_ARG);
  CHECK(lbm_batch_set_barrier_timeout(nullptr, 1.0) == LBM_ERR_INVALID_ARG);
  lbm_batch_destroy(nullptr);
  CHECK(lbm3d_step(nullptr, 1) == LBM_ERR_INVALID_ARG);
  lbm3d_destroy(nullptr);

  // A context on a pretend workspace: creation only records it; every call
  // that needs parameters refuses, parameter validation runs on the host.
  const lbm_geometry g = geom2d(200, 40, 64, 0);
  const size_t need = lbm_workspace_bytes(&g);
  lbm_ctx* c = nullptr;
  CHECK(lbm_create(&g, fake_ws(), need - 1, nullptr, &c) == LBM_ERR_INVALID_ARG);
  CHECK(lbm_create(&g, reinterpret_cast<char*>(fake_ws()) + 8, need, nullptr, &c) == LBM_ERR_INVALID_ARG);
  CHECK(lbm_create(&g, fake_ws(), need, nullptr, &c) == LBM_OK && c != nullptr);
  if (c) {
    CHECK(lbm_step(c, 1) == LBM_ERR_STATE);
    CHECK(lbm_init_equilibrium(c) == LBM_ERR_STATE);
    CHECK(lbm_observables(c, &o, nullptr, nullptr, nullptr) == LBM_ERR_STATE);
    CHECK(lbm_backward(c, 1.0, nullptr, nullptr, nullptr) == LBM_ERR_STATE);
    CHECK(std::strlen(lbm_last_error(c)) > 0);
    lbm_params bad = p;
    bad.tau_f = 0.5;
    CHECK(lbm_set_params(c, &bad, nullptr, nullptr, nullptr) == LBM_ERR_UNSTABLE_PARAMS);
    bad = p;
    bad.phi_gdl = 1.5;
    CHECK(lbm_set_params(c, &bad, nullptr, nullptr, nullptr) == LBM_ERR_UNSTABLE_PARAMS);
    bad = p;
    bad.Re = 1e6;
    CHECK(lbm_set_params(c, &bad, nullptr, nullptr, nullptr) == LBM_ERR_UNSTABLE_PARAMS);
    CHECK(lbm_set_params(c, &p, nullptr, nullptr, nullptr) != LBM_OK);  // no device to finish on
    lbm_destroy(c);
  }
  // A batch on a pretend workspace: host validation of every case first.
  lbm_geometry bg[2] = {geom2d(256, 64, 32, 0), geom2d(512, 64, 32, 0)};
  lbm_params bp[2] = {p, p};
  bp[1].tau_f = 0.4;
  lbm_batch* b = nullptr;
  const size_t bneed = lbm_batch_workspace_bytes(bg, 2);
  CHECK(lbm_batch_create(bg, bp, 2, fake_ws(), bneed, nullptr, &b) == LBM_ERR_UNSTABLE_PARAMS);
  if (b) CHECK(std::strlen(lbm_batch_last_error(b)) > 0);
  lbm_batch_destroy(b);
}

int main() {
  std::mt19937_64 rng(21030144);
  sweep_2d(rng);
  sweep_batch(rng);
  sweep_3d();
  null_and_order_checks();
  if (failures) {
    std::fprintf(stderr, "host checks: %d failed\n", failures);
    return 1;
  }
  std::printf("host checks: ok\n");
  return 0;
}
