// Host-side driver for the sanitizer build of libnlse's C ABI (test
// infrastructure, runs without a GPU).  Every source of the library is
// compiled for the host only with AddressSanitizer and UndefinedBehavior-
// Sanitizer; this program drives the host logic that needs no device:
// argument validation of every entry point, workspace sizing, the batched
// integrator's schedule planner over random problem sets and every compiled
// tile, the barrier-limit hook and the no-allocation reduction's size check.
// Each call's status is checked; a sanitizer report aborts the program.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "nlse.h"

extern "C" int nlse_internal_batch_plan(int nsims, const nlse_sim_desc* sims, int W, int tx, int ty, int* chunk_out,
                                        int64_t chunk_len, int* item_out, int64_t item_len, int* ngroups);
extern "C" int nlse_internal_batch_limits(int64_t out[3]);
extern "C" int nlse_internal_tile_supported(int ndim, int dtype, const int tile[3]);

static int failures = 0;
#define EXPECT(cond)                                                      \
  do {                                                                    \
    if (!(cond)) {                                                        \
      std::fprintf(stderr, "line %d: %s (%s)\n", __LINE__, #cond, nlse_last_error()); \
      ++failures;                                                         \
    }                                                                     \
  } while (0)

static nlse_sim_desc desc(int64_t nx, int64_t ny, int order, int bc, int64_t poff, int64_t voff) {
  nlse_sim_desc d{};
  d.ndim = 2;
  d.dims[0] = nx;
  d.dims[1] = ny;
  d.dims[2] = 1;
  d.h = 0.25;
  d.a = 1.0;
  d.s = -1.0;
  d.dt = 0.01;
  d.order = order;
  d.bc = bc;
  d.psi_offset = poff;
  d.v_offset = voff;
  return d;
}

static void validation() {
  size_t bytes = 0;
  const int64_t ok3[3] = {64, 32, 16}, bad[3] = {2, 32, 16}, bad1[3] = {64, 1, 5};
  EXPECT(nlse_workspace_bytes(3, ok3, NLSE_F32, NLSE_COMPENSATED, &bytes) == NLSE_OK && bytes > 0);
  EXPECT(nlse_workspace_bytes(3, bad, NLSE_F32, 0, &bytes) == NLSE_EINVAL);
  EXPECT(nlse_workspace_bytes(2, bad1, NLSE_F32, 0, &bytes) == NLSE_EINVAL);
  EXPECT(nlse_workspace_bytes(0, ok3, NLSE_F32, 0, &bytes) == NLSE_EINVAL);
  EXPECT(nlse_workspace_bytes(3, nullptr, NLSE_F32, 0, &bytes) == NLSE_EINVAL);
  EXPECT(nlse_workspace_bytes(3, ok3, NLSE_F64, NLSE_COMPENSATED, &bytes) != NLSE_OK);
  nlse_grid* g = nullptr;
  EXPECT(nlse_create_grid(&g, 3, ok3, 0.1, 1.0, 1.0, NLSE_F32, 0, nullptr, nullptr, 0, nullptr) == NLSE_EINVAL);
  EXPECT(nlse_create_grid(&g, 3, ok3, -0.1, 1.0, 1.0, NLSE_F32, 0, (void*)0x1000, (void*)0x1000, bytes, nullptr) ==
         NLSE_EINVAL);
  EXPECT(nlse_create_grid(&g, 3, ok3, 0.1, 1.0, 1.0, NLSE_F32, 0, (void*)0x1000, (void*)0x1000, 16, nullptr) ==
         NLSE_ENOMEM);
  EXPECT(g == nullptr);
  EXPECT(nlse_step_rk4(nullptr, 4, NLSE_BC_MSD, 0.01, 1) == NLSE_EINVAL);
  EXPECT(nlse_mass_energy(nullptr, 2, 0, nullptr, nullptr) == NLSE_EINVAL);
  EXPECT(nlse_destroy_grid(nullptr) == NLSE_EINVAL);
  double m = 0, e = 0;
  const int64_t huge[3] = {1024, 1024, 257};
  EXPECT(nlse_mass_energy_noalloc(3, huge, 0.1, 1.0, 1.0, NLSE_F32, 2, 0, (void*)0x1000, nullptr, nullptr, &m, &e) ==
         NLSE_EINVAL);
  EXPECT(nlse_mass_energy_noalloc(3, ok3, 0.1, 1.0, 1.0, NLSE_F32, 3, 0, (void*)0x1000, nullptr, nullptr, &m, &e) ==
         NLSE_EINVAL);
  EXPECT(nlse_dt_max(3, 4, 0.1, 0.5) > 0 && nlse_dt_max(0, 4, 0.1, 0.5) < 0);
  for (int s = 1; s >= -6; --s) EXPECT(nlse_strerror(s) != nullptr);
  int tile[3] = {32, 8, 16};
  EXPECT(nlse_internal_tile_supported(3, 0, tile) == 1);
  tile[0] = 48;
  EXPECT(nlse_internal_tile_supported(3, 0, tile) == 0);
  // surrogate
  size_t sb = 0;
  EXPECT(nlse_surrogate_workspace_bytes(256, 256, 4, &sb) == NLSE_OK && sb > 0);
  EXPECT(nlse_surrogate_workspace_bytes(250, 256, 4, &sb) != NLSE_OK);
  EXPECT(nlse_surrogate_param_count() > 0);
  // batches: validation and pools, before any device call
  std::vector<nlse_sim_desc> d = {desc(64, 64, 4, NLSE_BC_MSD, 0, -1), desc(100, 37, 2, NLSE_BC_L0, 4096, 0)};
  EXPECT(nlse_batch_workspace_bytes(2, d.data(), NLSE_F32, NLSE_COMPENSATED, &bytes) == NLSE_OK);
  nlse_batch* b = nullptr;
  EXPECT(nlse_batch_create(&b, 2, d.data(), NLSE_F32, 0, (void*)0x1000, 100, nullptr, 0, (void*)0x1000, bytes,
                           nullptr) == NLSE_EINVAL);
  d[0].dims[0] = 2;
  EXPECT(nlse_batch_workspace_bytes(2, d.data(), NLSE_F32, 0, &bytes) == NLSE_EINVAL);
  EXPECT(nlse_batch_step_rk4(nullptr, -1) == NLSE_EINVAL);
  EXPECT(nlse_batch_set_config(nullptr, 32, 8, 3, 0) == NLSE_EINVAL);
}

static void planner() {
  std::mt19937_64 rng(7);
  const int sizes[] = {3, 5, 40, 64, 100, 128, 192, 256, 384, 512, 700};
  const int tiles[3][2] = {{32, 8}, {64, 4}, {64, 8}};
  for (int trial = 0; trial < 60; ++trial) {
    const int nsims = 1 + (int)(rng() % 300);
    std::vector<nlse_sim_desc> d;
    int64_t off = 0;
    for (int j = 0; j < nsims; ++j) {
      const int nx = sizes[rng() % 11], ny = sizes[rng() % 11];
      d.push_back(desc(nx, ny, rng() % 2 ? 4 : 2, (int)(rng() % 3), off, j % 3 ? -1 : off));
      off += (int64_t)nx * ny;
    }
    const int W = 1 + (int)(rng() % 2048);
    for (const auto& t : tiles) {
      int64_t items = 0;
      for (const auto& s : d) items += ((s.dims[0] + t[0] - 1) / t[0]) * ((s.dims[1] + t[1] - 1) / t[1]);
      std::vector<int> chunk(5 * (size_t)W + 1), it(3 * (size_t)items);
      int ng = -1;
      EXPECT(nlse_internal_batch_plan(nsims, d.data(), W, t[0], t[1], chunk.data(), (int64_t)chunk.size(), it.data(),
                                      (int64_t)it.size(), &ng) == NLSE_OK);
      EXPECT(chunk[0] == 0 && chunk[W] == (int)items && ng >= 0 && ng <= W);
      // too-short outputs are refused, not overrun
      if (items > 0)
        EXPECT(nlse_internal_batch_plan(nsims, d.data(), W, t[0], t[1], chunk.data(), (int64_t)chunk.size(),
                                        it.data(), (int64_t)it.size() - 1, &ng) == NLSE_ENOMEM);
    }
    EXPECT(nlse_internal_batch_plan(nsims, d.data(), W, 48, 8, nullptr, 0, nullptr, 0, nullptr) != NLSE_OK);
  }
  int64_t lim[3];
  EXPECT(nlse_internal_batch_limits(lim) == NLSE_OK && lim[0] > 0 && lim[1] > 0 && lim[2] == 64);
}

int main() {
  validation();
  planner();
  if (failures) {
    std::fprintf(stderr, "%d failed checks\n", failures);
    return 1;
  }
  std::printf("sanitized host checks passed\n");
  return 0;
}
