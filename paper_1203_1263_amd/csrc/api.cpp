// C ABI of libnlse (declared in include/nlse.h): argument validation,
// workspace carving, stage sequencing and the tile autotuner.  All device
// work is enqueued on the caller's HIP stream.
#include "nlse.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "nlse_internal.h"

// ---------------------------------------------------------------- errors

static thread_local char g_last_error[512] = "";

int nlse_fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
  va_end(ap);
  return code;
}

int nlse_hip_fail(hipError_t e, const char* what) {
  return nlse_fail(NLSE_EDEVICE, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

#define fail nlse_fail
#define hip_fail nlse_hip_fail

extern "C" const char* nlse_last_error(void) { return g_last_error; }

extern "C" const char* nlse_strerror(int status) {
  switch (status) {
    case NLSE_OK: return "success";
    case NLSE_EINVAL: return "invalid argument";
    case NLSE_ENOMEM: return "out of memory or workspace too small";
    case NLSE_EDEVICE: return "HIP runtime error";
    case NLSE_EUNSTABLE: return "non-finite mass or energy (unstable run)";
    case NLSE_EUNSUPPORTED: return "unsupported combination";
    default: return "unknown status";
  }
}

// ---------------------------------------------------------------- shapes

struct Shape {
  int ndim;
  int64_t n[3];
  int64_t npts;
};

static int check_shape(int ndim, const int64_t dims[3], Shape* s) {
  if (ndim < 1 || ndim > 3) return fail(NLSE_EINVAL, "ndim must be 1, 2 or 3 (got %d)", ndim);
  if (!dims) return fail(NLSE_EINVAL, "dims is NULL");
  s->ndim = ndim;
  s->npts = 1;
  for (int d = 0; d < 3; ++d) {
    int64_t n = dims[d];
    if (d < ndim) {
      if (n < 3) return fail(NLSE_EINVAL, "extent %d is %lld; every active extent must be >= 3", d, (long long)n);
      if (n > (int64_t)1 << 30) return fail(NLSE_EINVAL, "extent %d is too large", d);
    } else if (n != 1) {
      return fail(NLSE_EINVAL, "extent %d must be 1 for a %dD grid", d, ndim);
    }
    s->n[d] = n;
    s->npts *= n;
  }
  if (s->n[0] * s->n[1] > ((int64_t)1 << 31) - 1)
    return fail(NLSE_EINVAL, "a single plane must hold fewer than 2^31 points");
  return NLSE_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Non-temporal own-point accesses pay off once a stage's fields (four
// field-sized arrays) no longer fit the 256 MB last-level cache; on smaller
// grids the next stage finds its input there.  1D grids never get here.
static bool use_streaming(const Shape& s, int dtype) {
  const double field = (double)s.npts * (dtype == NLSE_F32 ? 8.0 : 16.0);
  return s.ndim >= 2 && 4.0 * field > 256.0 * (1 << 20);
}

struct Layout {
  size_t acc, bufA, bufB, lo, partials, out, zero, total;
};

static Layout layout_for(const Shape& s, int dtype, unsigned flags) {
  const size_t esz = dtype == NLSE_F32 ? 8 : 16;
  const size_t field = align256((size_t)s.npts * esz);
  Layout L;
  size_t off = 0;
  L.acc = off;
  off += field;
  L.bufA = off;
  off += field;
  L.bufB = off;
  off += field;
  L.lo = off;
  if (flags & NLSE_COMPENSATED) off += field;
  L.partials = off;
  off += align256((size_t)nlse::reduce_blocks(s.npts) * 3 * sizeof(double));
  L.out = off;
  off += 256;
  L.zero = off;  // 256 zero bytes: stands in for V when there is no potential
  off += 256;
  L.total = off;
  return L;
}

// ---------------------------------------------------------------- grid

// Replayable step sequences: one HIP graph per (order, bc, dt, tile, steps).
struct GraphKey {
  int order, bc, steps;
  uint64_t dt_bits;
  int tile[3];
  bool operator<(const GraphKey& o) const {
    return std::tie(order, bc, steps, dt_bits, tile[0], tile[1], tile[2]) <
           std::tie(o.order, o.bc, o.steps, o.dt_bits, o.tile[0], o.tile[1], o.tile[2]);
  }
};

struct nlse_grid {
  Shape shape;
  int dtype;
  unsigned flags;
  double h, a, s;
  void* psi;
  char* work;
  size_t work_bytes;
  Layout lay;
  hipStream_t stream;
  const void* V;
  int tile[2][3];  // [0] CD2, [1] 2SHOC
  // 2D grids without NLSE_FUSED_PAIRS: stage pairs chosen by nlse_autotune
  // because they timed faster (per order slot, on a pair tile only)
  bool auto_pairs[2] = {false, false};
  hipStream_t cap = nullptr;  // private stream used only for graph capture
  std::map<GraphKey, hipGraphExec_t> graphs;
  hipStream_t copy = nullptr;  // frames: device-to-host copies
  hipEvent_t snap[2] = {nullptr, nullptr}, copied[2] = {nullptr, nullptr};
};

static void drop_graphs(nlse_grid* g) {
  for (auto& kv : g->graphs) (void)hipGraphExecDestroy(kv.second);
  g->graphs.clear();
}

// Read-only view of a grid for the other C-ABI translation units.
void nlse_grid_view(const nlse_grid* g, int* ndim, int64_t n[3], int* dtype, unsigned* flags, double* h,
                    void** psi, void** stream) {
  *ndim = g->shape.ndim;
  for (int d = 0; d < 3; ++d) n[d] = g->shape.n[d];
  *dtype = g->dtype;
  *flags = g->flags;
  *h = g->h;
  *psi = g->psi;
  *stream = g->stream;
}

extern "C" double nlse_dt_max(int ndim, int order, double h, double a) {
  if (ndim < 1 || ndim > 3 || (order != 2 && order != 4) || !(h > 0) || !(a > 0) || !std::isfinite(h) ||
      !std::isfinite(a))
    return -1.0;
  double k = h * h / ((double)ndim * std::sqrt(2.0) * a);
  return order == 4 ? 0.75 * k : k;
}

extern "C" int nlse_workspace_bytes(int ndim, const int64_t dims[3], int dtype, unsigned flags, size_t* bytes) {
  Shape s;
  int rc = check_shape(ndim, dims, &s);
  if (rc) return rc;
  if (dtype != NLSE_F32 && dtype != NLSE_F64) return fail(NLSE_EINVAL, "dtype must be NLSE_F32 or NLSE_F64");
  if (flags & ~(NLSE_COMPENSATED | NLSE_FUSED_PAIRS | NLSE_NO_GRAPH))
    return fail(NLSE_EINVAL, "unknown flag bits 0x%x", flags);
  if ((flags & NLSE_COMPENSATED) && dtype != NLSE_F32)
    return fail(NLSE_EUNSUPPORTED, "NLSE_COMPENSATED applies to FP32 grids only");
  if (!bytes) return fail(NLSE_EINVAL, "bytes is NULL");
  *bytes = layout_for(s, dtype, flags).total;
  return NLSE_OK;
}

// Default tile shapes (x-width, y-height, z-chunk) per dimension.
// A 3D FP32 2SHOC grid created with NLSE_FUSED_PAIRS runs each step as two
// fused launches (S1+S2, S3+S4) when its order-4 tile is 32x8.
static bool fused_eligible(const Shape& s, int dtype, unsigned flags, int order) {
  return s.ndim == 3 && dtype == NLSE_F32 && order == 4 && (flags & NLSE_FUSED_PAIRS);
}
// A 2D grid created with NLSE_FUSED_PAIRS runs each step as two stage-pair
// launches (every type, scheme and boundary condition) on the 64x16 tile if
// that is its tile, else on 32x32.
static bool pairs2d_eligible(const Shape& s, unsigned flags) { return s.ndim == 2 && (flags & NLSE_FUSED_PAIRS); }
static bool pair2d_tile(const int t[3]) { return (t[0] == 32 && t[1] == 32) || (t[0] == 64 && t[1] == 16); }

static void default_tile(const Shape& s, int dtype, unsigned flags, int order, int t[3]) {
  if (s.ndim == 1) {
    // grids that fit on chip run every step in one workgroup (tile 1024)
    t[0] = s.npts <= nlse_resident1d_max_points(dtype) ? 1024 : 256;
    t[1] = 1;
    t[2] = 1;
  } else if (s.ndim == 2) {
    t[0] = 64; t[1] = 4; t[2] = 1;
  } else {
    t[0] = 32; t[1] = 8;
    // z-chunk: each workgroup marches its planes one after another, so small
    // grids need short chunks (enough workgroups to hide the per-plane load
    // latency) and large ones long chunks (fewer re-read halo planes).
    // Aim at ~1024 workgroups with 1 <= cz <= 16 (measured best from 10^3 to
    // 256^3 points).
    const int64_t xy = ((s.n[0] + 31) / 32) * ((s.n[1] + 7) / 8);
    const int64_t nzi = s.n[2] - 2;
    int64_t cz = (nzi * xy + 1023) / 1024;
    if (cz < 1) cz = 1;
    if (cz > 16) cz = 16;
    // the fused kernels fill a 7-plane pipeline per chunk: longer chunks
    if (fused_eligible(s, dtype, flags, order)) cz = 32;
    if (cz > nzi) cz = nzi;
    t[2] = (int)cz;
  }
}

static int tile_slot(int order) { return order == 4 ? 1 : 0; }

// Whether steps of `order` on this grid with this tile run as stage pairs:
// always with NLSE_FUSED_PAIRS, else when the autotuner chose them.
static bool runs_pairs2d(const nlse_grid* g, int order, const int tile[3]) {
  if (g->shape.ndim != 2) return false;
  return (g->flags & NLSE_FUSED_PAIRS) || (g->auto_pairs[tile_slot(order)] && pair2d_tile(tile));
}

extern "C" int nlse_create_grid(nlse_grid** g, int ndim, const int64_t dims[3], double h, double a, double s,
                                int dtype, unsigned flags, void* psi_dev, void* work_dev, size_t work_bytes,
                                void* hip_stream) {
  if (!g) return fail(NLSE_EINVAL, "g is NULL");
  *g = nullptr;
  size_t need = 0;
  int rc = nlse_workspace_bytes(ndim, dims, dtype, flags, &need);
  if (rc) return rc;
  if (!(h > 0) || !std::isfinite(h)) return fail(NLSE_EINVAL, "h must be finite and > 0");
  if (!(a > 0) || !std::isfinite(a)) return fail(NLSE_EINVAL, "a must be finite and > 0");
  if (!std::isfinite(s)) return fail(NLSE_EINVAL, "s must be finite");
  if (!psi_dev) return fail(NLSE_EINVAL, "psi_dev is NULL");
  if (!work_dev) return fail(NLSE_EINVAL, "work_dev is NULL");
  if (((uintptr_t)psi_dev) % (dtype == NLSE_F32 ? 8 : 16))
    return fail(NLSE_EINVAL, "psi_dev is not aligned to one complex element");
  if (((uintptr_t)work_dev) % 256) return fail(NLSE_EINVAL, "work_dev must be 256-byte aligned");
  if (work_bytes < need)
    return fail(NLSE_ENOMEM, "workspace of %zu bytes is smaller than the %zu required", work_bytes, need);
  nlse_grid* G = new (std::nothrow) nlse_grid();
  if (!G) return fail(NLSE_ENOMEM, "host allocation failed");
  check_shape(ndim, dims, &G->shape);
  G->dtype = dtype;
  G->flags = flags;
  G->h = h;
  G->a = a;
  G->s = s;
  G->psi = psi_dev;
  G->work = static_cast<char*>(work_dev);
  G->work_bytes = work_bytes;
  G->lay = layout_for(G->shape, dtype, flags);
  G->stream = static_cast<hipStream_t>(hip_stream);
  G->V = nullptr;
  default_tile(G->shape, dtype, flags, 2, G->tile[0]);
  default_tile(G->shape, dtype, flags, 4, G->tile[1]);
  hipError_t e = nlse_launch_fill_zero(G->work + G->lay.zero, 256, G->stream);
  if (e == hipSuccess && (flags & NLSE_COMPENSATED))
    e = nlse_launch_fill_zero(G->work + G->lay.lo, (int64_t)G->shape.npts * 8, G->stream);
  if (e != hipSuccess) {
    delete G;
    return hip_fail(e, "clearing workspace");
  }
  *g = G;
  return NLSE_OK;
}

extern "C" int nlse_destroy_grid(nlse_grid* g) {
  if (!g) return fail(NLSE_EINVAL, "g is NULL");
  drop_graphs(g);
  if (g->cap) (void)hipStreamDestroy(g->cap);
  if (g->copy) (void)hipStreamDestroy(g->copy);
  for (int k = 0; k < 2; ++k) {
    if (g->snap[k]) (void)hipEventDestroy(g->snap[k]);
    if (g->copied[k]) (void)hipEventDestroy(g->copied[k]);
  }
  delete g;
  return NLSE_OK;
}

extern "C" int nlse_set_potential(nlse_grid* g, const void* V_dev) {
  if (!g) return fail(NLSE_EINVAL, "g is NULL");
  if (V_dev && ((uintptr_t)V_dev) % (g->dtype == NLSE_F32 ? 4 : 8))
    return fail(NLSE_EINVAL, "V_dev is misaligned");
  if (V_dev != g->V) drop_graphs(g);  // captured launches hold the old pointer
  g->V = V_dev;
  return NLSE_OK;
}

static int check_scheme(int order, int bc) {
  if (order != NLSE_CD2 && order != NLSE_2SHOC) return fail(NLSE_EINVAL, "order must be 2 (CD2) or 4 (2SHOC)");
  if (bc != NLSE_BC_DIRICHLET && bc != NLSE_BC_MSD && bc != NLSE_BC_L0)
    return fail(NLSE_EINVAL, "bc must be NLSE_BC_DIRICHLET, NLSE_BC_MSD or NLSE_BC_L0");
  return NLSE_OK;
}

// Enqueue one RK4 step (four stage launches) with the given tile.
// The grid-wide part of a stage launch.
static nlse::StageLaunch grid_launch(const nlse_grid* g, int order, int bc, const int tile[3]) {
  nlse::StageLaunch L;
  L.ndim = g->shape.ndim;
  L.dtype = g->dtype;
  L.order = order;
  L.bc = bc;
  for (int d = 0; d < 3; ++d) L.n[d] = g->shape.n[d];
  L.V = g->V;
  L.vzero = g->work + g->lay.zero;
  L.comp = (g->flags & NLSE_COMPENSATED) ? 1 : 0;
  L.stream = use_streaming(g->shape, g->dtype) ? 1 : 0;
  L.a = g->a;
  L.s = g->s;
  L.h = g->h;
  for (int d = 0; d < 3; ++d) L.tile[d] = tile[d];
  return L;
}

static hipError_t enqueue_step(const nlse_grid* g, int order, int bc, double dt, const int tile[3],
                               hipStream_t st) {
  nlse::StageLaunch L = grid_launch(g, order, bc, tile);
  void* psi = g->psi;
  void* acc = g->work + g->lay.acc;
  void* A = g->work + g->lay.bufA;
  void* B = g->work + g->lay.bufB;
  void* lo = L.comp ? g->work + g->lay.lo : nullptr;
  struct {
    const void* in;
    void* out;
    double ca, cn;
  } seq[4] = {{psi, A, dt / 6.0, dt / 2.0}, {A, B, dt / 3.0, dt / 2.0}, {B, A, dt / 3.0, dt}, {A, psi, dt / 6.0, 0.0}};
  for (int k = 0; k < 4; ++k) {
    L.stage = k + 1;
    L.uin = seq[k].in;
    L.uout = seq[k].out;
    L.psi = psi;
    L.acc = acc;
    L.lo = lo;
    L.c_acc = seq[k].ca;
    L.c_next = seq[k].cn;
    hipError_t e = nlse_launch_stage(L, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Enqueue nsteps RK4 steps on stream st (no host synchronisation).
static hipError_t enqueue_steps(const nlse_grid* g, int order, int bc, double dt, const int tile[3], int64_t nsteps,
                                hipStream_t st) {
  if (g->shape.ndim == 1 && tile[0] == 1024) {
    nlse::StageLaunch L = grid_launch(g, order, bc, tile);
    L.psi = g->psi;
    L.lo = L.comp ? g->work + g->lay.lo : nullptr;
    return nlse_launch_resident1d(L, nsteps, dt, st);
  }
  int64_t left = nsteps;
  if (runs_pairs2d(g, order, tile)) {
    // Pairs of steps Psi -> workspace -> Psi, as below; the first pass of
    // each step writes U2 to bufA
    nlse::StageLaunch L = grid_launch(g, order, bc, tile);
    if (!(tile[0] == 64 && tile[1] == 16)) {
      L.tile[0] = 32;
      L.tile[1] = 32;
    }
    void* acc = g->work + g->lay.acc;
    void* u2 = g->work + g->lay.bufA;
    void* alt = g->work + g->lay.bufB;
    void* lo = L.comp ? g->work + g->lay.lo : nullptr;
    for (; left >= 2; left -= 2) {
      hipError_t e = nlse_launch_pair2d(L, g->psi, alt, acc, u2, lo, dt, 1, st);
      if (e == hipSuccess) e = nlse_launch_pair2d(L, g->psi, alt, acc, u2, lo, dt, 2, st);
      if (e == hipSuccess) e = nlse_launch_pair2d(L, alt, g->psi, acc, u2, lo, dt, 1, st);
      if (e == hipSuccess) e = nlse_launch_pair2d(L, alt, g->psi, acc, u2, lo, dt, 2, st);
      if (e != hipSuccess) return e;
    }
  } else if (bc != NLSE_BC_L0 && fused_eligible(g->shape, g->dtype, g->flags, order) && tile[0] == 32 &&
             tile[1] == 8) {
    // Pairs of steps Psi -> workspace -> Psi (the fused launches cannot
    // update Psi in place); an odd last step takes the four-pass kernels,
    // which give the same bits.
    nlse::StageLaunch L = grid_launch(g, order, bc, tile);
    void* acc = g->work + g->lay.acc;
    void* mid = g->work + g->lay.bufA;
    void* alt = g->work + g->lay.bufB;
    void* lo = L.comp ? g->work + g->lay.lo : nullptr;
    for (; left >= 2; left -= 2) {
      hipError_t e = nlse_launch_fused3d(L, g->psi, alt, acc, mid, lo, dt, st);
      if (e == hipSuccess) e = nlse_launch_fused3d(L, alt, g->psi, acc, mid, lo, dt, st);
      if (e != hipSuccess) return e;
    }
  }
  for (; left > 0; --left) {
    hipError_t e = enqueue_step(g, order, bc, dt, tile, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

constexpr int kGraphSteps = 64;  // steps per captured graph
constexpr size_t kMaxGraphs = 32;

// The graph replaying `steps` steps with the grid's current settings,
// captured on first use.
static hipError_t step_graph(nlse_grid* g, int order, int bc, double dt, const int tile[3], int steps,
                             hipGraphExec_t* out) {
  GraphKey key;
  key.order = order;
  key.bc = bc;
  key.steps = steps;
  memcpy(&key.dt_bits, &dt, sizeof dt);
  for (int d = 0; d < 3; ++d) key.tile[d] = tile[d];
  auto found = g->graphs.find(key);
  if (found != g->graphs.end()) {
    *out = found->second;
    return hipSuccess;
  }
  if (g->graphs.size() >= kMaxGraphs) drop_graphs(g);
  hipError_t e = hipSuccess;
  if (!g->cap) e = hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking);
  if (e != hipSuccess) return e;
  hipGraph_t graph = nullptr;
  e = hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  hipError_t le = enqueue_steps(g, order, bc, dt, tile, steps, g->cap);
  e = hipStreamEndCapture(g->cap, &graph);
  if (le != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return le;
  }
  if (e != hipSuccess) return e;
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return e;
  g->graphs.emplace(key, exec);
  *out = exec;
  return hipSuccess;
}

extern "C" int nlse_step_rk4(nlse_grid* g, int order, int bc, double dt, int64_t nsteps) {
  if (!g) return fail(NLSE_EINVAL, "g is NULL");
  int rc = check_scheme(order, bc);
  if (rc) return rc;
  if (!(dt > 0) || !std::isfinite(dt)) return fail(NLSE_EINVAL, "dt must be finite and > 0");
  if (nsteps < 0) return fail(NLSE_EINVAL, "nsteps must be >= 0");
  const int* tile = g->tile[tile_slot(order)];
  if (g->flags & NLSE_NO_GRAPH) {
    hipError_t e = enqueue_steps(g, order, bc, dt, tile, nsteps, g->stream);
    return e == hipSuccess ? NLSE_OK : hip_fail(e, "stage launch");
  }
  // chunks of kGraphSteps steps (and one shorter chunk), each a replayed graph
  for (int64_t left = nsteps; left > 0;) {
    const int k = (int)std::min<int64_t>(left, kGraphSteps);
    hipGraphExec_t exec = nullptr;
    hipError_t e = step_graph(g, order, bc, dt, tile, k, &exec);
    if (e != hipSuccess) return hip_fail(e, "capturing the step graph");
    e = hipGraphLaunch(exec, g->stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    left -= k;
  }
  return NLSE_OK;
}

constexpr size_t kZeroCopyFrameMax = 1u << 20;  // bytes per frame

// Frames: after each chunk, Psi is snapshotted on the grid's stream into one
// half of the staging buffer (a copy kernel), and the copy stream moves that
// snapshot to the host while the next chunk integrates.  The host orders the
// two streams itself: it enqueues chunk j+1 first, then waits for snapshot j
// and only then enqueues copy j, which has no stream dependency.  (A
// device-to-host copy made to wait on the other stream's event did not
// overlap the kernels: frames then cost the full copy time.)  A half is
// refilled only after the host has seen the copy that last read it finish.
extern "C" int nlse_run_frames(nlse_grid* g, int order, int bc, double dt, int64_t chunk, int64_t nframes,
                               void* frames_host, void* stage_dev, size_t stage_bytes) {
  if (!g) return fail(NLSE_EINVAL, "g is NULL");
  int rc = check_scheme(order, bc);
  if (rc) return rc;
  if (!(dt > 0) || !std::isfinite(dt)) return fail(NLSE_EINVAL, "dt must be finite and > 0");
  if (chunk < 1) return fail(NLSE_EINVAL, "chunk must be >= 1");
  if (nframes < 0) return fail(NLSE_EINVAL, "nframes must be >= 0");
  if (nframes == 0) return NLSE_OK;
  const size_t fb = (size_t)g->shape.npts * (g->dtype == NLSE_F32 ? 8 : 16);
  if (!frames_host) return fail(NLSE_EINVAL, "frames_host is NULL");
  if (!stage_dev) return fail(NLSE_EINVAL, "stage_dev is NULL");
  if ((uintptr_t)stage_dev % 16) return fail(NLSE_EINVAL, "stage_dev must be 16-byte aligned");
  if (stage_bytes < 2 * fb) return fail(NLSE_ENOMEM, "stage_bytes %zu < 2 * %zu", stage_bytes, fb);
  hipError_t e = hipSuccess;
  if (!g->copy) e = hipStreamCreateWithFlags(&g->copy, hipStreamNonBlocking);
  for (int k = 0; k < 2 && e == hipSuccess; ++k) {
    if (!g->snap[k]) e = hipEventCreateWithFlags(&g->snap[k], hipEventDisableTiming);
    if (e == hipSuccess && !g->copied[k]) e = hipEventCreateWithFlags(&g->copied[k], hipEventDisableTiming);
  }
  if (e != hipSuccess) return hip_fail(e, "creating the copy stream / events");
  // Small frames into pinned memory the device can address: the copy kernel
  // writes each frame straight into host memory on the grid's stream (one
  // launch per frame, no second stream, no host waits).  Any other buffer
  // (pageable, or frames too large to copy without overlap) takes the
  // staged path below.
  if (fb <= kZeroCopyFrameMax) {
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, frames_host) == hipSuccess && at.type == hipMemoryTypeHost &&
        at.devicePointer) {
      char* dst = static_cast<char*>(at.devicePointer);
      for (int64_t j = 0; j < nframes; ++j) {
        rc = nlse_step_rk4(g, order, bc, dt, chunk);
        if (rc) break;
        e = nlse_launch_copy(dst + j * fb, g->psi, (int64_t)fb, g->stream);
        if (e != hipSuccess) break;
      }
      hipError_t se = hipStreamSynchronize(g->stream);
      if (rc) return rc;
      if (e == hipSuccess) e = se;
      return e == hipSuccess ? NLSE_OK : hip_fail(e, "frame copy");
    }
    (void)hipGetLastError();  // an unregistered pointer leaves an error behind
  }
  char* stage = static_cast<char*>(stage_dev);
  char* host = static_cast<char*>(frames_host);
  // frame j: wait until its snapshot is complete, then copy it out
  auto copy_out = [&](int64_t j) -> hipError_t {
    const int k = (int)(j & 1);
    hipError_t r = hipEventSynchronize(g->snap[k]);
    if (r == hipSuccess) r = hipMemcpyAsync(host + j * fb, stage + k * fb, fb, hipMemcpyDeviceToHost, g->copy);
    if (r == hipSuccess) r = hipEventRecord(g->copied[k], g->copy);
    return r;
  };
  // on an error, let copies already queued into the caller's buffer finish
  // before returning (the caller may free it)
  auto drain = [&]() { (void)hipStreamSynchronize(g->copy); };
  for (int64_t j = 0; j < nframes; ++j) {
    const int k = (int)(j & 1);
    rc = nlse_step_rk4(g, order, bc, dt, chunk);
    if (rc) {
      drain();
      return rc;
    }
    if (j >= 2) e = hipEventSynchronize(g->copied[k]);  // frame j-2 has left half k
    if (e == hipSuccess) e = nlse_launch_copy(stage + k * fb, g->psi, (int64_t)fb, g->stream);
    if (e == hipSuccess) e = hipEventRecord(g->snap[k], g->stream);
    if (e == hipSuccess && j >= 1) e = copy_out(j - 1);
    if (e != hipSuccess) {
      drain();
      return hip_fail(e, "frame copy");
    }
  }
  e = copy_out(nframes - 1);
  if (e == hipSuccess) e = hipStreamSynchronize(g->copy);
  else drain();
  if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
  return e == hipSuccess ? NLSE_OK : hip_fail(e, "frame synchronisation");
}

extern "C" int nlse_mass_energy(nlse_grid* g, int order, int bc, double* mass, double* energy) {
  if (!g) return fail(NLSE_EINVAL, "g is NULL");
  int rc = check_scheme(order, bc);
  if (rc) return rc;
  if (!mass || !energy) return fail(NLSE_EINVAL, "mass/energy pointers are NULL");
  nlse::ReduceLaunch R;
  R.ndim = g->shape.ndim;
  R.dtype = g->dtype;
  R.order = order;
  R.bc = bc;
  for (int d = 0; d < 3; ++d) R.n[d] = g->shape.n[d];
  R.psi = g->psi;
  R.V = g->V;
  R.a = g->a;
  R.s = g->s;
  R.h = g->h;
  R.partials = reinterpret_cast<double*>(g->work + g->lay.partials);
  R.out = reinterpret_cast<double*>(g->work + g->lay.out);
  // the stage buffers are idle between steps: bufA (and bufB after it, for
  // FP32) holds the FP64 D of the 2SHOC energy
  R.dscratch = g->work + g->lay.bufA;
  hipError_t e = nlse_launch_reduce(R, g->stream);
  if (e != hipSuccess) return hip_fail(e, "reduction launch");
  double host[3];
  e = hipMemcpyAsync(host, R.out, sizeof host, hipMemcpyDeviceToHost, g->stream);
  if (e != hipSuccess) return hip_fail(e, "copying the reduction result");
  e = hipStreamSynchronize(g->stream);
  if (e != hipSuccess) return hip_fail(e, "stream synchronize");
  const double hd = std::pow(g->h, (double)g->shape.ndim);
  *mass = hd * host[0];
  *energy = hd * (host[1] + host[2]);
  if (!std::isfinite(*mass) || !std::isfinite(*energy))
    return fail(NLSE_EUNSTABLE, "mass %g / energy %g is not finite", *mass, *energy);
  return NLSE_OK;
}

extern "C" int nlse_mass_energy_noalloc(int ndim, const int64_t dims[3], double h, double a, double s, int dtype,
                                        int order, int bc, const void* psi_dev, const void* V_dev, void* hip_stream,
                                        double* mass, double* energy) {
  Shape sh;
  int rc = check_shape(ndim, dims, &sh);
  if (rc) return rc;
  if (dtype != NLSE_F32 && dtype != NLSE_F64) return fail(NLSE_EINVAL, "dtype must be NLSE_F32 or NLSE_F64");
  rc = check_scheme(order, bc);
  if (rc) return rc;
  if (!(h > 0) || !std::isfinite(h)) return fail(NLSE_EINVAL, "h must be finite and > 0");
  if (!(a > 0) || !std::isfinite(a)) return fail(NLSE_EINVAL, "a must be finite and > 0");
  if (!std::isfinite(s)) return fail(NLSE_EINVAL, "s must be finite");
  if (!psi_dev) return fail(NLSE_EINVAL, "psi_dev is NULL");
  if (((uintptr_t)psi_dev) % (dtype == NLSE_F32 ? 8 : 16))
    return fail(NLSE_EINVAL, "psi_dev is not aligned to one complex element");
  if (V_dev && ((uintptr_t)V_dev) % (dtype == NLSE_F32 ? 4 : 8))
    return fail(NLSE_EINVAL, "V_dev is not aligned to one real element");
  if (!mass || !energy) return fail(NLSE_EINVAL, "mass/energy pointers are NULL");
  const int64_t max_pts = nlse::kStaticReduceBlocks * nlse::kReduceChunk;
  if (sh.npts > max_pts)
    return fail(NLSE_EINVAL, "grid of %lld points exceeds the %lld points the static scratch serves",
                (long long)sh.npts, (long long)max_pts);
  nlse::ReduceLaunch R;
  R.ndim = ndim;
  R.dtype = dtype;
  R.order = order;
  R.bc = bc;
  for (int d = 0; d < 3; ++d) R.n[d] = sh.n[d];
  R.psi = psi_dev;
  R.V = V_dev;
  R.a = a;
  R.s = s;
  R.h = h;
  R.dscratch = nullptr;  // 2SHOC: D recomputed where it is needed, nothing stored
  hipError_t e = nlse_static_reduce_scratch(&R.partials, &R.out);
  if (e != hipSuccess) return hip_fail(e, "looking up the static reduction scratch");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  e = nlse_launch_reduce(R, st);
  if (e != hipSuccess) return hip_fail(e, "reduction launch");
  double host[3];
  e = hipMemcpyAsync(host, R.out, sizeof host, hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return hip_fail(e, "copying the reduction result");
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "stream synchronize");
  const double hd = std::pow(h, (double)ndim);
  *mass = hd * host[0];
  *energy = hd * (host[1] + host[2]);
  if (!std::isfinite(*mass) || !std::isfinite(*energy))
    return fail(NLSE_EUNSTABLE, "mass %g / energy %g is not finite", *mass, *energy);
  return NLSE_OK;
}

extern "C" int nlse_get_state(nlse_grid* g, void* lo_dev) {
  if (!g) return fail(NLSE_EINVAL, "g is NULL");
  if (!(g->flags & NLSE_COMPENSATED)) return fail(NLSE_EINVAL, "grid has no compensation term");
  if (!lo_dev) return fail(NLSE_EINVAL, "lo_dev is NULL");
  hipError_t e = hipMemcpyAsync(lo_dev, g->work + g->lay.lo, (size_t)g->shape.npts * 8, hipMemcpyDeviceToDevice,
                                g->stream);
  return e == hipSuccess ? NLSE_OK : hip_fail(e, "copying the compensation term");
}

extern "C" int nlse_set_state(nlse_grid* g, const void* lo_dev) {
  if (!g) return fail(NLSE_EINVAL, "g is NULL");
  if (!(g->flags & NLSE_COMPENSATED)) return fail(NLSE_EINVAL, "grid has no compensation term");
  hipError_t e;
  if (!lo_dev)
    e = nlse_launch_fill_zero(g->work + g->lay.lo, (int64_t)g->shape.npts * 8, g->stream);
  else
    e = hipMemcpyAsync(g->work + g->lay.lo, lo_dev, (size_t)g->shape.npts * 8, hipMemcpyDeviceToDevice, g->stream);
  return e == hipSuccess ? NLSE_OK : hip_fail(e, "setting the compensation term");
}

// ---------------------------------------------------------------- tiles / autotuner

extern "C" int nlse_get_tile(const nlse_grid* g, int order, int tile[3]) {
  if (!g || !tile) return fail(NLSE_EINVAL, "NULL argument");
  if (order != 2 && order != 4) return fail(NLSE_EINVAL, "bad order");
  memcpy(tile, g->tile[tile_slot(order)], 3 * sizeof(int));
  return NLSE_OK;
}

// LDS bytes of the 3D stage kernel for a tile (must match stage.hip): a ring
// of stage-input planes with halo plus, for 2SHOC, three D planes.
static size_t lds_bytes_3d(int order, int dtype, int tx, int ty) {
  const size_t esz = dtype == NLSE_F32 ? 8 : 16;
  const int H = order == 4 ? 2 : 1;
  const int ns = order == 4 ? 6 : 4;
  size_t b = (size_t)ns * (tx + 2 * H) * (ty + 2 * H);
  if (order == 4) b += 3 * (size_t)(tx + 2) * (ty + 2);
  return b * esz;
}

static bool tile_fits(const nlse_grid* g, int order, const int t[3]) {
  if (!nlse_internal_tile_supported(g->shape.ndim, g->dtype, t)) return false;
  if (g->shape.ndim == 1 && t[0] == 1024 && g->shape.npts > nlse_resident1d_max_points(g->dtype)) return false;
  if (g->shape.ndim == 3) {
    if (t[2] > g->shape.n[2] - 2) return false;
    // keep each workgroup within 64 KiB of LDS so several fit on a CU
    if (lds_bytes_3d(order, g->dtype, t[0], t[1]) > 65536) return false;
  }
  return true;
}

extern "C" int nlse_set_tile(nlse_grid* g, int order, const int tile[3]) {
  if (!g || !tile) return fail(NLSE_EINVAL, "NULL argument");
  if (order != 2 && order != 4) return fail(NLSE_EINVAL, "bad order");
  if (!tile_fits(g, order, tile))
    return fail(NLSE_EUNSUPPORTED, "tile %dx%dx%d is not a compiled candidate for this grid", tile[0], tile[1],
                tile[2]);
  memcpy(g->tile[tile_slot(order)], tile, 3 * sizeof(int));
  if (g->auto_pairs[tile_slot(order)]) {  // a forced shape runs as four passes
    g->auto_pairs[tile_slot(order)] = false;
    drop_graphs(g);
  }
  return NLSE_OK;
}

static std::vector<std::array<int, 3>> candidates(const nlse_grid* g, int order) {
  std::vector<std::array<int, 3>> out;
  const Shape& s = g->shape;
  if (s.ndim == 1) {
    // the whole-grid kernel replaces four launches per step by none: when
    // it fits it is the only candidate (its runs would change the field)
    out.push_back({s.npts <= nlse_resident1d_max_points(g->dtype) ? 1024 : 256, 1, 1});
  } else if (s.ndim == 2 && pairs2d_eligible(s, g->flags)) {
    for (auto t : {std::array<int, 3>{32, 32, 1}, {64, 16, 1}}) out.push_back(t);
  } else if (s.ndim == 2) {
    for (auto t : {std::array<int, 3>{32, 8, 1}, {64, 4, 1}, {64, 8, 1}}) out.push_back(t);
  } else if (fused_eligible(s, g->dtype, g->flags, order)) {
    const int64_t nzi = s.n[2] - 2;
    for (int cz : {16, 32, 64, 128}) {
      std::array<int, 3> t = {32, 8, (int)std::min<int64_t>(cz, nzi)};
      bool dup = false;
      for (auto& o : out) dup |= (o == t);
      if (!dup) out.push_back(t);
    }
  } else {
    const int64_t nzi = s.n[2] - 2;
    for (auto xy : {std::array<int, 2>{32, 8}, {64, 4}, {64, 8}})
      for (int cz : {1, 2, 4, 8, 16, 32, 64}) {
        std::array<int, 3> t = {xy[0], xy[1], (int)std::min<int64_t>(cz, nzi)};
        bool dup = false;
        for (auto& o : out) dup |= (o == t);
        if (!dup) out.push_back(t);
      }
  }
  std::vector<std::array<int, 3>> ok;
  for (auto& t : out)
    if (tile_fits(g, order, t.data())) ok.push_back(t);
  return ok;
}

static std::string cache_key(const nlse_grid* g, int order, int bc) {
  char buf[160];
  snprintf(buf, sizeof buf, "d%d n%lldx%lldx%lld t%d o%d b%d c%d v%d p%d", g->shape.ndim, (long long)g->shape.n[0],
           (long long)g->shape.n[1], (long long)g->shape.n[2], g->dtype, order, bc,
           (g->flags & NLSE_COMPENSATED) ? 1 : 0, g->V ? 1 : 0, (g->flags & NLSE_FUSED_PAIRS) ? 1 : 0);
  return buf;
}

bool nlse_cache_lookup(const std::string& key, int* t, int n) {
  const char* path = getenv("NLSE_TUNE_CACHE");
  if (!path || !*path || n < 1 || n > 8) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char line[256];
  bool found = false;
  while (fgets(line, sizeof line, f)) {
    char* bar = strchr(line, '|');
    if (!bar) continue;
    *bar = 0;
    if (key != line) continue;
    int v[8], k = 0;
    const char* p = bar + 1;
    for (; k < n; ++k) {
      char* end = nullptr;
      const long x = strtol(p, &end, 10);
      if (end == p) break;
      v[k] = (int)x;
      p = end;
    }
    if (k == n) {
      for (int i = 0; i < n; ++i) t[i] = v[i];
      found = true;
    }
  }
  fclose(f);
  return found;
}

void nlse_cache_store(const std::string& key, const int* t, int n, float ms) {
  const char* path = getenv("NLSE_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s|", key.c_str());
  for (int i = 0; i < n; ++i) fprintf(f, "%d ", t[i]);
  fprintf(f, "%.6f\n", ms);
  fclose(f);
}

// Times stages 1-3 only (they read Psi but never write it), or the first
// fused pair (stages 1+2) of fused 3D and stage-pair 2D grids, so the field
// is left untouched; the accumulator and stage buffers are scratch.
extern "C" int nlse_autotune(nlse_grid* g, int order, int bc, double dt) {
  if (!g) return fail(NLSE_EINVAL, "g is NULL");
  int rc = check_scheme(order, bc);
  if (rc) return rc;
  if (!(dt > 0) || !std::isfinite(dt)) return fail(NLSE_EINVAL, "dt must be finite and > 0");
  const std::string key = cache_key(g, order, bc);
  const int slot = tile_slot(order);
  // 2D grids without NLSE_FUSED_PAIRS also choose between four passes and
  // stage pairs (the same bits either way)
  const bool choose_pairs = g->shape.ndim == 2 && !(g->flags & NLSE_FUSED_PAIRS);
  auto set_pairs = [&](bool on) {
    if (g->auto_pairs[slot] != on) drop_graphs(g);
    g->auto_pairs[slot] = on;
  };
  int cached[4];
  if (choose_pairs) {
    if (nlse_cache_lookup(key + " auto", cached, 4) && tile_fits(g, order, cached) &&
        (cached[3] == 0 || pair2d_tile(cached))) {
      memcpy(g->tile[slot], cached, 3 * sizeof(int));
      set_pairs(cached[3] != 0);
      return NLSE_OK;
    }
  } else if (nlse_cache_lookup(key, cached, 3) && tile_fits(g, order, cached)) {
    memcpy(g->tile[slot], cached, 3 * sizeof(int));
    return NLSE_OK;
  }
  auto cands = candidates(g, order);
  if (cands.empty()) return fail(NLSE_EUNSUPPORTED, "no tile candidate fits this grid");
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
  e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(e, "hipEventCreate");
  }
  nlse::StageLaunch L;
  L.ndim = g->shape.ndim;
  L.dtype = g->dtype;
  L.order = order;
  L.bc = bc;
  for (int d = 0; d < 3; ++d) L.n[d] = g->shape.n[d];
  L.V = g->V;
  L.vzero = g->work + g->lay.zero;
  L.comp = (g->flags & NLSE_COMPENSATED) ? 1 : 0;
  L.stream = use_streaming(g->shape, g->dtype) ? 1 : 0;
  L.a = g->a;
  L.s = g->s;
  L.h = g->h;
  L.psi = g->psi;
  L.acc = g->work + g->lay.acc;
  L.lo = L.comp ? g->work + g->lay.lo : nullptr;
  void* A = g->work + g->lay.bufA;
  void* B = g->work + g->lay.bufB;
  float best = 1e30f;
  std::array<int, 3> best_t = cands[0];
  const int reps = g->shape.npts > (1 << 20) ? 5 : 20;
  const bool fused = bc != NLSE_BC_L0 && fused_eligible(g->shape, g->dtype, g->flags, order);
  const bool pairs2d = pairs2d_eligible(g->shape, g->flags);
  for (auto& t : cands) {
    for (int d = 0; d < 3; ++d) L.tile[d] = t[d];
    auto run = [&](int n) -> hipError_t {
      if (pairs2d) {
        for (int r = 0; r < n; ++r) {
          hipError_t ee = nlse_launch_pair2d(L, g->psi, B, L.acc, A, nullptr, dt, 1, g->stream);
          if (ee != hipSuccess) return ee;
        }
        return hipSuccess;
      }
      if (fused) {
        for (int r = 0; r < n; ++r) {
          hipError_t ee = nlse_launch_fused3d_pair0(L, g->psi, L.acc, A, dt, g->stream);
          if (ee != hipSuccess) return ee;
        }
        return hipSuccess;
      }
      for (int r = 0; r < n; ++r)
        for (int k = 1; k <= 3; ++k) {
          L.stage = k;
          L.uin = k == 1 ? g->psi : (k == 2 ? A : B);
          L.uout = k == 2 ? B : A;
          L.c_acc = k == 1 ? dt / 6.0 : dt / 3.0;
          L.c_next = k == 3 ? dt : dt / 2.0;
          hipError_t ee = nlse_launch_stage(L, g->stream);
          if (ee != hipSuccess) return ee;
        }
      return hipSuccess;
    };
    if ((e = run(1)) != hipSuccess) break;  // warm-up
    (void)hipEventRecord(e0, g->stream);
    if ((e = run(reps)) != hipSuccess) break;
    (void)hipEventRecord(e1, g->stream);
    if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms < best) {
      best = ms;
      best_t = t;
    }
  }
  // Four passes or stage pairs: stages 1 and 2 at the best four-pass tile
  // against the first stage pair (stages 1 + 2 in one pass) on each pair
  // tile; both leave Psi untouched, and the second halves of a step compare
  // alike (stages 3 and 4 against the second pair).
  bool pick_pairs = false;
  if (e == hipSuccess && choose_pairs) {
    auto timed = [&](auto&& run, float* ms) -> hipError_t {
      hipError_t ee = run(1);  // warm-up
      if (ee != hipSuccess) return ee;
      (void)hipEventRecord(e0, g->stream);
      if ((ee = run(reps)) != hipSuccess) return ee;
      (void)hipEventRecord(e1, g->stream);
      if ((ee = hipEventSynchronize(e1)) != hipSuccess) return ee;
      return hipEventElapsedTime(ms, e0, e1);
    };
    float t4 = 0.f;
    for (int d = 0; d < 3; ++d) L.tile[d] = best_t[d];
    e = timed(
        [&](int n) -> hipError_t {
          for (int r = 0; r < n; ++r)
            for (int k = 1; k <= 2; ++k) {
              L.stage = k;
              L.uin = k == 1 ? g->psi : A;
              L.uout = k == 2 ? B : A;
              L.c_acc = k == 1 ? dt / 6.0 : dt / 3.0;
              L.c_next = dt / 2.0;
              hipError_t ee = nlse_launch_stage(L, g->stream);
              if (ee != hipSuccess) return ee;
            }
          return hipSuccess;
        },
        &t4);
    for (auto pt : {std::array<int, 3>{32, 32, 1}, {64, 16, 1}}) {
      if (e != hipSuccess || !tile_fits(g, order, pt.data())) continue;
      for (int d = 0; d < 3; ++d) L.tile[d] = pt[d];
      float tp = 0.f;
      e = timed(
          [&](int n) -> hipError_t {
            for (int r = 0; r < n; ++r) {
              hipError_t ee = nlse_launch_pair2d(L, g->psi, B, L.acc, A, nullptr, dt, 1, g->stream);
              if (ee != hipSuccess) return ee;
            }
            return hipSuccess;
          },
          &tp);
      if (e == hipSuccess && tp < t4) {
        t4 = tp;
        best_t = pt;
        pick_pairs = true;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(e, "autotune launch");
  memcpy(g->tile[slot], best_t.data(), 3 * sizeof(int));
  if (choose_pairs) {
    set_pairs(pick_pairs);
    const int rec[4] = {best_t[0], best_t[1], best_t[2], pick_pairs ? 1 : 0};
    nlse_cache_store(key + " auto", rec, 4, best / reps);
  } else {
    nlse_cache_store(key, best_t.data(), 3, best / reps);
  }
  return NLSE_OK;
}

extern "C" int nlse_get_stage_pairs(const nlse_grid* g, int order, int* on) {
  if (!g || !on) return fail(NLSE_EINVAL, "NULL argument");
  if (order != 2 && order != 4) return fail(NLSE_EINVAL, "bad order");
  const int* t = g->tile[tile_slot(order)];
  *on = (runs_pairs2d(g, order, t) ||
         (fused_eligible(g->shape, g->dtype, g->flags, order) && t[0] == 32 && t[1] == 8))
            ? 1
            : 0;
  return NLSE_OK;
}
