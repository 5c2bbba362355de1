// C ABI of the learned surrogate (declared in include/nlse.h): workspace
// carving, the layer sequence of forward and backward passes, Adam, batched
// mass checks and the block-advance loop with plain RK4 as the fallback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "api_common.h"
#include "nlse.h"
#include "nlse_internal.h"
#include "nlse_surrogate.h"

void nlse_grid_view(const nlse_grid* g, int* ndim, int64_t n[3], int* dtype, unsigned* flags, double* h,
                    void** psi, void** stream);

namespace {

struct Layer {
  int cin, cout, cinp, coutp;
  int kind;  // forward kernel kind
  size_t woff, boff;  // canonical offsets (floats) of W (cout, cin, 3, 3) and b (cout)
};

constexpr int kNL = 6;
constexpr int kChannels[kNL + 1] = {2, 48, 48, 48, 48, 48, 2};
constexpr int kWgradParts = 512;
constexpr int kLossParts = 1024;
constexpr int kMassChunks = 64;
constexpr int kBlockSteps = 16;  // RK4 steps one surrogate block stands for
// NLSE_SG_PATH_AUTO: the whole-network kernel while a batch has at most this
// many 16x16 tiles per CU (one workgroup per CU at a time)
constexpr int kFusedTilesPerCU = 2;

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

void layers(Layer L[kNL], int* nparams) {
  size_t off = 0;
  for (int l = 0; l < kNL; ++l) {
    L[l].cin = kChannels[l];
    L[l].cout = kChannels[l + 1];
    L[l].cinp = l == 0 ? 8 : kChannels[l];
    L[l].coutp = l == kNL - 1 ? 16 : kChannels[l + 1];
    L[l].kind = l == 0 ? kSgFirst : (l == kNL - 1 ? kSgLast : kSgHidden);
    L[l].woff = off;
    off += (size_t)L[l].cout * L[l].cin * 9;
    L[l].boff = off;
    off += (size_t)L[l].cout;
  }
  *nparams = (int)off;
}

struct SgLayout {
  size_t x8, act, pred, dz6, dzA, dzB, scratch, wf[kNL], wb[kNL], grad, m, v, wpart, lpart, mpart, mout, tmass,
      total;
};

SgLayout layout(int64_t P, int64_t fieldpts, int max_batch) {
  const int64_t tiles_per_field = fieldpts / 256;  // 16 x 16 pixel tiles
  Layer L[kNL];
  int np;
  layers(L, &np);
  SgLayout S;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += a256(bytes);
    return o;
  };
  S.x8 = take(P * 16);
  S.act = take(P * 96 * 5);
  S.pred = take(P * 8);
  S.dz6 = take(P * 32);
  S.dzA = take(P * 96);
  S.dzB = take(P * 96);
  S.scratch = take(fieldpts * 8);
  size_t maxpart = 0;
  for (int l = 0; l < kNL; ++l) {
    const size_t nw = (size_t)L[l].coutp * 9 * L[l].cinp;
    S.wf[l] = take(nw * 2);
    S.wb[l] = take(nw * 2);
    maxpart = std::max(maxpart, (size_t)L[l].coutp * (9 * L[l].cinp + 1));
  }
  S.grad = take((size_t)np * 4);
  S.m = take((size_t)np * 4);
  S.v = take((size_t)np * 4);
  S.wpart = take((size_t)kWgradParts * maxpart * 4);
  S.lpart = take((size_t)kLossParts * 8);
  S.mpart = take((size_t)max_batch * kMassChunks * 8);
  S.mout = take((size_t)max_batch * 8);
  S.tmass = take((size_t)max_batch * tiles_per_field * 8);
  S.total = off;
  return S;
}

int check_dims(int H, int W, int max_batch) {
  if (H < 16 || W < 16 || H % 16 || W % 16) return nlse_fail(NLSE_EINVAL, "H and W must be positive multiples of 16");
  if (max_batch < 1) return nlse_fail(NLSE_EINVAL, "max_batch must be >= 1");
  if ((int64_t)H * W * max_batch > ((int64_t)1 << 31) - 1) return nlse_fail(NLSE_EINVAL, "batch too large");
  return NLSE_OK;
}

}  // namespace

struct nlse_surrogate {
  int H, W, max_batch;
  double h;
  float* params;
  char* work;
  SgLayout lay;
  Layer L[kNL];
  int nparams;
  int64_t step;  // Adam step counter
  hipStream_t stream;
  // captured launch sequences: (input, output, batch, kind) -> graph; the
  // weights live at fixed workspace addresses, so a graph stays valid while
  // training updates them in place
  hipStream_t cap = nullptr;
  std::map<std::tuple<const void*, void*, int, int>, hipGraphExec_t> graphs;
  int path = NLSE_SG_PATH_AUTO;  // inference kernels
};

static void drop_graphs(nlse_surrogate* m) {
  for (auto& kv : m->graphs) (void)hipGraphExecDestroy(kv.second);
  m->graphs.clear();
}

// Replay the graph of `key`, capturing `enqueue` (which must enqueue on
// m->stream) the first time.  At most 16 graphs are kept.
template <typename F>
static hipError_t replay(nlse_surrogate* m, std::tuple<const void*, void*, int, int> key, F enqueue) {
  auto found = m->graphs.find(key);
  if (found == m->graphs.end()) {
    if (m->graphs.size() >= 16) drop_graphs(m);
    hipError_t e = hipSuccess;
    if (!m->cap) e = hipStreamCreateWithFlags(&m->cap, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    hipStream_t user = m->stream;
    m->stream = m->cap;
    hipGraph_t graph = nullptr;
    e = hipStreamBeginCapture(m->cap, hipStreamCaptureModeThreadLocal);
    hipError_t le = e == hipSuccess ? enqueue() : e;
    if (e == hipSuccess) e = hipStreamEndCapture(m->cap, &graph);
    m->stream = user;
    if (le != hipSuccess || e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return le != hipSuccess ? le : e;
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return e;
    found = m->graphs.emplace(key, exec).first;
  }
  return hipGraphLaunch(found->second, m->stream);
}

extern "C" int nlse_surrogate_param_count(void) {
  Layer L[kNL];
  int np;
  layers(L, &np);
  return np;
}

extern "C" int nlse_surrogate_workspace_bytes(int H, int W, int max_batch, size_t* bytes) {
  int rc = check_dims(H, W, max_batch);
  if (rc) return rc;
  if (!bytes) return nlse_fail(NLSE_EINVAL, "bytes is NULL");
  *bytes = layout((int64_t)H * W * max_batch, (int64_t)H * W, max_batch).total;
  return NLSE_OK;
}

static uint16_t* U16(nlse_surrogate* m, size_t off) { return reinterpret_cast<uint16_t*>(m->work + off); }
static float* F32(nlse_surrogate* m, size_t off) { return reinterpret_cast<float*>(m->work + off); }
static double* F64(nlse_surrogate* m, size_t off) { return reinterpret_cast<double*>(m->work + off); }
static uint16_t* act(nlse_surrogate* m, int k, int batch) {
  return U16(m, m->lay.act + (size_t)k * 96 * m->H * m->W * (size_t)batch);
}

static hipError_t refresh(nlse_surrogate* m) {
  for (int l = 0; l < kNL; ++l) {
    const Layer& L = m->L[l];
    hipError_t e = sg_prep_weights(m->params + L.woff, L.cout, L.cin, L.coutp, L.cinp, U16(m, m->lay.wf[l]),
                                   U16(m, m->lay.wb[l]), m->stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

extern "C" int nlse_surrogate_create(nlse_surrogate** out, int H, int W, int max_batch, double h, float* params_dev,
                                     void* work_dev, size_t work_bytes, void* hip_stream) {
  if (!out) return nlse_fail(NLSE_EINVAL, "m is NULL");
  *out = nullptr;
  int rc = check_dims(H, W, max_batch);
  if (rc) return rc;
  if (!(h > 0) || !std::isfinite(h)) return nlse_fail(NLSE_EINVAL, "h must be finite and > 0");
  if (!params_dev || ((uintptr_t)params_dev) % 4) return nlse_fail(NLSE_EINVAL, "params_dev is NULL or misaligned");
  if (!work_dev || ((uintptr_t)work_dev) % 256) return nlse_fail(NLSE_EINVAL, "work_dev must be 256-byte aligned");
  SgLayout S = layout((int64_t)H * W * max_batch, (int64_t)H * W, max_batch);
  if (work_bytes < S.total)
    return nlse_fail(NLSE_ENOMEM, "workspace of %zu bytes is smaller than the %zu required", work_bytes, S.total);
  nlse_surrogate* m = new (std::nothrow) nlse_surrogate();
  if (!m) return nlse_fail(NLSE_ENOMEM, "host allocation failed");
  m->H = H;
  m->W = W;
  m->max_batch = max_batch;
  m->h = h;
  m->params = params_dev;
  m->work = static_cast<char*>(work_dev);
  m->lay = S;
  layers(m->L, &m->nparams);
  m->step = 0;
  m->stream = static_cast<hipStream_t>(hip_stream);
  hipError_t e = refresh(m);
  if (e == hipSuccess) e = nlse_launch_fill_zero(m->work + S.m, (int64_t)m->nparams * 4, m->stream);
  if (e == hipSuccess) e = nlse_launch_fill_zero(m->work + S.v, (int64_t)m->nparams * 4, m->stream);
  if (e != hipSuccess) {
    delete m;
    return nlse_hip_fail(e, "initialising the surrogate");
  }
  *out = m;
  return NLSE_OK;
}

extern "C" int nlse_surrogate_refresh(nlse_surrogate* m) {
  if (!m) return nlse_fail(NLSE_EINVAL, "m is NULL");
  hipError_t e = refresh(m);
  if (e == hipSuccess) e = nlse_launch_fill_zero(m->work + m->lay.m, (int64_t)m->nparams * 4, m->stream);
  if (e == hipSuccess) e = nlse_launch_fill_zero(m->work + m->lay.v, (int64_t)m->nparams * 4, m->stream);
  m->step = 0;
  return e == hipSuccess ? NLSE_OK : nlse_hip_fail(e, "refreshing weights");
}

static int check_batch(nlse_surrogate* m, int batch) {
  if (!m) return nlse_fail(NLSE_EINVAL, "m is NULL");
  if (batch < 1 || batch > m->max_batch) return nlse_fail(NLSE_EINVAL, "batch must be in [1, max_batch]");
  return NLSE_OK;
}

// Compute units of the current device (queried once per process).
static int device_cus() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) ==
                                                 hipSuccess && n > 0)
      cus = n;
    else
      cus = 256;
  }
  return cus;
}

// Largest batch that NLSE_SG_PATH_AUTO sends through the whole-network kernel.
static int fused_max_batch(const nlse_surrogate* m) {
  const int tiles = (m->H / 16) * (m->W / 16);
  return std::max(1, (kFusedTilesPerCU * device_cus()) / tiles);
}

static bool use_fused(const nlse_surrogate* m, int batch) {
  return m->path == NLSE_SG_PATH_FUSED || (m->path == NLSE_SG_PATH_AUTO && batch <= fused_max_batch(m));
}

// Forward pass of `batch` fields.  With `checked`, the last layer also
// projects the boundary ring to the input's modulus (project) and sums
// |psi_out|^2 per tile, and the field masses go to the workspace (mout).
// Training passes (`infer` false) run layer by layer and leave every
// activation in the workspace for the backward pass; inference may take the
// whole-network kernel instead.
static hipError_t forward(nlse_surrogate* m, const void* psi_in, void* psi_out, int batch, bool checked = false,
                          bool project = false, bool infer = false) {
  if (infer && use_fused(m, batch)) {
    SgNet c;
    std::memset(&c, 0, sizeof c);
    c.x = psi_in;
    c.pred = psi_out;
    for (int l = 0; l < kNL; ++l) {
      c.w[l] = U16(m, m->lay.wf[l]);
      c.bias[l] = m->params + m->L[l].boff;
    }
    c.B = batch;
    c.H = m->H;
    c.W = m->W;
    c.project = checked && project ? 1 : 0;
    c.tile_mass = checked ? F64(m, m->lay.tmass) : nullptr;
    hipError_t e = sg_net_forward(c, m->stream);
    if (e == hipSuccess && checked)
      e = sg_tile_mass_final(F64(m, m->lay.tmass), batch, (m->H / 16) * (m->W / 16), m->h * m->h,
                             F64(m, m->lay.mout), m->stream);
    return e;
  }
  const int64_t P = (int64_t)batch * m->H * m->W;
  hipError_t e = sg_pack_input(psi_in, m->work + m->lay.x8, P, m->stream);
  for (int l = 0; l < kNL && e == hipSuccess; ++l) {
    SgConv c;
    std::memset(&c, 0, sizeof c);
    c.in = l == 0 ? U16(m, m->lay.x8) : act(m, l - 1, batch);
    c.w = U16(m, m->lay.wf[l]);
    c.bias = m->params + m->L[l].boff;
    c.out = l < kNL - 1 ? act(m, l, batch) : nullptr;
    c.x = psi_in;
    c.pred = psi_out;
    c.B = batch;
    c.H = m->H;
    c.W = m->W;
    if (l == kNL - 1 && checked) {
      c.project = project ? 1 : 0;
      c.tile_mass = F64(m, m->lay.tmass);
    }
    e = sg_conv(m->L[l].kind, c, m->stream);
  }
  if (e == hipSuccess && checked)
    e = sg_tile_mass_final(F64(m, m->lay.tmass), batch, (m->H / 16) * (m->W / 16), m->h * m->h, F64(m, m->lay.mout),
                           m->stream);
  return e;
}

extern "C" int nlse_surrogate_forward(nlse_surrogate* m, const void* psi_in, void* psi_out, int batch) {
  int rc = check_batch(m, batch);
  if (rc) return rc;
  if (!psi_in || !psi_out) return nlse_fail(NLSE_EINVAL, "NULL field");
  if (psi_in == psi_out) return nlse_fail(NLSE_EINVAL, "psi_in and psi_out must differ");
  // replayed graph: one launch instead of seven cuts the latency of a pass
  // that is waited for (batch 1: a surrogate block of forward, projection
  // and mass check 0.121 -> 0.114 ms), though back-to-back passes overlap
  // direct launches slightly better (0.069 vs 0.077 ms each)
  hipError_t e = replay(m, std::make_tuple(psi_in, psi_out, batch, 0),
                        [&]() { return forward(m, psi_in, psi_out, batch, false, false, true); });
  return e == hipSuccess ? NLSE_OK : nlse_hip_fail(e, "surrogate forward");
}

// Forward + backward into the workspace gradient (canonical layout).
static hipError_t loss_grad(nlse_surrogate* m, const void* psi_in, const void* tgt, int batch, float* grad) {
  const int64_t P = (int64_t)batch * m->H * m->W;
  void* pred = m->work + m->lay.pred;
  hipError_t e = forward(m, psi_in, pred, batch);
  if (e == hipSuccess) e = sg_loss(pred, tgt, U16(m, m->lay.dz6), F64(m, m->lay.lpart), kLossParts, P, m->stream);
  const uint16_t* dz = U16(m, m->lay.dz6);
  uint16_t* bufs[2] = {U16(m, m->lay.dzA), U16(m, m->lay.dzB)};
  const int ntiles = batch * (m->H / 8) * (m->W / 16);
  const int nparts = std::min(kWgradParts, ntiles);
  for (int l = kNL - 1; l >= 0 && e == hipSuccess; --l) {
    const Layer& L = m->L[l];
    const uint16_t* a_in = l == 0 ? U16(m, m->lay.x8) : act(m, l - 1, batch);
    e = sg_wgrad(L.kind, a_in, dz, F32(m, m->lay.wpart), nparts, batch, m->H, m->W, m->stream);
    if (e == hipSuccess)
      e = sg_wgrad_reduce(F32(m, m->lay.wpart), nparts, L.coutp, L.cinp, L.cout, L.cin, grad + L.woff,
                          grad + L.boff, m->stream);
    if (l == 0 || e != hipSuccess) break;
    SgConv c;
    std::memset(&c, 0, sizeof c);
    c.in = dz;
    c.w = U16(m, m->lay.wb[l]);
    c.out = bufs[l & 1];
    c.mask = act(m, l - 1, batch);
    c.B = batch;
    c.H = m->H;
    c.W = m->W;
    e = sg_conv(l == kNL - 1 ? kSgDgradLast : kSgDgradHidden, c, m->stream);
    dz = bufs[l & 1];
  }
  return e;
}

static int fetch_loss(nlse_surrogate* m, int batch, double* loss) {
  if (!loss) return NLSE_OK;
  std::vector<double> part(kLossParts);
  hipError_t e = hipMemcpyAsync(part.data(), m->work + m->lay.lpart, kLossParts * sizeof(double),
                                hipMemcpyDeviceToHost, m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) return nlse_hip_fail(e, "copying the loss");
  double s = 0.0;
  for (double v : part) s += v;
  *loss = s / (2.0 * (double)batch * m->H * m->W);
  return std::isfinite(*loss) ? NLSE_OK : nlse_fail(NLSE_EUNSTABLE, "non-finite loss");
}

extern "C" int nlse_surrogate_loss_grad(nlse_surrogate* m, const void* psi_in, const void* psi_target, int batch,
                                        float* grad_dev, double* loss) {
  int rc = check_batch(m, batch);
  if (rc) return rc;
  if (!psi_in || !psi_target) return nlse_fail(NLSE_EINVAL, "NULL field");
  float* grad = grad_dev ? grad_dev : F32(m, m->lay.grad);
  hipError_t e = loss_grad(m, psi_in, psi_target, batch, grad);
  if (e != hipSuccess) return nlse_hip_fail(e, "surrogate backward");
  return fetch_loss(m, batch, loss);
}

extern "C" int nlse_surrogate_train_step(nlse_surrogate* m, const void* psi_in, const void* psi_target, int batch,
                                         float lr, double* loss) {
  int rc = check_batch(m, batch);
  if (rc) return rc;
  if (!psi_in || !psi_target) return nlse_fail(NLSE_EINVAL, "NULL field");
  if (!(lr > 0) || !std::isfinite(lr)) return nlse_fail(NLSE_EINVAL, "lr must be finite and > 0");
  float* grad = F32(m, m->lay.grad);
  hipError_t e = loss_grad(m, psi_in, psi_target, batch, grad);
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  m->step += 1;
  const float c1 = (float)(1.0 - std::pow((double)b1, (double)m->step));
  const float c2 = (float)(1.0 - std::pow((double)b2, (double)m->step));
  if (e == hipSuccess)
    e = sg_adam(m->params, grad, F32(m, m->lay.m), F32(m, m->lay.v), m->nparams, lr, b1, b2, eps, c1, c2, m->stream);
  if (e == hipSuccess) e = refresh(m);
  if (e != hipSuccess) return nlse_hip_fail(e, "surrogate train step");
  return fetch_loss(m, batch, loss);
}

static int masses(nlse_surrogate* m, const void* psi, int batch, double* out_host) {
  hipError_t e = sg_field_mass(psi, batch, (int64_t)m->H * m->W, m->h * m->h, F64(m, m->lay.mpart), kMassChunks,
                               F64(m, m->lay.mout), m->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out_host, m->work + m->lay.mout, (size_t)batch * 8, hipMemcpyDeviceToHost, m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  return e == hipSuccess ? NLSE_OK : nlse_hip_fail(e, "field masses");
}

// The field masses a checked forward pass left in the workspace, to the host.
static int fetch_masses(nlse_surrogate* m, int batch, double* out_host) {
  hipError_t e = hipMemcpyAsync(out_host, m->work + m->lay.mout, (size_t)batch * 8, hipMemcpyDeviceToHost, m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  return e == hipSuccess ? NLSE_OK : nlse_hip_fail(e, "field masses");
}

extern "C" int nlse_surrogate_block(nlse_surrogate* m, const void* psi_in, void* psi_out, int batch, int project_msd,
                                    double* mass) {
  int rc = check_batch(m, batch);
  if (rc) return rc;
  if (!psi_in || !psi_out) return nlse_fail(NLSE_EINVAL, "NULL field");
  if (psi_in == psi_out) return nlse_fail(NLSE_EINVAL, "psi_in and psi_out must differ");
  if (!mass) return nlse_fail(NLSE_EINVAL, "mass is NULL");
  const bool project = project_msd != 0;
  hipError_t e = replay(m, std::make_tuple(psi_in, psi_out, batch, project ? 4 : 3),
                        [&]() { return forward(m, psi_in, psi_out, batch, true, project, true); });
  if (e != hipSuccess) return nlse_hip_fail(e, "surrogate block");
  return fetch_masses(m, batch, mass);
}

extern "C" int nlse_surrogate_field_mass(nlse_surrogate* m, const void* psi, int batch, double* mass) {
  int rc = check_batch(m, batch);
  if (rc) return rc;
  if (!psi || !mass) return nlse_fail(NLSE_EINVAL, "NULL argument");
  return masses(m, psi, batch, mass);
}

extern "C" int nlse_surrogate_project_msd(nlse_surrogate* m, const void* psi_in, void* psi_out, int batch) {
  int rc = check_batch(m, batch);
  if (rc) return rc;
  hipError_t e = sg_msd_project(psi_in, psi_out, batch, m->H, m->W, m->stream);
  return e == hipSuccess ? NLSE_OK : nlse_hip_fail(e, "MSD projection");
}

extern "C" int nlse_surrogate_advance(nlse_surrogate* m, nlse_grid* g, int order, int bc, double dt, int64_t nblocks,
                                      double drift_tol, int64_t* n_fallbacks) {
  if (!m || !g) return nlse_fail(NLSE_EINVAL, "NULL model or grid");
  int ndim, dtype;
  int64_t n[3];
  unsigned flags;
  double h;
  void *psi, *gst;
  nlse_grid_view(g, &ndim, n, &dtype, &flags, &h, &psi, &gst);
  if (ndim != 2 || dtype != NLSE_F32 || n[0] != m->W || n[1] != m->H)
    return nlse_fail(NLSE_EINVAL, "the grid must be a 2D FP32 field of the model's H x W");
  if (gst != (void*)m->stream) return nlse_fail(NLSE_EINVAL, "grid and model must share a stream");
  if (nblocks < 0 || !(drift_tol >= 0)) return nlse_fail(NLSE_EINVAL, "bad nblocks / drift_tol");
  if (bc != NLSE_BC_DIRICHLET && bc != NLSE_BC_MSD && bc != NLSE_BC_L0) return nlse_fail(NLSE_EINVAL, "bad bc");
  void* xin = m->work + m->lay.scratch;
  const size_t bytes = (size_t)m->H * m->W * 8;
  int64_t fb = 0;
  double Min = 0.0;
  int rc = masses(m, psi, 1, &Min);
  if (rc) return rc;
  // one block: keep its input, predict, project the boundary ring and sum
  // the new field's mass, all in the last layer's pass (captured)
  auto block = [&]() {
    hipError_t e = nlse_launch_copy(xin, psi, (int64_t)bytes, m->stream);
    if (e == hipSuccess) e = forward(m, xin, psi, 1, true, bc == NLSE_BC_MSD, true);
    return e;
  };
  for (int64_t k = 0; k < nblocks; ++k) {
    hipError_t e = replay(m, std::make_tuple((const void*)xin, psi, 1, bc == NLSE_BC_MSD ? 2 : 1), block);
    if (e != hipSuccess) return nlse_hip_fail(e, "surrogate block");
    double Mout = 0.0;
    if ((rc = fetch_masses(m, 1, &Mout))) return rc;
    const double drift = std::fabs(Mout - Min) / Min;
    if (!(drift <= drift_tol)) {  // also catches NaN
      e = hipMemcpyAsync(psi, xin, bytes, hipMemcpyDeviceToDevice, m->stream);
      if (e != hipSuccess) return nlse_hip_fail(e, "restoring the block input");
      if ((rc = nlse_step_rk4(g, order, bc, dt, kBlockSteps))) return rc;
      if ((rc = masses(m, psi, 1, &Mout))) return rc;
      ++fb;
    } else if (flags & NLSE_COMPENSATED) {
      if ((rc = nlse_set_state(g, nullptr))) return rc;
    }
    Min = Mout;
  }
  if (n_fallbacks) *n_fallbacks = fb;
  return NLSE_OK;
}

extern "C" int nlse_surrogate_set_path(nlse_surrogate* m, int path) {
  if (!m) return nlse_fail(NLSE_EINVAL, "m is NULL");
  if (path != NLSE_SG_PATH_AUTO && path != NLSE_SG_PATH_LAYERS && path != NLSE_SG_PATH_FUSED)
    return nlse_fail(NLSE_EINVAL, "path must be NLSE_SG_PATH_AUTO, _LAYERS or _FUSED");
  if (path != m->path) drop_graphs(m);  // captured passes name their kernels
  m->path = path;
  return NLSE_OK;
}

extern "C" int nlse_surrogate_fused_max_batch(const nlse_surrogate* m) {
  if (!m) return nlse_fail(NLSE_EINVAL, "m is NULL");
  return fused_max_batch(m);
}

extern "C" int nlse_surrogate_destroy(nlse_surrogate* m) {
  if (!m) return nlse_fail(NLSE_EINVAL, "m is NULL");
  drop_graphs(m);
  if (m->cap) (void)hipStreamDestroy(m->cap);
  delete m;
  return NLSE_OK;
}
