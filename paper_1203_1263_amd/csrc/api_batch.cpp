// C ABI of the batched integrator (declared in include/nlse.h): argument
// validation, workspace carving, the cost-balanced static schedule, HIP-graph
// capture of the persistent launch and per-problem reductions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "api_common.h"
#include "nlse.h"
#include "nlse_batch.h"
#include "nlse_internal.h"

namespace {

constexpr int kMaxChunks = 8192;          // upper bound of persistent workgroups
constexpr unsigned kSpinLimit = 1u << 25; // bounded barrier wait (~1-2 s)
constexpr int kDefaultWgPerCu = 3;        // persistent workgroups per CU (untuned)
constexpr int kMinWgPerCu = 1, kMaxWgPerCu = 5;  // the autotuner's range
constexpr int64_t kMaxBatchSteps = 1 << 24; // steps per nlse_batch_step_rk4 call
constexpr size_t kMaxBatchGraphs = 32;    // instantiated graphs kept per batch

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

struct BatchLayout {
  size_t acc, bufA, bufB, lo, items, chunks, barrier, zero, partials, out, total;
};

// Work items of a problem with tile tx x ty.
int64_t tiles_of(const nlse_sim_desc& d, int tx, int ty) {
  return ((d.dims[0] + tx - 1) / tx) * ((d.dims[1] + ty - 1) / ty);
}

bool tile_compiled(int tx, int ty) {
  for (const auto& t : nlse::kBatchTiles)
    if (t[0] == tx && t[1] == ty) return true;
  return false;
}

// *nitems: work items of the tile that makes the most (the workspace holds
// the descriptors of any compiled tile).
int validate(int nsims, const nlse_sim_desc* sims, int dtype, unsigned flags, int64_t* total_pts,
             int64_t* nitems, int64_t* max_blocks) {
  if (nsims < 1) return nlse_fail(NLSE_EINVAL, "nsims must be >= 1");
  if (!sims) return nlse_fail(NLSE_EINVAL, "sims is NULL");
  if (dtype != NLSE_F32 && dtype != NLSE_F64) return nlse_fail(NLSE_EINVAL, "bad dtype");
  if (flags & ~(NLSE_COMPENSATED | NLSE_NO_GRAPH)) return nlse_fail(NLSE_EINVAL, "unknown flag bits");
  if ((flags & NLSE_COMPENSATED) && dtype != NLSE_F32)
    return nlse_fail(NLSE_EUNSUPPORTED, "NLSE_COMPENSATED applies to FP32 only");
  int64_t tot = 0, mb = 1;
  int64_t items_t[nlse::kNumBatchTiles] = {};
  for (int j = 0; j < nsims; ++j) {
    const nlse_sim_desc& d = sims[j];
    if (d.ndim != 2) return nlse_fail(NLSE_EUNSUPPORTED, "problem %d: batches hold 2D problems only", j);
    if (d.dims[0] < 3 || d.dims[1] < 3 || d.dims[2] != 1 || d.dims[0] > (1 << 30) || d.dims[1] > (1 << 30))
      return nlse_fail(NLSE_EINVAL, "problem %d: dims must be {Nx>=3, Ny>=3, 1}", j);
    if ((int64_t)d.dims[0] * d.dims[1] > ((int64_t)1 << 31) - 1)
      return nlse_fail(NLSE_EINVAL, "problem %d is too large", j);
    if (!(d.h > 0) || !std::isfinite(d.h) || !(d.a > 0) || !std::isfinite(d.a) || !std::isfinite(d.s))
      return nlse_fail(NLSE_EINVAL, "problem %d: need h > 0, a > 0, finite s", j);
    if (!(d.dt > 0) || !std::isfinite(d.dt)) return nlse_fail(NLSE_EINVAL, "problem %d: dt must be > 0", j);
    if (d.order != NLSE_CD2 && d.order != NLSE_2SHOC) return nlse_fail(NLSE_EINVAL, "problem %d: bad order", j);
    if (d.bc != NLSE_BC_DIRICHLET && d.bc != NLSE_BC_MSD && d.bc != NLSE_BC_L0)
      return nlse_fail(NLSE_EINVAL, "problem %d: bad bc", j);
    if (d.psi_offset < 0 || d.v_offset < -1) return nlse_fail(NLSE_EINVAL, "problem %d: bad offsets", j);
    const int64_t n = d.dims[0] * d.dims[1];
    tot += n;
    for (int k = 0; k < nlse::kNumBatchTiles; ++k)
      items_t[k] += tiles_of(d, nlse::kBatchTiles[k][0], nlse::kBatchTiles[k][1]);
    mb = std::max(mb, nlse::reduce_blocks(n));
  }
  const int64_t items = *std::max_element(items_t, items_t + nlse::kNumBatchTiles);
  if (items > ((int64_t)1 << 31) - 1) return nlse_fail(NLSE_EINVAL, "too many work items");
  *total_pts = tot;
  *nitems = items;
  *max_blocks = mb;
  return NLSE_OK;
}

BatchLayout layout(int nsims, int dtype, unsigned flags, int64_t tot, int64_t nitems, int64_t max_blocks) {
  const size_t esz = dtype == NLSE_F32 ? 8 : 16;
  const size_t field = a256((size_t)tot * esz);
  BatchLayout L;
  size_t off = 0;
  L.acc = off; off += field;
  L.bufA = off; off += field;
  L.bufB = off; off += field;
  L.lo = off; if (flags & NLSE_COMPENSATED) off += field;
  L.items = off; off += a256(sizeof(nlse::BatchItem) * (size_t)nitems);
  L.chunks = off; off += a256(sizeof(int) * (size_t)(5 * kMaxChunks + 1));
  // two unsigned (the error flag is the second), then one 64-bit arrival
  // counter per group (at most one group per chunk)
  L.barrier = off; off += a256(8 + sizeof(unsigned long long) * (size_t)kMaxChunks);
  L.zero = off; off += 256;
  L.partials = off; off += a256((size_t)max_blocks * 3 * sizeof(double));
  L.out = off; off += a256((size_t)nsims * 3 * sizeof(double));
  L.total = off;
  return L;
}

}  // namespace

struct nlse_batch {
  int nsims, dtype;
  unsigned flags;
  std::vector<nlse_sim_desc> desc;
  int64_t total_pts, nitems;  // nitems: of the configured tile
  int nchunks, ngroups;
  int tx, ty, wg_per_cu;  // tile and persistent workgroups per CU
  int pairs;              // 1: two stage-pair passes per step
  int cus;
  unsigned spin_limit;
  void* psi;
  const void* vpool;
  char* work;
  BatchLayout lay;
  hipStream_t stream;
  hipStream_t cap;  // private stream used only for graph capture
  std::map<int64_t, hipGraphExec_t> graphs;
};

extern "C" int nlse_batch_workspace_bytes(int nsims, const nlse_sim_desc* sims, int dtype, unsigned flags,
                                          size_t* bytes) {
  int64_t tot, items, mb;
  int rc = validate(nsims, sims, dtype, flags, &tot, &items, &mb);
  if (rc) return rc;
  if (!bytes) return nlse_fail(NLSE_EINVAL, "bytes is NULL");
  *bytes = layout(nsims, dtype, flags, tot, items, mb).total;
  return NLSE_OK;
}

// One persistent launch of nsteps steps (preceded by the reset of the group
// arrival counters; the error flag before them stays sticky).  The stage-pair
// kernel runs even step counts, so an odd count under pairs starts with one
// step of the single-stage kernel.
static hipError_t launch(nlse_batch* b, int64_t nsteps, int pairs, hipStream_t st);

static hipError_t enqueue(nlse_batch* b, int64_t nsteps, hipStream_t st) {
  if (b->pairs && (nsteps & 1)) {
    hipError_t e = launch(b, 1, 0, st);
    if (e != hipSuccess || nsteps == 1) return e;
    return launch(b, nsteps - 1, 1, st);
  }
  return launch(b, nsteps, b->pairs, st);
}

static hipError_t launch(nlse_batch* b, int64_t nsteps, int pairs, hipStream_t st) {
  hipError_t e = nlse_launch_fill_zero(b->work + b->lay.barrier + 8, 8 * (int64_t)b->ngroups, st);
  if (e != hipSuccess) return e;
  nlse::BatchLaunch L;
  L.dtype = b->dtype;
  L.comp = (b->flags & NLSE_COMPENSATED) ? 1 : 0;
  L.nsteps = (int)nsteps;
  L.nchunks = b->nchunks;
  L.tx = b->tx;
  L.ty = b->ty;
  L.pairs = pairs;
  L.items = reinterpret_cast<const nlse::BatchItem*>(b->work + b->lay.items);
  L.chunk_off = reinterpret_cast<const int*>(b->work + b->lay.chunks);
  L.psi = b->psi;
  L.vpool = b->vpool;
  L.vzero = b->work + b->lay.zero;
  L.acc = b->work + b->lay.acc;
  L.bufA = b->work + b->lay.bufA;
  L.bufB = b->work + b->lay.bufB;
  L.lo = L.comp ? b->work + b->lay.lo : nullptr;
  L.barrier = reinterpret_cast<unsigned*>(b->work + b->lay.barrier);
  L.spin_limit = b->spin_limit;
  return nlse_launch_batch(L, st);
}

static void destroy_graphs(nlse_batch* b) {
  for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
  b->graphs.clear();
}

// Work items and the static schedule of a batch (host only): the tiles of
// every problem as device descriptors, and for W chunks the item offsets
// (W + 1) followed by four ints per chunk (group a, size a, group b,
// size b; -1 / 0 for none).  Returns the number of groups.
static int plan_schedule(int nsims, const nlse_sim_desc* sims, int W, int TX, int TY,
                         std::vector<nlse::BatchItem>& it, std::vector<int>& chunk) {
  // device descriptors: the same double constants the single-grid path uses
  std::vector<std::vector<nlse::BatchItem>> tiles(nsims);  // row-major tiles of each problem
  std::vector<double> pcost(nsims);                        // estimated cost of one stage
  int64_t woff = 0;
  for (int j = 0; j < nsims; ++j) {
    const nlse_sim_desc& d = sims[j];
    nlse::BatchItem s;
    std::memset(&s, 0, sizeof s);
    s.nx = (int)d.dims[0];
    s.ny = (int)d.dims[1];
    s.scheme = d.order | (d.bc << 8);
    s.psi_off = d.psi_offset;
    s.v_off = d.v_offset;
    s.woff = woff;
    woff += d.dims[0] * d.dims[1];
    s.a = d.a;
    s.s = d.s;
    s.inv_a = 1.0 / d.a;
    s.inv_h2 = 1.0 / (d.h * d.h);
    s.inv_6h2 = 1.0 / (6.0 * d.h * d.h);
    s.dt = d.dt;
    s.dt2 = d.dt / 2.0;
    s.dt3 = d.dt / 3.0;
    s.dt6 = d.dt / 6.0;
    s.af = (float)s.a;
    s.sf = (float)s.s;
    s.inv_af = (float)s.inv_a;
    s.inv_h2f = (float)s.inv_h2;
    s.inv_6h2f = (float)s.inv_6h2;
    s.dtf = (float)s.dt;
    s.dt2f = (float)s.dt2;
    s.dt3f = (float)s.dt3;
    s.dt6f = (float)s.dt6;
    s.sim = j;
    const int ntx = (s.nx + TX - 1) / TX, nty = (s.ny + TY - 1) / TY;
    const double c = (d.order == 4 ? 1.35 : 1.0) * (d.v_offset >= 0 ? 1.1 : 1.0);
    for (int ty = 0; ty < nty; ++ty)
      for (int tx = 0; tx < ntx; ++tx) {
        s.tx = tx;
        s.ty = ty;
        tiles[j].push_back(s);
      }
    pcost[j] = c * (double)tiles[j].size();
  }
  // Schedule: contiguous chunks of (problem, tile) items with balanced cost,
  // one per workgroup.  Problems are independent, so a problem inside one
  // chunk needs no barrier with any other chunk; a problem spread over
  // chunks c_a..c_b is a group whose chunks meet at a barrier after every
  // stage.  Only a chunk's first and last problem can spread beyond it, so
  // a chunk belongs to at most two groups.  Consecutive chunk numbers land on
  // one XCD, so most groups share an L2.
  it.clear();
  std::vector<double> cost;
  std::vector<int> owner;  // problem of each item
  for (int j = 0; j < nsims; ++j) {
    const double c = pcost[j] / (double)tiles[j].size();
    for (const auto& t : tiles[j]) {
      it.push_back(t);
      cost.push_back(c);
      owner.push_back(j);
    }
  }
  const int64_t items = (int64_t)it.size();
  chunk.assign(5 * (size_t)W + 1, -1);
  {
    double total = 0;
    for (double c : cost) total += c;
    double acc = 0;
    int k = 0;
    chunk[0] = 0;
    for (int64_t i = 0; i < items && k + 1 < W; ++i) {
      acc += cost[i];
      if (acc >= total * (k + 1) / W) chunk[++k] = (int)(i + 1);
    }
    for (int r = k + 1; r < W; ++r) chunk[r] = (int)items;
    chunk[W] = (int)items;
  }
  // chunk span of every problem, then its group
  std::vector<int> first(nsims, -1), last(nsims, -1);
  for (int c = 0; c < W; ++c)
    for (int i = chunk[c]; i < chunk[c + 1]; ++i) {
      const int j = owner[i];
      if (first[j] < 0) first[j] = c;
      last[j] = c;
    }
  int ngroups = 0;
  std::vector<int> gid(nsims, -1);
  for (int j = 0; j < nsims; ++j)
    if (first[j] >= 0 && last[j] > first[j]) gid[j] = ngroups++;
  for (int c = 0; c < W; ++c) {
    int ga = -1, gb = -1;
    if (chunk[c] < chunk[c + 1]) {
      const int ja = owner[chunk[c]], jb = owner[chunk[c + 1] - 1];
      ga = gid[ja];
      gb = (jb != ja) ? gid[jb] : -1;
      chunk[W + 1 + 4 * c + 1] = ga >= 0 ? last[ja] - first[ja] + 1 : 0;
      chunk[W + 1 + 4 * c + 3] = gb >= 0 ? last[jb] - first[jb] + 1 : 0;
    }
    chunk[W + 1 + 4 * c + 0] = ga;
    chunk[W + 1 + 4 * c + 2] = gb;
  }
  return ngroups;
}

// Test hook (host only, no device work): the schedule a batch with tile
// tx x ty builds for W chunks.  chunk_out receives 5 W + 1 ints (see
// plan_schedule), item_out 3 ints per work item (problem, tile x index,
// tile y index), *ngroups the number of groups.  NLSE_ENOMEM if an output is
// shorter than that.
extern "C" int nlse_internal_batch_plan(int nsims, const nlse_sim_desc* sims, int W, int tx, int ty, int* chunk_out,
                                        int64_t chunk_len, int* item_out, int64_t item_len, int* ngroups) {
  int64_t tot, items, mb;
  int rc = validate(nsims, sims, NLSE_F32, 0, &tot, &items, &mb);
  if (rc) return rc;
  if (W < 1 || W > kMaxChunks || !chunk_out || !item_out || !ngroups) return nlse_fail(NLSE_EINVAL, "bad argument");
  if (!tile_compiled(tx, ty)) return nlse_fail(NLSE_EUNSUPPORTED, "tile %dx%d is not compiled", tx, ty);
  std::vector<nlse::BatchItem> it;
  std::vector<int> chunk;
  const int ng = plan_schedule(nsims, sims, W, tx, ty, it, chunk);
  if ((int64_t)chunk.size() > chunk_len || 3 * (int64_t)it.size() > item_len)
    return nlse_fail(NLSE_ENOMEM, "output arrays too short");
  std::copy(chunk.begin(), chunk.end(), chunk_out);
  for (size_t i = 0; i < it.size(); ++i) {
    item_out[3 * i] = it[i].sim;
    item_out[3 * i + 1] = it[i].tx;
    item_out[3 * i + 2] = it[i].ty;
  }
  *ngroups = ng;
  return NLSE_OK;
}

// Test hook (host only): the limits behind the group barrier's arithmetic.
// out[0] = largest nsteps of one call, out[1] = largest number of chunks
// (so of chunks in one group), out[2] = bits of an arrival counter.  The
// barrier target of the last stage of a call is 4 * nsteps * group size.
extern "C" int nlse_internal_batch_limits(int64_t out[3]) {
  if (!out) return nlse_fail(NLSE_EINVAL, "out is NULL");
  out[0] = kMaxBatchSteps;
  out[1] = kMaxChunks;
  out[2] = 8 * (int64_t)sizeof(unsigned long long);
  return NLSE_OK;
}

// Tile, workgroups per CU, pass structure and the static schedule of a
// batch: the persistent grid is min(wg_per_cu, what fits) x CUs workgroups;
// the work items and chunk table are rebuilt and uploaded, and captured
// graphs (which hold the grid size, tile and kernel) are dropped.
// Synchronises the stream.
static int configure(nlse_batch* b, int tx, int ty, int wg_per_cu, int pairs) {
  if (!tile_compiled(tx, ty)) return nlse_fail(NLSE_EUNSUPPORTED, "tile %dx%d is not compiled", tx, ty);
  if (wg_per_cu < 1 || wg_per_cu > 16) return nlse_fail(NLSE_EINVAL, "wg_per_cu must be 1..16");
  if (pairs != 0 && pairs != 1) return nlse_fail(NLSE_EINVAL, "pairs must be 0 or 1");
  // the grid must be resident at once for every kernel it runs (with pairs,
  // an odd step count also runs the single-stage kernel on it)
  int occ = 0, occ1 = 0;
  const int comp = (b->flags & NLSE_COMPENSATED) ? 1 : 0;
  hipError_t e = nlse_batch_occupancy(b->dtype, comp, tx, ty, pairs, &occ);
  if (e == hipSuccess && pairs) e = nlse_batch_occupancy(b->dtype, comp, tx, ty, 0, &occ1);
  if (e != hipSuccess) return nlse_hip_fail(e, "querying occupancy");
  if (pairs) occ = std::min(occ, occ1);
  if (occ < 1) return nlse_fail(NLSE_EDEVICE, "the batched kernel does not fit on a CU");
  int64_t items = 0;
  for (const auto& d : b->desc) items += tiles_of(d, tx, ty);
  const int64_t nchunks = std::min<int64_t>({(int64_t)std::min(occ, wg_per_cu) * b->cus, items, (int64_t)kMaxChunks});
  std::vector<nlse::BatchItem> it;
  std::vector<int> chunk;
  const int ngroups = plan_schedule(b->nsims, b->desc.data(), (int)nchunks, tx, ty, it, chunk);
  if ((int64_t)it.size() != items) return nlse_fail(NLSE_EDEVICE, "internal error: schedule lost work items");
  e = hipStreamSynchronize(b->stream);  // no launch still reads the old tables
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->work + b->lay.items, it.data(), sizeof(nlse::BatchItem) * it.size(),
                       hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->work + b->lay.chunks, chunk.data(), sizeof(int) * chunk.size(), hipMemcpyHostToDevice,
                       b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return nlse_hip_fail(e, "uploading the batch schedule");
  destroy_graphs(b);
  b->tx = tx;
  b->ty = ty;
  b->wg_per_cu = wg_per_cu;
  b->pairs = pairs;
  b->nchunks = (int)nchunks;
  b->ngroups = ngroups;
  b->nitems = items;
  return NLSE_OK;
}

extern "C" int nlse_batch_create(nlse_batch** out, int nsims, const nlse_sim_desc* sims, int dtype, unsigned flags,
                                 void* psi_pool, size_t psi_pool_elems, const void* v_pool, size_t v_pool_elems,
                                 void* work_dev, size_t work_bytes, void* hip_stream) {
  if (!out) return nlse_fail(NLSE_EINVAL, "b is NULL");
  *out = nullptr;
  int64_t tot, items, mb;
  int rc = validate(nsims, sims, dtype, flags, &tot, &items, &mb);
  if (rc) return rc;
  if (!psi_pool || !work_dev) return nlse_fail(NLSE_EINVAL, "psi_pool / work_dev is NULL");
  if (((uintptr_t)work_dev) % 256) return nlse_fail(NLSE_EINVAL, "work_dev must be 256-byte aligned");
  if (((uintptr_t)psi_pool) % (dtype == NLSE_F32 ? 8 : 16)) return nlse_fail(NLSE_EINVAL, "psi_pool misaligned");
  BatchLayout L = layout(nsims, dtype, flags, tot, items, mb);
  if (work_bytes < L.total)
    return nlse_fail(NLSE_ENOMEM, "workspace of %zu bytes is smaller than the %zu required", work_bytes, L.total);
  for (int j = 0; j < nsims; ++j) {
    const int64_t n = sims[j].dims[0] * sims[j].dims[1];
    if ((size_t)(sims[j].psi_offset + n) > psi_pool_elems)
      return nlse_fail(NLSE_EINVAL, "problem %d lies outside psi_pool", j);
    if (sims[j].v_offset >= 0 && (!v_pool || (size_t)(sims[j].v_offset + n) > v_pool_elems))
      return nlse_fail(NLSE_EINVAL, "problem %d: potential lies outside v_pool", j);
  }

  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return nlse_hip_fail(e, "querying the device");
  if (cus < 1) return nlse_fail(NLSE_EDEVICE, "no compute units");

  nlse_batch* B = new (std::nothrow) nlse_batch();
  if (!B) return nlse_fail(NLSE_ENOMEM, "host allocation failed");
  B->nsims = nsims;
  B->dtype = dtype;
  B->flags = flags;
  B->desc.assign(sims, sims + nsims);
  B->total_pts = tot;
  B->nitems = items;
  B->cus = cus;
  B->spin_limit = kSpinLimit;
  if (const char* sl = getenv("NLSE_BATCH_SPIN_LIMIT")) {
    const long v = strtol(sl, nullptr, 10);
    if (v > 0 && v <= (long)kSpinLimit) B->spin_limit = (unsigned)v;  // a shorter wait only
  }
  B->psi = psi_pool;
  B->vpool = v_pool;
  B->work = static_cast<char*>(work_dev);
  B->lay = L;
  B->stream = static_cast<hipStream_t>(hip_stream);
  B->cap = nullptr;

  hipStream_t st = B->stream;
  e = nlse_launch_fill_zero(B->work + L.zero, 256, st);
  if (e == hipSuccess) e = nlse_launch_fill_zero(B->work + L.barrier, (int64_t)(L.zero - L.barrier), st);
  if (e == hipSuccess && (flags & NLSE_COMPENSATED)) e = nlse_launch_fill_zero(B->work + L.lo, tot * 8, st);
  if (e == hipSuccess && !(flags & NLSE_NO_GRAPH)) e = hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete B;
    return nlse_hip_fail(e, "creating the batch");
  }
  rc = configure(B, 32, 8, kDefaultWgPerCu, 0);
  if (rc) {
    if (B->cap) (void)hipStreamDestroy(B->cap);
    delete B;
    return rc;
  }
  *out = B;
  return NLSE_OK;
}

extern "C" int nlse_batch_set_config(nlse_batch* b, int tx, int ty, int wg_per_cu, int pairs) {
  if (!b) return nlse_fail(NLSE_EINVAL, "b is NULL");
  return configure(b, tx, ty, wg_per_cu, pairs);
}

extern "C" int nlse_batch_get_config(const nlse_batch* b, int cfg[4]) {
  if (!b || !cfg) return nlse_fail(NLSE_EINVAL, "NULL argument");
  cfg[0] = b->tx;
  cfg[1] = b->ty;
  cfg[2] = b->wg_per_cu;
  cfg[3] = b->pairs;
  return NLSE_OK;
}

// Cache key of a batch: element type, mode and a hash (FNV-1a) of every
// problem's shape, scheme, boundary condition and whether it has a potential.
static std::string batch_key(const nlse_batch* b) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](int64_t v) {
    for (int i = 0; i < 8; ++i) {
      h ^= (uint64_t)((v >> (8 * i)) & 0xff);
      h *= 1099511628211ull;
    }
  };
  for (const auto& d : b->desc) {
    mix(d.dims[0]);
    mix(d.dims[1]);
    mix(d.order);
    mix(d.bc);
    mix(d.v_offset >= 0 ? 1 : 0);
  }
  char buf[128];
  snprintf(buf, sizeof buf, "batch4 t%d c%d n%d h%016llx", b->dtype, (b->flags & NLSE_COMPENSATED) ? 1 : 0, b->nsims,
           (unsigned long long)h);
  return buf;
}

// Copies every problem's Psi (packed by work offset) and the compensation
// term between the batch and `save` (to = true: into save).
static hipError_t copy_fields(nlse_batch* b, char* save, bool to) {
  const size_t esz = b->dtype == NLSE_F32 ? 8 : 16;
  size_t woff = 0;
  hipError_t e = hipSuccess;
  for (const auto& d : b->desc) {
    const size_t n = (size_t)(d.dims[0] * d.dims[1]);
    char* p = static_cast<char*>(b->psi) + (size_t)d.psi_offset * esz;
    char* q = save + woff * esz;
    e = hipMemcpyAsync(to ? q : p, to ? p : q, n * esz, hipMemcpyDeviceToDevice, b->stream);
    if (e != hipSuccess) return e;
    woff += n;
  }
  if (b->flags & NLSE_COMPENSATED) {
    char* lo = b->work + b->lay.lo;
    char* q = save + (size_t)b->total_pts * esz;
    e = hipMemcpyAsync(to ? q : lo, to ? lo : q, (size_t)b->total_pts * esz, hipMemcpyDeviceToDevice, b->stream);
  }
  return e;
}

// Times whole RK4 steps of every candidate (tile x workgroups per CU x
// single-stage / stage-pair passes) on the batch itself, each with its own
// schedule; Psi and the compensation term are saved to a temporary device
// buffer first and restored afterwards, so the fields end as they began.
extern "C" int nlse_batch_autotune(nlse_batch* b) {
  if (!b) return nlse_fail(NLSE_EINVAL, "b is NULL");
  const std::string key = batch_key(b);
  int cached[4];
  if (nlse_cache_lookup(key, cached, 4) && tile_compiled(cached[0], cached[1]) && cached[2] >= 1 &&
      cached[2] <= 16 && (cached[3] == 0 || cached[3] == 1))
    return configure(b, cached[0], cached[1], cached[2], cached[3]);
  const size_t esz = b->dtype == NLSE_F32 ? 8 : 16;
  const size_t save_bytes = (size_t)b->total_pts * esz * ((b->flags & NLSE_COMPENSATED) ? 2 : 1);
  char* save = nullptr;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&save), save_bytes);
  if (e != hipSuccess) return nlse_hip_fail(e, "allocating the autotuner's copy of the fields");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  e = copy_fields(b, save, true);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  const int reps = (int)std::max<int64_t>(2, std::min<int64_t>(50, (int64_t)3e8 / std::max<int64_t>(b->total_pts, 1)));
  float best = 1e30f;
  int best_c[4] = {32, 8, kDefaultWgPerCu, 0};
  int rc = NLSE_OK;
  for (int pairs = 0; pairs <= 1 && e == hipSuccess && rc == NLSE_OK; ++pairs)
    for (const auto& t : nlse::kBatchTiles) {
      int occ = 0;
      e = nlse_batch_occupancy(b->dtype, (b->flags & NLSE_COMPENSATED) ? 1 : 0, t[0], t[1], pairs, &occ);
      if (e != hipSuccess) break;
      for (int w = kMinWgPerCu; w <= std::min(kMaxWgPerCu, occ); ++w) {
        if ((rc = configure(b, t[0], t[1], w, pairs)) != NLSE_OK) break;
        if ((e = enqueue(b, 2, b->stream)) != hipSuccess) break;  // warm-up
        (void)hipEventRecord(e0, b->stream);
        if ((e = enqueue(b, reps, b->stream)) != hipSuccess) break;
        (void)hipEventRecord(e1, b->stream);
        if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) {
          best = ms;
          best_c[0] = t[0];
          best_c[1] = t[1];
          best_c[2] = w;
          best_c[3] = pairs;
        }
      }
      if (rc != NLSE_OK || e != hipSuccess) break;
    }
  // restore the fields whatever happened above
  hipError_t er = copy_fields(b, save, false);
  if (er == hipSuccess) er = hipStreamSynchronize(b->stream);
  (void)hipFree(save);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (rc != NLSE_OK) return rc;
  if (e != hipSuccess) return nlse_hip_fail(e, "batch autotune launch");
  if (er != hipSuccess) return nlse_hip_fail(er, "restoring the fields after autotuning");
  rc = configure(b, best_c[0], best_c[1], best_c[2], best_c[3]);
  if (rc == NLSE_OK) nlse_cache_store(key, best_c, 4, best / reps);
  return rc;
}

extern "C" int nlse_batch_step_rk4(nlse_batch* b, int64_t nsteps) {
  if (nsteps < 0 || nsteps > kMaxBatchSteps) return nlse_fail(NLSE_EINVAL, "nsteps out of range");
  if (!b) return nlse_fail(NLSE_EINVAL, "b is NULL");
  if (nsteps == 0) return NLSE_OK;
  hipError_t e;
  if (b->flags & NLSE_NO_GRAPH) {
    e = enqueue(b, nsteps, b->stream);
    return e == hipSuccess ? NLSE_OK : nlse_hip_fail(e, "batch launch");
  }
  auto found = b->graphs.find(nsteps);
  if (found == b->graphs.end()) {
    if (b->graphs.size() >= kMaxBatchGraphs) destroy_graphs(b);
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return nlse_hip_fail(e, "hipStreamBeginCapture");
    hipError_t le = enqueue(b, nsteps, b->cap);
    e = hipStreamEndCapture(b->cap, &graph);
    if (le != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return nlse_hip_fail(le, "capturing the batch launch");
    }
    if (e != hipSuccess) return nlse_hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return nlse_hip_fail(e, "hipGraphInstantiate");
    found = b->graphs.emplace(nsteps, exec).first;
  }
  e = hipGraphLaunch(found->second, b->stream);
  return e == hipSuccess ? NLSE_OK : nlse_hip_fail(e, "hipGraphLaunch");
}

extern "C" int nlse_batch_mass_energy(nlse_batch* b, double* mass, double* energy) {
  if (!b || !mass || !energy) return nlse_fail(NLSE_EINVAL, "NULL argument");
  double* out = reinterpret_cast<double*>(b->work + b->lay.out);
  for (int j = 0; j < b->nsims; ++j) {
    const nlse_sim_desc& d = b->desc[j];
    nlse::ReduceLaunch R;
    R.ndim = 2;
    R.dtype = b->dtype;
    R.order = d.order;
    R.bc = d.bc;
    R.n[0] = d.dims[0];
    R.n[1] = d.dims[1];
    R.n[2] = 1;
    const size_t esz = b->dtype == NLSE_F32 ? 8 : 16;
    R.psi = static_cast<char*>(b->psi) + (size_t)d.psi_offset * esz;
    R.V = d.v_offset >= 0 ? static_cast<const char*>(b->vpool) + (size_t)d.v_offset * (esz / 2) : nullptr;
    R.a = d.a;
    R.s = d.s;
    R.h = d.h;
    R.partials = reinterpret_cast<double*>(b->work + b->lay.partials);
    R.out = out + 3 * j;
    R.dscratch = b->work + b->lay.bufA;  // idle between steps; bufB follows it
    hipError_t e = nlse_launch_reduce(R, b->stream);
    if (e != hipSuccess) return nlse_hip_fail(e, "reduction launch");
  }
  std::vector<double> host((size_t)b->nsims * 3);
  hipError_t e = hipMemcpyAsync(host.data(), out, host.size() * sizeof(double), hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return nlse_hip_fail(e, "copying the reductions");
  bool finite = true;
  for (int j = 0; j < b->nsims; ++j) {
    const double h2 = b->desc[j].h * b->desc[j].h;
    mass[j] = h2 * host[3 * j];
    energy[j] = h2 * (host[3 * j + 1] + host[3 * j + 2]);
    finite = finite && std::isfinite(mass[j]) && std::isfinite(energy[j]);
  }
  return finite ? NLSE_OK : nlse_fail(NLSE_EUNSTABLE, "a problem has non-finite mass or energy");
}

extern "C" int nlse_batch_status(nlse_batch* b) {
  if (!b) return nlse_fail(NLSE_EINVAL, "b is NULL");
  unsigned flag[2] = {0, 0};
  hipError_t e = hipMemcpyAsync(flag, b->work + b->lay.barrier, sizeof flag, hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return nlse_hip_fail(e, "reading the batch status");
  return flag[1] ? nlse_fail(NLSE_EDEVICE, "a barrier of the batched kernel timed out") : NLSE_OK;
}

extern "C" int nlse_batch_info(const nlse_batch* b, int64_t info[4]) {
  if (!b || !info) return nlse_fail(NLSE_EINVAL, "NULL argument");
  info[0] = b->nchunks;
  info[1] = b->nitems;
  info[2] = b->total_pts;
  info[3] = (int64_t)b->graphs.size();
  return NLSE_OK;
}

extern "C" int nlse_batch_destroy(nlse_batch* b) {
  if (!b) return nlse_fail(NLSE_EINVAL, "b is NULL");
  destroy_graphs(b);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
  return NLSE_OK;
}
