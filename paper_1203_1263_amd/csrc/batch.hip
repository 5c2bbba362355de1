// Batched persistent RK4 integrator for many independent 2D problems of
// uneven size and parameters (a, s, V, h, dt, scheme, boundary condition).
//
// One launch advances every problem nsteps RK4 steps.  The launch is
// persistent: its grid is sized to what the device holds at once, and each
// workgroup owns a fixed, cost-balanced chunk of (problem, tile) work items
// computed on the host.  For every stage a workgroup runs the 2D tile body of
// the single-grid kernel (tile2d.hpp) on each of its items, then waits for
// the workgroups its next stage depends on (a stage of a problem reads the
// previous stage of its neighbouring tiles).  Problems are independent: a
// problem inside one chunk needs only a workgroup barrier between stages,
// and a problem spread over consecutive chunks is a group whose chunks meet
// at a barrier (a monotonically increasing arrival counter per group with a
// bounded wait).  A chunk belongs to at most two groups (its first and last
// problem).  A wait that exceeds the spin limit raises an error flag and
// every waiting workgroup then leaves the kernel, so the grid always drains.
//
// Within a stage the items of a chunk are software-pipelined: while item i
// is computed, the loads of item i+1 are in flight in a second register set
// and the descriptor of item i+2 in a third, so a workgroup never waits a
// full memory round trip per item.  Descriptors are read with vector loads
// (one dword per lane) and broadcast with readlane, which keeps their wait
// separate from the LDS traffic of the item being computed.  Two LDS
// buffers for the stage-input box alternate between consecutive items.
#include <cstddef>

#include "nlse_batch.h"
#include "tile2d.hpp"

namespace nlse {

template <typename T>
struct BatchArgs {
  const BatchItem* items;
  const int* chunk_off;  // items of chunk c: [chunk_off[c], chunk_off[c+1]);
                         // then per chunk (group a, size a, group b, size b),
                         // -1 for no group
  cpx<T>* psi;           // caller's pool
  const T* vpool;        // caller's potential pool (may be null)
  const T* vzero;        // one zero element
  cpx<T>* acc;           // work pools, indexed by BatchItem::woff
  cpx<T>* bufA;
  cpx<T>* bufB;
  cpx<T>* lo;
  unsigned* flag;        // sticky error flag
  unsigned long long* arrivals;  // arrivals of group g
  unsigned spin_limit;
};

// Barrier number `k` (1, 2, ...) of the groups (ga, size sa) and (gb, size
// sb) a chunk belongs to (-1: none): the workgroup adds one arrival to each
// group's counter and waits until each holds k * size arrivals.  The
// counters and targets are 64-bit: k reaches 4 * nsteps and a group spans up
// to every chunk, so a 32-bit target could wrap within one launch.  One
// release before the arrivals and one acquire after the waits, and only
// thread 0 crosses device scope:
// the workgroup barrier first orders every wave's stores before thread 0's
// agent-scope release (on this chip a release writes back the XCD's L2 and
// an acquire invalidates it, so one of each per workgroup instead of one
// per wave), and the workgroup barrier after thread 0's agent-scope acquire
// orders every wave's later loads after it.  Returns false if the wait
// timed out or another workgroup reported an error.
__device__ __forceinline__ bool group_barrier(unsigned* flag, unsigned long long* cnt, int ga, unsigned sa, int gb,
                                              unsigned sb, unsigned long long k, unsigned spin_limit) {
  __shared__ int ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long* ca = cnt + (ga >= 0 ? ga : 0);
    unsigned long long* cb = cnt + (gb >= 0 ? gb : 0);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (ga >= 0) __hip_atomic_fetch_add(ca, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (gb >= 0) __hip_atomic_fetch_add(cb, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    auto arrived = [&](const unsigned long long* c, int g, unsigned size) {
      return g < 0 || __hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= k * size;
    };
    unsigned spins = 0;
    int good = 1;
    // poll with relaxed loads (an acquire per poll would invalidate the
    // caches under the workgroups still computing); acquire once below
    while (!(arrived(ca, ga, sa) && arrived(cb, gb, sb))) {
      if (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u || ++spins > spin_limit) {
        good = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    if (!good) __hip_atomic_store(flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    ok = good;
  }
  __syncthreads();
  return ok != 0;
}

// Dword k of the descriptor words held one per lane, broadcast to the
// whole wave.
__device__ __forceinline__ int word_i32(unsigned w, int k) { return __builtin_amdgcn_readlane((int)w, k); }
__device__ __forceinline__ int64_t word_i64(unsigned w, int k) {
  return (int64_t)(((uint64_t)(unsigned)word_i32(w, k + 1) << 32) | (uint64_t)(unsigned)word_i32(w, k));
}
__device__ __forceinline__ double word_f64(unsigned w, int k) {
  return __builtin_bit_cast(double, (uint64_t)word_i64(w, k));
}
// A physical constant in the element type: the FP32 copy (one dword) for
// FP32 kernels, the double for FP64 ones.
template <typename T>
__device__ __forceinline__ T word_t(unsigned w, int kd, int kf) {
  if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(float, word_i32(w, kf));
  else
    return word_f64(w, kd);
}
#define NLSE_WORD(field) ((int)(offsetof(BatchItem, field) / 4))
#define NLSE_WORD_T(field) word_t<T>(w, NLSE_WORD(field), NLSE_WORD(field##f))

// The descriptor of item `it`, one dword per lane.
__device__ __forceinline__ unsigned item_words(const BatchItem* items, int it) {
  return reinterpret_cast<const unsigned*>(items + it)[threadIdx.x & 63];
}

template <typename T>
struct ItemArgs {
  StageArgs<T> A;
  int order, bc, tx, ty;
};

// Stage arguments of one item, from its descriptor words.
template <typename T, int STAGE>
__device__ __forceinline__ ItemArgs<T> decode(const BatchArgs<T>& B, unsigned w) {
  ItemArgs<T> I;
  StageArgs<T>& A = I.A;
  const int64_t psi_off = word_i64(w, NLSE_WORD(psi_off)), v_off = word_i64(w, NLSE_WORD(v_off));
  const int64_t woff = word_i64(w, NLSE_WORD(woff));
  cpx<T>* psi = B.psi + psi_off;
  cpx<T>* a = B.bufA + woff;
  cpx<T>* b = B.bufB + woff;
  A.uin = STAGE == 1 ? psi : (STAGE == 2 ? a : (STAGE == 3 ? b : a));
  A.uout = STAGE == 1 ? a : (STAGE == 2 ? b : (STAGE == 3 ? a : psi));
  A.psi = psi;
  A.acc = B.acc + woff;
  A.lo = B.lo ? B.lo + woff : nullptr;
  A.V = v_off >= 0 ? B.vpool + v_off : B.vzero;
  A.vs = v_off >= 0 ? 1 : 0;
  A.nx = word_i32(w, NLSE_WORD(nx));
  A.ny = word_i32(w, NLSE_WORD(ny));
  A.nz = 1;
  A.ph.a = NLSE_WORD_T(a);
  A.ph.s = NLSE_WORD_T(s);
  A.ph.inv_a = NLSE_WORD_T(inv_a);
  A.ph.inv_h2 = NLSE_WORD_T(inv_h2);
  A.ph.inv_6h2 = NLSE_WORD_T(inv_6h2);
  A.c_acc = (STAGE == 1 || STAGE == 4) ? NLSE_WORD_T(dt6) : NLSE_WORD_T(dt3);
  A.c_next = STAGE == 3 ? NLSE_WORD_T(dt) : NLSE_WORD_T(dt2);
  A.c_acc_d = (STAGE == 1 || STAGE == 4) ? word_f64(w, NLSE_WORD(dt6)) : word_f64(w, NLSE_WORD(dt3));
  const int scheme = word_i32(w, NLSE_WORD(scheme));
  I.order = scheme & 0xff;
  I.bc = scheme >> 8;
  I.tx = word_i32(w, NLSE_WORD(tx));
  I.ty = word_i32(w, NLSE_WORD(ty));
  return I;
}

// Arguments of one item of a stage pair, from its descriptor words.  Psi of
// the step lives in the caller's pool or, on alternate steps, in bufA
// (src_a); the second pair writes the new Psi to the other one (dst_a).
template <typename T>
struct PairItem {
  PairArgs<T> A;
  int order, bc, tx, ty;
};

template <typename T, int PAIR>
__device__ __forceinline__ PairItem<T> decode_pair(const BatchArgs<T>& B, unsigned w, bool src_a, bool dst_a) {
  PairItem<T> I;
  PairArgs<T>& A = I.A;
  const int64_t psi_off = word_i64(w, NLSE_WORD(psi_off)), v_off = word_i64(w, NLSE_WORD(v_off));
  const int64_t woff = word_i64(w, NLSE_WORD(woff));
  cpx<T>* psi_src = src_a ? B.bufA + woff : B.psi + psi_off;
  cpx<T>* u2 = B.bufB + woff;
  A.uin = PAIR == 1 ? psi_src : u2;
  A.psi = psi_src;
  A.acc = B.acc + woff;
  A.out = PAIR == 1 ? u2 : (dst_a ? B.bufA + woff : B.psi + psi_off);
  A.lo = B.lo ? B.lo + woff : nullptr;
  A.V = v_off >= 0 ? B.vpool + v_off : B.vzero;
  A.vs = v_off >= 0 ? 1 : 0;
  A.nx = word_i32(w, NLSE_WORD(nx));
  A.ny = word_i32(w, NLSE_WORD(ny));
  A.ph.a = NLSE_WORD_T(a);
  A.ph.s = NLSE_WORD_T(s);
  A.ph.inv_a = NLSE_WORD_T(inv_a);
  A.ph.inv_h2 = NLSE_WORD_T(inv_h2);
  A.ph.inv_6h2 = NLSE_WORD_T(inv_6h2);
  // the coefficients of stages 1, 2 (PAIR 1) or 3, 4 (PAIR 2) as decode gives them
  A.ca1 = PAIR == 1 ? NLSE_WORD_T(dt6) : NLSE_WORD_T(dt3);
  A.cn1 = PAIR == 1 ? NLSE_WORD_T(dt2) : NLSE_WORD_T(dt);
  A.ca2 = PAIR == 1 ? NLSE_WORD_T(dt3) : NLSE_WORD_T(dt6);
  A.cn2 = NLSE_WORD_T(dt2);  // stage 2; stage 4 has none
  A.ca2_d = PAIR == 1 ? word_f64(w, NLSE_WORD(dt3)) : word_f64(w, NLSE_WORD(dt6));
  const int scheme = word_i32(w, NLSE_WORD(scheme));
  I.order = scheme & 0xff;
  I.bc = scheme >> 8;
  I.tx = word_i32(w, NLSE_WORD(tx));
  I.ty = word_i32(w, NLSE_WORD(ty));
  return I;
}
#undef NLSE_WORD
#undef NLSE_WORD_T

// The items [i0, i1) of a chunk, software-pipelined.  Item `it`: its loads
// are in flight in `cur`, its descriptor words (long arrived) are in `wc`,
// the words of item it+1 are in flight in `wn`.  Decode both items, reuse
// `wc` for the words of item it+2, start the loads of item it+1 into `nxt`,
// then compute item it.  The next item swaps the roles of (wc, wn) and
// (cur, nxt), so no register that a load is still writing is ever copied.
// The scheduling barrier keeps the descriptor load ahead of the tile loads:
// waiting for it later must not mean waiting for them.  Past the end of the
// chunk the last item is loaded again (and not computed), which keeps the
// memory operations straight-line code.  `compute` gets the LDS buffer
// parity of the item (consecutive items alternate), the next item's
// arguments and registers (its loads in flight) and whether it exists and
// whether the item is the first of the chunk.
template <typename Regs, typename Dec, typename Issue, typename Compute>
__device__ __forceinline__ void run_items(const BatchItem* items, int i0, int i1, Dec dec, Issue issue,
                                          Compute compute) {
  auto words = [&](int it) { return item_words(items, min(it, i1 - 1)); };
  auto body = [&](int it, const Regs& cur, Regs& nxt, unsigned& wc, unsigned wn, int buf) {
    const auto Icur = dec(wc);
    const auto Inxt = dec(wn);
    wc = words(it + 2);
    __builtin_amdgcn_sched_barrier(0);
    issue(Inxt, nxt);
    compute(Icur, cur, buf, Inxt, nxt, it + 1 < i1, it == i0);
  };
  if (i0 >= i1) return;
  unsigned wa = words(i0), wb = words(i0 + 1);
  Regs ra, rb;
  const auto I0 = dec(wa);
  __builtin_amdgcn_sched_barrier(0);
  issue(I0, ra);
  int it = i0;
  for (; it + 1 < i1; it += 2) {
    body(it, ra, rb, wa, wb, 0);      // wa <- words(it + 2)
    body(it + 1, rb, ra, wb, wa, 1);  // wb <- words(it + 3)
  }
  if (it < i1) body(it, ra, rb, wa, wb, 0);
}

template <typename T, int TX, int TY>
struct BatchLds {
  static constexpr int BSZ = (TX + 4) * (TY + 4);
  cpx<T> u[2][BSZ];  // stage-input box, alternating between items
  T v[2][BSZ];       // potential box, alternating between items
  cpx<T> d[(TX + 2) * (TY + 2)];
};

// LDS of a stage pair: input and potential box with the 2SHOC pair halo of
// 4 and the first stage's D box (the second stage's D is smaller and
// reuses it), alternating between consecutive items, and the first stage's
// output on the tile and its ring of 2.  An item stores the next item's box
// before its own last barrier, so the next item's first D pass may run
// while slower waves still finish this item's second stage.
template <typename T, int TX, int TY>
struct PairLds {
  static constexpr int BSZ = (TX + 8) * (TY + 8);
  cpx<T> u[2][BSZ];
  T v[2][BSZ];
  cpx<T> d[2][(TX + 6) * (TY + 6)];
  cpx<T> m[(TX + 4) * (TY + 4)];
};

// One stage over the items [i0, i1) of this workgroup's chunk.
template <typename T, int STAGE, int COMP, int TX, int TY>
__device__ __forceinline__ void batch_stage(const BatchArgs<T>& B, int i0, int i1, BatchLds<T, TX, TY>& S) {
  using Regs = TileRegs<T, TX, TY>;
  auto dec = [&](unsigned w) { return decode<T, STAGE>(B, w); };
  auto issue = [&](const ItemArgs<T>& I, Regs& r) {
    if (I.order == 4)
      tile2d_load<T, STAGE, COMP, TX, TY, 2, true>(I.A, I.tx, I.ty, r);
    else
      tile2d_load<T, STAGE, COMP, TX, TY, 1, true>(I.A, I.tx, I.ty, r);
  };
  auto compute = [&](const ItemArgs<T>& I, const Regs& r, int buf, const ItemArgs<T>&, const Regs&, bool, bool) {
    cpx<T>* sU = S.u[buf];
    T* sV = S.v[buf];
    if (I.order == 4)
      tile2d_compute<T, 4, kAnyBC, STAGE, COMP, TX, TY, true>(I.A, I.tx, I.ty, r, sU, sV, S.d, I.bc);
    else
      tile2d_compute<T, 2, kAnyBC, STAGE, COMP, TX, TY, true>(I.A, I.tx, I.ty, r, sU, sV, S.d, I.bc);
  };
  run_items<Regs>(B.items, i0, i1, dec, issue, compute);
}

// One stage pair (PAIR 1: stages 1+2, PAIR 2: stages 3+4) over the items
// [i0, i1) of this workgroup's chunk.
template <typename T, int PAIR, int COMP, int TX, int TY>
__device__ __forceinline__ void batch_pair(const BatchArgs<T>& B, int i0, int i1, PairLds<T, TX, TY>& S, bool src_a,
                                           bool dst_a) {
  using Regs = PairRegs<T, TX, TY>;
  auto dec = [&](unsigned w) { return decode_pair<T, PAIR>(B, w, src_a, dst_a); };
  auto issue = [&](const PairItem<T>& I, Regs& r) {
    if (I.order == 4)
      pair2d_load<T, PAIR, COMP, TX, TY, 2, true>(I.A, I.tx, I.ty, r);
    else
      pair2d_load<T, PAIR, COMP, TX, TY, 1, true>(I.A, I.tx, I.ty, r);
  };
  auto compute = [&](const PairItem<T>& I, const Regs& r, int buf, const PairItem<T>& In, const Regs& rn,
                     bool has_next, bool first) {
    // the first item of the chunk stores its own box; every item stores the
    // next one's (with that item's halo) into the other buffers
    auto before_last = [&] {
      if (has_next) {
        if (In.order == 4)
          pair2d_put<T, TX, TY, 2>(rn, S.u[buf ^ 1], S.v[buf ^ 1]);
        else
          pair2d_put<T, TX, TY, 1>(rn, S.u[buf ^ 1], S.v[buf ^ 1]);
      }
    };
    if (I.order == 4)
      pair2d_compute<T, 4, kAnyBC, PAIR, COMP, TX, TY, true>(I.A, I.tx, I.ty, r, S.u[buf], S.v[buf], S.d[buf],
                                                             S.m, I.bc, !first, before_last);
    else
      pair2d_compute<T, 2, kAnyBC, PAIR, COMP, TX, TY, true>(I.A, I.tx, I.ty, r, S.u[buf], S.v[buf], S.d[buf],
                                                             S.m, I.bc, !first, before_last);
  };
  run_items<Regs>(B.items, i0, i1, dec, issue, compute);
}

// The chunk of this workgroup and its barrier between passes: a chunk whose
// problems all lie inside it reads only its own earlier stores (a workgroup
// barrier orders them); otherwise it meets its groups.
struct ChunkSync {
  int i0, i1, ga, gb;
  unsigned sa, sb;
  unsigned long long k;
  template <typename T>
  __device__ __forceinline__ ChunkSync(const BatchArgs<T>& B) : k(0) {
    const int c = xcd_swizzle(blockIdx.x, gridDim.x);
    i0 = B.chunk_off[c];
    i1 = B.chunk_off[c + 1];
    const int* meta = B.chunk_off + gridDim.x + 1 + 4 * c;
    ga = meta[0];
    gb = meta[2];
    sa = (unsigned)meta[1];
    sb = (unsigned)meta[3];
  }
  template <typename T>
  __device__ __forceinline__ bool operator()(const BatchArgs<T>& B) {
    if (ga < 0 && gb < 0) {
      __syncthreads();
      return true;
    }
    return group_barrier(B.flag, B.arrivals, ga, sa, gb, sb, ++k, B.spin_limit);
  }
};

// nsteps RK4 steps, four single-stage passes each.
template <typename T, int COMP, int TX, int TY>
__global__ __launch_bounds__(TX* TY) void batch2d_kernel(BatchArgs<T> B, int nsteps) {
  __shared__ BatchLds<T, TX, TY> S;
  ChunkSync sync(B);
  const int i0 = sync.i0, i1 = sync.i1;
  for (int n = 0; n < nsteps; ++n) {
    batch_stage<T, 1, COMP, TX, TY>(B, i0, i1, S);
    if (!sync(B)) return;
    batch_stage<T, 2, COMP, TX, TY>(B, i0, i1, S);
    if (!sync(B)) return;
    batch_stage<T, 3, COMP, TX, TY>(B, i0, i1, S);
    if (!sync(B)) return;
    batch_stage<T, 4, COMP, TX, TY>(B, i0, i1, S);
    if (!sync(B)) return;
  }
}

// nsteps RK4 steps (nsteps even), two stage-pair passes each.  The second
// pass reads Psi on its tiles' rings, which neighbouring tiles are
// overwriting in the same pass, so the new Psi goes to the other of
// (caller's pool, bufA): odd steps read bufA and write the caller's pool,
// even steps the reverse, so the last step ends in the caller's pool.  (An
// odd step count starts with one step of batch2d_kernel, whose stage 4
// reads Psi at its own points only and writes it in place.)
template <typename T, int COMP, int TX, int TY>
__global__ __launch_bounds__(TX* TY) void batch2d_pair_kernel(BatchArgs<T> B, int nsteps) {
  __shared__ PairLds<T, TX, TY> S;
  ChunkSync sync(B);
  const int i0 = sync.i0, i1 = sync.i1;
  for (int n = 0; n < nsteps; ++n) {
    const bool odd = n & 1;
    batch_pair<T, 1, COMP, TX, TY>(B, i0, i1, S, odd, !odd);
    if (!sync(B)) return;
    batch_pair<T, 2, COMP, TX, TY>(B, i0, i1, S, odd, !odd);
    if (!sync(B)) return;
  }
}

template <typename T, int COMP>
static const void* kernel_ptr(int tx, int ty, int pairs) {
#define NLSE_KP(TX_, TY_)                                                                       \
  if (tx == TX_ && ty == TY_)                                                                   \
    return pairs ? reinterpret_cast<const void*>(&batch2d_pair_kernel<T, COMP, TX_, TY_>)       \
                 : reinterpret_cast<const void*>(&batch2d_kernel<T, COMP, TX_, TY_>);
  NLSE_KP(32, 8)
  NLSE_KP(64, 4)
  NLSE_KP(64, 8)
  NLSE_KP(128, 4)
  NLSE_KP(64, 16)
  NLSE_KP(32, 16)
  NLSE_KP(32, 32)
#undef NLSE_KP
  return nullptr;
}

template <typename T, int COMP>
static hipError_t launch_typed(const BatchLaunch& L, hipStream_t st) {
  if (L.pairs && (L.nsteps & 1)) return hipErrorInvalidValue;  // the pair kernel runs even step counts
  BatchArgs<T> B;
  B.items = L.items;
  B.chunk_off = L.chunk_off;
  B.psi = static_cast<cpx<T>*>(L.psi);
  B.vpool = static_cast<const T*>(L.vpool);
  B.vzero = static_cast<const T*>(L.vzero);
  B.acc = static_cast<cpx<T>*>(L.acc);
  B.bufA = static_cast<cpx<T>*>(L.bufA);
  B.bufB = static_cast<cpx<T>*>(L.bufB);
  B.lo = static_cast<cpx<T>*>(L.lo);
  B.flag = L.barrier + 1;
  B.arrivals = reinterpret_cast<unsigned long long*>(L.barrier + 2);
  B.spin_limit = L.spin_limit;
#define NLSE_LB(TX_, TY_)                                                                                          \
  if (L.tx == TX_ && L.ty == TY_) {                                                                                \
    if (L.pairs)                                                                                                   \
      hipLaunchKernelGGL((batch2d_pair_kernel<T, COMP, TX_, TY_>), dim3(L.nchunks), dim3(TX_ * TY_), 0, st, B,     \
                         L.nsteps);                                                                                \
    else                                                                                                           \
      hipLaunchKernelGGL((batch2d_kernel<T, COMP, TX_, TY_>), dim3(L.nchunks), dim3(TX_ * TY_), 0, st, B, L.nsteps); \
    return hipGetLastError();                                                                                      \
  }
  NLSE_LB(32, 8)
  NLSE_LB(64, 4)
  NLSE_LB(64, 8)
  NLSE_LB(128, 4)
  NLSE_LB(64, 16)
  NLSE_LB(32, 16)
  NLSE_LB(32, 32)
#undef NLSE_LB
  return hipErrorInvalidValue;
}

}  // namespace nlse

hipError_t nlse_launch_batch(const nlse::BatchLaunch& L, hipStream_t st) {
  if (L.dtype == 0) return L.comp ? nlse::launch_typed<float, 1>(L, st) : nlse::launch_typed<float, 0>(L, st);
  return nlse::launch_typed<double, 0>(L, st);
}

// Workgroups of the batched kernel with tile tx x ty (stage pairs or not)
// that one CU holds at once.
hipError_t nlse_batch_occupancy(int dtype, int comp, int tx, int ty, int pairs, int* blocks_per_cu) {
  const void* k = dtype == 0 ? (comp ? nlse::kernel_ptr<float, 1>(tx, ty, pairs) : nlse::kernel_ptr<float, 0>(tx, ty, pairs))
                             : nlse::kernel_ptr<double, 0>(tx, ty, pairs);
  if (!k) return hipErrorInvalidValue;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, tx * ty, 0);
}
