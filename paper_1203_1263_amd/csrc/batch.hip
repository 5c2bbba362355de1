// Batched persistent RK4 integrator for many independent 2D problems of
// uneven size and parameters (a, s, V, h, dt, scheme, boundary condition).
//
// One launch advances every problem nsteps RK4 steps.  The launch is
// persistent: its grid is sized to what the device holds at once, and each
// workgroup owns a fixed, cost-balanced chunk of (problem, tile) work items
// computed on the host.  For every stage a workgroup runs the 2D tile body of
// the single-grid kernel (tile2d.hpp) on each of its items, then all
// workgroups meet at a grid-wide barrier before the next stage (a stage of a
// problem reads the previous stage of its neighbouring tiles).  The barrier
// is a monotonically increasing arrival counter with a bounded wait: a wait
// that exceeds the spin limit raises an error flag and every workgroup then
// leaves the kernel, so the grid always drains.
#include "nlse_batch.h"
#include "tile2d.hpp"

namespace nlse {

template <typename T>
struct BatchArgs {
  const BatchSim* sims;
  const BatchItem* items;
  const int* chunk_off;  // items of chunk c: [chunk_off[c], chunk_off[c+1])
  cpx<T>* psi;           // caller's pool
  const T* vpool;        // caller's potential pool (may be null)
  const T* vzero;        // one zero element
  cpx<T>* acc;           // work pools, indexed by BatchSim::woff
  cpx<T>* bufA;
  cpx<T>* bufB;
  cpx<T>* lo;
  unsigned* barrier;     // [0] arrival counter, [1] error flag
  unsigned spin_limit;
};

// Grid-wide barrier number `k` (1, 2, ...): every workgroup adds one arrival
// and waits for k * gridDim.x arrivals.  Device-scope release before the
// arrival and acquire after it make the stage's stores visible to every
// workgroup.  Returns false if the wait timed out or another workgroup
// reported an error.
__device__ __forceinline__ bool grid_barrier(unsigned* bar, unsigned k, unsigned spin_limit) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  __shared__ int ok;
  if (threadIdx.x == 0) {
    const unsigned target = k * gridDim.x;
    __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    unsigned spins = 0;
    int good = 1;
    // poll with relaxed loads (an acquire per poll would invalidate the
    // CU's L1 under the workgroups still computing); acquire once below
    while (__hip_atomic_load(&bar[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u || ++spins > spin_limit) {
        good = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    if (!good) __hip_atomic_store(&bar[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    ok = good;
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return ok != 0;
}

template <typename T, int STAGE>
__device__ __forceinline__ StageArgs<T> sim_args(const BatchArgs<T>& B, const BatchSim& d) {
  StageArgs<T> A;
  cpx<T>* psi = B.psi + d.psi_off;
  cpx<T>* a = B.bufA + d.woff;
  cpx<T>* b = B.bufB + d.woff;
  A.uin = STAGE == 1 ? psi : (STAGE == 2 ? a : (STAGE == 3 ? b : a));
  A.uout = STAGE == 1 ? a : (STAGE == 2 ? b : (STAGE == 3 ? a : psi));
  A.psi = psi;
  A.acc = B.acc + d.woff;
  A.lo = B.lo ? B.lo + d.woff : nullptr;
  A.V = d.v_off >= 0 ? B.vpool + d.v_off : B.vzero;
  A.vs = d.v_off >= 0 ? 1 : 0;
  A.nx = d.nx;
  A.ny = d.ny;
  A.nz = 1;
  A.ph.a = (T)d.a;
  A.ph.s = (T)d.s;
  A.ph.inv_a = (T)d.inv_a;
  A.ph.inv_h2 = (T)d.inv_h2;
  A.ph.inv_6h2 = (T)d.inv_6h2;
  const double ca = (STAGE == 1 || STAGE == 4) ? d.dt6 : d.dt3;
  const double cn = STAGE == 3 ? d.dt : d.dt2;
  A.c_acc = (T)ca;
  A.c_next = (T)cn;
  A.c_acc_d = ca;
  return A;
}

template <typename T, int STAGE, int COMP>
__device__ __forceinline__ void run_item(const BatchArgs<T>& B, const BatchItem& w, cpx<T>* sU, cpx<T>* sD) {
  const BatchSim d = B.sims[w.sim];
  const StageArgs<T> A = sim_args<T, STAGE>(B, d);
  if (d.order == 4) {
    if (d.bc == kMSD)
      tile2d<T, 4, kMSD, STAGE, COMP, kBatchTX, kBatchTY>(A, w.tx, w.ty, sU, sD);
    else
      tile2d<T, 4, kDirichlet, STAGE, COMP, kBatchTX, kBatchTY>(A, w.tx, w.ty, sU, sD);
  } else {
    if (d.bc == kMSD)
      tile2d<T, 2, kMSD, STAGE, COMP, kBatchTX, kBatchTY>(A, w.tx, w.ty, sU, sD);
    else
      tile2d<T, 2, kDirichlet, STAGE, COMP, kBatchTX, kBatchTY>(A, w.tx, w.ty, sU, sD);
  }
}

template <typename T, int COMP>
__global__ __launch_bounds__(kBatchTX* kBatchTY) void batch2d_kernel(BatchArgs<T> B, int nsteps) {
  __shared__ cpx<T> sU[(kBatchTY + 4) * (kBatchTX + 4)];
  __shared__ cpx<T> sD[(kBatchTY + 2) * (kBatchTX + 2)];
  const int c = xcd_swizzle(blockIdx.x, gridDim.x);
  const int i0 = B.chunk_off[c], i1 = B.chunk_off[c + 1];
  unsigned k = 0;
  for (int n = 0; n < nsteps; ++n) {
    for (int stage = 1; stage <= 4; ++stage) {
      for (int it = i0; it < i1; ++it) {
        const BatchItem w = B.items[it];
        __syncthreads();  // the previous item's LDS reads are done
        switch (stage) {
          case 1: run_item<T, 1, COMP>(B, w, sU, sD); break;
          case 2: run_item<T, 2, COMP>(B, w, sU, sD); break;
          case 3: run_item<T, 3, COMP>(B, w, sU, sD); break;
          default: run_item<T, 4, COMP>(B, w, sU, sD); break;
        }
      }
      if (!grid_barrier(B.barrier, ++k, B.spin_limit)) return;
    }
  }
}

template <typename T, int COMP>
static const void* kernel_ptr() {
  return reinterpret_cast<const void*>(&batch2d_kernel<T, COMP>);
}

template <typename T, int COMP>
static hipError_t launch_typed(const BatchLaunch& L, hipStream_t st) {
  BatchArgs<T> B;
  B.sims = L.sims;
  B.items = L.items;
  B.chunk_off = L.chunk_off;
  B.psi = static_cast<cpx<T>*>(L.psi);
  B.vpool = static_cast<const T*>(L.vpool);
  B.vzero = static_cast<const T*>(L.vzero);
  B.acc = static_cast<cpx<T>*>(L.acc);
  B.bufA = static_cast<cpx<T>*>(L.bufA);
  B.bufB = static_cast<cpx<T>*>(L.bufB);
  B.lo = static_cast<cpx<T>*>(L.lo);
  B.barrier = L.barrier;
  B.spin_limit = L.spin_limit;
  hipLaunchKernelGGL((batch2d_kernel<T, COMP>), dim3(L.nchunks), dim3(kBatchTX * kBatchTY), 0, st, B, L.nsteps);
  return hipGetLastError();
}

}  // namespace nlse

hipError_t nlse_launch_batch(const nlse::BatchLaunch& L, hipStream_t st) {
  if (L.dtype == 0) return L.comp ? nlse::launch_typed<float, 1>(L, st) : nlse::launch_typed<float, 0>(L, st);
  return nlse::launch_typed<double, 0>(L, st);
}

// Workgroups of the batched kernel that one CU holds at once.
hipError_t nlse_batch_occupancy(int dtype, int comp, int* blocks_per_cu) {
  const void* k = dtype == 0 ? (comp ? nlse::kernel_ptr<float, 1>() : nlse::kernel_ptr<float, 0>())
                             : nlse::kernel_ptr<double, 0>();
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, nlse::kBatchTX * nlse::kBatchTY, 0);
}
