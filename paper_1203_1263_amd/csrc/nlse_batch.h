// Internal structures of the batched persistent integrator (batch.hip and
// api_batch.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nlse {

// Tiles the batched kernel is compiled for (x-width, y-height; up to 1024
// threads, one per point); 32 x 8 is the default, the autotuner picks among
// all of them.
constexpr int kNumBatchTiles = 7;
constexpr int kBatchTiles[kNumBatchTiles][2] = {{32, 8}, {64, 4}, {64, 8}, {128, 4}, {64, 16}, {32, 16}, {32, 32}};

// One work item (a tile of one problem) as the device sees it: 256 bytes,
// read by the kernel as 64 dwords, one per lane.  The physical constants are
// the exact double values the single-grid path converts to the element type,
// and the same values rounded to FP32 on the host (round to nearest, as the
// device conversion does) for the FP32 kernels, so a problem computes the
// same bits alone or inside a batch.
struct BatchItem {
  double a, s, inv_a, inv_h2, inv_6h2;
  double dt, dt2, dt3, dt6;
  int64_t psi_off;  // complex elements into the caller's field pool
  int64_t v_off;    // real elements into the caller's potential pool, -1 = V == 0
  int64_t woff;     // complex elements into the work pools
  float af, sf, inv_af, inv_h2f, inv_6h2f;
  float dtf, dt2f, dt3f, dt6f;
  int nx, ny;
  int tx, ty;    // tile indices
  int scheme;    // order | bc << 8
  int sim;
  int pad[24];
};
static_assert(sizeof(BatchItem) == 256, "BatchItem is read as 64 dwords");

struct BatchLaunch {
  int dtype, comp, nsteps, nchunks;
  int tx, ty;  // tile (one of kBatchTiles)
  int pairs;   // 1: two stage-pair passes per step (Psi alternates with bufA
               // inside a launch; nsteps must be even), 0: four single-stage passes
  const BatchItem* items;
  const int* chunk_off;  // nchunks + 1 item offsets, then per chunk its group
                         // (-1: the chunk owns whole problems), then the group size
  void* psi;
  const void* vpool;
  const void* vzero;
  void *acc, *bufA, *bufB, *lo;
  unsigned* barrier;  // [1] sticky error flag; 64-bit arrival counters from byte 8
  unsigned spin_limit;
};

}  // namespace nlse

hipError_t nlse_launch_batch(const nlse::BatchLaunch& L, hipStream_t st);
hipError_t nlse_batch_occupancy(int dtype, int comp, int tx, int ty, int pairs, int* blocks_per_cu);
