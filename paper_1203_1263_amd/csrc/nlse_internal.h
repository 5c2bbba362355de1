// Internal interfaces between the C-ABI layer (api.cpp) and the kernel
// translation units of libnlse.  Not installed; no HIP types in the public
// header.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nlse {

// Everything one stage launch needs.  Element pointers are device addresses
// of interleaved complex arrays of the grid's element type (dtype 0 = FP32,
// 1 = FP64); V is real or nullptr.
struct StageLaunch {
  int ndim, dtype, order, bc;
  int64_t n[3];
  const void* uin;
  const void* psi;
  void* acc;
  void* uout;
  void* lo;
  const void* V;
  const void* vzero;  // device zero of the element type, read when V is null
  int stage, comp;
  int stream;  // non-temporal own-point accesses (fields far larger than the last-level cache)
  double a, s, h;
  double c_acc, c_next;
  int tile[3];
};

// Mass / energy reduction over one grid.
struct ReduceLaunch {
  int ndim, dtype, order, bc;
  int64_t n[3];
  const void* psi;
  const void* V;
  double a, s, h;
  double* partials;  // >= reduce_blocks(npts) * 3 doubles
  void* dscratch;    // order 4: npts complex doubles for the stored 2SHOC D
  double* out;       // 3 doubles: sum rho, sum kinetic, sum potential
};

constexpr int kReduceChunk = 4096;  // points per reduction workgroup (fixed)

inline int64_t reduce_blocks(int64_t npts) { return (npts + kReduceChunk - 1) / kReduceChunk; }

// Reduction workgroups the library's static scratch holds partial sums for
// (nlse_mass_energy_noalloc): grids of at most kStaticReduceBlocks *
// kReduceChunk = 2^28 points.
constexpr int64_t kStaticReduceBlocks = (int64_t)1 << 16;

}  // namespace nlse

hipError_t nlse_launch_stage(const nlse::StageLaunch& L, hipStream_t st);
// One RK4 step of a 3D FP32 2SHOC grid as two fused launches (stages 1+2
// into acc and mid = U2, stages 3+4 into psi_out and lo); psi_out must not
// be psi_in.  L.tile[2] = z-chunk.
hipError_t nlse_launch_fused3d(const nlse::StageLaunch& L, const void* psi_in, void* psi_out, void* acc, void* mid,
                               void* lo, double dt, hipStream_t st);
// Only the first fused launch (reads psi, writes acc and mid): for timing.
hipError_t nlse_launch_fused3d_pair0(const nlse::StageLaunch& L, const void* psi, void* acc, void* mid, double dt,
                                     hipStream_t st);
// One stage pair of a 2D grid (pair 1: stages 1+2 from psi_in into acc and
// u2 = U2; pair 2: stages 3+4 from u2 into psi_out and lo); psi_out must not
// be psi_in.  L.tile = 32x32 or 64x16 (hipErrorInvalidValue otherwise).
hipError_t nlse_launch_pair2d(const nlse::StageLaunch& L, const void* psi_in, void* psi_out, void* acc, void* u2,
                              void* lo, double dt, int pair, hipStream_t st);
hipError_t nlse_launch_reduce(const nlse::ReduceLaunch& R, hipStream_t st);
// Device addresses, on the current device, of the library's static reduction
// scratch: kStaticReduceBlocks * 3 partial doubles and 3 result doubles
// (looked up once per device with hipGetSymbolAddress).
hipError_t nlse_static_reduce_scratch(double** partials, double** out);
// Whole-grid 1D integrator (one workgroup, grid on chip): nsteps RK4 steps of
// size dt in one launch, updating L.psi (and L.lo) in place; bitwise equal
// to the per-stage kernels.  Grids of 3 .. nlse_resident1d_max_points(dtype).
hipError_t nlse_launch_resident1d(const nlse::StageLaunch& L, int64_t nsteps, double dt, hipStream_t st);
int64_t nlse_resident1d_max_points(int dtype);
hipError_t nlse_launch_fill_zero(void* p, int64_t nbytes, hipStream_t st);
hipError_t nlse_launch_copy(void* dst, const void* src, int64_t nbytes, hipStream_t st);
extern "C" int nlse_internal_tile_supported(int ndim, int dtype, const int tile[3]);
