// Fused RK4 stage kernel, 2D: one workgroup = one TX x TY tile (tile body in
// tile2d.hpp), tiles mapped XCD-aware.
#include "tile2d.hpp"

namespace nlse {

template <typename T, int ORDER, int BC, int STAGE, int COMP, int TX, int TY, bool STREAM>
__global__ __launch_bounds__(TX* TY) void stage2d_kernel(StageArgs<T> A) {
  __shared__ TileLds<T, TX, TY, ORDER == 4 ? 2 : 1> S;
  const int ntx = (A.nx + TX - 1) / TX;
  const int t = xcd_swizzle(blockIdx.x, gridDim.x);
  tile2d<T, ORDER, BC, STAGE, COMP, TX, TY, STREAM>(A, t % ntx, t / ntx, S);
}

template <typename T, int O, int B, int S, int C>
struct Launch2D {
  static hipError_t run(const StageLaunch& L, hipStream_t st) {
    StageArgs<T> A = make_args<T>(L);
    const int tx = L.tile[0], ty = L.tile[1];
    const int nb = cdiv(L.n[0], tx) * cdiv(L.n[1], ty);
#define NLSE_L2(TX_, TY_)                                                                                      \
  if (tx == TX_ && ty == TY_) {                                                                                \
    if (L.stream)                                                                                              \
      hipLaunchKernelGGL((stage2d_kernel<T, O, B, S, C, TX_, TY_, true>), dim3(nb), dim3(TX_ * TY_), 0, st, A);  \
    else                                                                                                       \
      hipLaunchKernelGGL((stage2d_kernel<T, O, B, S, C, TX_, TY_, false>), dim3(nb), dim3(TX_ * TY_), 0, st, A); \
    return hipGetLastError();                                                                                  \
  }
    NLSE_L2(32, 8)
    NLSE_L2(64, 4)
    NLSE_L2(64, 8)
    NLSE_L2(128, 4)
    NLSE_L2(64, 16)
    NLSE_L2(32, 16)
    NLSE_L2(32, 32)
#undef NLSE_L2
    return hipErrorInvalidValue;
  }
};

}  // namespace nlse

hipError_t nlse_launch_stage_2d(const nlse::StageLaunch& L, hipStream_t st) {
  return nlse::dispatch_all<nlse::Launch2D>(L, st);
}
