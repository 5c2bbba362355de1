// Fused RK4 stage kernel, 2D: one workgroup = one TX x TY tile (tile body in
// tile2d.hpp), tiles mapped XCD-aware.
#include <type_traits>

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

// One stage pair (PAIR 1: stages 1+2, PAIR 2: stages 3+4) of one tile per
// workgroup (pair body in tile2d.hpp); the boundary condition is a run-time
// value, which keeps one kernel per (type, scheme, pair, tile).
template <typename T, int ORDER, int PAIR, int COMP, int TX, int TY, bool STREAM>
__global__ __launch_bounds__(TX* TY) void pair2d_kernel(PairArgs<T> A, int bc) {
  constexpr int H = ORDER == 4 ? 2 : 1;
  __shared__ cpx<T> sU[(TX + 4 * H) * (TY + 4 * H)];
  __shared__ T sV[(TX + 4 * H) * (TY + 4 * H)];
  __shared__ cpx<T> sD[ORDER == 4 ? (TX + 2 * H + 2) * (TY + 2 * H + 2) : 1];
  __shared__ cpx<T> sM[(TX + 2 * H) * (TY + 2 * H)];
  const int ntx = (A.nx + TX - 1) / TX;
  const int t = xcd_swizzle(blockIdx.x, gridDim.x);
  PairRegs<T, TX, TY> R;
  pair2d_load<T, PAIR, COMP, TX, TY, H, STREAM>(A, t % ntx, t / ntx, R);
  pair2d_compute<T, ORDER, kAnyBC, PAIR, COMP, TX, TY, STREAM>(A, t % ntx, t / ntx, R, sU, sV, sD, sM, bc, false,
                                                                [] {});
}

template <typename T, int COMP>
static hipError_t launch_pair2d_typed(const StageLaunch& L, const void* psi_in, void* psi_out, void* acc, void* u2,
                                      void* lo, double dt, int pair, hipStream_t st) {
  PairArgs<T> A;
  const StageArgs<T> S = make_args<T>(L);
  A.uin = static_cast<const cpx<T>*>(pair == 1 ? psi_in : u2);
  A.psi = static_cast<const cpx<T>*>(psi_in);
  A.acc = static_cast<cpx<T>*>(acc);
  A.out = static_cast<cpx<T>*>(pair == 1 ? u2 : psi_out);
  A.lo = static_cast<cpx<T>*>(lo);
  A.V = S.V;
  A.vs = S.vs;
  A.nx = S.nx;
  A.ny = S.ny;
  A.ph = S.ph;
  // the coefficients of the four single-stage launches, converted on the
  // host as they are
  A.ca1 = (T)(pair == 1 ? dt / 6.0 : dt / 3.0);
  A.cn1 = (T)(pair == 1 ? dt / 2.0 : dt);
  A.ca2 = (T)(pair == 1 ? dt / 3.0 : dt / 6.0);
  A.cn2 = (T)(dt / 2.0);
  A.ca2_d = pair == 1 ? dt / 3.0 : dt / 6.0;
  const int tx = L.tile[0], ty = L.tile[1];
  const int nb = cdiv(L.n[0], tx) * cdiv(L.n[1], ty);
#define NLSE_P2(TX_, TY_)                                                                                    \
  if (tx == TX_ && ty == TY_) {                                                                              \
    auto go = [&](auto o, auto p, auto s) {                                                                  \
      hipLaunchKernelGGL((pair2d_kernel<T, decltype(o)::value, decltype(p)::value, COMP, TX_, TY_,           \
                                        decltype(s)::value>),                                                \
                         dim3(nb), dim3(TX_ * TY_), 0, st, A, L.bc);                                         \
    };                                                                                                       \
    using O2 = std::integral_constant<int, 2>;                                                               \
    using O4 = std::integral_constant<int, 4>;                                                               \
    using P1 = std::integral_constant<int, 1>;                                                               \
    using P2 = std::integral_constant<int, 2>;                                                               \
    auto by_stream = [&](auto o, auto p) {                                                                   \
      if (L.stream) go(o, p, std::true_type{});                                                              \
      else go(o, p, std::false_type{});                                                                      \
    };                                                                                                       \
    auto by_pair = [&](auto o) {                                                                             \
      if (pair == 1) by_stream(o, P1{});                                                                     \
      else by_stream(o, P2{});                                                                               \
    };                                                                                                       \
    if (L.order == 4) by_pair(O4{});                                                                         \
    else by_pair(O2{});                                                                                      \
    return hipGetLastError();                                                                                \
  }
  NLSE_P2(32, 32)
  NLSE_P2(64, 16)
#undef NLSE_P2
  return hipErrorInvalidValue;
}

}  // namespace nlse

hipError_t nlse_launch_stage_2d(const nlse::StageLaunch& L, hipStream_t st) {
  return nlse::dispatch_all<nlse::Launch2D>(L, st);
}

hipError_t nlse_launch_pair2d(const nlse::StageLaunch& L, const void* psi_in, void* psi_out, void* acc, void* u2,
                              void* lo, double dt, int pair, hipStream_t st) {
  if ((pair != 1 && pair != 2) || psi_in == psi_out) return hipErrorInvalidValue;
  if (L.bc != nlse::kDirichlet && L.bc != nlse::kMSD && L.bc != nlse::kL0) return hipErrorInvalidValue;
  if (L.dtype == 0)
    return L.comp ? nlse::launch_pair2d_typed<float, 1>(L, psi_in, psi_out, acc, u2, lo, dt, pair, st)
                  : nlse::launch_pair2d_typed<float, 0>(L, psi_in, psi_out, acc, u2, lo, dt, pair, st);
  return nlse::launch_pair2d_typed<double, 0>(L, psi_in, psi_out, acc, u2, lo, dt, pair, st);
}
