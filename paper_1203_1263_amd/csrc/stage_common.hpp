// Helpers shared by the 1D/2D/3D stage kernels: difference-form stencil
// pieces, argument packing and the compile-time dispatch over element type,
// scheme, boundary condition, RK4 stage and compensation mode.
#pragma once

#include <type_traits>

#include "nlse_device.hpp"
#include "nlse_internal.h"

namespace nlse {

// 2SHOC step 2 in difference form:
//   L = c0 D0 - (1/12) sum_faces (D_f - D0) + 1/(6h^2) sum_edges (u_e - u0)
// with c0 = 1, 2/3, 1/3 in 1D, 2D, 3D (the centre weights 14, 12, 10 of the
// paper's step-2 stencils minus the face count 2d, divided by -12).
template <typename T, int DIM>
__device__ __forceinline__ cpx<T> shoc_combine(const Phys<T>& p, cpx<T> D0, T fr, T fi, T er, T ei) {
  constexpr double c0d = DIM == 1 ? 1.0 : (DIM == 2 ? 2.0 / 3.0 : 1.0 / 3.0);
  const T c0 = T(c0d);
  const T m12 = T(-1.0 / 12.0);
  return mk<T>(fmaT(c0, D0.re, fmaT(m12, fr, p.inv_6h2 * er)), fmaT(c0, D0.im, fmaT(m12, fi, p.inv_6h2 * ei)));
}

// Sums of differences start at -0: -0 + x == x exactly for every x, so the
// compiler drops the first addition without fast-math.
template <typename T>
__device__ __forceinline__ void add_diff(T& sr, T& si, cpx<T> v, cpx<T> c) {
  sr += v.re - c.re;
  si += v.im - c.im;
}

template <typename T>
inline StageArgs<T> make_args(const StageLaunch& L) {
  StageArgs<T> A;
  A.uin = static_cast<const cpx<T>*>(L.uin);
  A.psi = static_cast<const cpx<T>*>(L.psi);
  A.acc = static_cast<cpx<T>*>(L.acc);
  A.uout = static_cast<cpx<T>*>(L.uout);
  A.lo = static_cast<cpx<T>*>(L.lo);
  A.V = static_cast<const T*>(L.V ? L.V : L.vzero);
  A.vs = L.V ? 1 : 0;
  A.nx = (int)L.n[0];
  A.ny = (int)L.n[1];
  A.nz = (int)L.n[2];
  A.ph.a = (T)L.a;
  A.ph.s = (T)L.s;
  A.ph.inv_a = (T)(1.0 / L.a);
  A.ph.inv_h2 = (T)(1.0 / (L.h * L.h));
  A.ph.inv_6h2 = (T)(1.0 / (6.0 * L.h * L.h));
  A.c_acc = (T)L.c_acc;
  A.c_next = (T)L.c_next;
  A.c_acc_d = L.c_acc;
  return A;
}

inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// F<T, ORDER, BC, STAGE, COMP>::run(L, stream) for the values in L.
// Compensation exists for FP32 only.
template <typename T, int O, int B, template <typename, int, int, int, int> class F>
hipError_t dispatch_stage(const StageLaunch& L, hipStream_t st) {
  if constexpr (std::is_same<T, float>::value) {
    if (L.comp) {
      switch (L.stage) {
        case 1: return F<T, O, B, 1, 1>::run(L, st);
        case 2: return F<T, O, B, 2, 1>::run(L, st);
        case 3: return F<T, O, B, 3, 1>::run(L, st);
        case 4: return F<T, O, B, 4, 1>::run(L, st);
        default: return hipErrorInvalidValue;
      }
    }
  }
  switch (L.stage) {
    case 1: return F<T, O, B, 1, 0>::run(L, st);
    case 2: return F<T, O, B, 2, 0>::run(L, st);
    case 3: return F<T, O, B, 3, 0>::run(L, st);
    case 4: return F<T, O, B, 4, 0>::run(L, st);
    default: return hipErrorInvalidValue;
  }
}

template <template <typename, int, int, int, int> class F>
hipError_t dispatch_all(const StageLaunch& L, hipStream_t st) {
  if (L.bc != kDirichlet && L.bc != kMSD && L.bc != kL0) return hipErrorInvalidValue;
  const int k = (L.dtype ? 6 : 0) + (L.order == 4 ? 3 : 0) + L.bc;
  switch (k) {
    case 0: return dispatch_stage<float, 2, kDirichlet, F>(L, st);
    case 1: return dispatch_stage<float, 2, kMSD, F>(L, st);
    case 2: return dispatch_stage<float, 2, kL0, F>(L, st);
    case 3: return dispatch_stage<float, 4, kDirichlet, F>(L, st);
    case 4: return dispatch_stage<float, 4, kMSD, F>(L, st);
    case 5: return dispatch_stage<float, 4, kL0, F>(L, st);
    case 6: return dispatch_stage<double, 2, kDirichlet, F>(L, st);
    case 7: return dispatch_stage<double, 2, kMSD, F>(L, st);
    case 8: return dispatch_stage<double, 2, kL0, F>(L, st);
    case 9: return dispatch_stage<double, 4, kDirichlet, F>(L, st);
    case 10: return dispatch_stage<double, 4, kMSD, F>(L, st);
    default: return dispatch_stage<double, 4, kL0, F>(L, st);
  }
}

}  // namespace nlse
