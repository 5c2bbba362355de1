// Whole-grid 1D integrator for small grids (up to 1024 FP64 / 2048 FP32
// points).  Four kernel launches per RK4 step cost more than the arithmetic
// of a grid this small, so one workgroup keeps the whole grid on chip and
// runs every stage of nsteps steps in one launch: the stage input and the
// 2SHOC temporary D (Eq. 2shoc1d) live in LDS, the own-point RK4 state (Psi,
// the accumulator, Psi_lo) in registers, and workgroup barriers stand in for
// the launches between stages.  The stencil, boundary forms (Eqs. BCDdt,
// BCDlap, msd, BCMSDlap, BCL0dt, BCL0lap) and stage update (Eq. RK4 in the
// four-pass order) are the same helper functions, applied to the same values
// in the same order, as in the per-stage 1D kernel, so both give the same
// bits.
#include "stage_common.hpp"

namespace nlse {

constexpr int kResThreads = 1024;

template <typename T>
struct ResArgs {
  cpx<T>* psi;  // field, updated in place at the end
  cpx<T>* lo;   // compensation term (compensated FP32 only)
  const T* V;   // potential, or a one-element zero array with vs = 0
  int64_t vs;
  int nx;
  Phys<T> ph;
  T ca[4], cn[4];  // per-stage k/6, k/3, k/3, k/6 and k/2, k/2, k, 0
  double ca4_d;    // k/6 in FP64 (compensated stage 4)
};

template <typename T, int ORDER, int BC, int COMP, int PPT>
__global__ __launch_bounds__(kResThreads) void resident1d_kernel(ResArgs<T> A, int64_t nsteps) {
  constexpr int NMAX = kResThreads * PPT;
  __shared__ cpx<T> sU[2][NMAX];                // stage input / output (ping-pong)
  __shared__ cpx<T> sD[ORDER == 4 ? NMAX : 1];  // 2SHOC step 1
  __shared__ T sV[NMAX];
  const int nx = A.nx;
  const int tid = threadIdx.x;
  const Phys<T>& ph = A.ph;

  // thread tid owns points tid, tid + 1024, ... (consecutive lanes, consecutive points)
  cpx<T> psi[PPT], acc[PPT], lo[PPT];
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int i = tid + k * kResThreads;
    psi[k] = acc[k] = lo[k] = czero<T>();
    if (i < nx) {
      psi[k] = A.psi[i];
      if constexpr (COMP) lo[k] = A.lo[i];
      sU[0][i] = psi[k];
      sV[i] = A.V[i * A.vs];
    }
  }
  __syncthreads();

  int b = 0;
  auto stage = [&](auto stage_tag) {
    constexpr int S = decltype(stage_tag)::value;
    const cpx<T>* U = sU[b];
    cpx<T>* O = sU[b ^ 1];
    if constexpr (ORDER == 4) {
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        const int i = tid + k * kResThreads;
        if (i >= nx) continue;
        const cpx<T> c = U[i];
        cpx<T> d = czero<T>();
        if (i != 0 && i != nx - 1) {
          T sr = T(-0.0), si = T(-0.0);
          add_diff(sr, si, U[i + 1], c);
          add_diff(sr, si, U[i - 1], c);
          d = mk<T>(sr * ph.inv_h2, si * ph.inv_h2);
        } else if constexpr (BC != kL0) {  // L0: D_b = 0
          const T Nb = nlin(ph, c, sV[i]);
          if (BC == kDirichlet) {
            d = dirichlet_lap(ph, c, Nb);
          } else {
            const int q = i + inward(i, nx);
            const cpx<T> uq = U[q];
            T sr = T(-0.0), si = T(-0.0);
            add_diff(sr, si, U[q + 1], uq);
            add_diff(sr, si, U[q - 1], uq);
            const cpx<T> dq = mk<T>(sr * ph.inv_h2, si * ph.inv_h2);
            d = msd_lap(ph, dq, uq, nlin(ph, uq, sV[q]), c, Nb);
          }
        }
        sD[i] = d;
      }
      __syncthreads();
    }
    const T ca = A.ca[S - 1], cn = A.cn[S - 1];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const int i = tid + k * kResThreads;
      if (i >= nx) continue;
      const bool bnd = (i == 0 || i == nx - 1);
      const cpx<T> u0 = U[i];
      cpx<T> K = czero<T>();
      if (bnd && BC == kL0) {
        K = l0_rhs(u0, nlin(ph, u0, sV[i]));
      } else if (!bnd || BC == kMSD) {
        // F at the point itself, or for an MSD boundary point at its
        // interior neighbour q
        const int q = i + (bnd ? inward(i, nx) : 0);
        const cpx<T> uq = U[q];
        cpx<T> L;
        if constexpr (ORDER == 2) {
          T sr = T(-0.0), si = T(-0.0);
          add_diff(sr, si, U[q + 1], uq);
          add_diff(sr, si, U[q - 1], uq);
          L = mk<T>(sr * ph.inv_h2, si * ph.inv_h2);
        } else {
          const cpx<T> D0 = sD[q];
          T fr = T(-0.0), fi = T(-0.0);
          add_diff(fr, fi, sD[q + 1], D0);
          add_diff(fr, fi, sD[q - 1], D0);
          L = shoc_combine<T, 1>(ph, D0, fr, fi, T(0), T(0));
        }
        const cpx<T> Kq = rhs(ph, L, uq, nlin(ph, uq, sV[q]));
        K = bnd ? msd_rhs(Kq, uq, u0) : Kq;
      }  // Dirichlet boundary: K = 0
      // the stage update of the four-pass kernels, on registers
      if constexpr (S == 1) {
        acc[k] = COMP ? mk<T>(ca * K.re, ca * K.im) : mk<T>(fmaT(ca, K.re, u0.re), fmaT(ca, K.im, u0.im));
        O[i] = mk<T>(fmaT(cn, K.re, u0.re), fmaT(cn, K.im, u0.im));
      } else if constexpr (S == 2 || S == 3) {
        acc[k] = mk<T>(fmaT(ca, K.re, acc[k].re), fmaT(ca, K.im, acc[k].im));
        O[i] = mk<T>(fmaT(cn, K.re, psi[k].re), fmaT(cn, K.im, psi[k].im));
      } else if constexpr (!COMP) {
        psi[k] = mk<T>(fmaT(ca, K.re, acc[k].re), fmaT(ca, K.im, acc[k].im));
        O[i] = psi[k];
      } else {
        const double inc_r = __builtin_fma(A.ca4_d, (double)K.re, (double)acc[k].re);
        const double inc_i = __builtin_fma(A.ca4_d, (double)K.im, (double)acc[k].im);
        const double sr = ((double)psi[k].re + (double)lo[k].re) + inc_r;
        const double si = ((double)psi[k].im + (double)lo[k].im) + inc_i;
        const T hr = (T)sr, hi = (T)si;
        psi[k] = mk<T>(hr, hi);
        lo[k] = mk<T>((T)(sr - (double)hr), (T)(si - (double)hi));
        O[i] = psi[k];
      }
    }
    __syncthreads();  // O complete; every read of U and D of this stage done
    b ^= 1;
  };
  for (int64_t n = 0; n < nsteps; ++n) {
    stage(std::integral_constant<int, 1>{});
    stage(std::integral_constant<int, 2>{});
    stage(std::integral_constant<int, 3>{});
    stage(std::integral_constant<int, 4>{});
  }
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int i = tid + k * kResThreads;
    if (i < nx) {
      A.psi[i] = psi[k];
      if constexpr (COMP) A.lo[i] = lo[k];
    }
  }
}

template <typename T, int ORDER, int BC, int COMP>
hipError_t launch_resident(const ResArgs<T>& A, int64_t nsteps, hipStream_t st) {
  if (A.nx <= kResThreads) {
    hipLaunchKernelGGL((resident1d_kernel<T, ORDER, BC, COMP, 1>), dim3(1), dim3(kResThreads), 0, st, A, nsteps);
  } else {
    if constexpr (std::is_same<T, float>::value) {
      if (A.nx > 2 * kResThreads) return hipErrorInvalidValue;
      hipLaunchKernelGGL((resident1d_kernel<T, ORDER, BC, COMP, 2>), dim3(1), dim3(kResThreads), 0, st, A, nsteps);
    } else {
      return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

template <typename T, int COMP>
hipError_t resident_typed(const StageLaunch& L, int64_t nsteps, double dt, hipStream_t st) {
  ResArgs<T> A;
  A.psi = static_cast<cpx<T>*>(const_cast<void*>(L.psi));
  A.lo = static_cast<cpx<T>*>(L.lo);
  A.V = static_cast<const T*>(L.V ? L.V : L.vzero);
  A.vs = L.V ? 1 : 0;
  A.nx = (int)L.n[0];
  // the same conversions as the per-stage launches
  A.ph.a = (T)L.a;
  A.ph.s = (T)L.s;
  A.ph.inv_a = (T)(1.0 / L.a);
  A.ph.inv_h2 = (T)(1.0 / (L.h * L.h));
  A.ph.inv_6h2 = (T)(1.0 / (6.0 * L.h * L.h));
  const double ca[4] = {dt / 6.0, dt / 3.0, dt / 3.0, dt / 6.0};
  const double cn[4] = {dt / 2.0, dt / 2.0, dt, 0.0};
  for (int s = 0; s < 4; ++s) {
    A.ca[s] = (T)ca[s];
    A.cn[s] = (T)cn[s];
  }
  A.ca4_d = dt / 6.0;
  if (L.order == 4) {
    if (L.bc == kMSD) return launch_resident<T, 4, kMSD, COMP>(A, nsteps, st);
    if (L.bc == kL0) return launch_resident<T, 4, kL0, COMP>(A, nsteps, st);
    return launch_resident<T, 4, kDirichlet, COMP>(A, nsteps, st);
  }
  if (L.bc == kMSD) return launch_resident<T, 2, kMSD, COMP>(A, nsteps, st);
  if (L.bc == kL0) return launch_resident<T, 2, kL0, COMP>(A, nsteps, st);
  return launch_resident<T, 2, kDirichlet, COMP>(A, nsteps, st);
}

}  // namespace nlse

int64_t nlse_resident1d_max_points(int dtype) { return dtype == 0 ? 2 * nlse::kResThreads : nlse::kResThreads; }

hipError_t nlse_launch_resident1d(const nlse::StageLaunch& L, int64_t nsteps, double dt, hipStream_t st) {
  if (L.ndim != 1 || L.n[0] < 3 || L.n[0] > nlse_resident1d_max_points(L.dtype) || nsteps < 0)
    return hipErrorInvalidValue;
  if (L.bc != nlse::kDirichlet && L.bc != nlse::kMSD && L.bc != nlse::kL0) return hipErrorInvalidValue;
  if (nsteps == 0) return hipSuccess;
  if (L.dtype == 0)
    return L.comp ? nlse::resident_typed<float, 1>(L, nsteps, dt, st) : nlse::resident_typed<float, 0>(L, nsteps, dt, st);
  return nlse::resident_typed<double, 0>(L, nsteps, dt, st);
}
