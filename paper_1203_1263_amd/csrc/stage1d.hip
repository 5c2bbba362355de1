// Fused RK4 stage kernel, 1D.  One launch is one RK4 stage over the grid: the
// stage input of a 256-point tile plus halo is staged in LDS, the 2SHOC
// temporary D (Eq. 2shoc1d) is formed in LDS on the tile plus one point each
// side, the Laplacian (CD2, or Eq. 2shoc1d2), F, the boundary forms (Eqs.
// BCDdt, BCDlap, msd, BCMSDlap, BCL0dt, BCL0lap) and the stage accumulation
// follow, and only
// the RK4 arrays touch HBM.
#include "stage_common.hpp"

namespace nlse {

template <typename T, int ORDER, int BC, int STAGE, int COMP, int TX>
__global__ __launch_bounds__(TX) void stage1d_kernel(StageArgs<T> A) {
  constexpr int H = ORDER == 4 ? 2 : 1;
  constexpr int BW = TX + 2 * H;
  constexpr int DW = TX + 2;
  __shared__ cpx<T> sU[BW];
  __shared__ cpx<T> sD[ORDER == 4 ? DW : 1];

  const int nx = A.nx;
  const int t = xcd_swizzle(blockIdx.x, gridDim.x);
  const int x0 = tile_origin(t, TX, nx);
  const int lx = threadIdx.x;
  const int x = x0 + lx;
  const bool valid = x < nx;
  const bool store = valid && x >= t * TX;
  const int xc = valid ? x : nx - 1;  // clamped: every load is in bounds
  // MSD boundary points evaluate F at their interior neighbour q themselves
  // (L0 needs only the point's own values)
  const bool bnd = valid && (x == 0 || x == nx - 1);
  const int qlx = lx + ((BC != kL0 && bnd) ? inward(x, nx) : 0);
  const Phys<T>& ph = A.ph;

  Own<T> own;
  load_own<T, STAGE, COMP>(A, xc, own);
  const T vq = vload(A, valid ? x0 + qlx : xc);

  for (int i = lx; i < BW; i += TX) {
    int gx = min(max(x0 - H + i, 0), nx - 1);
    sU[i] = A.uin[gx];
  }
  __syncthreads();

  if constexpr (ORDER == 4) {
    for (int i = lx; i < DW; i += TX) {
      int gx = x0 - 1 + i;
      int b = i + 1;  // position in sU
      cpx<T> d = czero<T>();
      if (gx >= 0 && gx < nx) {
        cpx<T> c = sU[b];
        if (gx != 0 && gx != nx - 1) {
          T sr = T(-0.0), si = T(-0.0);
          add_diff(sr, si, sU[b + 1], c);
          add_diff(sr, si, sU[b - 1], c);
          d = mk<T>(sr * ph.inv_h2, si * ph.inv_h2);
        } else if constexpr (BC != kL0) {  // L0: D_b = 0
          T Nb = nlin(ph, c, vload(A, gx));
          if (BC == kDirichlet) {
            d = dirichlet_lap(ph, c, Nb);
          } else {
            int q = inward(gx, nx);
            cpx<T> uq = sU[b + q];
            T sr = T(-0.0), si = T(-0.0);
            add_diff(sr, si, sU[b + q + 1], uq);
            add_diff(sr, si, sU[b + q - 1], uq);
            cpx<T> dq = mk<T>(sr * ph.inv_h2, si * ph.inv_h2);
            d = msd_lap(ph, dq, uq, nlin(ph, uq, vload(A, gx + q)), c, Nb);
          }
        }
      }
      sD[i] = d;
    }
    __syncthreads();
  }

  const cpx<T> u0 = sU[lx + H];
  const cpx<T> uq = sU[qlx + H];
  cpx<T> Kq = czero<T>();
  if (valid) {
    cpx<T> L;
    if constexpr (ORDER == 2) {
      T sr = T(-0.0), si = T(-0.0);
      add_diff(sr, si, sU[qlx + H + 1], uq);
      add_diff(sr, si, sU[qlx + H - 1], uq);
      L = mk<T>(sr * ph.inv_h2, si * ph.inv_h2);
    } else {
      cpx<T> D0 = sD[qlx + 1];
      T fr = T(-0.0), fi = T(-0.0);
      add_diff(fr, fi, sD[qlx + 2], D0);
      add_diff(fr, fi, sD[qlx], D0);
      L = shoc_combine<T, 1>(ph, D0, fr, fi, T(0), T(0));
    }
    Kq = rhs(ph, L, uq, nlin(ph, uq, vq));
  }
  cpx<T> K = Kq;
  if (bnd) {
    if constexpr (BC == kMSD) K = msd_rhs(Kq, uq, u0);
    else if constexpr (BC == kL0) K = l0_rhs(u0, nlin(ph, u0, vq));
    else K = czero<T>();
  }
  if (store) stage_update<T, STAGE, COMP>(A, x, u0, K, own);
}

template <typename T, int O, int B, int S, int C>
struct Launch1D {
  static hipError_t run(const StageLaunch& L, hipStream_t st) {
    if (L.tile[0] != 256) return hipErrorInvalidValue;
    StageArgs<T> A = make_args<T>(L);
    hipLaunchKernelGGL((stage1d_kernel<T, O, B, S, C, 256>), dim3(cdiv(L.n[0], 256)), dim3(256), 0, st, A);
    return hipGetLastError();
  }
};

}  // namespace nlse

hipError_t nlse_launch_stage_1d(const nlse::StageLaunch& L, hipStream_t st) {
  return nlse::dispatch_all<nlse::Launch1D>(L, st);
}
