// The 2D stage tile body shared by the single-grid 2D stage kernel and the
// batched persistent kernel, so a simulation computes the same bits whether
// it runs alone or inside a batch.
//
// One TX x TY tile: the stage input of the tile plus a 1-cell (CD2) or 2-cell
// (2SHOC) halo is staged in LDS, D (Eq. 2d2shocs1) is formed in LDS on the
// tile plus a one-cell ring, then the Laplacian (CD2, or Eq. 2d2shocs2), F,
// the boundary forms (Eqs. BCDdt, BCDlap, msd, BCMSDlap) and the stage
// accumulation follow.  Loads are coalesced along x; every load address is
// clamped into the grid so the memory operations are straight-line code.
#pragma once

#include "stage_common.hpp"

namespace nlse {

// One TX x TY tile (tile indices tx, ty) of one RK4 stage.  Called by the
// single-grid kernel below and by the batched persistent kernel; sU and sD
// are the workgroup's LDS buffers ((TY+2H)(TX+2H) and (TY+2)(TX+2) points).
// Contains barriers: every thread of the workgroup must call it.
template <typename T, int ORDER, int BC, int STAGE, int COMP, int TX, int TY>
__device__ __forceinline__ void tile2d(const StageArgs<T>& A, int tx, int ty, cpx<T>* __restrict__ sU,
                                       cpx<T>* __restrict__ sD) {
  constexpr int NT = TX * TY;
  constexpr int H = ORDER == 4 ? 2 : 1;
  constexpr int BW = TX + 2 * H, BH = TY + 2 * H;
  constexpr int DW = TX + 2, DH = TY + 2;

  const int nx = A.nx, ny = A.ny;
  const int x0 = tile_origin(tx, TX, nx), y0 = tile_origin(ty, TY, ny);
  const int tid = threadIdx.x, lx = tid % TX, ly = tid / TX;
  const int x = x0 + lx, y = y0 + ly;
  const bool valid = x < nx && y < ny;
  const bool store = valid && x >= tx * TX && y >= ty * TY;
  const int64_t idx = (int64_t)min(y, ny - 1) * nx + min(x, nx - 1);  // clamped
  // MSD boundary points evaluate F at their interior neighbour q themselves
  const bool bnd = valid && (x == 0 || x == nx - 1 || y == 0 || y == ny - 1);
  const int qlx = lx + (bnd ? inward(x, nx) : 0), qly = ly + (bnd ? inward(y, ny) : 0);
  const int64_t qidx = valid ? (int64_t)(y0 + qly) * nx + (x0 + qlx) : idx;
  const Phys<T>& ph = A.ph;

  Own<T> own;
  load_own<T, STAGE, COMP>(A, idx, own);
  const T vq = vload(A, qidx);

  for (int i = tid; i < BW * BH; i += NT) {
    int r = i / BW, c = i - r * BW;
    int gx = min(max(x0 - H + c, 0), nx - 1), gy = min(max(y0 - H + r, 0), ny - 1);
    sU[i] = A.uin[(int64_t)gy * nx + gx];
  }
  __syncthreads();

  auto U = [&](int r, int c) -> cpx<T> { return sU[r * BW + c]; };
  auto cd2 = [&](int r, int c) -> cpx<T> {
    cpx<T> u = U(r, c);
    T sr = T(0), si = T(0);
    add_diff(sr, si, U(r, c + 1), u);
    add_diff(sr, si, U(r, c - 1), u);
    add_diff(sr, si, U(r + 1, c), u);
    add_diff(sr, si, U(r - 1, c), u);
    return mk<T>(sr * ph.inv_h2, si * ph.inv_h2);
  };

  if constexpr (ORDER == 4) {
    for (int i = tid; i < DW * DH; i += NT) {
      int r = i / DW, c = i - r * DW;
      int gx = x0 - 1 + c, gy = y0 - 1 + r;
      int br = r + 1, bc = c + 1;  // position in the stage-input box
      cpx<T> d = czero<T>();
      if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
        int qx = inward(gx, nx), qy = inward(gy, ny);
        if (qx == 0 && qy == 0) {
          d = cd2(br, bc);
        } else {
          cpx<T> ub = U(br, bc);
          T Nb = nlin(ph, ub, vload(A, (int64_t)gy * nx + gx));
          if (BC == kDirichlet) {
            d = dirichlet_lap(ph, ub, Nb);
          } else {
            cpx<T> uq = U(br + qy, bc + qx);
            T vq2 = vload(A, (int64_t)(gy + qy) * nx + gx + qx);
            d = msd_lap(ph, cd2(br + qy, bc + qx), uq, nlin(ph, uq, vq2), ub, Nb);
          }
        }
      }
      sD[i] = d;
    }
    __syncthreads();
  }

  const cpx<T> u0 = U(ly + H, lx + H);
  const cpx<T> uq = U(qly + H, qlx + H);
  cpx<T> Kq = czero<T>();
  if (valid) {
    cpx<T> L;
    if constexpr (ORDER == 2) {
      L = cd2(qly + H, qlx + H);
    } else {
      auto Dv = [&](int r, int c) -> cpx<T> { return sD[r * DW + c]; };
      const int r = qly + 1, c = qlx + 1;
      cpx<T> D0 = Dv(r, c);
      T fr = T(0), fi = T(0);
      add_diff(fr, fi, Dv(r, c + 1), D0);
      add_diff(fr, fi, Dv(r, c - 1), D0);
      add_diff(fr, fi, Dv(r + 1, c), D0);
      add_diff(fr, fi, Dv(r - 1, c), D0);
      const int br = qly + H, bc = qlx + H;
      T er = T(0), ei = T(0);
      add_diff(er, ei, U(br + 1, bc + 1), uq);
      add_diff(er, ei, U(br + 1, bc - 1), uq);
      add_diff(er, ei, U(br - 1, bc + 1), uq);
      add_diff(er, ei, U(br - 1, bc - 1), uq);
      L = shoc_combine<T, 2>(ph, D0, fr, fi, er, ei);
    }
    Kq = rhs(ph, L, uq, nlin(ph, uq, vq));
  }
  cpx<T> K = Kq;
  if (bnd) K = (BC == kMSD) ? msd_rhs(Kq, uq, u0) : czero<T>();
  if (store) stage_update<T, STAGE, COMP>(A, idx, u0, K, own);
}

}  // namespace nlse
