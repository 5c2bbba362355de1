// The 2D stage tile body shared by the single-grid 2D stage kernel and the
// batched persistent kernel, so a simulation computes the same bits whether
// it runs alone or inside a batch.
//
// One TX x TY tile: the stage input of the tile plus a 1-cell (CD2) or 2-cell
// (2SHOC) halo and the potential on the same box are staged in LDS, D (Eq.
// 2d2shocs1) is formed in LDS on the tile plus a one-cell ring, then the
// Laplacian (CD2, or Eq. 2d2shocs2), F, the boundary forms (Eqs. BCDdt,
// BCDlap, msd, BCMSDlap) and the stage accumulation follow.
//
// The body is split in two so the batched kernel can overlap one tile's
// loads with the previous tile's arithmetic: tile2d_load issues every global
// load of a tile into registers (straight-line code: each address is clamped
// into the grid), tile2d_compute consumes them.  Loads are coalesced along x.
#pragma once

#include "stage_common.hpp"

namespace nlse {

// Registers that carry one tile's loads from tile2d_load to tile2d_compute.
// PF covers the larger (2SHOC) box, so one type serves both halos.
template <typename T, int TX, int TY>
struct TileRegs {
  static constexpr int NT = TX * TY;
  static constexpr int PF = ((TX + 4) * (TY + 4) + NT - 1) / NT;
  cpx<T> u[PF];  // stage input on the box
  T v[PF];       // potential on the box
  Own<T> own;    // own-point operands of the stage update
};

// Box elements per thread for halo H (at most TileRegs::PF).
template <int TX, int TY, int H>
constexpr int box_pf() {
  return ((TX + 2 * H) * (TY + 2 * H) + TX * TY - 1) / (TX * TY);
}

// Index of box element k of this thread (clamped, so every thread moves
// box_pf elements; duplicates carry the same value to the same place).
template <int TX, int TY, int H>
__device__ __forceinline__ int box_elem(int k) {
  constexpr int BW = TX + 2 * H, BSZ = BW * (TY + 2 * H);
  return min((int)threadIdx.x + k * TX * TY, BSZ - 1);
}

// Issue all global loads of tile (tx, ty) with halo H into R.
template <typename T, int STAGE, int COMP, int TX, int TY, int H, bool STREAM = false>
__device__ __forceinline__ void tile2d_load(const StageArgs<T>& A, int tx, int ty, TileRegs<T, TX, TY>& R) {
  constexpr int BW = TX + 2 * H;
  const int nx = A.nx, ny = A.ny;
  const int x0 = tile_origin(tx, TX, nx), y0 = tile_origin(ty, TY, ny);
  const int tid = threadIdx.x;
  const int x = min(x0 + tid % TX, nx - 1), y = min(y0 + tid / TX, ny - 1);
  constexpr int PF = box_pf<TX, TY, H>();
  int off[PF];
#pragma unroll
  for (int k = 0; k < PF; ++k) {
    const int i = box_elem<TX, TY, H>(k);
    const int r = i / BW, c = i - r * BW;
    const int gx = min(max(x0 - H + c, 0), nx - 1), gy = min(max(y0 - H + r, 0), ny - 1);
    off[k] = gy * nx + gx;
  }
#pragma unroll
  for (int k = 0; k < PF; ++k) R.u[k] = A.uin[off[k]];
#pragma unroll
  for (int k = 0; k < PF; ++k) R.v[k] = vload(A, off[k]);
  load_own<T, STAGE, COMP, STREAM>(A, (int64_t)y * nx + x, R.own);
}

// Stage tile (tx, ty) from the loads in R.  sU, sV hold the (TY+2H)(TX+2H)
// box, sD the (TY+2)(TX+2) D ring.  Contains barriers: every thread of the
// workgroup must call it.  The first barrier orders the LDS writes here
// after this workgroup's earlier reads of sU and sV only through the caller
// (a single-tile kernel has none; the batched kernel alternates two sU / sV
// buffers), while sD is rewritten only after that barrier.
template <typename T, int ORDER, int BC, int STAGE, int COMP, int TX, int TY, bool STREAM = false>
__device__ __forceinline__ void tile2d_compute(const StageArgs<T>& A, int tx, int ty, const TileRegs<T, TX, TY>& R,
                                               cpx<T>* __restrict__ sU, T* __restrict__ sV,
                                               cpx<T>* __restrict__ sD) {
  constexpr int NT = TX * TY;
  constexpr int H = ORDER == 4 ? 2 : 1;
  constexpr int BW = TX + 2 * H;
  constexpr int DW = TX + 2, DH = TY + 2;

  const int nx = A.nx, ny = A.ny;
  const int x0 = tile_origin(tx, TX, nx), y0 = tile_origin(ty, TY, ny);
  const int tid = threadIdx.x, lx = tid % TX, ly = tid / TX;
  const int x = x0 + lx, y = y0 + ly;
  const bool valid = x < nx && y < ny;
  const bool store = valid && x >= tx * TX && y >= ty * TY;
  const int64_t idx = (int64_t)min(y, ny - 1) * nx + min(x, nx - 1);  // clamped
  // MSD boundary points evaluate F at their interior neighbour q themselves
  // (L0 needs only the point's own values)
  const bool bnd = valid && (x == 0 || x == nx - 1 || y == 0 || y == ny - 1);
  const bool shift = BC != kL0 && bnd;
  const int qlx = lx + (shift ? inward(x, nx) : 0), qly = ly + (shift ? inward(y, ny) : 0);
  const Phys<T>& ph = A.ph;

#pragma unroll
  for (int k = 0; k < box_pf<TX, TY, H>(); ++k) {
    const int i = box_elem<TX, TY, H>(k);
    sU[i] = R.u[k];
    sV[i] = R.v[k];
  }
  __syncthreads();

  auto U = [&](int r, int c) -> cpx<T> { return sU[r * BW + c]; };
  auto Vb = [&](int r, int c) -> T { return sV[r * BW + c]; };
  auto cd2 = [&](int r, int c) -> cpx<T> {
    cpx<T> u = U(r, c);
    T sr = T(-0.0), si = T(-0.0);
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
        } else if constexpr (BC != kL0) {  // L0: D_b = 0
          cpx<T> ub = U(br, bc);
          T Nb = nlin(ph, ub, Vb(br, bc));
          if (BC == kDirichlet) {
            d = dirichlet_lap(ph, ub, Nb);
          } else {
            cpx<T> uq = U(br + qy, bc + qx);
            d = msd_lap(ph, cd2(br + qy, bc + qx), uq, nlin(ph, uq, Vb(br + qy, bc + qx)), ub, Nb);
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
      T fr = T(-0.0), fi = T(-0.0);
      add_diff(fr, fi, Dv(r, c + 1), D0);
      add_diff(fr, fi, Dv(r, c - 1), D0);
      add_diff(fr, fi, Dv(r + 1, c), D0);
      add_diff(fr, fi, Dv(r - 1, c), D0);
      const int br = qly + H, bc = qlx + H;
      T er = T(-0.0), ei = T(-0.0);
      add_diff(er, ei, U(br + 1, bc + 1), uq);
      add_diff(er, ei, U(br + 1, bc - 1), uq);
      add_diff(er, ei, U(br - 1, bc + 1), uq);
      add_diff(er, ei, U(br - 1, bc - 1), uq);
      L = shoc_combine<T, 2>(ph, D0, fr, fi, er, ei);
    }
    Kq = rhs(ph, L, uq, nlin(ph, uq, Vb(qly + H, qlx + H)));
  }
  cpx<T> K = Kq;
  if (bnd) {
    if constexpr (BC == kMSD) K = msd_rhs(Kq, uq, u0);
    else if constexpr (BC == kL0) K = l0_rhs(u0, nlin(ph, u0, Vb(ly + H, lx + H)));
    else K = czero<T>();
  }
  if (store) stage_update<T, STAGE, COMP, STREAM>(A, idx, u0, K, R.own);
}

// LDS of one tile: box of the stage input and of the potential, D ring.
template <typename T, int TX, int TY, int H>
struct TileLds {
  static constexpr int BSZ = (TX + 2 * H) * (TY + 2 * H);
  static constexpr int DSZ = (TX + 2) * (TY + 2);
  cpx<T> u[BSZ];
  T v[BSZ];
  cpx<T> d[H == 2 ? DSZ : 1];  // D ring (2SHOC only)
};

// One TX x TY tile (tile indices tx, ty) of one RK4 stage, loads then
// arithmetic.  Contains barriers: every thread of the workgroup must call it.
template <typename T, int ORDER, int BC, int STAGE, int COMP, int TX, int TY, bool STREAM>
__device__ __forceinline__ void tile2d(const StageArgs<T>& A, int tx, int ty,
                                       TileLds<T, TX, TY, ORDER == 4 ? 2 : 1>& S) {
  TileRegs<T, TX, TY> R;
  tile2d_load<T, STAGE, COMP, TX, TY, ORDER == 4 ? 2 : 1, STREAM>(A, tx, ty, R);
  tile2d_compute<T, ORDER, BC, STAGE, COMP, TX, TY, STREAM>(A, tx, ty, R, S.u, S.v, S.d);
}

}  // namespace nlse
