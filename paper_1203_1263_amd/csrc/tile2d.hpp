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
//
// The per-point pieces (d_at, k_at, and stage_values in nlse_device.hpp)
// also make up the stage-pair body further down (pair2d_load /
// pair2d_compute: two RK4 stages per pass, the first on the tile and its
// halo ring), so one stage, two stages per pass and a batch all give the
// same bits.
#pragma once

#include <type_traits>

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

// A field staged in LDS, addressed in grid coordinates: row width W (a
// compile-time constant, so neighbours are immediate offsets from one
// address), grid coordinates (ox, oy) of its first element.
template <typename E, int W_>
struct LdsView {
  static constexpr int W = W_;
  const E* p;
  int ox, oy;
  __device__ __forceinline__ const E* at(int gx, int gy) const { return p + ((gy - oy) * W + (gx - ox)); }
  __device__ __forceinline__ E operator()(int gx, int gy) const { return *at(gx, gy); }
};

// CD2 Laplacian at the LDS element c of a field with row width W.
template <typename T, int W>
__device__ __forceinline__ cpx<T> cd2_ptr(const Phys<T>& ph, const cpx<T>* c) {
  const cpx<T> u = c[0];
  T sr = T(-0.0), si = T(-0.0);
  add_diff(sr, si, c[1], u);
  add_diff(sr, si, c[-1], u);
  add_diff(sr, si, c[W], u);
  add_diff(sr, si, c[-W], u);
  return mk<T>(sr * ph.inv_h2, si * ph.inv_h2);
}

// Boundary conditions are a template parameter of the stage bodies (each
// single-grid kernel is compiled for one) or, with kAnyBC, a value read at
// run time: the batched kernel runs problems of every boundary condition,
// and one body per scheme instead of per (scheme, condition) keeps its
// register footprint small.  The boundary forms touch boundary points only,
// so the run-time test is not on the interior path.
enum { kAnyBC = -1 };

// D of 2SHOC (Eq. 2d2shocs1) at grid point (gx, gy): the CD2 Laplacian in
// the interior, the boundary condition's Laplacian form on the boundary
// (Eqs. BCDlap, BCMSDlap; 0 for L0) and 0 outside the grid.
// IN: the caller knows (gx, gy) is an interior point of the grid.
template <typename T, bool IN, class UV, class VV>
__device__ __forceinline__ cpx<T> d_at(const Phys<T>& ph, const UV& U, const VV& V, int gx, int gy, int nx, int ny,
                                       int bc) {
  if constexpr (IN) return cd2_ptr<T, UV::W>(ph, U.at(gx, gy));
  cpx<T> d = czero<T>();
  if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
    const int qx = inward(gx, nx), qy = inward(gy, ny);
    const cpx<T>* u = U.at(gx, gy);
    if (qx == 0 && qy == 0) {
      d = cd2_ptr<T, UV::W>(ph, u);
    } else if (bc != kL0) {  // L0: D_b = 0
      const cpx<T> ub = u[0];
      const T Nb = nlin(ph, ub, V(gx, gy));
      if (bc == kDirichlet) {
        d = dirichlet_lap(ph, ub, Nb);
      } else {
        const cpx<T>* q = U.at(gx + qx, gy + qy);
        const cpx<T> uq = q[0];
        d = msd_lap(ph, cd2_ptr<T, UV::W>(ph, q), uq, nlin(ph, uq, V(gx + qx, gy + qy)), ub, Nb);
      }
    }
  }
  return d;
}

// D at every point of the LDS box sD (row width DW, DH rows, grid origin
// (ox, oy)), the workgroup's threads striding over it.
template <typename T, bool IN, int NT, int DW, int DH, class UV, class VV>
__device__ __forceinline__ void d_box(const Phys<T>& ph, const UV& U, const VV& V, cpx<T>* __restrict__ sD, int ox,
                                      int oy, int nx, int ny, int bc) {
  for (int i = threadIdx.x; i < DW * DH; i += NT) {
    const int r = i / DW, c = i - r * DW;
    sD[i] = d_at<T, IN>(ph, U, V, ox + c, oy + r, nx, ny, bc);
  }
}

// K = F(U) at grid point (x, y) of the grid: the Laplacian (CD2, or Eq.
// 2d2shocs2 from the D box) and F in the interior; on the boundary the time
// forms: MSD (Eq. msd) from F at the inward neighbour q, L0 (Eq. BCL0dt),
// Dirichlet (Eq. BCDdt) 0.  IN: the caller knows (x, y) is an interior
// point.
template <typename T, int ORDER, bool IN, class UV, class VV, class DV>
__device__ __forceinline__ cpx<T> k_at(const Phys<T>& ph, const UV& U, const VV& V, const DV& D, int x, int y,
                                       int nx, int ny, int bc) {
  constexpr int UW = UV::W, DW = DV::W;
  const bool bnd = !IN && (x == 0 || x == nx - 1 || y == 0 || y == ny - 1);
  const bool shift = bc != kL0 && bnd;
  const int qx = x + (shift ? inward(x, nx) : 0), qy = y + (shift ? inward(y, ny) : 0);
  const cpx<T>* q = U.at(qx, qy);
  const cpx<T> u0 = U(x, y), uq = q[0];
  cpx<T> L;
  if constexpr (ORDER == 2) {
    L = cd2_ptr<T, UW>(ph, q);
  } else {
    const cpx<T>* dq = D.at(qx, qy);
    const cpx<T> D0 = dq[0];
    T fr = T(-0.0), fi = T(-0.0);
    add_diff(fr, fi, dq[1], D0);
    add_diff(fr, fi, dq[-1], D0);
    add_diff(fr, fi, dq[DW], D0);
    add_diff(fr, fi, dq[-DW], D0);
    T er = T(-0.0), ei = T(-0.0);
    add_diff(er, ei, q[UW + 1], uq);
    add_diff(er, ei, q[UW - 1], uq);
    add_diff(er, ei, q[-UW + 1], uq);
    add_diff(er, ei, q[-UW - 1], uq);
    L = shoc_combine<T, 2>(ph, D0, fr, fi, er, ei);
  }
  const cpx<T> Kq = rhs(ph, L, uq, nlin(ph, uq, V(qx, qy)));
  cpx<T> K = Kq;
  if (bnd) {
    if (bc == kMSD) K = msd_rhs(Kq, uq, u0);
    else if (bc == kL0) K = l0_rhs(u0, nlin(ph, u0, V(x, y)));
    else K = czero<T>();
  }
  return K;
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
                                               cpx<T>* __restrict__ sD, int rt_bc = kAnyBC) {
  const int bc = BC == kAnyBC ? rt_bc : BC;
  constexpr int NT = TX * TY;
  constexpr int H = ORDER == 4 ? 2 : 1;
  constexpr int BW = TX + 2 * H;

  const int nx = A.nx, ny = A.ny;
  const int x0 = tile_origin(tx, TX, nx), y0 = tile_origin(ty, TY, ny);
  const int tid = threadIdx.x, lx = tid % TX, ly = tid / TX;
  const int x = x0 + lx, y = y0 + ly;
  const bool valid = x < nx && y < ny;
  const bool store = valid && x >= tx * TX && y >= ty * TY;
  const Phys<T>& ph = A.ph;

#pragma unroll
  for (int k = 0; k < box_pf<TX, TY, H>(); ++k) {
    const int i = box_elem<TX, TY, H>(k);
    sU[i] = R.u[k];
    sV[i] = R.v[k];
  }
  __syncthreads();

  const LdsView<cpx<T>, BW> U{sU, x0 - H, y0 - H};
  const LdsView<T, BW> V{sV, x0 - H, y0 - H};
  const LdsView<cpx<T>, TX + 2> D{sD, x0 - 1, y0 - 1};
  // IN: every point whose D or F this tile evaluates is interior, so no
  // boundary test is needed (uniform over the workgroup)
  auto body = [&](auto in_c) {
    constexpr bool IN = decltype(in_c)::value;
    if constexpr (ORDER == 4) {
      d_box<T, IN, NT, TX + 2, TY + 2>(ph, U, V, sD, x0 - 1, y0 - 1, nx, ny, bc);
      __syncthreads();
    }
    if (store) {
      const cpx<T> K = k_at<T, ORDER, IN>(ph, U, V, D, x, y, nx, ny, bc);
      stage_update<T, STAGE, COMP, STREAM>(A, (int64_t)y * nx + x, U(x, y), K, R.own);
    }
  };
  if (x0 >= 2 && x0 + TX <= nx - 2 && y0 >= 2 && y0 + TY <= ny - 2)
    body(std::true_type{});
  else
    body(std::false_type{});
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

// ---------------------------------------------------------------- stage pairs
//
// Two RK4 stages of one tile in one pass (stages 1+2, or 3+4; Eq. RK4_GPU
// regrouped in pairs).  The first stage is evaluated on the tile and on the
// ring of H cells around it that the second stage's stencil reads (halo H:
// 1 for CD2, 2 for 2SHOC), into LDS; the second stage then runs on the tile
// from there.  Its input box therefore carries a halo of 2H.  Every point
// value goes through the single-stage helpers (d_at, k_at, stage_values), so
// a pair gives the bits of two single-stage passes; the ring is computed
// again by each neighbouring tile instead of travelling through memory.
// Ring points outside the grid hold 0: no point of the grid reads them
// (D is 0 there and every Laplacian that reaches past the edge belongs to a
// boundary point whose time form discards it).

// Operands of a stage pair.  out never aliases uin or psi: the second pass
// of a step reads Psi on the ring of neighbouring tiles while it writes the
// new Psi.
template <typename T>
struct PairArgs {
  const cpx<T>* uin;  // first stage's input: Psi (stages 1+2) or U2 (stages 3+4)
  const cpx<T>* psi;  // Psi, at own and ring points
  cpx<T>* acc;        // RK4 accumulator: written by stages 1+2, read by 3+4
  cpx<T>* out;        // U2 (stages 1+2) or the new Psi (stages 3+4)
  cpx<T>* lo;         // compensation term (stages 3+4, compensated; own points)
  const T* V;         // potential; a one-element zero array when V == 0
  int64_t vs;         // 1 with a potential, 0 without
  int nx, ny;
  Phys<T> ph;
  T ca1, cn1;    // accumulation / next-input coefficients of the first stage
  T ca2, cn2;    // and of the second
  double ca2_d;  // k/6 in FP64 (compensated stage 4)
};

// Ring of h cells around a TX x TY tile: the (TX+2h)(TY+2h) box minus the
// tile, numbered top rows, bottom rows, then the left and right h cells of
// each tile row.  (r, c) is the position in the box.
template <int TX, int TY, int HR>
constexpr int ring_n() {
  return (TX + 2 * HR) * (TY + 2 * HR) - TX * TY;
}

template <int TX, int TY, int HR>
__device__ __forceinline__ void ring_pos(int j, int& r, int& c) {
  constexpr int RW = TX + 2 * HR, TOP = HR * RW;
  if (j < TOP) {
    r = j / RW;
    c = j - r * RW;
  } else if (j < 2 * TOP) {
    const int k = j - TOP, q = k / RW;
    r = HR + TY + q;
    c = k - q * RW;
  } else {
    const int k = j - 2 * TOP, q = k / (2 * HR), m = k - q * 2 * HR;
    r = HR + q;
    c = m < HR ? m : TX + m;
  }
}

// Registers that carry one tile's loads from pair2d_load to pair2d_compute,
// sized for the larger (2SHOC) halo.
template <typename T, int TX, int TY>
struct PairRegs {
  static constexpr int NT = TX * TY;
  static constexpr int PF = box_pf<TX, TY, 4>();
  static constexpr int RP = (ring_n<TX, TY, 2>() + NT - 1) / NT;
  cpx<T> u[PF];     // first stage's input on the box (halo 2H)
  T v[PF];          // potential on the box
  Own<T> own;       // Psi, acc, lo at the own point (stages 3+4)
  cpx<T> rpsi[RP];  // Psi at this thread's ring points (stages 3+4)
};

// Issue all global loads of pair PAIR (1: stages 1+2, 2: stages 3+4) on
// tile (tx, ty) with first-stage halo H.  Psi at own and ring points is
// read through the cache: the ring of one tile is the interior of its
// neighbours.
template <typename T, int PAIR, int COMP, int TX, int TY, int H, bool STREAM = false>
__device__ __forceinline__ void pair2d_load(const PairArgs<T>& A, int tx, int ty, PairRegs<T, TX, TY>& R) {
  constexpr int G = 2 * H, BW = TX + 2 * G, NT = TX * TY;
  const int nx = A.nx, ny = A.ny;
  const int x0 = tile_origin(tx, TX, nx), y0 = tile_origin(ty, TY, ny);
  const int tid = threadIdx.x;
  constexpr int PF = box_pf<TX, TY, G>();
  constexpr int NR = ring_n<TX, TY, H>(), RP = (NR + NT - 1) / NT;
  // A tile that takes the interior body of pair2d_compute (its first D
  // pass stays H + 1 cells inside the edges) has its whole 2H box inside
  // the grid, so its offsets need no clamping (uniform over the workgroup).
  const bool in = x0 - H - 1 >= 1 && x0 + TX + H <= nx - 2 && y0 - H - 1 >= 1 && y0 + TY + H <= ny - 2;
  int off[PF], roff[RP];
  if (in) {
    const int base = (y0 - G) * nx + (x0 - G);
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const int i = box_elem<TX, TY, G>(k);
      const int r = i / BW, c = i - r * BW;
      off[k] = base + r * nx + c;
    }
    const int rbase = (y0 - H) * nx + (x0 - H);
#pragma unroll
    for (int k = 0; k < RP; ++k) {
      int r, c;
      ring_pos<TX, TY, H>(min(tid + k * NT, NR - 1), r, c);
      roff[k] = rbase + r * nx + c;
    }
  } else {
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const int i = box_elem<TX, TY, G>(k);
      const int r = i / BW, c = i - r * BW;
      const int gx = min(max(x0 - G + c, 0), nx - 1), gy = min(max(y0 - G + r, 0), ny - 1);
      off[k] = gy * nx + gx;
    }
#pragma unroll
    for (int k = 0; k < RP; ++k) {
      int r, c;
      ring_pos<TX, TY, H>(min(tid + k * NT, NR - 1), r, c);
      const int gx = min(max(x0 - H + c, 0), nx - 1), gy = min(max(y0 - H + r, 0), ny - 1);
      roff[k] = gy * nx + gx;
    }
  }
#pragma unroll
  for (int k = 0; k < PF; ++k) R.u[k] = A.uin[off[k]];
#pragma unroll
  for (int k = 0; k < PF; ++k) R.v[k] = A.V[(int64_t)off[k] * A.vs];
  if constexpr (PAIR == 2) {
    const int x = min(x0 + tid % TX, nx - 1), y = min(y0 + tid / TX, ny - 1);
    const int64_t i = (int64_t)y * nx + x;
    R.own.psi = A.psi[i];
    R.own.acc = ld_own<T, STREAM>(A.acc + i);
    if constexpr (COMP) R.own.lo = ld_own<T, STREAM>(A.lo + i);
#pragma unroll
    for (int k = 0; k < RP; ++k) R.rpsi[k] = A.psi[roff[k]];
  }
}

// The input and potential box of a pair with first-stage halo H (box halo
// 2H) from the loads in R into LDS.
template <typename T, int TX, int TY, int H>
__device__ __forceinline__ void pair2d_put(const PairRegs<T, TX, TY>& R, cpx<T>* __restrict__ sU,
                                           T* __restrict__ sV) {
#pragma unroll
  for (int k = 0; k < box_pf<TX, TY, 2 * H>(); ++k) {
    const int i = box_elem<TX, TY, 2 * H>(k);
    sU[i] = R.u[k];
    sV[i] = R.v[k];
  }
}

// Pair PAIR of tile (tx, ty) from the loads in R.  sU, sV hold the input and
// potential box (halo 2H), sD the D box of either stage ((TY+2H+2)(TX+2H+2)
// elements), sM the first stage's output on the tile and its H ring.
// Contains barriers: every thread of the workgroup must call it.
// Unless box_in_lds (the caller stored this tile's box and made it visible
// with a barrier), the box is stored from R first and a barrier follows; as
// in tile2d_compute, that barrier orders the stores after earlier reads of
// sU and sV only through the caller.  before_last() runs once in every
// thread just before the last barrier, after every write of sD and sM: a
// caller that alternates sU, sV and sD between consecutive items stores the
// next item's box into the other sU and sV there, and the next item (if
// 2SHOC) starts its first D pass, into the other sD, without a barrier.  sM
// is written only after a barrier of the item (its D barrier for 2SHOC, a
// first barrier kept for CD2), so one sM serves consecutive items.
template <typename T, int ORDER, int BC, int PAIR, int COMP, int TX, int TY, bool STREAM = false, class Before>
__device__ __forceinline__ void pair2d_compute(const PairArgs<T>& A, int tx, int ty, const PairRegs<T, TX, TY>& R,
                                               cpx<T>* __restrict__ sU, T* __restrict__ sV,
                                               cpx<T>* __restrict__ sD, cpx<T>* __restrict__ sM, int rt_bc,
                                               bool box_in_lds, Before&& before_last) {
  const int bc = BC == kAnyBC ? rt_bc : BC;
  constexpr int NT = TX * TY;
  constexpr int H = ORDER == 4 ? 2 : 1, G = 2 * H;
  constexpr int BW = TX + 2 * G, RW = TX + 2 * H, RH = TY + 2 * H;
  constexpr int S1 = PAIR == 1 ? 1 : 3, S2 = S1 + 1;
  constexpr int NR = ring_n<TX, TY, H>();

  const int nx = A.nx, ny = A.ny;
  const int x0 = tile_origin(tx, TX, nx), y0 = tile_origin(ty, TY, ny);
  const int tid = threadIdx.x, lx = tid % TX, ly = tid / TX;
  const int x = x0 + lx, y = y0 + ly;
  const bool valid = x < nx && y < ny;
  const bool store = valid && x >= tx * TX && y >= ty * TY;
  const Phys<T>& ph = A.ph;
  const cpx<T> z = czero<T>();

  if (!box_in_lds) pair2d_put<T, TX, TY, H>(R, sU, sV);
  if (!box_in_lds || ORDER == 2) __syncthreads();

  const LdsView<cpx<T>, BW> U{sU, x0 - G, y0 - G};
  const LdsView<T, BW> V{sV, x0 - G, y0 - G};
  const LdsView<cpx<T>, RW + 2> D1{sD, x0 - H - 1, y0 - H - 1};
  const LdsView<cpx<T>, RW> M{sM, x0 - H, y0 - H};
  const LdsView<cpx<T>, TX + 2> D2{sD, x0 - 1, y0 - 1};
  // IN: every point whose D or F this tile evaluates (the first stage's D
  // box reaches H + 1 cells past the tile) is interior, so no boundary or
  // grid-edge test is needed (uniform over the workgroup)
  auto body = [&](auto in_c) {
    constexpr bool IN = decltype(in_c)::value;
    if constexpr (ORDER == 4) {
      d_box<T, IN, NT, RW + 2, RH + 2>(ph, U, V, sD, x0 - H - 1, y0 - H - 1, nx, ny, bc);
      __syncthreads();
    }

    // first stage: own point (its accumulator stays in a register), then the ring
    cpx<T> acc1 = z;
    {
      cpx<T> m = z;
      if (IN || valid) {
        const cpx<T> K = k_at<T, ORDER, IN>(ph, U, V, D1, x, y, nx, ny, bc);
        Own<T> o;
        o.psi = PAIR == 1 ? z : R.own.psi;
        o.acc = PAIR == 1 ? z : R.own.acc;
        o.lo = z;
        const StageOut<T> r = stage_values<T, S1, COMP>(A.ca1, A.cn1, 0.0, U(x, y), K, o);
        acc1 = r.acc;
        m = r.out;
      }
      sM[(ly + H) * RW + lx + H] = m;
    }
#pragma unroll
    for (int k = 0; k < (NR + NT - 1) / NT; ++k) {
      const int j = tid + k * NT;
      if (j < NR) {
        int r, c;
        ring_pos<TX, TY, H>(j, r, c);
        const int gx = x0 - H + c, gy = y0 - H + r;
        cpx<T> m = z;
        if (IN || (gx >= 0 && gx < nx && gy >= 0 && gy < ny)) {
          const cpx<T> K = k_at<T, ORDER, IN>(ph, U, V, D1, gx, gy, nx, ny, bc);
          Own<T> o;
          o.psi = PAIR == 1 ? z : R.rpsi[k];
          o.acc = z;
          o.lo = z;
          m = stage_values<T, S1, COMP>(A.ca1, A.cn1, 0.0, U(gx, gy), K, o).out;
        }
        sM[r * RW + c] = m;
      }
    }
    if constexpr (ORDER == 4) {
      __syncthreads();
      d_box<T, IN, NT, TX + 2, TY + 2>(ph, M, V, sD, x0 - 1, y0 - 1, nx, ny, bc);
    }
    before_last();
    __syncthreads();
    if (store) {
      const cpx<T> K = k_at<T, ORDER, IN>(ph, M, V, D2, x, y, nx, ny, bc);
      Own<T> o;
      o.acc = acc1;
      o.psi = PAIR == 1 ? U(x, y) : R.own.psi;
      o.lo = (PAIR == 2 && COMP) ? R.own.lo : z;
      const StageOut<T> r = stage_values<T, S2, COMP>(A.ca2, A.cn2, A.ca2_d, M(x, y), K, o);
      const int64_t i = (int64_t)y * nx + x;
      if constexpr (PAIR == 1) st_own<T, STREAM>(A.acc + i, r.acc);
      st_own<T, STREAM>(A.out + i, r.out);
      if constexpr (PAIR == 2 && COMP) st_own<T, STREAM>(A.lo + i, r.lo);
    }
  };
  if (x0 - H - 1 >= 1 && x0 + TX + H <= nx - 2 && y0 - H - 1 >= 1 && y0 + TY + H <= ny - 2)
    body(std::true_type{});
  else
    body(std::false_type{});
}

}  // namespace nlse
