// Fused RK4 stage kernels for the NLSE on 1D/2D/3D grids (gfx950).
//
// One launch = one RK4 stage over the whole grid: the stage input is staged
// in LDS with its halo, the 2SHOC temporary D (step 1 of Eqs. 2shoc1d /
// 2d2shocs1 / 3d2shocs) is formed in LDS on the tile plus a one-cell ring,
// the Laplacian (CD2, or 2SHOC step 2 of Eqs. 2shoc1d2 / 2d2shocs2 /
// 3d2shocs2), the right-hand side, the Dirichlet / MSD boundary forms (Eqs.
// BCDdt, BCDlap, msd, BCMSDlap) and the RK4 stage accumulation are applied,
// and only the RK4 arrays touch HBM.  The paper splits each stage into a
// compute_D and a compute_F kernel with D in global memory; here D never
// leaves the chip.
//
// 3D marches along z: each workgroup owns an x-y tile and a run of z planes,
// keeps a ring of stage-input planes (with halo) in LDS and the centre-column
// values it needs from neighbouring planes in registers, and prefetches the
// plane it will need next while it computes the current one.
//
// Laplacians are evaluated in difference form, sum_j c_j (u_j - u_0), which
// keeps FP32 rounding proportional to the local variation of the field
// instead of its magnitude.  Per point the operation sequence is fixed, so
// every tile shape gives bitwise identical results.
#include "nlse_device.hpp"
#include "nlse_internal.h"

namespace nlse {

// ---------------------------------------------------------------- helpers

// 2SHOC step 2 in difference form:
//   L = c0 D0 - (1/12) sum_faces (D_f - D0) + 1/(6h^2) sum_edges (u_e - u0)
// with c0 = 1, 2/3, 1/3 in 1D, 2D, 3D (the centre weights 14, 12, 10 of the
// paper's stencils minus the face count 2d, divided by -12).
template <typename T, int DIM>
__device__ __forceinline__ cpx<T> shoc_combine(const Phys<T>& p, cpx<T> D0, T fr, T fi, T er, T ei) {
  constexpr double c0d = DIM == 1 ? 1.0 : (DIM == 2 ? 2.0 / 3.0 : 1.0 / 3.0);
  const T c0 = T(c0d);
  const T m12 = T(-1.0 / 12.0);
  return mk<T>(fmaT(c0, D0.re, fmaT(m12, fr, p.inv_6h2 * er)),
               fmaT(c0, D0.im, fmaT(m12, fi, p.inv_6h2 * ei)));
}

template <typename T>
__device__ __forceinline__ void add_diff(T& sr, T& si, cpx<T> v, cpx<T> c) {
  sr += v.re - c.re;
  si += v.im - c.im;
}

// ================================================================ 1D

template <typename T, int ORDER, int BC, int TX>
__global__ __launch_bounds__(TX) void stage1d_kernel(StageArgs<T> A) {
  constexpr int H = ORDER == 4 ? 2 : 1;
  constexpr int BW = TX + 2 * H;
  constexpr int DW = TX + 2;
  __shared__ cpx<T> sU[BW];
  __shared__ cpx<T> sD[ORDER == 4 ? DW : 1];
  __shared__ cpx<T> sK[BC == kMSD ? TX : 1];

  const int nx = A.nx;
  const int t = xcd_swizzle(blockIdx.x, gridDim.x);
  const int x0 = tile_origin(t, TX, nx);
  const int lx = threadIdx.x;
  const int x = x0 + lx;
  const bool valid = x < nx;
  const bool store = valid && x >= t * TX;
  const Phys<T>& ph = A.ph;

  Own<T> own = store ? load_own(A, x) : Own<T>{};
  T v0 = (valid && A.V) ? A.V[x] : T(0);

  for (int i = lx; i < BW; i += TX) {
    int gx = x0 - H + i;
    sU[i] = (gx >= 0 && gx < nx) ? A.uin[gx] : czero<T>();
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
          T sr = T(0), si = T(0);
          add_diff(sr, si, sU[b + 1], c);
          add_diff(sr, si, sU[b - 1], c);
          d = mk<T>(sr * ph.inv_h2, si * ph.inv_h2);
        } else {
          T vb = A.V ? A.V[gx] : T(0);
          T Nb = nlin(ph, c, vb);
          if (BC == kDirichlet) {
            d = dirichlet_lap(ph, c, Nb);
          } else {
            int q = inward(gx, nx);
            cpx<T> uq = sU[b + q];
            T sr = T(0), si = T(0);
            add_diff(sr, si, sU[b + q + 1], uq);
            add_diff(sr, si, sU[b + q - 1], uq);
            cpx<T> dq = mk<T>(sr * ph.inv_h2, si * ph.inv_h2);
            T vq = A.V ? A.V[gx + q] : T(0);
            d = msd_lap(ph, dq, uq, nlin(ph, uq, vq), c, Nb);
          }
        }
      }
      sD[i] = d;
    }
    __syncthreads();
  }

  const cpx<T> u0 = sU[lx + H];
  const bool bnd = valid && (x == 0 || x == nx - 1);
  cpx<T> K = czero<T>();
  if (valid && !bnd) {
    cpx<T> L;
    if constexpr (ORDER == 2) {
      T sr = T(0), si = T(0);
      add_diff(sr, si, sU[lx + H + 1], u0);
      add_diff(sr, si, sU[lx + H - 1], u0);
      L = mk<T>(sr * ph.inv_h2, si * ph.inv_h2);
    } else {
      cpx<T> D0 = sD[lx + 1];
      T fr = T(0), fi = T(0);
      add_diff(fr, fi, sD[lx + 2], D0);
      add_diff(fr, fi, sD[lx], D0);
      L = shoc_combine<T, 1>(ph, D0, fr, fi, T(0), T(0));
    }
    K = rhs(ph, L, u0, nlin(ph, u0, v0));
  }
  if constexpr (BC == kMSD) {
    sK[lx] = K;
    __syncthreads();
    if (bnd) {
      int q = lx + inward(x, nx);
      K = msd_rhs(sK[q], sU[q + H], u0);
    }
  }
  if (store) stage_update(A, x, u0, K, own);
}

// ================================================================ 2D

template <typename T, int ORDER, int BC, int TX, int TY>
__global__ __launch_bounds__(TX* TY) void stage2d_kernel(StageArgs<T> A) {
  constexpr int NT = TX * TY;
  constexpr int H = ORDER == 4 ? 2 : 1;
  constexpr int BW = TX + 2 * H, BH = TY + 2 * H;
  constexpr int DW = TX + 2, DH = TY + 2;
  __shared__ cpx<T> sU[BH * BW];
  __shared__ cpx<T> sD[ORDER == 4 ? DH * DW : 1];
  __shared__ cpx<T> sK[BC == kMSD ? NT : 1];

  const int nx = A.nx, ny = A.ny;
  const int ntx = (nx + TX - 1) / TX;
  const int t = xcd_swizzle(blockIdx.x, gridDim.x);
  const int tx = t % ntx, ty = t / ntx;
  const int x0 = tile_origin(tx, TX, nx), y0 = tile_origin(ty, TY, ny);
  const int tid = threadIdx.x, lx = tid % TX, ly = tid / TX;
  const int x = x0 + lx, y = y0 + ly;
  const bool valid = x < nx && y < ny;
  const bool store = valid && x >= tx * TX && y >= ty * TY;
  const int64_t idx = (int64_t)y * nx + x;
  const Phys<T>& ph = A.ph;

  Own<T> own = store ? load_own(A, idx) : Own<T>{};
  T v0 = (valid && A.V) ? A.V[idx] : T(0);

  for (int i = tid; i < BW * BH; i += NT) {
    int r = i / BW, c = i - r * BW;
    int gx = x0 - H + c, gy = y0 - H + r;
    sU[i] = (gx >= 0 && gx < nx && gy >= 0 && gy < ny) ? A.uin[(int64_t)gy * nx + gx] : czero<T>();
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
          T vb = A.V ? A.V[(int64_t)gy * nx + gx] : T(0);
          T Nb = nlin(ph, ub, vb);
          if (BC == kDirichlet) {
            d = dirichlet_lap(ph, ub, Nb);
          } else {
            cpx<T> uq = U(br + qy, bc + qx);
            T vq = A.V ? A.V[(int64_t)(gy + qy) * nx + gx + qx] : T(0);
            d = msd_lap(ph, cd2(br + qy, bc + qx), uq, nlin(ph, uq, vq), ub, Nb);
          }
        }
      }
      sD[i] = d;
    }
    __syncthreads();
  }

  const cpx<T> u0 = U(ly + H, lx + H);
  const bool bnd = valid && (x == 0 || x == nx - 1 || y == 0 || y == ny - 1);
  cpx<T> K = czero<T>();
  if (valid && !bnd) {
    cpx<T> L;
    if constexpr (ORDER == 2) {
      L = cd2(ly + 1, lx + 1);
    } else {
      auto Dv = [&](int r, int c) -> cpx<T> { return sD[r * DW + c]; };
      const int r = ly + 1, c = lx + 1;
      cpx<T> D0 = Dv(r, c);
      T fr = T(0), fi = T(0);
      add_diff(fr, fi, Dv(r, c + 1), D0);
      add_diff(fr, fi, Dv(r, c - 1), D0);
      add_diff(fr, fi, Dv(r + 1, c), D0);
      add_diff(fr, fi, Dv(r - 1, c), D0);
      const int br = ly + H, bc = lx + H;
      T er = T(0), ei = T(0);
      add_diff(er, ei, U(br + 1, bc + 1), u0);
      add_diff(er, ei, U(br + 1, bc - 1), u0);
      add_diff(er, ei, U(br - 1, bc + 1), u0);
      add_diff(er, ei, U(br - 1, bc - 1), u0);
      L = shoc_combine<T, 2>(ph, D0, fr, fi, er, ei);
    }
    K = rhs(ph, L, u0, nlin(ph, u0, v0));
  }
  if constexpr (BC == kMSD) {
    sK[tid] = K;
    __syncthreads();
    if (bnd) {
      int qx = lx + inward(x, nx), qy = ly + inward(y, ny);
      K = msd_rhs(sK[qy * TX + qx], U(qy + H, qx + H), u0);
    }
  }
  if (store) stage_update(A, idx, u0, K, own);
}

// ================================================================ 3D

template <typename T, int ORDER, int BC, int TX, int TY>
__global__ __launch_bounds__(TX* TY) void stage3d_kernel(StageArgs<T> A, int cz) {
  constexpr int NT = TX * TY;
  constexpr int H = ORDER == 4 ? 2 : 1;
  constexpr int BW = TX + 2 * H, BH = TY + 2 * H, BSZ = BW * BH;
  constexpr int NS = ORDER == 4 ? 5 : 4;  // stage-input planes kept in LDS
  constexpr int DW = TX + 2, DH = TY + 2;
  constexpr int PF = (BSZ + NT - 1) / NT;  // prefetch registers per thread
  __shared__ cpx<T> sU[NS * BSZ];
  __shared__ cpx<T> sD[ORDER == 4 ? 2 * DW * DH : 1];
  __shared__ cpx<T> sK[BC == kMSD ? NT : 1];

  const int nx = A.nx, ny = A.ny, nz = A.nz;
  const int64_t ps = (int64_t)nx * ny;
  const int ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY;
  const int t = xcd_swizzle(blockIdx.x, gridDim.x);
  const int tx = t % ntx, ty = (t / ntx) % nty, zc = t / (ntx * nty);
  const int x0 = tile_origin(tx, TX, nx), y0 = tile_origin(ty, TY, ny);
  const int tid = threadIdx.x, lx = tid % TX, ly = tid / TX;
  const int x = x0 + lx, y = y0 + ly;
  const bool valid = x < nx && y < ny;
  const bool store = valid && x >= tx * TX && y >= ty * TY;
  const bool bnd = valid && (x == 0 || x == nx - 1 || y == 0 || y == ny - 1);
  const int64_t cidx = (int64_t)y * nx + x;  // column offset within a plane
  const int zb = 1 + zc * cz;
  const int ze = min(zb + cz, nz - 1);
  const Phys<T>& ph = A.ph;
  // in-tile position of this column's MSD interior neighbour
  const int qlx = lx + (bnd ? inward(x, nx) : 0), qly = ly + (bnd ? inward(y, ny) : 0);

  auto slot = [&](int z) -> cpx<T>* { return sU + (z % NS) * BSZ; };
  auto load_regs = [&](int z, cpx<T>(&r)[PF]) {
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      int i = tid + k * NT;
      cpx<T> v = czero<T>();
      if (i < BSZ) {
        int rr = i / BW, cc = i - rr * BW;
        int gx = x0 - H + cc, gy = y0 - H + rr;
        if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) v = A.uin[(int64_t)z * ps + (int64_t)gy * nx + gx];
      }
      r[k] = v;
    }
  };
  auto put_regs = [&](int z, const cpx<T>(&r)[PF]) {
    cpx<T>* s = slot(z);
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      int i = tid + k * NT;
      if (i < BSZ) s[i] = r[k];
    }
  };
  // CD2 at box position (r, c) of plane zc_, with z-neighbours from planes
  // zc_-1 and zc_+1 (all in LDS).
  auto cd2 = [&](int zp, int r, int c) -> cpx<T> {
    const cpx<T>* P = slot(zp);
    const cpx<T>* Pm = slot(zp - 1);
    const cpx<T>* Pp = slot(zp + 1);
    int i = r * BW + c;
    cpx<T> u = P[i];
    T sr = T(0), si = T(0);
    add_diff(sr, si, P[i + 1], u);
    add_diff(sr, si, P[i - 1], u);
    add_diff(sr, si, P[i + BW], u);
    add_diff(sr, si, P[i - BW], u);
    add_diff(sr, si, Pp[i], u);
    add_diff(sr, si, Pm[i], u);
    return mk<T>(sr * ph.inv_h2, si * ph.inv_h2);
  };
  auto vat = [&](int64_t i) -> T { return A.V ? A.V[i] : T(0); };

  // D of plane zp on the tile plus a one-cell ring, into sD buffer `buf`.
  // Interior points: CD2.  Boundary points: the Laplacian form of the
  // boundary condition; on the last plane every point is a boundary point
  // and its MSD neighbour lies in plane zp-1.
  auto compute_D = [&](int zp, int buf) {
    cpx<T>* Dd = sD + buf * DW * DH;
    const bool zbnd = (zp == nz - 1);
    for (int i = tid; i < DW * DH; i += NT) {
      int r = i / DW, c = i - r * DW;
      int gx = x0 - 1 + c, gy = y0 - 1 + r;
      int br = r + 1, bc = c + 1;
      cpx<T> d = czero<T>();
      if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
        int qx = inward(gx, nx), qy = inward(gy, ny);
        if (!zbnd && qx == 0 && qy == 0) {
          d = cd2(zp, br, bc);
        } else {
          cpx<T> ub = slot(zp)[br * BW + bc];
          int64_t gi = (int64_t)zp * ps + (int64_t)gy * nx + gx;
          T Nb = nlin(ph, ub, vat(gi));
          if (BC == kDirichlet) {
            d = dirichlet_lap(ph, ub, Nb);
          } else {
            int qz = zbnd ? -1 : 0;
            cpx<T> uq = slot(zp + qz)[(br + qy) * BW + bc + qx];
            int64_t qi = gi + (int64_t)qz * ps + (int64_t)qy * nx + qx;
            d = msd_lap(ph, cd2(zp + qz, br + qy, bc + qx), uq, nlin(ph, uq, vat(qi)), ub, Nb);
          }
        }
      }
      Dd[i] = d;
    }
  };

  // Boundary plane zb_ (0 or nz-1) of this column, once plane zq = zb_ +- 1
  // has its interior K in sK.
  auto boundary_plane = [&](int zbp, int zq) {
    int64_t gi = (int64_t)zbp * ps + cidx;
    Own<T> o = load_own(A, gi);
    cpx<T> ub = slot(zbp)[(ly + H) * BW + lx + H];
    cpx<T> Kb = czero<T>();
    if constexpr (BC == kMSD) Kb = msd_rhs(sK[qly * TX + qlx], slot(zq)[(qly + H) * BW + qlx + H], ub);
    stage_update(A, gi, ub, Kb, o);
  };

  // ---- prologue: planes zb-1 .. zb+NS-3 into LDS
  {
    const int last = min(zb + (NS - 3), nz - 1);
    for (int z = zb - 1; z <= last; ++z) {
      cpx<T> r[PF];
      load_regs(z, r);
      put_regs(z, r);
    }
  }
  cpx<T> um2 = czero<T>();
  if (ORDER == 4 && zb - 2 >= 0 && valid) um2 = A.uin[(int64_t)(zb - 2) * ps + cidx];
  __syncthreads();

  int cur = 0;
  cpx<T> dm = czero<T>();  // D of plane z-1 at this column (register queue)
  if constexpr (ORDER == 4) {
    if (valid && !bnd) {
      const int ci = (ly + H) * BW + lx + H;
      if (zb - 1 == 0) {
        cpx<T> ub = slot(0)[ci];
        T Nb = nlin(ph, ub, vat(cidx));
        if (BC == kDirichlet) {
          dm = dirichlet_lap(ph, ub, Nb);
        } else {
          cpx<T> uq = slot(1)[ci];
          dm = msd_lap(ph, cd2(1, ly + H, lx + H), uq, nlin(ph, uq, vat(ps + cidx)), ub, Nb);
        }
      } else {
        const cpx<T>* P = slot(zb - 1);
        cpx<T> u = P[ci];
        T sr = T(0), si = T(0);
        add_diff(sr, si, P[ci + 1], u);
        add_diff(sr, si, P[ci - 1], u);
        add_diff(sr, si, P[ci + BW], u);
        add_diff(sr, si, P[ci - BW], u);
        add_diff(sr, si, slot(zb)[ci], u);
        add_diff(sr, si, um2, u);
        dm = mk<T>(sr * ph.inv_h2, si * ph.inv_h2);
      }
    }
    compute_D(zb, 0);
  }

  for (int z = zb; z < ze; ++z) {
    const bool pf = (z + NS - 2 <= nz - 1) && (z + 1 < ze);
    cpx<T> reg[PF];
    if (pf) load_regs(z + NS - 2, reg);
    const int64_t gi = (int64_t)z * ps + cidx;
    Own<T> own = store ? load_own(A, gi) : Own<T>{};
    const T v0 = valid ? vat(gi) : T(0);
    __syncthreads();
    if constexpr (ORDER == 4) {
      compute_D(z + 1, cur ^ 1);
      __syncthreads();
    }
    const int ci = (ly + H) * BW + lx + H;
    const cpx<T>* P0 = slot(z);
    const cpx<T>* Pm = slot(z - 1);
    const cpx<T>* Pp = slot(z + 1);
    const cpx<T> u0 = P0[ci];
    cpx<T> K = czero<T>();
    if (valid && !bnd) {
      cpx<T> L;
      if constexpr (ORDER == 2) {
        T sr = T(0), si = T(0);
        add_diff(sr, si, P0[ci + 1], u0);
        add_diff(sr, si, P0[ci - 1], u0);
        add_diff(sr, si, P0[ci + BW], u0);
        add_diff(sr, si, P0[ci - BW], u0);
        add_diff(sr, si, Pp[ci], u0);
        add_diff(sr, si, Pm[ci], u0);
        L = mk<T>(sr * ph.inv_h2, si * ph.inv_h2);
      } else {
        const cpx<T>* Dc = sD + cur * DW * DH;
        const cpx<T>* Dn = sD + (cur ^ 1) * DW * DH;
        const int di = (ly + 1) * DW + lx + 1;
        cpx<T> D0 = Dc[di];
        T fr = T(0), fi = T(0);
        add_diff(fr, fi, Dc[di + 1], D0);
        add_diff(fr, fi, Dc[di - 1], D0);
        add_diff(fr, fi, Dc[di + DW], D0);
        add_diff(fr, fi, Dc[di - DW], D0);
        add_diff(fr, fi, Dn[di], D0);
        add_diff(fr, fi, dm, D0);
        T er = T(0), ei = T(0);
        add_diff(er, ei, P0[ci + BW + 1], u0);
        add_diff(er, ei, P0[ci + BW - 1], u0);
        add_diff(er, ei, P0[ci - BW + 1], u0);
        add_diff(er, ei, P0[ci - BW - 1], u0);
        add_diff(er, ei, Pp[ci + 1], u0);
        add_diff(er, ei, Pp[ci - 1], u0);
        add_diff(er, ei, Pp[ci + BW], u0);
        add_diff(er, ei, Pp[ci - BW], u0);
        add_diff(er, ei, Pm[ci + 1], u0);
        add_diff(er, ei, Pm[ci - 1], u0);
        add_diff(er, ei, Pm[ci + BW], u0);
        add_diff(er, ei, Pm[ci - BW], u0);
        L = shoc_combine<T, 3>(ph, D0, fr, fi, er, ei);
      }
      K = rhs(ph, L, u0, nlin(ph, u0, v0));
    }
    if constexpr (BC == kMSD) {
      sK[tid] = K;
      __syncthreads();
      if (bnd) K = msd_rhs(sK[qly * TX + qlx], P0[(qly + H) * BW + qlx + H], u0);
    }
    if (store) stage_update(A, gi, u0, K, own);
    if (store && z == 1) boundary_plane(0, 1);
    if (store && z == nz - 2) boundary_plane(nz - 1, nz - 2);
    if constexpr (ORDER == 4) dm = sD[cur * DW * DH + (ly + 1) * DW + lx + 1];
    if (pf) put_regs(z + NS - 2, reg);
    cur ^= 1;
  }
}

// ================================================================ launchers

template <typename T>
static StageArgs<T> make_args(const StageLaunch& L) {
  StageArgs<T> A;
  A.uin = static_cast<const cpx<T>*>(L.uin);
  A.psi = static_cast<const cpx<T>*>(L.psi);
  A.acc = static_cast<cpx<T>*>(L.acc);
  A.uout = static_cast<cpx<T>*>(L.uout);
  A.lo = static_cast<cpx<T>*>(L.lo);
  A.V = static_cast<const T*>(L.V);
  A.nx = (int)L.n[0];
  A.ny = (int)L.n[1];
  A.nz = (int)L.n[2];
  A.stage = L.stage;
  A.comp = L.comp;
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

static inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

template <typename T, int ORDER, int BC>
static hipError_t launch_typed(const StageLaunch& L, hipStream_t st) {
  StageArgs<T> A = make_args<T>(L);
  const int tx = L.tile[0], ty = L.tile[1];
  if (L.ndim == 1) {
    int nb = cdiv(L.n[0], 256);
    if (tx != 256) return hipErrorInvalidValue;
    hipLaunchKernelGGL((stage1d_kernel<T, ORDER, BC, 256>), dim3(nb), dim3(256), 0, st, A);
    return hipGetLastError();
  }
  if (L.ndim == 2) {
    int nb = cdiv(L.n[0], tx) * cdiv(L.n[1], ty);
#define NLSE_L2(TX_, TY_)                                                                          \
  if (tx == TX_ && ty == TY_) {                                                                    \
    hipLaunchKernelGGL((stage2d_kernel<T, ORDER, BC, TX_, TY_>), dim3(nb), dim3(TX_ * TY_), 0, st, \
                       A);                                                                         \
    return hipGetLastError();                                                                      \
  }
    NLSE_L2(64, 4)
    NLSE_L2(64, 8)
    NLSE_L2(128, 4)
    NLSE_L2(32, 8)
#undef NLSE_L2
    return hipErrorInvalidValue;
  }
  {
    const int cz = L.tile[2];
    if (cz < 1) return hipErrorInvalidValue;
    int nb = cdiv(L.n[0], tx) * cdiv(L.n[1], ty) * cdiv(L.n[2] - 2, cz);
#define NLSE_L3(TX_, TY_)                                                                          \
  if (tx == TX_ && ty == TY_) {                                                                    \
    hipLaunchKernelGGL((stage3d_kernel<T, ORDER, BC, TX_, TY_>), dim3(nb), dim3(TX_ * TY_), 0, st, \
                       A, cz);                                                                     \
    return hipGetLastError();                                                                      \
  }
    NLSE_L3(64, 4)
    NLSE_L3(64, 2)
    NLSE_L3(32, 8)
    NLSE_L3(128, 2)
#undef NLSE_L3
    return hipErrorInvalidValue;
  }
}

}  // namespace nlse

// Tile candidates compiled above; see nlse_internal.h.
extern "C" int nlse_internal_tile_supported(int ndim, int dtype, const int tile[3]) {
  const int tx = tile[0], ty = tile[1], cz = tile[2];
  if (ndim == 1) return tx == 256 && ty == 1 && cz == 1;
  if (ndim == 2) {
    if (cz != 1) return 0;
    return (tx == 64 && ty == 4) || (tx == 64 && ty == 8) || (tx == 128 && ty == 4) ||
           (tx == 32 && ty == 8);
  }
  if (cz < 1 || cz > 4096) return 0;
  bool ok = (tx == 64 && ty == 4) || (tx == 64 && ty == 2) || (tx == 32 && ty == 8) ||
            (tx == 128 && ty == 2);
  (void)dtype;
  return ok;
}

hipError_t nlse_launch_stage(const nlse::StageLaunch& L, hipStream_t st) {
  using namespace nlse;
  if (L.dtype == 0) {
    if (L.order == 2 && L.bc == kDirichlet) return launch_typed<float, 2, kDirichlet>(L, st);
    if (L.order == 2 && L.bc == kMSD) return launch_typed<float, 2, kMSD>(L, st);
    if (L.order == 4 && L.bc == kDirichlet) return launch_typed<float, 4, kDirichlet>(L, st);
    if (L.order == 4 && L.bc == kMSD) return launch_typed<float, 4, kMSD>(L, st);
  } else {
    if (L.order == 2 && L.bc == kDirichlet) return launch_typed<double, 2, kDirichlet>(L, st);
    if (L.order == 2 && L.bc == kMSD) return launch_typed<double, 2, kMSD>(L, st);
    if (L.order == 4 && L.bc == kDirichlet) return launch_typed<double, 4, kDirichlet>(L, st);
    if (L.order == 4 && L.bc == kMSD) return launch_typed<double, 4, kMSD>(L, st);
  }
  return hipErrorInvalidValue;
}
