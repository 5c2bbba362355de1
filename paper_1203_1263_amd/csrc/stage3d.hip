// Fused RK4 stage kernel, 3D, marching along z.
//
// One workgroup owns a TX x TY column tile and a chunk [zb, ze) of interior
// planes (plus plane 0 / nz-1 when the chunk touches them).  LDS holds a ring
// of stage-input planes with halo (planes z-1 .. z+3 for 2SHOC, z-1 .. z+1 for
// CD2) and a ring of three 2SHOC D planes (z .. z+2, Eq. 3d2shocs on the tile
// plus a one-cell ring); the D value of plane z-1 at the thread's column is
// carried in a register.  Iteration z:
//   1. issue the loads for iteration z+1 (next stage-input plane into
//      registers, own operands of plane z+1) -- they stay in flight while
//      this iteration computes;
//   2. one barrier;
//   3. D of plane z+2 into the D ring;
//   4. L (CD2, or 2SHOC step 2 of Eq. 3d2shocs2), F, boundary forms (Eqs.
//      BCDdt, BCDlap, msd, BCMSDlap) and the stage update of plane z;
//   5. the plane loaded one iteration earlier goes into the LDS ring.
// The loop is unrolled by two with two alternating register sets so no
// in-flight load is ever copied or overwritten; every load address is
// clamped into the grid so the memory operations are straight-line code.
// MSD: a boundary column evaluates F at its interior neighbour column itself
// (exactly the values the neighbour's thread computes), so no barrier is
// needed for it; the boundary planes 0 and nz-1 reuse that F at z = 1 / nz-2.
#include "stage_common.hpp"

// Iterations of loads in flight: 1 (two register sets) or 2 (three sets,
// one wave less occupancy at 32x8; measured slower at 256^3).
#ifndef NLSE_3D_EXTRA_LDS
#define NLSE_3D_EXTRA_LDS 0
#endif
#ifndef NLSE_3D_DEPTH
#define NLSE_3D_DEPTH 1
#endif

namespace nlse {

// The compensated MSD stage 4 on the 32x8 tile holds the most registers
// (102, four waves per SIMD); asking for five waves costs it one
// loop-invariant 8-byte reload per plane and is slightly faster (Dirichlet
// and L0 would spill 11-12 registers, so they keep four).
template <int STAGE, int COMP, int BC, int TX, int TY>
constexpr int stage3d_min_waves() {
  return (STAGE == 4 && COMP && BC == kMSD && TX == 32 && TY == 8) ? 5 : 1;
}

template <typename T, int ORDER, int BC, int STAGE, int COMP, int TX, int TY, bool STREAM>
__global__ __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(stage3d_min_waves<STAGE, COMP, BC, TX, TY>())))
void stage3d_kernel(StageArgs<T> A, int cz) {
  constexpr int NT = TX * TY;
  constexpr int H = ORDER == 4 ? 2 : 1;
  constexpr int BW = TX + 2 * H, BH = TY + 2 * H, BSZ = BW * BH;
  constexpr int LOOK = ORDER == 4 ? 4 : 2;  // plane put into LDS during iteration z is z+LOOK
  constexpr int NS = LOOK + 2;              // planes z-1 .. z+LOOK
  constexpr int DW = TX + 2, DH = TY + 2, DSZ = DW * DH;
  constexpr int PF = (BSZ + NT - 1) / NT;   // plane elements per thread
  constexpr int DEPTH = NLSE_3D_DEPTH;      // planes of loads in flight
  __shared__ cpx<T> sU[NS * BSZ];
  __shared__ cpx<T> sD[ORDER == 4 ? 3 * DSZ : 1];

  struct Pipe {
    cpx<T> r[PF];
    Own<T> own;
    T vq;
  };

  const int nx = A.nx, ny = A.ny, nz = A.nz;
  // points per plane: below 2^31 (checked on the host), so every plane
  // offset is a widening 32 x 32-bit product on the scalar unit
  const int ps = nx * ny;
  const int ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY;
  const int t = xcd_swizzle(blockIdx.x, gridDim.x);
  const int tx = t % ntx, ty = (t / ntx) % nty, zc = t / (ntx * nty);
  const int x0 = tile_origin(tx, TX, nx), y0 = tile_origin(ty, TY, ny);
  const int tid = threadIdx.x, lx = tid % TX, ly = tid / TX;
  const int x = x0 + lx, y = y0 + ly;
  const bool valid = x < nx && y < ny;
  const bool store = valid && x >= tx * TX && y >= ty * TY;
  const bool bnd = valid && (x == 0 || x == nx - 1 || y == 0 || y == ny - 1);
  const int64_t cidx = (int64_t)min(y, ny - 1) * nx + min(x, nx - 1);  // clamped own column
  // interior column whose F this thread evaluates: its own, or for a
  // boundary column the MSD neighbour one step inward on each boundary axis
  // (L0 needs only the point's own values)
  const bool shift = BC != kL0 && bnd;
  const int qlx = lx + (shift ? inward(x, nx) : 0), qly = ly + (shift ? inward(y, ny) : 0);
  const int64_t qidx = valid ? (int64_t)(y0 + qly) * nx + (x0 + qlx) : cidx;
  const int zb = 1 + zc * cz;
  const int ze = min(zb + cz, nz - 1);
  const int zmax = ORDER == 4 ? min(ze + 1, nz - 1) : ze;  // highest plane read
  const Phys<T>& ph = A.ph;
  const int ci = (qly + H) * BW + qlx + H;  // q column in a stage-input plane
  const int di = (qly + 1) * DW + qlx + 1;  // q column in a D plane
  const int oi = (ly + H) * BW + lx + H;    // own column in a stage-input plane

  auto slot = [&](int z) -> cpx<T>* { return sU + (z % NS) * BSZ; };
  auto dslot = [&](int z) -> cpx<T>* { return sD + (z % 3) * DSZ; };
  // 32-bit in-plane offsets; plane bases are uniform (scalar) pointers
  const int c32 = (int)cidx, q32 = (int)qidx;
  // the arrays of one plane, as uniform pointers
  auto plane_args = [&](int z) -> StageArgs<T> {
    StageArgs<T> P = A;
    const int64_t o = (int64_t)z * ps;
    P.uin += o;
    P.psi += o;
    P.acc += o;
    P.uout += o;
    if (COMP) P.lo += o;
    P.V += o * P.vs;
    return P;
  };
  // per-thread constants of the stage-input plane box, hoisted out of the
  // z loop: LDS index and clamped in-plane offset of each element it moves
  int bidx[PF], boff[PF];
#pragma unroll
  for (int k = 0; k < PF; ++k) {
    const int i = min(tid + k * NT, BSZ - 1);
    const int rr = i / BW, cc = i - rr * BW;
    const int gx = min(max(x0 - H + cc, 0), nx - 1), gy = min(max(y0 - H + rr, 0), ny - 1);
    bidx[k] = i;
    boff[k] = gy * nx + gx;
  }
  auto load_regs = [&](int z, cpx<T>(&r)[PF]) {
    const cpx<T>* P = A.uin + (int64_t)z * ps;
#pragma unroll
    for (int k = 0; k < PF; ++k) r[k] = P[boff[k]];
  };
  auto put_regs = [&](int z, const cpx<T>(&r)[PF]) {
    cpx<T>* s = slot(z);
#pragma unroll
    for (int k = 0; k < PF; ++k) s[bidx[k]] = r[k];
  };
  auto load_pipe = [&](int zplane, int zown, Pipe& p) {
    load_regs(zplane, p.r);
    const StageArgs<T> Po = plane_args(zown);
    load_own<T, STAGE, COMP, STREAM>(Po, c32, p.own);
    p.vq = vload(Po, q32);
  };
  // CD2 at stage-input position i of plane zp (z-neighbours from LDS too).
  auto cd2 = [&](int zp, int i) -> cpx<T> {
    const cpx<T>* P = slot(zp);
    const cpx<T>* Pm = slot(zp - 1);
    const cpx<T>* Pp = slot(zp + 1);
    cpx<T> u = P[i];
    T sr = T(-0.0), si = T(-0.0);
    add_diff(sr, si, P[i + 1], u);
    add_diff(sr, si, P[i - 1], u);
    add_diff(sr, si, P[i + BW], u);
    add_diff(sr, si, P[i - BW], u);
    add_diff(sr, si, Pp[i], u);
    add_diff(sr, si, Pm[i], u);
    return mk<T>(sr * ph.inv_h2, si * ph.inv_h2);
  };
  // The D points (tile plus a one-cell ring) this thread computes on every
  // plane, hoisted out of the z loop: LDS index, in-plane offsets of the point
  // and of its in-plane MSD neighbour, and whether it is in the domain /
  // interior in x and y.
  constexpr int DPF = (DSZ + NT - 1) / NT;
  int dbi[DPF], dqi[DPF], dgo[DPF], dgq[DPF];
  bool din[DPF], dint[DPF];
#pragma unroll
  for (int k = 0; k < DPF; ++k) {
    const int i = tid + k * NT;
    const int r = i / DW, c = i - r * DW;
    const int gx = x0 - 1 + c, gy = y0 - 1 + r;
    din[k] = i < DSZ && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
    const int qx = din[k] ? inward(gx, nx) : 0, qy = din[k] ? inward(gy, ny) : 0;
    dint[k] = qx == 0 && qy == 0;
    dbi[k] = (r + 1) * BW + c + 1;
    dqi[k] = dbi[k] + qy * BW + qx;
    dgo[k] = din[k] ? gy * nx + gx : 0;
    dgq[k] = din[k] ? (gy + qy) * nx + gx + qx : 0;
  }
  // D of plane zp on the tile plus a one-cell ring.  Interior points: CD2.
  // Boundary points: the Laplacian form of the boundary condition; on the
  // last plane every point is a boundary point, with its MSD neighbour in
  // plane zp-1.
  auto compute_D = [&](int zp) {
    cpx<T>* Dd = dslot(zp);
    const bool zbnd = (zp == nz - 1);
#pragma unroll
    for (int k = 0; k < DPF; ++k) {
      const int i = tid + k * NT;
      if (i >= DSZ) break;
      cpx<T> d = czero<T>();
      if (din[k]) {
        if (!zbnd && dint[k]) {
          d = cd2(zp, dbi[k]);
        } else if constexpr (BC != kL0) {  // L0: D_b = 0
          const StageArgs<T> Pz = plane_args(zp);
          cpx<T> ub = slot(zp)[dbi[k]];
          T Nb = nlin(ph, ub, vload(Pz, dgo[k]));
          if (BC == kDirichlet) {
            d = dirichlet_lap(ph, ub, Nb);
          } else {
            const int qz = zbnd ? -1 : 0;
            const StageArgs<T> Pq = plane_args(zp + qz);
            cpx<T> uq = slot(zp + qz)[dqi[k]];
            d = msd_lap(ph, cd2(zp + qz, dqi[k]), uq, nlin(ph, uq, vload(Pq, dgq[k])), ub, Nb);
          }
        }
      }
      Dd[i] = d;
    }
  };

  // ---- prologue: planes zb-1 .. zb+LOOK-1 into LDS.  Every load of the
  // prologue (those planes, the column below them, the first pipeline set)
  // is issued before the first LDS store, so the workgroup waits for one
  // memory round trip instead of one per plane.
  cpx<T> pro[LOOK + 1][PF];
#pragma unroll
  for (int k = 0; k <= LOOK; ++k) load_regs(min(zb - 1 + k, zmax), pro[k]);
  cpx<T> um2 = czero<T>();
  if constexpr (ORDER == 4) um2 = A.uin[(int64_t)max(zb - 2, 0) * ps + qidx];
  Pipe pa, pb, pc;
  load_pipe(min(zb + LOOK, zmax), zb, pa);
  if constexpr (DEPTH == 2) load_pipe(min(zb + 1 + LOOK, zmax), min(zb + 1, ze - 1), pb);
#pragma unroll
  for (int k = 0; k <= LOOK; ++k)
    if (zb - 1 + k <= zmax) put_regs(zb - 1 + k, pro[k]);
  __syncthreads();

  cpx<T> dm = czero<T>();  // D of plane z-1 at the q column
  if constexpr (ORDER == 4) {
    if (zb - 1 == 0) {
      cpx<T> ub = slot(0)[ci];
      T Nb = nlin(ph, ub, vload(A, qidx));
      if (BC == kL0) {
        dm = czero<T>();
      } else if (BC == kDirichlet) {
        dm = dirichlet_lap(ph, ub, Nb);
      } else {
        cpx<T> uq = slot(1)[ci];
        dm = msd_lap(ph, cd2(1, ci), uq, nlin(ph, uq, vload(A, ps + qidx)), ub, Nb);
      }
    } else {
      const cpx<T>* P = slot(zb - 1);
      cpx<T> u = P[ci];
      T sr = T(-0.0), si = T(-0.0);
      add_diff(sr, si, P[ci + 1], u);
      add_diff(sr, si, P[ci - 1], u);
      add_diff(sr, si, P[ci + BW], u);
      add_diff(sr, si, P[ci - BW], u);
      add_diff(sr, si, slot(zb)[ci], u);
      add_diff(sr, si, um2, u);
      dm = mk<T>(sr * ph.inv_h2, si * ph.inv_h2);
    }
    compute_D(zb);
    compute_D(zb + 1);
  }

  auto body = [&](int z, Pipe& cur, Pipe& nxt) {
    load_pipe(min(z + DEPTH + LOOK, zmax), min(z + DEPTH, ze - 1), nxt);
    __syncthreads();
    if constexpr (ORDER == 4) {
      if (z + 2 <= ze) compute_D(z + 2);
    }
    const cpx<T>* P0 = slot(z);
    const cpx<T>* Pm = slot(z - 1);
    const cpx<T>* Pp = slot(z + 1);
    const cpx<T> u0 = P0[oi];
    const cpx<T> uq = P0[ci];
    cpx<T> L;
    if constexpr (ORDER == 2) {
      T sr = T(-0.0), si = T(-0.0);
      add_diff(sr, si, P0[ci + 1], uq);
      add_diff(sr, si, P0[ci - 1], uq);
      add_diff(sr, si, P0[ci + BW], uq);
      add_diff(sr, si, P0[ci - BW], uq);
      add_diff(sr, si, Pp[ci], uq);
      add_diff(sr, si, Pm[ci], uq);
      L = mk<T>(sr * ph.inv_h2, si * ph.inv_h2);
    } else {
      const cpx<T>* Dc = dslot(z);
      cpx<T> D0 = Dc[di];
      T fr = T(-0.0), fi = T(-0.0);
      add_diff(fr, fi, Dc[di + 1], D0);
      add_diff(fr, fi, Dc[di - 1], D0);
      add_diff(fr, fi, Dc[di + DW], D0);
      add_diff(fr, fi, Dc[di - DW], D0);
      add_diff(fr, fi, dslot(z + 1)[di], D0);
      add_diff(fr, fi, dm, D0);
      T er = T(-0.0), ei = T(-0.0);
      add_diff(er, ei, P0[ci + BW + 1], uq);
      add_diff(er, ei, P0[ci + BW - 1], uq);
      add_diff(er, ei, P0[ci - BW + 1], uq);
      add_diff(er, ei, P0[ci - BW - 1], uq);
      add_diff(er, ei, Pp[ci + 1], uq);
      add_diff(er, ei, Pp[ci - 1], uq);
      add_diff(er, ei, Pp[ci + BW], uq);
      add_diff(er, ei, Pp[ci - BW], uq);
      add_diff(er, ei, Pm[ci + 1], uq);
      add_diff(er, ei, Pm[ci - 1], uq);
      add_diff(er, ei, Pm[ci + BW], uq);
      add_diff(er, ei, Pm[ci - BW], uq);
      L = shoc_combine<T, 3>(ph, D0, fr, fi, er, ei);
    }
    const cpx<T> Kq = rhs(ph, L, uq, nlin(ph, uq, cur.vq));
    cpx<T> K = Kq;
    if (bnd) {
      if constexpr (BC == kMSD) K = msd_rhs(Kq, uq, u0);
      else if constexpr (BC == kL0) K = l0_rhs(u0, nlin(ph, u0, cur.vq));
      else K = czero<T>();
    }
    if (store) stage_update<T, STAGE, COMP, STREAM>(plane_args(z), c32, u0, K, cur.own);
    // boundary planes: F_b from the interior neighbour in plane 1 / nz-2
    if (z == 1 || z == nz - 2) {
      for (int zz = 0; zz < 2; ++zz) {
        const int zbp = zz == 0 ? 0 : nz - 1;
        if ((zz == 0 && z != 1) || (zz == 1 && z != nz - 2)) continue;
        const StageArgs<T> Pb = plane_args(zbp);
        Own<T> o;
        load_own<T, STAGE, COMP, STREAM>(Pb, c32, o);
        const cpx<T> ub = slot(zbp)[oi];
        cpx<T> Kb = czero<T>();
        if constexpr (BC == kMSD) Kb = msd_rhs(Kq, uq, ub);
        else if constexpr (BC == kL0) Kb = l0_rhs(ub, nlin(ph, ub, vload(Pb, c32)));
        if (store) stage_update<T, STAGE, COMP, STREAM>(Pb, c32, ub, Kb, o);
      }
    }
    if constexpr (ORDER == 4) dm = dslot(z)[di];
    if (z + LOOK <= zmax) put_regs(z + LOOK, cur.r);
  };

  int z = zb;
  if constexpr (DEPTH == 1) {
    for (; z + 1 < ze; z += 2) {
      body(z, pa, pb);
      body(z + 1, pb, pa);
    }
    if (z < ze) body(z, pa, pb);
  } else {
    for (; z + 2 < ze; z += 3) {
      body(z, pa, pc);
      body(z + 1, pb, pa);
      body(z + 2, pc, pb);
    }
    if (z < ze) body(z, pa, pc);
    if (z + 1 < ze) body(z + 1, pb, pa);
  }
}

template <typename T, int O, int B, int S, int C>
struct Launch3D {
  static hipError_t run(const StageLaunch& L, hipStream_t st) {
    StageArgs<T> A = make_args<T>(L);
    const int tx = L.tile[0], ty = L.tile[1], cz = L.tile[2];
    if (cz < 1) return hipErrorInvalidValue;
    const int nb = cdiv(L.n[0], tx) * cdiv(L.n[1], ty) * cdiv(L.n[2] - 2, cz);
#define NLSE_L3(TX_, TY_)                                                                          \
  if (tx == TX_ && ty == TY_) {                                                                    \
    if (L.stream)                                                                                  \
      hipLaunchKernelGGL((stage3d_kernel<T, O, B, S, C, TX_, TY_, true>), dim3(nb), dim3(TX_ * TY_), \
                         NLSE_3D_EXTRA_LDS, st, A, cz);                                            \
    else                                                                                           \
      hipLaunchKernelGGL((stage3d_kernel<T, O, B, S, C, TX_, TY_, false>), dim3(nb), dim3(TX_ * TY_), \
                         NLSE_3D_EXTRA_LDS, st, A, cz);                                            \
    return hipGetLastError();                                                                      \
  }
    NLSE_L3(32, 8)
    NLSE_L3(64, 4)
    NLSE_L3(64, 8)
#undef NLSE_L3
    return hipErrorInvalidValue;
  }
};

}  // namespace nlse

hipError_t nlse_launch_stage_3d(const nlse::StageLaunch& L, hipStream_t st) {
  return nlse::dispatch_all<nlse::Launch3D>(L, st);
}
