// Fused RK4 stage pairs, 3D 2SHOC, FP32: one launch runs S1+S2, a second
// S3+S4, so the intermediate stage input (U1, U3) and the first stage's
// accumulator contribution never travel to HBM.
//
// Per RK4 step the four-pass kernels move 168 B per point (compensated);
// the pair kernels move 28 B (S1+S2: read Psi, V; write acc, U2) + 52 B
// (S3+S4: read U2, Psi, acc, Psi_lo, V; write Psi, Psi_lo) = 80 B.  The price
// is redundant arithmetic in the in-plane halo: the first stage of a pair is
// evaluated on the tile plus a 2-cell ring, its D (Eq. 3d2shocs) on a 3-cell
// ring, because the second stage's stencil reaches 2 cells.
//
// Every point is computed with exactly the operations, in exactly the order,
// of the four-pass kernels, so both paths give the same bits.
//
// A workgroup owns a 32x8 column tile and a chunk [zb, ze) of planes of the
// second stage, and marches along z.  Iteration z, between two barriers:
//   phase A:  D of the stage input at plane z+4   (ring of 3 D planes)
//             D of the first stage's output at plane z+1 (ring of 3)
//   phase B:  first stage at plane z+3 on the tile + 2-cell ring
//             second stage at plane z on the tile; results to HBM
// and the stage-input plane z+6 (loaded one iteration earlier into
// registers, as are every other operand of the next iteration) goes into a
// ring of 5 planes with a 4-cell halo.  Each phase reads only what earlier
// phases or iterations wrote.  The lags make the first iterations of a chunk
// a pipeline fill in which the later phases are idle.
//
// The second launch evaluates stage 3 on the halo too, so it reads Psi of
// points that neighbouring workgroups update in the same launch: the new Psi
// therefore goes to a second buffer (Psi alternates between the caller's
// array and a workspace array over pairs of steps).  Psi_lo and acc are read
// and written at the own point only and stay in place.
//
// z boundaries: plane 0 is processed with plane 1 and plane nz-1 with plane
// nz-2 (their F comes from the interior neighbour, Eqs. BCDdt, msd), except
// that the first stage's plane nz-1 is stored one iteration later, when its
// ring slot is free.  D of the boundary planes uses the Laplacian forms
// (Eqs. BCDlap, BCMSDlap).
#include <type_traits>

#include "stage_common.hpp"

namespace nlse {

template <int V>
using IC = std::integral_constant<int, V>;

namespace fz {
constexpr int TX = 32, TY = 8, NT = TX * TY;
constexpr int W4 = TX + 8, H4 = TY + 8;  // stage input, 4-cell halo
constexpr int W3 = TX + 6, H3 = TY + 6;  // D of the stage input, 3-cell halo
constexpr int W2 = TX + 4, H2 = TY + 4;  // first stage's output, 2-cell halo
constexpr int W1 = TX + 2, H1 = TY + 2;  // D of the first stage's output, 1-cell halo
constexpr int NIN = 5, NDIN = 3, NMID = 5, NDMID = 3;
constexpr int PIN = (W4 * H4 + NT - 1) / NT;   // stage-input elements per thread (3)
constexpr int PDIN = (W3 * H3 + NT - 1) / NT;  // D points per thread (3)
constexpr int PDMID = (W1 * H1 + NT - 1) / NT; // D points per thread (2)
constexpr int RING2 = W2 * H2 - NT;            // first-stage points outside the tile (176)
static_assert(RING2 <= NT, "one extra first-stage point per thread");
}  // namespace fz

struct FusedArgs {
  const cpx<float>* in;  // stage input of the first stage: Psi (pair 0) or U2 (pair 1)
  const cpx<float>* psi; // Psi at the start of the step (Psi_hi when compensated)
  cpx<float>* acc;       // pair 0 writes it, pair 1 reads it
  cpx<float>* out;       // pair 0: U2; pair 1: Psi after the step (not psi: see below)
  cpx<float>* lo;        // compensation term (pair 1, compensated)
  const float* V;        // potential, or a one-element zero array
  int64_t vs;            // 1 with a potential, 0 without
  int nx, ny, nz;
  Phys<float> ph;
  float c1a, c1n;        // first stage: accumulator and next-input coefficients
  float c2a, c2n;        // second stage
  double c2a_d;          // second stage accumulator coefficient in FP64 (S4)
};

template <int BC, int PAIR, int COMP, bool STREAM>
__global__ __launch_bounds__(fz::NT) void fused3d_kernel(FusedArgs A, int cz) {
  using namespace fz;
  using T = float;
  using C = cpx<T>;
  constexpr int STAGE2 = PAIR == 0 ? 2 : 4;
  __shared__ C sIn[NIN][W4 * H4];
  __shared__ C sDin[NDIN][W3 * H3];
  __shared__ C sMid[NMID][W2 * H2];
  __shared__ C sDmid[NDMID][W1 * H1];

  const int nx = A.nx, ny = A.ny, nz = A.nz;
  const int64_t ps = (int64_t)nx * ny;
  const int ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY;
  const int t = xcd_swizzle(blockIdx.x, gridDim.x);
  const int tx = t % ntx, ty = (t / ntx) % nty, zc = t / (ntx * nty);
  const int x0 = tile_origin(tx, TX, nx), y0 = tile_origin(ty, TY, ny);
  const int tid = threadIdx.x, lx = tid % TX, ly = tid / TX;
  const int zb = 1 + zc * cz;
  const int ze = min(zb + cz, nz - 1);
  const Phys<T>& ph = A.ph;

  // own point of the second stage
  const int ox = x0 + lx, oy = y0 + ly;
  const bool valid = ox < nx && oy < ny;
  const bool store = valid && ox >= tx * TX && oy >= ty * TY;
  const bool bnd = valid && (ox == 0 || ox == nx - 1 || oy == 0 || oy == ny - 1);
  const int oidx = min(oy, ny - 1) * nx + min(ox, nx - 1);  // clamped
  const int oqx = lx + (bnd ? inward(ox, nx) : 0), oqy = ly + (bnd ? inward(oy, ny) : 0);
  const int oqidx = valid ? (y0 + oqy) * nx + (x0 + oqx) : oidx;

  // the points of the first stage handled by this thread: its own tile
  // point, and (threads < RING2) one point of the 2-cell ring
  int frx[2], fry[2];
  frx[0] = lx;
  fry[0] = ly;
  {
    const int j = min(tid, RING2 - 1);
    if (j < 2 * W2) {
      fry[1] = -2 + j / W2;
      frx[1] = -2 + j % W2;
    } else if (j < 4 * W2) {
      fry[1] = TY + (j - 2 * W2) / W2;
      frx[1] = -2 + (j - 2 * W2) % W2;
    } else if (j < 4 * W2 + 2 * TY) {
      frx[1] = -2 + (j - 4 * W2) / TY;
      fry[1] = (j - 4 * W2) % TY;
    } else {
      frx[1] = TX + (j - 4 * W2 - 2 * TY) / TY;
      fry[1] = (j - 4 * W2 - 2 * TY) % TY;
    }
  }
  const int nfirst = tid < RING2 ? 2 : 1;

  auto in_dom = [&](int gx, int gy) { return gx >= 0 && gx < nx && gy >= 0 && gy < ny; };
  auto clampi = [&](int gx, int gy) { return min(max(gy, 0), ny - 1) * nx + min(max(gx, 0), nx - 1); };
  auto i4 = [&](int rx, int ry) { return (ry + 4) * W4 + rx + 4; };
  auto i3 = [&](int rx, int ry) { return (ry + 3) * W3 + rx + 3; };
  auto i2 = [&](int rx, int ry) { return (ry + 2) * W2 + rx + 2; };
  auto i1 = [&](int rx, int ry) { return (ry + 1) * W1 + rx + 1; };
  auto rin = [&](int p) -> C* { return sIn[p % NIN]; };
  auto rdin = [&](int p) -> C* { return sDin[p % NDIN]; };
  auto rmid = [&](int p) -> C* { return sMid[p % NMID]; };
  auto rdmid = [&](int p) -> C* { return sDmid[p % NDMID]; };
  auto vat = [&](int p, int gidx) -> T { return A.V[((int64_t)p * ps + gidx) * A.vs]; };

  // CD2 at LDS position i of plane P (neighbours below Pm / above Pp), row width W
  auto cd2 = [&](const C* P, const C* Pm, const C* Pp, int i, int W) -> C {
    C u = P[i];
    T sr = T(-0.0), si = T(-0.0);
    add_diff(sr, si, P[i + 1], u);
    add_diff(sr, si, P[i - 1], u);
    add_diff(sr, si, P[i + W], u);
    add_diff(sr, si, P[i - W], u);
    add_diff(sr, si, Pp[i], u);
    add_diff(sr, si, Pm[i], u);
    return mk<T>(sr * ph.inv_h2, si * ph.inv_h2);
  };

  // D of plane p of a ring (U: stage values with halo HU, D: output with
  // halo HD = HU - 1) on the D region.  Boundary points take the Laplacian
  // form of the boundary condition; on planes 0 and nz-1 every point is a
  // boundary point with its MSD neighbour one plane inward.
  auto compute_D = [&](auto ring_u, C* Dd, int p, auto iu, auto id, auto wd, auto hdim, auto wu) {
    constexpr int WD = decltype(wd)::value, HD = decltype(hdim)::value, WU = decltype(wu)::value;
    constexpr int hd = (WD - TX) / 2;
    const bool zlo = p == 0, zhi = p == nz - 1;
    const C* U0 = ring_u(p);
    const C* Um = ring_u(p > 0 ? p - 1 : p);
    const C* Up = ring_u(p < nz - 1 ? p + 1 : p);
#pragma unroll
    for (int k = 0; k * NT < WD * HD; ++k) {
      const int i = tid + k * NT;
      if (i >= WD * HD) break;
      const int rx = i % WD - hd, ry = i / WD - hd;
      const int gx = x0 + rx, gy = y0 + ry;
      C d = czero<T>();
      if (in_dom(gx, gy)) {
        const int qx = inward(gx, nx), qy = inward(gy, ny);
        const int ui = iu(rx, ry);
        if (!zlo && !zhi && qx == 0 && qy == 0) {
          d = cd2(U0, Um, Up, ui, WU);
        } else {
          const C ub = U0[ui];
          const T Nb = nlin(ph, ub, vat(p, gy * nx + gx));
          if (BC == kDirichlet) {
            d = dirichlet_lap(ph, ub, Nb);
          } else {
            const int pq = zlo ? 1 : (zhi ? nz - 2 : p);
            const C* Q0 = ring_u(pq);
            const C* Qm = ring_u(pq - 1 >= 0 ? pq - 1 : pq);
            const C* Qp = ring_u(pq + 1 <= nz - 1 ? pq + 1 : pq);
            const int uq = iu(rx + qx, ry + qy);
            const C uqv = Q0[uq];
            d = msd_lap(ph, cd2(Q0, Qm, Qp, uq, WU), uqv, nlin(ph, uqv, vat(pq, (gy + qy) * nx + gx + qx)), ub,
                        Nb);
          }
        }
      }
      Dd[id(rx, ry)] = d;
    }
  };

  // 2SHOC Laplacian (Eq. 3d2shocs2) at position (rx, ry) of plane p, from D
  // planes Dm/Dc/Dp (index fd, row width WD) and stage planes Um/Uc/Up
  // (index fu, row width WU).
  auto shoc_L = [&](const C* Dm, const C* Dc, const C* Dp, int di, int WD, const C* Um, const C* Uc, const C* Up,
                    int ui, int WU) -> C {
    const C D0 = Dc[di];
    T fr = T(-0.0), fi = T(-0.0);
    add_diff(fr, fi, Dc[di + 1], D0);
    add_diff(fr, fi, Dc[di - 1], D0);
    add_diff(fr, fi, Dc[di + WD], D0);
    add_diff(fr, fi, Dc[di - WD], D0);
    add_diff(fr, fi, Dp[di], D0);
    add_diff(fr, fi, Dm[di], D0);
    const C uq = Uc[ui];
    T er = T(-0.0), ei = T(-0.0);
    add_diff(er, ei, Uc[ui + WU + 1], uq);
    add_diff(er, ei, Uc[ui + WU - 1], uq);
    add_diff(er, ei, Uc[ui - WU + 1], uq);
    add_diff(er, ei, Uc[ui - WU - 1], uq);
    add_diff(er, ei, Up[ui + 1], uq);
    add_diff(er, ei, Up[ui - 1], uq);
    add_diff(er, ei, Up[ui + WU], uq);
    add_diff(er, ei, Up[ui - WU], uq);
    add_diff(er, ei, Um[ui + 1], uq);
    add_diff(er, ei, Um[ui - 1], uq);
    add_diff(er, ei, Um[ui + WU], uq);
    add_diff(er, ei, Um[ui - WU], uq);
    return shoc_combine<T, 3>(ph, D0, fr, fi, er, ei);
  };

  // Registers carried from one iteration's loads to the next iteration.
  struct Pre {
    C in[PIN];          // stage-input plane z+7 (put at the end of iteration z+1)
    T vq1[2];           // V at the MSD neighbours of the first-stage points, plane z+4
    C psi1[2];          // pair 1: Psi at the first-stage points, plane z+4
    C acc1;             // pair 1: acc at the own point, plane z+4
    T vq2;              // V at the own MSD neighbour, plane z+1
    C psi2, lo2;        // pair 1: Psi, Psi_lo at the own point, plane z+1
  };
  int boff[PIN], bidx[PIN];
#pragma unroll
  for (int k = 0; k < PIN; ++k) {
    const int i = min(tid + k * NT, W4 * H4 - 1);
    bidx[k] = i;
    boff[k] = clampi(x0 - 4 + i % W4, y0 - 4 + i / W4);
  }
  int fidx[2], fqidx[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int gx = x0 + frx[k], gy = y0 + fry[k];
    fidx[k] = clampi(gx, gy);
    const bool ok = in_dom(gx, gy);
    const int qx = ok ? inward(gx, nx) : 0, qy = ok ? inward(gy, ny) : 0;
    fqidx[k] = clampi(gx + qx, gy + qy);
  }
  auto clampz = [&](int p) { return min(max(p, 0), nz - 1); };
  auto issue = [&](int z, Pre& r) {  // loads for iteration z
    const int64_t pin = (int64_t)clampz(z + 6) * ps;
#pragma unroll
    for (int k = 0; k < PIN; ++k) r.in[k] = A.in[pin + boff[k]];
    const int p1 = clampz(z + 3);
    const int64_t o1 = (int64_t)p1 * ps;
#pragma unroll
    for (int k = 0; k < 2; ++k) r.vq1[k] = A.V[(o1 + fqidx[k]) * A.vs];
    if constexpr (PAIR == 1) {
#pragma unroll
      for (int k = 0; k < 2; ++k) r.psi1[k] = A.psi[o1 + fidx[k]];
      r.acc1 = ld_own<T, STREAM>(A.acc + o1 + oidx);
    }
    const int64_t o2 = (int64_t)clampz(z) * ps;
    r.vq2 = A.V[(o2 + oqidx) * A.vs];
    if constexpr (PAIR == 1) {
      r.psi2 = ld_own<T, STREAM>(A.psi + o2 + oidx);
      if constexpr (COMP) r.lo2 = ld_own<T, STREAM>(A.lo + o2 + oidx);
    }
  };

  // queue of the first stage's own-point values for the second stage:
  // qa = accumulator contribution, qp = Psi (pair 0); index 0 = plane z
  C qa[4], qp[4];
  C qa0 = czero<T>(), qp0 = czero<T>(), qaL = czero<T>(), qpL = czero<T>();
  // first stage's values of plane nz-1, stored one iteration later
  C lastK[2], lastU[2];

  // First stage at plane p (interior, 1 <= p <= nz-2) on this thread's points.
  auto first_stage = [&](int p, const Pre& r) {
    const C* Dm = rdin(p - 1);
    const C* Dc = rdin(p);
    const C* Dp = rdin(p + 1);
    const C* Um = rin(p - 1);
    const C* Uc = rin(p);
    const C* Up = rin(p + 1);
    C* Mo = rmid(p);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (k >= nfirst) break;
      const int rx = frx[k], ry = fry[k];
      const int gx = x0 + rx, gy = y0 + ry;
      if (!in_dom(gx, gy)) continue;
      const bool b = gx == 0 || gx == nx - 1 || gy == 0 || gy == ny - 1;
      const int qx = inward(gx, nx), qy = inward(gy, ny);
      const C L = shoc_L(Dm, Dc, Dp, i3(rx + qx, ry + qy), W3, Um, Uc, Up, i4(rx + qx, ry + qy), W4);
      const C uq = Uc[i4(rx + qx, ry + qy)];
      const C Kq = rhs(ph, L, uq, nlin(ph, uq, r.vq1[k]));
      const C u = Uc[i4(rx, ry)];
      C K = Kq;
      if (b) K = (BC == kMSD) ? msd_rhs(Kq, uq, u) : czero<T>();
      // the point's own values: Psi (pair 0: the stage input itself)
      const C pv = PAIR == 0 ? u : r.psi1[k];
      Mo[i2(rx, ry)] = mk<T>(fmaT(A.c1n, K.re, pv.re), fmaT(A.c1n, K.im, pv.im));
      if (k == 0) {
        if constexpr (PAIR == 0)
          qa[3] = COMP ? mk<T>(A.c1a * K.re, A.c1a * K.im) : mk<T>(fmaT(A.c1a, K.re, u.re), fmaT(A.c1a, K.im, u.im));
        else
          qa[3] = mk<T>(fmaT(A.c1a, K.re, r.acc1.re), fmaT(A.c1a, K.im, r.acc1.im));
        qp[3] = u;
      }
      // boundary planes from the interior neighbour plane
      auto zplane = [&](int pb, C& qaB, C& qpB, bool now) {
        const int64_t ob = (int64_t)pb * ps;
        const C ub = rin(pb)[i4(rx, ry)];
        const C Kb = (BC == kMSD) ? msd_rhs(Kq, uq, ub) : czero<T>();
        const C pvb = PAIR == 0 ? ub : A.psi[ob + gy * nx + gx];
        if (now) {
          rmid(pb)[i2(rx, ry)] = mk<T>(fmaT(A.c1n, Kb.re, pvb.re), fmaT(A.c1n, Kb.im, pvb.im));
        } else {
          lastK[k] = Kb;
          lastU[k] = pvb;
        }
        if (k == 0) {
          if constexpr (PAIR == 0) {
            qaB = COMP ? mk<T>(A.c1a * Kb.re, A.c1a * Kb.im) : mk<T>(fmaT(A.c1a, Kb.re, ub.re), fmaT(A.c1a, Kb.im, ub.im));
          } else {
            const C ab = ld_own<T, STREAM>(A.acc + ob + oidx);
            qaB = mk<T>(fmaT(A.c1a, Kb.re, ab.re), fmaT(A.c1a, Kb.im, ab.im));
          }
          qpB = ub;
        }
      };
      if (p == 1) zplane(0, qa0, qp0, true);
      if (p == nz - 2) zplane(nz - 1, qaL, qpL, false);
    }
  };
  // the first stage's plane nz-1, one iteration after plane nz-2
  auto first_stage_last = [&]() {
    C* Mo = rmid(nz - 1);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (k >= nfirst) break;
      const int gx = x0 + frx[k], gy = y0 + fry[k];
      if (!in_dom(gx, gy)) continue;
      Mo[i2(frx[k], fry[k])] = mk<T>(fmaT(A.c1n, lastK[k].re, lastU[k].re), fmaT(A.c1n, lastK[k].im, lastU[k].im));
    }
  };

  // Second stage at plane z (interior) on the own point, and planes 0 /
  // nz-1 with planes 1 / nz-2.
  auto second_stage = [&](int z, const Pre& r) {
    const C* Dm = rdmid(z - 1);
    const C* Dc = rdmid(z);
    const C* Dp = rdmid(z + 1);
    const C* Um = rmid(z - 1);
    const C* Uc = rmid(z);
    const C* Up = rmid(z + 1);
    const C L = shoc_L(Dm, Dc, Dp, i1(oqx, oqy), W1, Um, Uc, Up, i2(oqx, oqy), W2);
    const C uq = Uc[i2(oqx, oqy)];
    const C u0 = Uc[i2(lx, ly)];
    const C Kq = rhs(ph, L, uq, nlin(ph, uq, r.vq2));
    C K = Kq;
    if (bnd) K = (BC == kMSD) ? msd_rhs(Kq, uq, u0) : czero<T>();
    StageArgs<T> S;
    S.uin = nullptr;
    S.psi = A.psi;
    S.acc = A.acc;
    S.uout = A.out;
    S.lo = A.lo;
    S.V = A.V;
    S.vs = A.vs;
    S.nx = nx;
    S.ny = ny;
    S.nz = nz;
    S.ph = ph;
    S.c_acc = A.c2a;
    S.c_next = A.c2n;
    S.c_acc_d = A.c2a_d;
    auto put = [&](int pz, C ub, C Kb, C qaz, C qpz) {
      StageArgs<T> P = S;
      const int64_t o = (int64_t)pz * ps;
      P.psi += o;
      P.acc += o;
      P.uout += o;
      if (COMP) P.lo += o;
      Own<T> own;
      own.acc = qaz;
      if constexpr (PAIR == 0) {
        own.psi = qpz;
      } else {
        own.psi = pz == z ? r.psi2 : ld_own<T, STREAM>(A.psi + o + oidx);
        if constexpr (COMP) own.lo = pz == z ? r.lo2 : ld_own<T, STREAM>(A.lo + o + oidx);
      }
      if (store) stage_update<T, STAGE2, COMP, STREAM>(P, oidx, ub, Kb, own);
    };
    put(z, u0, K, qa[0], qp[0]);
    if (z == 1) {
      const C ub = rmid(0)[i2(lx, ly)];
      put(0, ub, (BC == kMSD) ? msd_rhs(Kq, uq, ub) : czero<T>(), qa0, qp0);
    }
    if (z == nz - 2) {
      const C ub = rmid(nz - 1)[i2(lx, ly)];
      put(nz - 1, ub, (BC == kMSD) ? msd_rhs(Kq, uq, ub) : czero<T>(), qaL, qpL);
    }
  };

  // ---- pipeline ranges (planes each phase produces for this chunk)
  const int dinlo = max(zb - 3, 0), dinhi = min(ze + 2, nz - 1);    // D of the stage input
  const int firlo = max(zb - 2, 1), firhi = min(ze + 1, nz - 2);    // first stage (interior planes)
  const int dmdlo = max(zb - 1, 0), dmdhi = min(ze, nz - 1);        // D of the first stage's output
  const int inlo = max(zb - 4, 0), inhi = min(ze + 3, nz - 1);      // stage-input planes in LDS
  const int z0 = zb - 7;

  // prologue: stage-input planes read by the first iterations
  for (int p = z0 + 3; p <= z0 + 5; ++p) {
    if (p < inlo || p > inhi) continue;
    const int64_t o = (int64_t)p * ps;
    C* s = rin(p);
#pragma unroll
    for (int k = 0; k < PIN; ++k) s[bidx[k]] = A.in[o + boff[k]];
  }
  Pre pa, pb;
  issue(z0, pa);

  auto body = [&](int z, Pre& cur, Pre& nxt) {
    issue(z + 1, nxt);
    __syncthreads();
    // phase A
    {
      const int p = z + 4;
      if (p >= dinlo && p <= dinhi && p != 0) {
        compute_D(rin, rdin(p), p, i4, i3, IC<W3>{}, IC<H3>{}, IC<W4>{});
        if (p == 1) compute_D(rin, rdin(0), 0, i4, i3, IC<W3>{}, IC<H3>{}, IC<W4>{});
      }
    }
    {
      const int p = z + 1;
      if (p >= dmdlo && p <= dmdhi && p != 0) {
        compute_D(rmid, rdmid(p), p, i2, i1, IC<W1>{}, IC<H1>{}, IC<W2>{});
        if (p == 1) compute_D(rmid, rdmid(0), 0, i2, i1, IC<W1>{}, IC<H1>{}, IC<W2>{});
      }
    }
    __syncthreads();
    // phase B
    {
      const int p = z + 3;
      if (p >= firlo && p <= firhi) first_stage(p, cur);
      if (p == nz - 1 && nz - 2 >= firlo && nz - 2 <= firhi) first_stage_last();
    }
    if (z >= zb && z < ze) second_stage(z, cur);
    {
      const int p = z + 6;
      if (p >= inlo && p <= inhi) {
        C* s = rin(p);
#pragma unroll
        for (int k = 0; k < PIN; ++k) s[bidx[k]] = cur.in[k];
      }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      qa[k] = qa[k + 1];
      qp[k] = qp[k + 1];
    }
  };

  int z = z0;
  for (; z + 1 < ze; z += 2) {
    body(z, pa, pb);
    body(z + 1, pb, pa);
  }
  if (z < ze) body(z, pa, pb);
}

template <int BC, int PAIR, int COMP>
static hipError_t launch_fused(const FusedArgs& A, int cz, int nb, bool stream, hipStream_t st) {
  if (stream)
    hipLaunchKernelGGL((fused3d_kernel<BC, PAIR, COMP, true>), dim3(nb), dim3(fz::NT), 0, st, A, cz);
  else
    hipLaunchKernelGGL((fused3d_kernel<BC, PAIR, COMP, false>), dim3(nb), dim3(fz::NT), 0, st, A, cz);
  return hipGetLastError();
}

}  // namespace nlse

namespace {

nlse::FusedArgs fused_args(const nlse::StageLaunch& L, const void* psi, void* acc, void* lo) {
  using namespace nlse;
  FusedArgs A;
  A.psi = static_cast<const cpx<float>*>(psi);
  A.acc = static_cast<cpx<float>*>(acc);
  A.lo = static_cast<cpx<float>*>(lo);
  A.V = static_cast<const float*>(L.V ? L.V : L.vzero);
  A.vs = L.V ? 1 : 0;
  A.nx = (int)L.n[0];
  A.ny = (int)L.n[1];
  A.nz = (int)L.n[2];
  A.ph.a = (float)L.a;
  A.ph.s = (float)L.s;
  A.ph.inv_a = (float)(1.0 / L.a);
  A.ph.inv_h2 = (float)(1.0 / (L.h * L.h));
  A.ph.inv_6h2 = (float)(1.0 / (6.0 * L.h * L.h));
  return A;
}

// Pair 0: stages 1 + 2 (in = Psi; writes acc and mid = U2).
hipError_t pair0(const nlse::StageLaunch& L, nlse::FusedArgs A, const void* psi, void* mid, double dt,
                 hipStream_t st) {
  using namespace nlse;
  const int cz = L.tile[2];
  const int nb = cdiv(L.n[0], fz::TX) * cdiv(L.n[1], fz::TY) * cdiv(L.n[2] - 2, cz);
  const bool comp = L.comp != 0, stream = L.stream != 0;
  A.in = static_cast<const cpx<float>*>(psi);
  A.out = static_cast<cpx<float>*>(mid);
  A.c1a = (float)(dt / 6.0);
  A.c1n = (float)(dt / 2.0);
  A.c2a = (float)(dt / 3.0);
  A.c2n = (float)(dt / 2.0);
  A.c2a_d = dt / 3.0;
  if (L.bc == kMSD)
    return comp ? launch_fused<kMSD, 0, 1>(A, cz, nb, stream, st) : launch_fused<kMSD, 0, 0>(A, cz, nb, stream, st);
  return comp ? launch_fused<kDirichlet, 0, 1>(A, cz, nb, stream, st)
              : launch_fused<kDirichlet, 0, 0>(A, cz, nb, stream, st);
}

// Pair 1: stages 3 + 4 (in = mid = U2, Psi read from A.psi; writes the new
// Psi to psi_out and, compensated, lo).
hipError_t pair1(const nlse::StageLaunch& L, nlse::FusedArgs A, void* psi, const void* mid, double dt,
                 hipStream_t st) {
  using namespace nlse;
  const int cz = L.tile[2];
  const int nb = cdiv(L.n[0], fz::TX) * cdiv(L.n[1], fz::TY) * cdiv(L.n[2] - 2, cz);
  const bool comp = L.comp != 0, stream = L.stream != 0;
  A.in = static_cast<const cpx<float>*>(mid);
  A.out = static_cast<cpx<float>*>(psi);
  A.c1a = (float)(dt / 3.0);
  A.c1n = (float)dt;
  A.c2a = (float)(dt / 6.0);
  A.c2n = 0.0f;
  A.c2a_d = dt / 6.0;
  if (L.bc == kMSD)
    return comp ? launch_fused<kMSD, 1, 1>(A, cz, nb, stream, st) : launch_fused<kMSD, 1, 0>(A, cz, nb, stream, st);
  return comp ? launch_fused<kDirichlet, 1, 1>(A, cz, nb, stream, st)
              : launch_fused<kDirichlet, 1, 0>(A, cz, nb, stream, st);
}

bool fused_ok(const nlse::StageLaunch& L) {
  return L.ndim == 3 && L.dtype == 0 && L.order == 4 && (L.bc == nlse::kDirichlet || L.bc == nlse::kMSD) &&
         L.tile[0] == nlse::fz::TX && L.tile[1] == nlse::fz::TY && L.tile[2] >= 1 && L.n[2] >= 3;
}

}  // namespace

hipError_t nlse_launch_fused3d(const nlse::StageLaunch& L, const void* psi_in, void* psi_out, void* acc, void* mid,
                               void* lo, double dt, hipStream_t st) {
  if (!fused_ok(L) || psi_in == psi_out) return hipErrorInvalidValue;
  const nlse::FusedArgs A = fused_args(L, psi_in, acc, lo);
  hipError_t e = pair0(L, A, psi_in, mid, dt, st);
  if (e != hipSuccess) return e;
  return pair1(L, A, psi_out, mid, dt, st);
}

hipError_t nlse_launch_fused3d_pair0(const nlse::StageLaunch& L, const void* psi, void* acc, void* mid, double dt,
                                     hipStream_t st) {
  if (!fused_ok(L)) return hipErrorInvalidValue;
  return pair0(L, fused_args(L, psi, acc, nullptr), psi, mid, dt, st);
}
