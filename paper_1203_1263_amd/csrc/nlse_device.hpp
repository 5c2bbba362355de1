// Device-side building blocks shared by the stage and reduction kernels of
// libnlse: complex storage type, per-point physics (right-hand side and the
// boundary forms), RK4 stage accumulation and the tile mapping.
//
// All arithmetic is written out explicitly; the library is compiled with
// -ffp-contract=off so every fused multiply-add below is deliberate and the
// value computed for a grid point never depends on the tile shape, launch
// shape or batch packing around it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nlse {

enum { kDirichlet = 0, kMSD = 1, kL0 = 2 };

// Interleaved complex value; 8-byte (FP32) / 16-byte (FP64) aligned so a
// lane moves one point with a single vector memory instruction.
template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T re, im;
};

__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
__device__ __forceinline__ cpx<T> czero() {
  cpx<T> z;
  z.re = T(0);
  z.im = T(0);
  return z;
}

template <typename T>
__device__ __forceinline__ cpx<T> mk(T r, T i) {
  cpx<T> z;
  z.re = r;
  z.im = i;
  return z;
}

// Physical constants of one problem, pre-converted to the compute type.
template <typename T>
struct Phys {
  T a, s, inv_a, inv_h2, inv_6h2;
};

// N = s|u|^2 - V  (the factor named N_b in Eq. BCMSDlap).
template <typename T>
__device__ __forceinline__ T nlin(const Phys<T>& p, cpx<T> u, T v) {
  T rho = fmaT(u.re, u.re, u.im * u.im);
  return fmaT(p.s, rho, -v);
}

// F = i (a L + N u): the right-hand side under Eq. RK4 (split form Eq. fsplit).
template <typename T>
__device__ __forceinline__ cpx<T> rhs(const Phys<T>& p, cpx<T> L, cpx<T> u, T N) {
  T wr = fmaT(p.a, L.re, N * u.re);
  T wi = fmaT(p.a, L.im, N * u.im);
  return mk<T>(-wi, wr);
}

// MSD time form (Eq. msd): F_b = i Im(F_q / u_q) u_b; a zero |u_q| gives 0.
template <typename T>
__device__ __forceinline__ cpx<T> msd_rhs(cpx<T> Fq, cpx<T> uq, cpx<T> ub) {
  T m = fmaT(uq.re, uq.re, uq.im * uq.im);
  T w = (m == T(0)) ? T(0) : fmaT(Fq.im, uq.re, -(Fq.re * uq.im)) / m;
  return mk<T>(-(w * ub.im), w * ub.re);
}

// Laplacian-zero time form (Eq. BCL0dt): F_b = i N_b u_b.  Its Laplacian
// form (Eq. BCL0lap) is D_b = 0.
template <typename T>
__device__ __forceinline__ cpx<T> l0_rhs(cpx<T> ub, T Nb) {
  return mk<T>(-(Nb * ub.im), Nb * ub.re);
}

// Dirichlet Laplacian form (Eq. BCDlap): D_b = -(1/a) N_b u_b.
template <typename T>
__device__ __forceinline__ cpx<T> dirichlet_lap(const Phys<T>& p, cpx<T> ub, T Nb) {
  T f = -(Nb * p.inv_a);
  return mk<T>(f * ub.re, f * ub.im);
}

// MSD Laplacian form (Eq. BCMSDlap, with Im(i z) = Re z):
//   D_b = [ Re(D_q / u_q) + (N_q - N_b)/a ] u_b.
template <typename T>
__device__ __forceinline__ cpx<T> msd_lap(const Phys<T>& p, cpx<T> Dq, cpx<T> uq, T Nq,
                                          cpx<T> ub, T Nb) {
  T m = fmaT(uq.re, uq.re, uq.im * uq.im);
  T r = (m == T(0)) ? T(0) : fmaT(Dq.re, uq.re, Dq.im * uq.im) / m;
  T f = fmaT(Nq - Nb, p.inv_a, r);
  return mk<T>(f * ub.re, f * ub.im);
}

// One step inward on a boundary axis: +1 at index 0, -1 at n-1, else 0.
__device__ __forceinline__ int inward(int i, int n) { return i == 0 ? 1 : (i == n - 1 ? -1 : 0); }

// ---------------------------------------------------------------- RK4 stages
//
// One RK4 step is four passes (Eq. RK4 regrouped so each pass evaluates F
// once, as in Eq. RK4_GPU):
//   S1: acc  = [Psi +] k/6 K1,  out = Psi + k/2 K1      (in = Psi)
//   S2: acc += k/3 K2,          out = Psi + k/2 K2      (in = U1)
//   S3: acc += k/3 K3,          out = Psi + k   K3      (in = U2)
//   S4: Psi  = acc + k/6 K4                             (in = U3)
// Plain mode stores Psi inside acc; compensated mode (COMP) keeps acc as the
// pure increment and finishes S4 in FP64 on the pair Psi_hi + Psi_lo.
// The stage number and the mode are template parameters so the memory
// operations of a stage are straight-line code.
template <typename T>
struct StageArgs {
  const cpx<T>* uin;  // stage input (neighbours are read)
  const cpx<T>* psi;  // Psi (own point; stages 2 and 3)
  cpx<T>* acc;        // RK4 accumulator
  cpx<T>* uout;       // next stage input; Psi itself at stage 4
  cpx<T>* lo;         // compensation term (stage 4, compensated)
  const T* V;         // potential; a one-element zero array when V == 0
  int64_t vs;         // 1 with a potential, 0 without (V index multiplier)
  int nx, ny, nz;
  Phys<T> ph;
  T c_acc;            // k/6, k/3, k/3, k/6
  T c_next;           // k/2, k/2, k,   (unused)
  double c_acc_d;     // k/6 in FP64 (compensated stage 4)
};

template <typename T>
__device__ __forceinline__ T vload(const StageArgs<T>& A, int64_t i) {
  return A.V[i * A.vs];
}

// Own-point operands of the stage update.
template <typename T>
struct Own {
  cpx<T> psi, acc, lo;
};

// Own-point operands are read once and stage results written once per
// launch.  When a grid's fields are much larger than the last-level cache
// (STREAM = true) these accesses are non-temporal, which leaves the caches to
// the stencil's halo data; on grids that fit, ordinary accesses let the
// next stage find its input in the cache.
template <typename T, bool STREAM>
__device__ __forceinline__ cpx<T> ld_own(const cpx<T>* p) {
  if constexpr (STREAM) {
    typedef T v2 __attribute__((ext_vector_type(2)));
    const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
    return mk<T>(v.x, v.y);
  } else {
    return *p;
  }
}

template <typename T, bool STREAM>
__device__ __forceinline__ void st_own(cpx<T>* p, cpx<T> c) {
  if constexpr (STREAM) {
    typedef T v2 __attribute__((ext_vector_type(2)));
    const v2 v = {c.re, c.im};
    __builtin_nontemporal_store(v, reinterpret_cast<v2*>(p));
  } else {
    *p = c;
  }
}

template <typename T, int STAGE, int COMP, bool STREAM = false>
__device__ __forceinline__ void load_own(const StageArgs<T>& A, int64_t i, Own<T>& o) {
  if constexpr (STAGE == 2 || STAGE == 3) {
    o.psi = ld_own<T, STREAM>(A.psi + i);
    o.acc = ld_own<T, STREAM>(A.acc + i);
  } else if constexpr (STAGE == 4) {
    o.acc = ld_own<T, STREAM>(A.acc + i);
    if constexpr (COMP) {
      o.psi = ld_own<T, STREAM>(A.uout + i);
      o.lo = ld_own<T, STREAM>(A.lo + i);
    }
  }
}

// The values a stage writes for one point: the accumulator (stages 1-3),
// the next stage input or, at stage 4, Psi, and (stage 4, compensated) the
// new compensation term.  u is the point's stage input (Psi itself at stage
// 1); o its own operands.
template <typename T>
struct StageOut {
  cpx<T> acc, out, lo;
};

template <typename T, int STAGE, int COMP>
__device__ __forceinline__ StageOut<T> stage_values(T ca, T cn, double ca_d, cpx<T> u, cpx<T> K, const Own<T>& o) {
  StageOut<T> r;
  if constexpr (STAGE == 1) {
    r.acc = COMP ? mk<T>(ca * K.re, ca * K.im) : mk<T>(fmaT(ca, K.re, u.re), fmaT(ca, K.im, u.im));
    r.out = mk<T>(fmaT(cn, K.re, u.re), fmaT(cn, K.im, u.im));
  } else if constexpr (STAGE == 2 || STAGE == 3) {
    r.acc = mk<T>(fmaT(ca, K.re, o.acc.re), fmaT(ca, K.im, o.acc.im));
    r.out = mk<T>(fmaT(cn, K.re, o.psi.re), fmaT(cn, K.im, o.psi.im));
  } else if constexpr (!COMP) {
    r.out = mk<T>(fmaT(ca, K.re, o.acc.re), fmaT(ca, K.im, o.acc.im));
  } else {
    // Psi_hi + Psi_lo + (acc + k/6 K4), summed in FP64 and split back.
    double inc_r = __builtin_fma(ca_d, (double)K.re, (double)o.acc.re);
    double inc_i = __builtin_fma(ca_d, (double)K.im, (double)o.acc.im);
    double sr = ((double)o.psi.re + (double)o.lo.re) + inc_r;
    double si = ((double)o.psi.im + (double)o.lo.im) + inc_i;
    T hr = (T)sr, hi = (T)si;
    r.out = mk<T>(hr, hi);
    r.lo = mk<T>((T)(sr - (double)hr), (T)(si - (double)hi));
  }
  return r;
}

template <typename T, int STAGE, int COMP, bool STREAM = false>
__device__ __forceinline__ void stage_update(const StageArgs<T>& A, int64_t i, cpx<T> u, cpx<T> K,
                                             const Own<T>& o) {
  const StageOut<T> r = stage_values<T, STAGE, COMP>(A.c_acc, A.c_next, A.c_acc_d, u, K, o);
  if constexpr (STAGE <= 3) st_own<T, STREAM>(A.acc + i, r.acc);
  st_own<T, STREAM>(A.uout + i, r.out);
  if constexpr (STAGE == 4 && COMP) st_own<T, STREAM>(A.lo + i, r.lo);
}

// ---------------------------------------------------------------- tiles

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous run of tile indices so tiles that share halos share an L2.
__device__ __forceinline__ int xcd_swizzle(int bid, int nb) {
  int q = nb >> 3, r = nb & 7;
  int xcd = bid & 7, local = bid >> 3;
  return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

// Tile origin along one axis.  The last tile is shifted back so it ends at
// n-1 (it never holds fewer than min(T, n) >= 2 points), which keeps every
// boundary point and its MSD interior neighbour in the same tile.  Points of
// the overlap are stored only by the earlier tile.
__device__ __forceinline__ int tile_origin(int t, int T, int n) {
  int o = t * T;
  return (o + T > n) ? (n > T ? n - T : 0) : o;
}

}  // namespace nlse
