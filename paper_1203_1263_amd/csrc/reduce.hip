// Mass and energy of a grid (the standard NLSE invariants; the paper defines
// neither):
//   M = h^d sum |Psi|^2
//   E = h^d [ sum_interior -a Re(conj(Psi) L Psi) + sum ( V|Psi|^2 - (s/2)|Psi|^4 ) ]
// with L the scheme Laplacian (CD2, or 2SHOC reading the boundary D of the
// chosen condition, Eqs. BCDlap / BCMSDlap / BCL0lap).  Stored values are promoted to
// FP64 and every operation below runs in FP64.
//
// Determinism: workgroup b always reduces the fixed index range
// [b*C, (b+1)*C) with a fixed per-lane order, a fixed wavefront shuffle tree
// and a fixed cross-wave order; a single workgroup then sums the partials in
// a fixed order.  The result is bitwise reproducible and independent of the
// stage kernels' tile shapes.
#include <algorithm>
#include <mutex>

#include "nlse_device.hpp"
#include "nlse_internal.h"

namespace nlse {

// ND (the number of active axes) is a template parameter so every loop over
// the axes unrolls and the coordinate arrays stay in registers.
template <typename T, int ND>
struct View {
  const cpx<T>* u;
  const T* V;
  int n[3];
  int64_t st[3];
  double a, s, inv_a, inv_h2, inv_6h2;
};

template <typename T, int ND>
__device__ __forceinline__ cpx<double> ldd(const View<T, ND>& g, const int c[3]) {
  cpx<T> v = g.u[c[0] * g.st[0] + c[1] * g.st[1] + c[2] * g.st[2]];
  return mk<double>((double)v.re, (double)v.im);
}

template <typename T, int ND>
__device__ __forceinline__ double vd(const View<T, ND>& g, const int c[3]) {
  return g.V ? (double)g.V[c[0] * g.st[0] + c[1] * g.st[1] + c[2] * g.st[2]] : 0.0;
}

template <typename T, int ND>
__device__ __forceinline__ bool on_bnd(const View<T, ND>& g, const int c[3]) {
#pragma unroll
  for (int d = 0; d < ND; ++d)
    if (c[d] == 0 || c[d] == g.n[d] - 1) return true;
  return false;
}

template <typename T, int ND>
__device__ cpx<double> cd2_at(const View<T, ND>& g, const int c[3]) {
  cpx<double> u = ldd(g, c);
  double sr = 0.0, si = 0.0;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    int p[3] = {c[0], c[1], c[2]};
    p[d] = c[d] + 1;
    cpx<double> a = ldd(g, p);
    p[d] = c[d] - 1;
    cpx<double> b = ldd(g, p);
    sr += (a.re - u.re) + (b.re - u.re);
    si += (a.im - u.im) + (b.im - u.im);
  }
  return mk<double>(sr * g.inv_h2, si * g.inv_h2);
}

template <typename T, int ND>
__device__ __forceinline__ double nl_d(const View<T, ND>& g, cpx<double> u, double v) {
  return g.s * (u.re * u.re + u.im * u.im) - v;
}

// 2SHOC step-1 value D at any point: CD2 inside, boundary form on the edge.
template <typename T, int ND>
__device__ cpx<double> D_at(const View<T, ND>& g, int bc, const int c[3]) {
  if (!on_bnd(g, c)) return cd2_at(g, c);
  if (bc == kL0) return mk<double>(0.0, 0.0);  // Eq. BCL0lap
  cpx<double> ub = ldd(g, c);
  double Nb = nl_d(g, ub, vd(g, c));
  if (bc == kDirichlet) {
    double f = -Nb * g.inv_a;
    return mk<double>(f * ub.re, f * ub.im);
  }
  int q[3] = {c[0], c[1], c[2]};
#pragma unroll
  for (int d = 0; d < ND; ++d) q[d] += inward(c[d], g.n[d]);
  cpx<double> uq = ldd(g, q);
  cpx<double> Dq = cd2_at(g, q);
  double m = uq.re * uq.re + uq.im * uq.im;
  double r = (m == 0.0) ? 0.0 : (Dq.re * uq.re + Dq.im * uq.im) / m;
  double f = r + (nl_d(g, uq, vd(g, q)) - Nb) * g.inv_a;
  return mk<double>(f * ub.re, f * ub.im);
}

// Coordinates of linear index i (x fastest): 32-bit divisions when the grid
// has fewer than 2^31 points (64-bit division costs far more).
template <typename T, int ND>
__device__ __forceinline__ void coords(const View<T, ND>& g, int64_t i, int c[3]) {
  if (i <= 0x7fffffff) {
    const unsigned u = (unsigned)i, n0 = (unsigned)g.n[0], n1 = (unsigned)g.n[1];
    const unsigned q = u / n0;
    c[0] = (int)(u - q * n0);
    c[1] = (int)(q % n1);
    c[2] = (int)(q / n1);
  } else {
    c[0] = (int)(i % g.n[0]);
    c[1] = (int)((i / g.n[0]) % g.n[1]);
    c[2] = (int)(i / ((int64_t)g.n[0] * g.n[1]));
  }
}

template <typename T, int ND>
__device__ __forceinline__ int64_t lin(const View<T, ND>& g, const int c[3]) {
  return c[0] * g.st[0] + c[1] * g.st[1] + c[2] * g.st[2];
}

// 2SHOC step 1 at every point, stored once (FP64) for the energy pass: the
// Laplacian of each interior point then reads its own and its 2d
// neighbours' D instead of recomputing them.
template <typename T, int ND>
__global__ __launch_bounds__(256) void reduce_d_kernel(View<T, ND> g, int bc, int64_t npts, cpx<double>* D) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < npts; i += (int64_t)gridDim.x * 256) {
    int c[3];
    coords(g, i, c);
    D[i] = D_at(g, bc, c);
  }
}

// 2SHOC D of a point: read from the stored pass, or (no D array) computed
// on the spot by the same function the stored pass runs, so both give the
// same value.
template <bool STORED, typename T, int ND>
__device__ __forceinline__ cpx<double> D_get(const View<T, ND>& g, int bc, const cpx<double>* D, const int c[3]) {
  if constexpr (STORED) return D[lin(g, c)];
  else return D_at(g, bc, c);
}

// Scheme Laplacian at an interior point (2SHOC from the stored D, or from D
// recomputed at the point and its 2d face neighbours).
template <bool STORED, typename T, int ND>
__device__ cpx<double> L_at(const View<T, ND>& g, int order, int bc, const cpx<double>* D, const int c[3]) {
  if (order == 2) return cd2_at(g, c);
  cpx<double> D0 = D_get<STORED>(g, bc, D, c);
  cpx<double> u0 = ldd(g, c);
  double fr = 0.0, fi = 0.0, er = 0.0, ei = 0.0;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    for (int sgn = -1; sgn <= 1; sgn += 2) {
      int p[3] = {c[0], c[1], c[2]};
      p[d] += sgn;
      cpx<double> Df = D_get<STORED>(g, bc, D, p);
      fr += Df.re - D0.re;
      fi += Df.im - D0.im;
    }
  }
#pragma unroll
  for (int d1 = 0; d1 < ND; ++d1)
    for (int d2 = d1 + 1; d2 < ND; ++d2)
      for (int s1 = -1; s1 <= 1; s1 += 2)
        for (int s2 = -1; s2 <= 1; s2 += 2) {
          int p[3] = {c[0], c[1], c[2]};
          p[d1] += s1;
          p[d2] += s2;
          cpx<double> ue = ldd(g, p);
          er += ue.re - u0.re;
          ei += ue.im - u0.im;
        }
  double c0 = ND == 1 ? 1.0 : (ND == 2 ? 2.0 / 3.0 : 1.0 / 3.0);
  return mk<double>(c0 * D0.re - fr / 12.0 + g.inv_6h2 * er, c0 * D0.im - fi / 12.0 + g.inv_6h2 * ei);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <bool STORED, typename T, int ND>
__global__ __launch_bounds__(256) void reduce_partial_kernel(View<T, ND> g, int order, int bc, const cpx<double>* D,
                                                             int64_t npts, double* partials) {
  __shared__ double red[3][4];
  const int64_t b0 = (int64_t)blockIdx.x * kReduceChunk;
  const int64_t b1 = min(b0 + (int64_t)kReduceChunk, npts);
  double m = 0.0, kin = 0.0, pot = 0.0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += 256) {
    int c[3];
    coords(g, i, c);
    cpx<double> u = ldd(g, c);
    double rho = u.re * u.re + u.im * u.im;
    m += rho;
    pot += vd(g, c) * rho - 0.5 * g.s * rho * rho;
    if (!on_bnd(g, c)) {
      cpx<double> L = L_at<STORED>(g, order, bc, D, c);
      kin += -g.a * (u.re * L.re + u.im * L.im);
    }
  }
  m = wave_sum(m);
  kin = wave_sum(kin);
  pot = wave_sum(pot);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = m;
    red[1][w] = kin;
    red[2][w] = pot;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int k = threadIdx.x;
    partials[blockIdx.x * 3 + k] = (red[k][0] + red[k][1]) + (red[k][2] + red[k][3]);
  }
}

__global__ __launch_bounds__(256) void reduce_final_kernel(const double* partials, int64_t nb, double* out) {
  __shared__ double red[3][256];
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t j = threadIdx.x; j < nb; j += 256)
    for (int k = 0; k < 3; ++k) acc[k] += partials[j * 3 + k];
  for (int k = 0; k < 3; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int s = 128; s >= 1; s >>= 1) {
    if (threadIdx.x < s)
      for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < 3) out[threadIdx.x] = red[threadIdx.x][0];
}

__global__ void fill_zero_kernel(uint32_t* p, int64_t nwords) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < nwords; i += stride) p[i] = 0u;
}

__global__ void copy_words_kernel(const uint2* __restrict__ src, uint2* __restrict__ dst, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) dst[i] = src[i];
}

template <typename T, int ND>
static hipError_t reduce_dim(const ReduceLaunch& R, hipStream_t st) {
  View<T, ND> g;
  g.u = static_cast<const cpx<T>*>(R.psi);
  g.V = static_cast<const T*>(R.V);
  for (int d = 0; d < 3; ++d) g.n[d] = (int)R.n[d];
  g.st[0] = 1;
  g.st[1] = R.n[0];
  g.st[2] = R.n[0] * R.n[1];
  g.a = R.a;
  g.s = R.s;
  g.inv_a = 1.0 / R.a;
  g.inv_h2 = 1.0 / (R.h * R.h);
  g.inv_6h2 = 1.0 / (6.0 * R.h * R.h);
  const int64_t npts = R.n[0] * R.n[1] * R.n[2];
  const int64_t nb = reduce_blocks(npts);
  cpx<double>* D = nullptr;
  if (R.order == 4 && R.dscratch) {
    D = static_cast<cpx<double>*>(R.dscratch);
    const int64_t blocks = std::min<int64_t>((npts + 255) / 256, 8192);
    hipLaunchKernelGGL((reduce_d_kernel<T, ND>), dim3((unsigned)blocks), dim3(256), 0, st, g, R.bc, npts, D);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (D)
    hipLaunchKernelGGL((reduce_partial_kernel<true, T, ND>), dim3((unsigned)nb), dim3(256), 0, st, g, R.order, R.bc,
                       D, npts, R.partials);
  else
    hipLaunchKernelGGL((reduce_partial_kernel<false, T, ND>), dim3((unsigned)nb), dim3(256), 0, st, g, R.order,
                       R.bc, D, npts, R.partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(256), 0, st, R.partials, nb, R.out);
  return hipGetLastError();
}

template <typename T>
static hipError_t reduce_typed(const ReduceLaunch& R, hipStream_t st) {
  switch (R.ndim) {
    case 1: return reduce_dim<T, 1>(R, st);
    case 2: return reduce_dim<T, 2>(R, st);
    case 3: return reduce_dim<T, 3>(R, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace nlse

hipError_t nlse_launch_reduce(const nlse::ReduceLaunch& R, hipStream_t st) {
  return R.dtype == 0 ? nlse::reduce_typed<float>(R, st) : nlse::reduce_typed<double>(R, st);
}

// Device-to-device copy of nbytes (a multiple of 8, both pointers 8-byte
// aligned) as a kernel: it runs at HBM speed on the given stream, where a
// runtime copy may go to a copy engine of far lower bandwidth.
hipError_t nlse_launch_copy(void* dst, const void* src, int64_t nbytes, hipStream_t st) {
  int64_t n = nbytes / 8;
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(nlse::copy_words_kernel, dim3((unsigned)blocks), dim3(256), 0, st,
                     static_cast<const uint2*>(src), static_cast<uint2*>(dst), n);
  return hipGetLastError();
}

// Clears nbytes (a multiple of 4) with a kernel instead of a memset node, so
// the call is safe inside a captured graph.
hipError_t nlse_launch_fill_zero(void* p, int64_t nbytes, hipStream_t st) {
  int64_t nw = nbytes / 4;
  if (nw <= 0) return hipSuccess;
  int64_t blocks = (nw + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(nlse::fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, st,
                     static_cast<uint32_t*>(p), nw);
  return hipGetLastError();
}

// ---------------------------------------------------------------- static scratch

// Partial sums (three per reduction workgroup) and the three result doubles
// of nlse_mass_energy_noalloc, so that entry point needs no device
// allocation.  A file-scope device array: every device the library runs on
// holds its own copy from module load until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol); it uses the device address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double scratch[nlse::kStaticReduceBlocks * 3 + 32];

hipError_t nlse_static_reduce_scratch(double** partials, double** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static double* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[dev] = static_cast<double*>(p);
  }
  *partials = addr[dev];
  *out = addr[dev] + nlse::kStaticReduceBlocks * 3;
  return hipSuccess;
}
