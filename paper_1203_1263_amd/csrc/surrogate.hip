// Learned surrogate of 16 RK4 steps: a 6-layer 3x3 convolutional residual
// network on the field's two real channels (2 -> 48 -> 48 -> 48 -> 48 -> 48
// -> 2, ReLU after layers 1-5, zero "same" padding, pred = psi + net(psi)).
// BF16 weights and activations, FP32 accumulation on the matrix cores
// (v_mfma_f32_16x16x32_bf16), FP32 master weights and Adam.
//
// Activations are NHWC BF16 with the channel count padded to a multiple of 8
// (input 2 -> 8, last-layer output 2 -> 16).  A 3x3 convolution is an implicit
// GEMM: D[co][pixel] = sum_k W[co][k] X[k][pixel] with k = (tap, ci), tap =
// 3 ky + kx.  A persistent workgroup computes 16x16 pixel tiles for every
// output channel: the weights ([co][tap][ci], K contiguous, staged once) and
// the input tile with a one-pixel halo ([pixel][ci]) sit in LDS; each wave
// owns four pixel rows and all channel blocks.  The backward data pass is the same kernel with flipped
// taps and transposed channels, masked by the ReLU of the stored activation.
// The weight gradient is a second MFMA kernel (pixels are the reduction
// dimension) writing per-workgroup partials that a fixed-order pass sums, so
// gradients are bitwise reproducible.
#include <stdint.h>

#include <algorithm>

#include "nlse_device.hpp"
#include "nlse_surrogate.h"

namespace nlse {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }
__device__ __forceinline__ uint4 zero4() { return make_uint4(0u, 0u, 0u, 0u); }

__device__ __forceinline__ uint16_t bf16_bits(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float bf16_val(uint16_t b) { return (float)__builtin_bit_cast(__bf16, b); }

// ---------------------------------------------------------------- packing

// complex64 field [n] -> BF16 [n][8] = (re, im, 0, ..., 0)
__global__ void pack_input_kernel(const float2* __restrict__ psi, uint4* __restrict__ x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    float2 v = psi[i];
    uint4 o;
    o.x = (uint32_t)bf16_bits(v.x) | ((uint32_t)bf16_bits(v.y) << 16);
    o.y = o.z = o.w = 0u;
    x[i] = o;
  }
}

// ---------------------------------------------------------------- conv

struct ConvArgs {
  const uint16_t* in;    // [B][H][W][CIN] BF16
  const uint16_t* w;     // [COUT][9][CIN] BF16
  const float* bias;     // [COUT] (forward) or null
  uint16_t* out;         // [B][H][W][COUT] BF16 (relu / dgrad)
  const float2* x;       // network input field (last layer)
  float2* pred;          // prediction (last layer)
  const uint16_t* mask;  // dgrad: activation whose sign gates the gradient, [B][H][W][COUT]
  int H, W;
  int project;           // last layer: MSD projection of the boundary ring
  double* tile_mass;     // last layer, or null: sum of |pred|^2 of every tile
};

enum { kEpiRelu = 0, kEpiLast = 1, kEpiDgrad = 2 };

// Persistent: a workgroup stages the layer's weights in LDS once and then
// walks pixel tiles tile = blockIdx.x, + gridDim.x, ...; the input of its
// next tile is loaded into registers while the current tile is computed.
// LDS rows are padded by 16 bytes (weights: K + 8, pixels: CIN + 8 BF16
// values) so the 16-byte operand reads of 16 lanes hit distinct banks.
// NW waves per workgroup, each owning 16 / NW pixel rows of the tile and
// every output channel block; launch bounds ask for two workgroups per CU
// (NW / 2 waves per SIMD).
template <int CIN, int COUT, int EPI, int NW>
__global__ __launch_bounds__(64 * NW, NW / 2) void conv3x3_kernel(ConvArgs a, int ntiles) {
  constexpr int NTH = 64 * NW;  // threads
  constexpr int RPW = 16 / NW;  // pixel rows per wave
  constexpr int K = 9 * CIN;
  constexpr int KP = K + 8;    // padded weight row
  constexpr int CP = CIN + 8;  // padded input pixel
  constexpr int KSTEPS = (K + 31) / 32;
  constexpr int NCB = COUT / 16;
  constexpr int CH = CIN / 8;  // 16-byte chunks per input pixel
  constexpr int NCHUNK = 18 * 18 * CH;
  constexpr int NLD = (NCHUNK + NTH - 1) / NTH;
  __shared__ __attribute__((aligned(16))) uint16_t sIn[18 * 18 * CP];
  __shared__ __attribute__((aligned(16))) uint16_t sW[COUT * KP];
  __shared__ double sMass[NW];

  const int tid = threadIdx.x;
  const int tilesx = a.W / 16, tilesy = a.H / 16;

  // weights -> LDS once (16-byte chunks; K is a multiple of 8)
  {
    const uint4* src = reinterpret_cast<const uint4*>(a.w);
    uint4* dst = reinterpret_cast<uint4*>(sW);
    for (int i = tid; i < COUT * K / 8; i += NTH) {
      const int row = i / (K / 8), c = i - row * (K / 8);
      dst[row * (KP / 8) + c] = src[i];
    }
  }

  // input tile with a one-pixel halo, zero outside the image
  uint4 pre[NLD];
  auto load_tile = [&](int t) {
    const int b = t / (tilesx * tilesy);
    const int ty = (t / tilesx) % tilesy, tx = t % tilesx;
    const int64_t img = (int64_t)b * a.H * a.W;
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
      const int i = tid + NTH * k;
      uint4 v = zero4();
      if (i < NCHUNK) {
        const int pp = i / CH, part = i - pp * CH;
        const int py = pp / 18, px = pp - py * 18;
        const int gy = ty * 16 - 1 + py, gx = tx * 16 - 1 + px;
        if (gy >= 0 && gy < a.H && gx >= 0 && gx < a.W)
          v = reinterpret_cast<const uint4*>(a.in + (img + (int64_t)gy * a.W + gx) * CIN)[part];
      }
      pre[k] = v;
    }
  };
  auto store_tile = [&]() {
    uint4* dst = reinterpret_cast<uint4*>(sIn);
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
      const int i = tid + NTH * k;
      if (i < NCHUNK) {
        const int pp = i / CH, part = i - pp * CH;
        dst[pp * (CP / 8) + part] = pre[k];
      }
    }
  };

  const int wave = tid >> 6, lane = tid & 63;
  const int j = lane & 15, g = lane >> 4;
  int t = blockIdx.x;
  if (t < ntiles) load_tile(t);
  for (; t < ntiles; t += gridDim.x) {
    __syncthreads();  // the previous tile's operand reads are done (and the weights are in)
    store_tile();
    __syncthreads();
    if (t + (int)gridDim.x < ntiles) load_tile(t + gridDim.x);

    const int b = t / (tilesx * tilesy);
    const int ty = (t / tilesx) % tilesy, tx = t % tilesx;
    const int x0 = tx * 16, y0 = ty * 16;
    const int64_t img = (int64_t)b * a.H * a.W;

    f32x4 acc[NCB][RPW];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int rr = 0; rr < RPW; ++rr) acc[cb][rr] = f32x4{0.f, 0.f, 0.f, 0.f};
    // backward data from the 16-channel last layer: the ReLU mask of this
    // lane's outputs is loaded before the k-loop so its latency overlaps the
    // MFMAs (the 48-channel variant has no registers left for it: at 128 it
    // spills and was measured slower, so it loads the mask in the epilogue)
    constexpr bool kMaskEarly = EPI == kEpiDgrad && CIN < 48;
    uint2 mk[RPW][NCB];
    if constexpr (kMaskEarly) {
#pragma unroll
      for (int rr = 0; rr < RPW; ++rr)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          const int64_t pix = img + (int64_t)(y0 + RPW * wave + rr) * a.W + (x0 + j);
          mk[rr][cb] = *reinterpret_cast<const uint2*>(a.mask + pix * COUT + 16 * cb + 4 * g);
        }
    }

    // operands of k-step ks (weights: 16 output channels x 32 k; input: 32 k
    // x 16 pixels of one row), read from LDS
    auto frags = [&](int ks, bf16x8 (&af)[NCB], bf16x8 (&bfr)[RPW]) {
      const int k0 = 32 * ks + 8 * g;
      const bool kv = k0 < K;
      const int tap = kv ? k0 / CIN : 0, ci0 = kv ? k0 % CIN : 0;
      const int dy = tap / 3, dx = tap - 3 * dy;
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
        af[cb] = as_bf16x8(kv ? *reinterpret_cast<const uint4*>(&sW[(16 * cb + j) * KP + k0]) : zero4());
#pragma unroll
      for (int rr = 0; rr < RPW; ++rr) {
        const int row = RPW * wave + rr;
        bfr[rr] = as_bf16x8(kv ? *reinterpret_cast<const uint4*>(&sIn[((row + dy) * 18 + j + dx) * CP + ci0]) : zero4());
      }
    };
    auto mfmas = [&](const bf16x8 (&af)[NCB], const bf16x8 (&bfr)[RPW]) {
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int rr = 0; rr < RPW; ++rr)
          acc[cb][rr] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[cb], bfr[rr], acc[cb][rr], 0, 0, 0);
    };
    if constexpr (NW == 4) {
      // two operand sets: the reads of step ks+1 are in flight while the
      // matrix cores work on step ks (each accumulator still sums the
      // k-steps in ascending order)
      bf16x8 a0[NCB], b0[RPW], a1[NCB], b1[RPW];
      frags(0, a0, b0);
      int ks = 0;
      for (; ks + 1 < KSTEPS; ks += 2) {
        frags(ks + 1, a1, b1);
        mfmas(a0, b0);
        if (ks + 2 < KSTEPS) frags(ks + 2, a0, b0);
        mfmas(a1, b1);
      }
      if (ks < KSTEPS) mfmas(a0, b0);
    } else {
      // one operand set: the other waves of the SIMD cover the LDS latency
      bf16x8 a0[NCB], b0[RPW];
      for (int ks = 0; ks < KSTEPS; ++ks) {
        frags(ks, a0, b0);
        mfmas(a0, b0);
      }
    }

    // lane holds D[co = 16 cb + 4 g + r][pixel (row, j)], r = 0..3
    double mass = 0.0;  // last layer: |pred|^2 of this lane's pixels, rows in order
#pragma unroll
    for (int rr = 0; rr < RPW; ++rr) {
      const int row = RPW * wave + rr;
      const int64_t pix = img + (int64_t)(y0 + row) * a.W + (x0 + j);
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const int co = 16 * cb + 4 * g;
        float v[4] = {acc[cb][rr][0], acc[cb][rr][1], acc[cb][rr][2], acc[cb][rr][3]};
        if constexpr (EPI == kEpiRelu) {
#pragma unroll
          for (int r = 0; r < 4; ++r) v[r] = fmaxf(v[r] + a.bias[co + r], 0.f);
        } else if constexpr (EPI == kEpiDgrad) {
          const uint2 m = kMaskEarly ? mk[rr][cb] : *reinterpret_cast<const uint2*>(a.mask + pix * COUT + co);
          const uint16_t mb[4] = {(uint16_t)(m.x & 0xffffu), (uint16_t)(m.x >> 16), (uint16_t)(m.y & 0xffffu),
                                  (uint16_t)(m.y >> 16)};
#pragma unroll
          for (int r = 0; r < 4; ++r) v[r] = bf16_val(mb[r]) > 0.f ? v[r] : 0.f;
        }
        if constexpr (EPI == kEpiLast) {
          if (g == 0) {  // channels 0, 1 are the real and imaginary increments
            const float2 xv = a.x[pix];
            float2 p = make_float2(xv.x + (v[0] + a.bias[0]), xv.y + (v[1] + a.bias[1]));
            const int py = y0 + row, px = x0 + j;
            if (a.project && (py == 0 || py == a.H - 1 || px == 0 || px == a.W - 1)) {
              // the operations of msd_project_kernel, so both give the same bits
              const float mi = sqrtf(xv.x * xv.x + xv.y * xv.y), mo = sqrtf(p.x * p.x + p.y * p.y);
              if (mo > 0.f) p = make_float2(p.x * (mi / mo), p.y * (mi / mo));
            }
            a.pred[pix] = p;
            mass += (double)p.x * p.x + (double)p.y * p.y;
          }
        } else {
          uint2 o;
          o.x = (uint32_t)bf16_bits(v[0]) | ((uint32_t)bf16_bits(v[1]) << 16);
          o.y = (uint32_t)bf16_bits(v[2]) | ((uint32_t)bf16_bits(v[3]) << 16);
          *reinterpret_cast<uint2*>(a.out + pix * COUT + co) = o;
        }
      }
    }
    if constexpr (EPI == kEpiLast) {
      // tile mass in a fixed order: lanes (a fixed shuffle tree), then the
      // waves in ascending order
      if (a.tile_mass) {
        for (int off = 32; off >= 1; off >>= 1) mass += __shfl_xor(mass, off, 64);
        if (lane == 0) sMass[wave] = mass;
        __syncthreads();
        if (tid == 0) {
          double t_m = 0.0;
#pragma unroll
          for (int w = 0; w < NW; ++w) t_m += sMass[w];
          a.tile_mass[t] = t_m;
        }
      }
    }
  }
}

// ---------------------------------------------------------------- whole network, small batches

// Inference for small batches: one workgroup takes one 16x16 output tile
// through all six layers, with the activations in LDS instead of HBM.  Layer
// l (1..6) is evaluated on the tile plus a ring of 6 - l pixels (26^2, 24^2,
// ..., 16^2 pixels), which is exactly what the layers after it read; ring
// pixels outside the image are stored as zero, the padding the layer-by-layer
// pass applies.  Activations are stored channel-chunk major
// ([ci / 8][pixel][8 values]), so the 16 lanes of an operand read take 256
// contiguous bytes (no bank conflicts without padding, which would not fit:
// weights 42 KB + the two largest regions 117 KB).  Every accumulator takes
// the k-steps, operands and MFMAs of conv3x3_kernel in the same order and
// the epilogues are the same operations, so both passes give the same bits.
// The next layer's weights are loaded into registers while a layer computes.
struct NetArgs {
  const float2* x;            // network input fields [B][H][W]
  float2* pred;               // prediction
  const uint16_t* w[6];       // forward-layout BF16 weights of each layer
  const float* bias[6];       // FP32 biases
  int H, W;
  int project;                // MSD projection of the boundary ring
  double* tile_mass;          // or null: per 16x16 tile, sum of |pred|^2
};

constexpr int kNetWaves = 8;
constexpr int kNetThreads = 64 * kNetWaves;
constexpr int kNetPre = (48 * 9 * 48 / 8 + kNetThreads - 1) / kNetThreads;  // 16-byte weight chunks per thread

template <int CIN, int COUT>
__device__ __forceinline__ void net_load_w(const uint16_t* w, uint4 (&r)[kNetPre], int tid) {
  constexpr int N = COUT * 9 * CIN / 8;
  const uint4* src = reinterpret_cast<const uint4*>(w);
#pragma unroll
  for (int k = 0; k < kNetPre; ++k) {
    const int i = tid + kNetThreads * k;
    uint4 v = zero4();
    if (i < N) v = src[i];
    r[k] = v;
  }
}

// weights [COUT][9 CIN] into LDS rows padded to 9 CIN + 8 values
template <int CIN, int COUT>
__device__ __forceinline__ void net_put_w(uint16_t* sW, const uint4 (&r)[kNetPre], int tid) {
  constexpr int K = 9 * CIN, KP = K + 8, N = COUT * K / 8;
  uint4* dst = reinterpret_cast<uint4*>(sW);
#pragma unroll
  for (int k = 0; k < kNetPre; ++k) {
    const int i = tid + kNetThreads * k;
    if (i < N) {
      const int row = i / (K / 8), c = i - row * (K / 8);
      dst[row * (KP / 8) + c] = r[k];
    }
  }
}

// The layer's input offset of every (k-step, lane group): k0 = 32 ks + 8 g =
// tap CIN + ci0, tap = 3 dy + dx -> (ci0 / 8) SI^2 + dy SI + dx
template <int CIN>
__device__ __forceinline__ void net_put_off(int* sOff, int SI, int tid) {
  constexpr int K = 9 * CIN, KSTEPS = (K + 31) / 32;
  if (tid < 4 * KSTEPS) {
    const int k0 = 32 * (tid >> 2) + 8 * (tid & 3);
    int off = 0;
    if (k0 < K) {
      const int tap = k0 / CIN, ci0 = k0 - tap * CIN;
      const int dy = tap / 3, dx = tap - 3 * dy;
      off = (ci0 >> 3) * SI * SI + dy * SI + dx;
    }
    sOff[tid] = off;
  }
}

// One layer: activation region `in` (SI x SI pixels) -> region of
// SO = SI - 2 pixels whose first pixel is (gx0, gy0) in image `img`.  Wave w
// takes the pixel-block pairs w, w + kNetWaves, ... (16 pixels per block, in
// region order); on the last layer (SO = 16) that is rows 2w, 2w + 1 of the
// tile, the rows conv3x3_kernel gives its wave w.
template <int CIN, int COUT, bool LAST>
__device__ __forceinline__ void net_layer(NetArgs a, const float* bias, const uint16_t* sW, const uint16_t* in, int SI,
                                          uint16_t* out, int gx0, int gy0, int64_t img, double* sMass, int t,
                                          const float2 (&xq)[2], const int* sOff) {
  constexpr int K = 9 * CIN;
  constexpr int KP = K + 8;
  constexpr int KSTEPS = (K + 31) / 32;
  constexpr int NCB = COUT / 16;
  const int SO = SI - 2, npo = SO * SO, npi = SI * SI;
  const int npairs = (npo + 31) / 32;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int j = lane & 15, g = lane >> 4;
  double mass = 0.0;
  for (int q = wave; q < npairs; q += kNetWaves) {
    int base[2];
#pragma unroll
    for (int rr = 0; rr < 2; ++rr) {
      const int n = min(32 * q + 16 * rr + j, npo - 1);
      const int py = n / SO, px = n - py * SO;
      base[rr] = py * SI + px;
    }
    f32x4 acc[NCB][2];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int rr = 0; rr < 2; ++rr) acc[cb][rr] = f32x4{0.f, 0.f, 0.f, 0.f};
    // operands of k-step ks (weights: 16 output channels x 32 k; input: 32 k
    // x 16 pixels), two sets: the LDS reads of step ks + 1 are in flight
    // while the matrix cores work on step ks (each accumulator still sums
    // the k-steps in ascending order)
    // Operands of k-step ks (weights: 16 output channels x 32 k; input: 32 k
    // x 16 pixels).  The input offset of lane group g comes from the layer's
    // table, (ci0 / 8) npi + dy SI + dx for k0 = 32 ks + 8 g = CIN tap + ci0;
    // the entry of step ks + 1 is read while step ks loads.  The first
    // KF = K / 32 steps have every lane group in range; K = 432 or 72 leaves
    // one partial step, peeled off the loop, whose out-of-range groups read
    // in-range operands (offset 0) and mask them to zero.  Two operand sets:
    // the reads of step ks + 1 are in flight while the matrix cores work on
    // step ks; each accumulator sums the k-steps in ascending order.
    constexpr int KF = K / 32;
    constexpr bool TAIL = K % 32 != 0;
    static_assert(KF >= 2, "at least two full k-steps");
    int offn = sOff[g];
    auto frags = [&](int ks, bf16x8 (&af)[NCB], bf16x8 (&bfr)[2]) {
      const int off = offn;
      if (ks + 1 < KSTEPS) offn = sOff[4 * (ks + 1) + g];
      const int k0 = 32 * ks + 8 * g;
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) af[cb] = as_bf16x8(*reinterpret_cast<const uint4*>(&sW[(16 * cb + j) * KP + k0]));
#pragma unroll
      for (int rr = 0; rr < 2; ++rr) bfr[rr] = as_bf16x8(*reinterpret_cast<const uint4*>(&in[(off + base[rr]) * 8]));
    };
    auto frags_tail = [&](bf16x8 (&af)[NCB], bf16x8 (&bfr)[2]) {
      const int k0 = 32 * KF + 8 * g;
      const uint32_t msk = k0 < K ? 0xffffffffu : 0u;  // offn is 0 where k0 >= K
      const int kc = k0 < K ? k0 : 0;
      auto mask = [&](uint4 v) { return make_uint4(v.x & msk, v.y & msk, v.z & msk, v.w & msk); };
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
        af[cb] = as_bf16x8(mask(*reinterpret_cast<const uint4*>(&sW[(16 * cb + j) * KP + kc])));
#pragma unroll
      for (int rr = 0; rr < 2; ++rr)
        bfr[rr] = as_bf16x8(mask(*reinterpret_cast<const uint4*>(&in[(offn + base[rr]) * 8])));
    };
    auto mfmas = [&](const bf16x8 (&af)[NCB], const bf16x8 (&bfr)[2]) {
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int rr = 0; rr < 2; ++rr)
          acc[cb][rr] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[cb], bfr[rr], acc[cb][rr], 0, 0, 0);
    };
    bf16x8 a0[NCB], b0[2], a1[NCB], b1[2];
    frags(0, a0, b0);
#pragma unroll 1
    for (int ks = 0; ks + 2 < KF; ks += 2) {
      frags(ks + 1, a1, b1);
      mfmas(a0, b0);
      frags(ks + 2, a0, b0);
      mfmas(a1, b1);
    }
    // a0 holds full step KE; the full step KE + 1 (if any) and the tail remain
    constexpr int KE = 2 * ((KF - 1) / 2);
    if constexpr (KE + 1 < KF) {
      frags(KE + 1, a1, b1);
      mfmas(a0, b0);
      if constexpr (TAIL) {
        frags_tail(a0, b0);
        mfmas(a1, b1);
        mfmas(a0, b0);
      } else {
        mfmas(a1, b1);
      }
    } else {
      if constexpr (TAIL) {
        frags_tail(a1, b1);
        mfmas(a0, b0);
        mfmas(a1, b1);
      } else {
        mfmas(a0, b0);
      }
    }
    // lane holds D[co = 16 cb + 4 g + r][pixel n], r = 0..3
#pragma unroll
    for (int rr = 0; rr < 2; ++rr) {
      const int n = 32 * q + 16 * rr + j;
      if (n >= npo) continue;
      const int py = n / SO, px = n - py * SO;
      const int gy = gy0 + py, gx = gx0 + px;
      const int64_t pix = img + (int64_t)gy * a.W + gx;
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const int co = 16 * cb + 4 * g;
        float v[4] = {acc[cb][rr][0], acc[cb][rr][1], acc[cb][rr][2], acc[cb][rr][3]};
        if constexpr (LAST) {
          if (g == 0) {  // channels 0, 1 are the real and imaginary increments
            const float2 xv = xq[rr];  // a.x[pix], loaded when the tile started
            float2 p = make_float2(xv.x + (v[0] + bias[0]), xv.y + (v[1] + bias[1]));
            if (a.project && (gy == 0 || gy == a.H - 1 || gx == 0 || gx == a.W - 1)) {
              // the operations of msd_project_kernel, so both give the same bits
              const float mi = sqrtf(xv.x * xv.x + xv.y * xv.y), mo = sqrtf(p.x * p.x + p.y * p.y);
              if (mo > 0.f) p = make_float2(p.x * (mi / mo), p.y * (mi / mo));
            }
            a.pred[pix] = p;
            mass += (double)p.x * p.x + (double)p.y * p.y;
          }
        } else {
          uint2 o = make_uint2(0u, 0u);
          if (gy >= 0 && gy < a.H && gx >= 0 && gx < a.W) {
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] = fmaxf(v[r] + bias[co + r], 0.f);
            o.x = (uint32_t)bf16_bits(v[0]) | ((uint32_t)bf16_bits(v[1]) << 16);
            o.y = (uint32_t)bf16_bits(v[2]) | ((uint32_t)bf16_bits(v[3]) << 16);
          }
          *reinterpret_cast<uint2*>(&out[((co >> 3) * npo + n) * 8 + (co & 7)]) = o;
        }
      }
    }
  }
  if constexpr (LAST) {
    // tile mass in the order of conv3x3_kernel: lanes (a fixed shuffle
    // tree), then the waves that hold rows in ascending order
    if (a.tile_mass) {
      for (int off = 32; off >= 1; off >>= 1) mass += __shfl_xor(mass, off, 64);
      if (lane == 0 && wave < 8) sMass[wave] = mass;
      __syncthreads();
      if (tid == 0) {
        double t_m = 0.0;
#pragma unroll
        for (int w = 0; w < 8; ++w) t_m += sMass[w];
        a.tile_mass[t] = t_m;
      }
    }
  }
}

__global__ __launch_bounds__(kNetThreads, 1) void net_forward_kernel(NetArgs a, int ntiles) {
  // weights of one layer; regions: X = input (28^2 x 8), layer 2 (24^2 x 48),
  // layer 4 (20^2 x 48); Y = layer 1 (26^2 x 48), layer 3, layer 5
  __shared__ __attribute__((aligned(16))) uint16_t sW[48 * (9 * 48 + 8)];
  __shared__ __attribute__((aligned(16))) uint16_t sX[24 * 24 * 48];
  __shared__ __attribute__((aligned(16))) uint16_t sY[26 * 26 * 48];
  __shared__ double sMass[8];
  __shared__ float sBias[5 * 48 + 2];
  __shared__ int sOff[14 * 4];  // input offsets of the current layer's k-steps
  const int tid = threadIdx.x;
  const int tilesx = a.W / 16, tilesy = a.H / 16;
  // biases once (the last layer has 2 real output channels); visible after
  // the first barrier of the tile loop
  for (int i = tid; i < 5 * 48 + 2; i += kNetThreads) {
    const int l = i / 48, c = i - l * 48;
    sBias[i] = a.bias[l][c];
  }
  uint4 wr[kNetPre];
  float2 xq[2];  // last layer: the input at this lane's two output pixels
  int t = blockIdx.x;
  if (t < ntiles) net_load_w<8, 48>(a.w[0], wr, tid);
  for (; t < ntiles; t += gridDim.x) {
    const int b = t / (tilesx * tilesy);
    const int ty = (t / tilesx) % tilesy, tx = t % tilesx;
    const int x0 = tx * 16, y0 = ty * 16;
    const int64_t img = (int64_t)b * a.H * a.W;
    {
      const int wave = tid >> 6, j = tid & 15;
#pragma unroll
      for (int rr = 0; rr < 2; ++rr)
        xq[rr] = (wave < 8 && (tid & 63) < 16) ? a.x[img + (int64_t)(y0 + 2 * wave + rr) * a.W + x0 + j]
                                                : make_float2(0.f, 0.f);
    }
    __syncthreads();  // the previous tile's reads of sW and sY are done
    net_put_w<8, 48>(sW, wr, tid);
    net_put_off<8>(sOff, 28, tid);
    // network input on the tile plus a 6-pixel ring: (re, im, 0, ..., 0) as
    // BF16, zero outside the image (the conversion of pack_input_kernel)
    for (int p = tid; p < 28 * 28; p += kNetThreads) {
      const int py = p / 28, px = p - py * 28;
      const int gy = y0 - 6 + py, gx = x0 - 6 + px;
      uint4 o = zero4();
      if (gy >= 0 && gy < a.H && gx >= 0 && gx < a.W) {
        const float2 v = a.x[img + (int64_t)gy * a.W + gx];
        o.x = (uint32_t)bf16_bits(v.x) | ((uint32_t)bf16_bits(v.y) << 16);
      }
      reinterpret_cast<uint4*>(sX)[p] = o;
    }
    __syncthreads();
    net_load_w<48, 48>(a.w[1], wr, tid);
    net_layer<8, 48, false>(a, sBias + 0, sW, sX, 28, sY, x0 - 5, y0 - 5, img, sMass, t, xq, sOff);
    __syncthreads();
    net_put_w<48, 48>(sW, wr, tid);
    net_put_off<48>(sOff, 26, tid);
    __syncthreads();
    net_load_w<48, 48>(a.w[2], wr, tid);
    net_layer<48, 48, false>(a, sBias + 48, sW, sY, 26, sX, x0 - 4, y0 - 4, img, sMass, t, xq, sOff);
    __syncthreads();
    net_put_w<48, 48>(sW, wr, tid);
    net_put_off<48>(sOff, 24, tid);
    __syncthreads();
    net_load_w<48, 48>(a.w[3], wr, tid);
    net_layer<48, 48, false>(a, sBias + 96, sW, sX, 24, sY, x0 - 3, y0 - 3, img, sMass, t, xq, sOff);
    __syncthreads();
    net_put_w<48, 48>(sW, wr, tid);
    net_put_off<48>(sOff, 22, tid);
    __syncthreads();
    net_load_w<48, 48>(a.w[4], wr, tid);
    net_layer<48, 48, false>(a, sBias + 144, sW, sY, 22, sX, x0 - 2, y0 - 2, img, sMass, t, xq, sOff);
    __syncthreads();
    net_put_w<48, 48>(sW, wr, tid);
    net_put_off<48>(sOff, 20, tid);
    __syncthreads();
    net_load_w<48, 16>(a.w[5], wr, tid);
    net_layer<48, 48, false>(a, sBias + 192, sW, sX, 20, sY, x0 - 1, y0 - 1, img, sMass, t, xq, sOff);
    __syncthreads();
    net_put_w<48, 16>(sW, wr, tid);
    net_put_off<48>(sOff, 18, tid);
    __syncthreads();
    if (t + (int)gridDim.x < ntiles) net_load_w<8, 48>(a.w[0], wr, tid);
    net_layer<48, 16, true>(a, sBias + 240, sW, sY, 18, nullptr, x0, y0, img, sMass, t, xq, sOff);
  }
}

// ---------------------------------------------------------------- loss

// d = pred - target; partial sums of |d|^2 per workgroup (FP64, fixed order);
// dz6 = 2 d / nel as BF16 channels 0, 1 of a 16-channel gradient.
__global__ __launch_bounds__(256) void loss_kernel(const float2* __restrict__ pred, const float2* __restrict__ tgt,
                                                   uint16_t* __restrict__ dz, double* __restrict__ partial,
                                                   int64_t n, float scale) {
  __shared__ double red[4];
  double s = 0.0;
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * chunk, i1 = min(n, i0 + chunk);
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
    const float2 p = pred[i], q = tgt[i];
    const float dr = p.x - q.x, di = p.y - q.y;
    s += (double)dr * dr + (double)di * di;
    uint4 o0, o1;
    o0.x = (uint32_t)bf16_bits(scale * dr) | ((uint32_t)bf16_bits(scale * di) << 16);
    o0.y = o0.z = o0.w = 0u;
    o1 = zero4();
    uint4* d = reinterpret_cast<uint4*>(dz + i * 16);
    d[0] = o0;
    d[1] = o1;
  }
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// ---------------------------------------------------------------- weight gradient

struct WgradArgs {
  const uint16_t* a;   // [B][H][W][CIN] layer input (BF16)
  const uint16_t* dz;  // [B][H][W][COUT] gradient of the layer output (BF16)
  float* partial;      // [gridDim.x][COUT][9*CIN + 1]: weight and bias partial sums
  int B, H, W;
};

// dW[co][tap][ci] = sum_pixels dz[p][co] a[p + off(tap)][ci] and
// db[co] = sum_pixels dz[p][co].  Tiles of 16 x 8 pixels; workgroup w takes
// tiles w, w + G, w + 2G, ... in order, so each partial has a fixed order.
template <int CIN, int COUT>
__global__ __launch_bounds__(256, 2) void wgrad_kernel(WgradArgs A) {
  constexpr int N = 9 * CIN;
  constexpr int NB = (N + 15) / 16;
  constexpr int MB = COUT / 16;
  constexpr int NBLK = MB * NB;
  constexpr int PER = (NBLK + 3) / 4;  // output blocks per wave
  // With many column blocks, wave w owns column blocks w, w + 4, ... for
  // every row block: one B fragment read from LDS then feeds MB MFMAs and
  // each A fragment is read once per k-step (LDS read bandwidth, not the
  // MFMAs, bounds this loop otherwise).  Each accumulator still takes the
  // same MFMAs in the same order.
  constexpr bool BYCOL = NB >= 8;
  constexpr int QN = (NB + 3) / 4;
  constexpr int NACC = BYCOL ? QN * MB : PER;
  constexpr int CH = CIN / 8, CHZ = COUT / 8;
  // Rows are padded by 8 values (16 bytes) so the 16 lanes of an operand
  // read (consecutive channels) fall on distinct LDS banks.
  constexpr int APL = 10 * 16 + 8;  // one (dx, ci) plane of the input tile
  constexpr int ZPL = 128 + 8;      // one output channel of the gradient tile
  __shared__ __attribute__((aligned(16))) uint16_t sA[3 * CIN * APL];  // [dx][ci][row][col]
  __shared__ __attribute__((aligned(16))) uint16_t sZ[COUT * ZPL];     // [co][row][col]

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int j = lane & 15, g = lane >> 4;
  const int tilesx = A.W / 16, tilesy = A.H / 8;
  const int ntiles = A.B * tilesx * tilesy;
  f32x4 acc[NACC];
#pragma unroll
  for (int q = 0; q < NACC; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bacc = 0.f;  // bias partial of channel tid / 4 (lanes with tid % 4 == 0, tid < 4 COUT)

  // Tile staging in two halves: the global loads of tile t + G are issued
  // into registers before the MFMAs of tile t and written to LDS (unpacked
  // into the channel-major layouts) after them, so their latency is hidden.
  constexpr int AITEMS = 10 * 18 * CH, ZITEMS = 128 * CHZ;
  constexpr int NA = (AITEMS + 255) / 256, NZ = (ZITEMS + 255) / 256;
  uint4 ra[NA], rz[NZ];
  auto gload = [&](int t) {
    const int b = t / (tilesx * tilesy);
    const int ty = (t / tilesx) % tilesy, tx = t % tilesx;
    const int x0 = tx * 16, y0 = ty * 8;
    const int64_t img = (int64_t)b * A.H * A.W;
    // input halo tile (10 rows x 18 cols); consecutive lanes take
    // consecutive pixels of one 8-channel part
#pragma unroll
    for (int k = 0; k < NA; ++k) {
      const int i = tid + 256 * k;
      ra[k] = zero4();
      if (i < AITEMS) {
        const int part = i / (10 * 18), pp = i - part * (10 * 18);
        const int r = pp / 18, c = pp - r * 18;
        const int gy = y0 - 1 + r, gx = x0 - 1 + c;
        if (gy >= 0 && gy < A.H && gx >= 0 && gx < A.W)
          ra[k] = reinterpret_cast<const uint4*>(A.a + (img + (int64_t)gy * A.W + gx) * CIN)[part];
      }
    }
    // output-gradient tile (8 rows x 16 cols)
#pragma unroll
    for (int k = 0; k < NZ; ++k) {
      const int i = tid + 256 * k;
      rz[k] = zero4();
      if (i < ZITEMS) {
        const int part = i / 128, pp = i - part * 128;
        const int r = pp / 16, c = pp - r * 16;
        rz[k] = reinterpret_cast<const uint4*>(A.dz + (img + (int64_t)(y0 + r) * A.W + x0 + c) * COUT)[part];
      }
    }
  };
  auto lstore = [&]() {
    // three x-shifted channel-major copies of the input tile; adjacent lanes'
    // 2-byte stores are adjacent
#pragma unroll
    for (int k = 0; k < NA; ++k) {
      const int i = tid + 256 * k;
      if (i >= AITEMS) break;
      const int part = i / (10 * 18), pp = i - part * (10 * 18);
      const int r = pp / 18, c = pp - r * 18;
      const uint4 v = ra[k];
      const uint16_t e[8] = {(uint16_t)(v.x & 0xffffu), (uint16_t)(v.x >> 16), (uint16_t)(v.y & 0xffffu),
                             (uint16_t)(v.y >> 16), (uint16_t)(v.z & 0xffffu), (uint16_t)(v.z >> 16),
                             (uint16_t)(v.w & 0xffffu), (uint16_t)(v.w >> 16)};
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const int cc = c - dx;
        if (cc < 0 || cc >= 16) continue;
#pragma unroll
        for (int q = 0; q < 8; ++q) sA[(dx * CIN + part * 8 + q) * APL + r * 16 + cc] = e[q];
      }
    }
    // the output-gradient tile, channel-major
#pragma unroll
    for (int k = 0; k < NZ; ++k) {
      const int i = tid + 256 * k;
      if (i >= ZITEMS) break;
      const int part = i / 128, pp = i - part * 128;
      const uint4 v = rz[k];
      const uint16_t e[8] = {(uint16_t)(v.x & 0xffffu), (uint16_t)(v.x >> 16), (uint16_t)(v.y & 0xffffu),
                             (uint16_t)(v.y >> 16), (uint16_t)(v.z & 0xffffu), (uint16_t)(v.z >> 16),
                             (uint16_t)(v.w & 0xffffu), (uint16_t)(v.w >> 16)};
#pragma unroll
      for (int q = 0; q < 8; ++q) sZ[(part * 8 + q) * ZPL + pp] = e[q];
    }
  };

  if ((int)blockIdx.x < ntiles) gload(blockIdx.x);
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    __syncthreads();  // previous tile's LDS reads are done
    lstore();
    __syncthreads();
    if (t + (int)gridDim.x < ntiles) gload(t + gridDim.x);
    // bias gradient: four lanes per channel (lanes 4c .. 4c+3 of the first
    // 4 COUT threads) sum 32 pixels each, then two fixed-order shuffles
    {
      float s = 0.f;
      if (tid < 4 * COUT) {
        const uint16_t* z = &sZ[(tid >> 2) * ZPL + 32 * (tid & 3)];
#pragma unroll 8
        for (int p = 0; p < 32; ++p) s += bf16_val(z[p]);
      }
      s += __shfl_xor(s, 1, 64);
      s += __shfl_xor(s, 2, 64);
      if (tid < 4 * COUT && (tid & 3) == 0) bacc += s;
    }
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int p0 = 32 * ks + 8 * g;  // 8 consecutive pixels in one row
      const int py = p0 >> 4, px = p0 & 15;
      auto bfrag = [&](int nb) {
        const int n = 16 * nb + j;
        uint4 bv = zero4();
        if (n < N) {
          const int tap = n / CIN, ci = n - tap * CIN;
          const int dy = tap / 3, dx = tap - 3 * dy;
          bv = *reinterpret_cast<const uint4*>(&sA[(dx * CIN + ci) * APL + (py + dy) * 16 + px]);
        }
        return as_bf16x8(bv);
      };
      if constexpr (BYCOL) {
        bf16x8 af[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
          af[mb] = as_bf16x8(*reinterpret_cast<const uint4*>(&sZ[(16 * mb + j) * ZPL + p0]));
#pragma unroll
        for (int qn = 0; qn < QN; ++qn) {
          const int nb = wave + 4 * qn;
          if (nb >= NB) break;
          const bf16x8 bf = bfrag(nb);
#pragma unroll
          for (int mb = 0; mb < MB; ++mb)
            acc[qn * MB + mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[mb], bf, acc[qn * MB + mb], 0, 0, 0);
        }
      } else {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
          const int blk = wave + 4 * q;
          if (blk >= NBLK) break;
          const int mb = blk / NB, nb = blk - mb * NB;
          const bf16x8 af = as_bf16x8(*reinterpret_cast<const uint4*>(&sZ[(16 * mb + j) * ZPL + p0]));
          acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bfrag(nb), acc[q], 0, 0, 0);
        }
      }
    }
  }
  // lane holds D[co = 16 mb + 4 g + r][n = 16 nb + j]
  float* P = A.partial + (int64_t)blockIdx.x * COUT * (N + 1);
#pragma unroll
  for (int q = 0; q < NACC; ++q) {
    int mb, nb;
    if constexpr (BYCOL) {
      mb = q % MB;
      nb = wave + 4 * (q / MB);
      if (nb >= NB) break;
    } else {
      const int blk = wave + 4 * q;
      if (blk >= NBLK) break;
      mb = blk / NB;
      nb = blk - mb * NB;
    }
    const int n = 16 * nb + j;
    if (n < N)
#pragma unroll
      for (int r = 0; r < 4; ++r) P[(16 * mb + 4 * g + r) * (N + 1) + n] = acc[q][r];
  }
  if (tid < 4 * COUT && (tid & 3) == 0) P[(tid >> 2) * (N + 1) + N] = bacc;
}

// Fixed-order sum of the partials into the canonical gradient of one layer:
// W (Cout, Cin, 3, 3) then b (Cout), real channels only.  A workgroup takes
// 64 consecutive partial columns of one output channel; wave w sums parts
// w, w + 8, ... in ascending order (each load of a wave is one contiguous
// 256-byte row of one part), then wave 0 adds the 8 wave sums in order.
// The result depends only on nparts, not on timing.
__global__ __launch_bounds__(512) void wgrad_reduce_kernel(const float* __restrict__ partial, int nparts,
                                                           int coutp, int cinp, int cout, int cin,
                                                           float* __restrict__ gw, float* __restrict__ gb) {
  __shared__ double red[8][64];
  const int N = 9 * cinp;
  const int nblk = (N + 1 + 63) / 64;
  const int co = blockIdx.x / nblk;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int col = (blockIdx.x - co * nblk) * 64 + lane;
  double s = 0.0;
  if (col <= N) {
    const float* src = partial + (int64_t)co * (N + 1) + col;
    const int64_t stride = (int64_t)coutp * (N + 1);
#pragma unroll 8
    for (int p = w; p < nparts; p += 8) s += (double)src[p * stride];
  }
  red[w][lane] = s;
  __syncthreads();
  if (w == 0 && col <= N) {
    double t = red[0][lane];
#pragma unroll
    for (int k = 1; k < 8; ++k) t += red[k][lane];
    if (col == N) {
      gb[co] = (float)t;
    } else {
      const int tap = col / cinp, ci = col - tap * cinp;
      if (ci < cin) gw[(co * cin + ci) * 9 + tap] = (float)t;
    }
  }
}

// ---------------------------------------------------------------- weights, optimiser

// Canonical FP32 layer (W (cout, cin, 3, 3), b) -> BF16 kernel layouts:
// forward [coutp][tap][cinp]; backward-data [cinp][tap'][coutp] with tap'
// the point-reflected tap (8 - tap).  Padded entries are zero.
__global__ void prep_weights_kernel(const float* __restrict__ w, int cout, int cin, int coutp, int cinp,
                                    uint16_t* __restrict__ fwd, uint16_t* __restrict__ bwd) {
  const int nf = coutp * 9 * cinp;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nf; e += gridDim.x * blockDim.x) {
    // forward
    {
      const int co = e / (9 * cinp), rem = e - co * 9 * cinp;
      const int tap = rem / cinp, ci = rem - tap * cinp;
      const float v = (co < cout && ci < cin) ? w[(co * cin + ci) * 9 + tap] : 0.f;
      fwd[e] = bf16_bits(v);
    }
    if (bwd) {
      const int ci = e / (9 * coutp), rem = e - ci * 9 * coutp;
      const int tp = rem / coutp, co = rem - tp * coutp;
      const int tap = 8 - tp;
      const float v = (co < cout && ci < cin) ? w[(co * cin + ci) * 9 + tap] : 0.f;
      bwd[e] = bf16_bits(v);
    }
  }
}

// Adam (Kingma & Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// p -= lr mhat / (sqrt(vhat) + eps) with bias corrections c1 = 1 - b1^t, c2 = 1 - b2^t.
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// ---------------------------------------------------------------- checks

// Per-field mass h^2 sum |psi|^2 of B fields of n points: workgroup (f, c)
// reduces a fixed chunk in FP64; then a fixed-order pass per field.
__global__ __launch_bounds__(256) void field_mass_partial_kernel(const float2* __restrict__ psi, int64_t n,
                                                                 int chunks, double* __restrict__ partial) {
  __shared__ double red[4];
  const int f = blockIdx.x / chunks, c = blockIdx.x - f * chunks;
  const int64_t len = (n + chunks - 1) / chunks;
  const int64_t i0 = (int64_t)c * len, i1 = min(n, i0 + len);
  const float2* P = psi + (int64_t)f * n;
  double s = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
    const float2 v = P[i];
    s += (double)v.x * v.x + (double)v.y * v.y;
  }
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void field_mass_final_kernel(const double* __restrict__ partial, int fields, int chunks, double h2,
                                        double* __restrict__ out) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= fields) return;
  double s = 0.0;
  for (int c = 0; c < chunks; ++c) s += partial[f * chunks + c];
  out[f] = h2 * s;
}

// Field masses from the last layer's tile sums, one workgroup per field:
// thread i adds tiles i, i + 256, ... in order, then a fixed tree over the
// threads (lanes by shuffles, then the four waves in order); h^2 times that.
__global__ __launch_bounds__(256) void tile_mass_final_kernel(const double* __restrict__ tile_mass, int tiles,
                                                              double h2, double* __restrict__ out) {
  __shared__ double red[4];
  const int f = blockIdx.x;
  double s = 0.0;
  for (int c = threadIdx.x; c < tiles; c += 256) s += tile_mass[(int64_t)f * tiles + c];
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[f] = h2 * ((red[0] + red[1]) + (red[2] + red[3]));
}

// MSD boundary projection: boundary points of the prediction keep their
// phase and take the modulus of the input (|psi_b|^2 is the fixed value of
// the modulus-squared Dirichlet condition, Eq. BCMSDdef).
__global__ void msd_project_kernel(const float2* __restrict__ in, float2* __restrict__ out, int B, int H, int W) {
  const int per = 2 * W + 2 * (H - 2);
  const int64_t total = (int64_t)B * per;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(e / per);
    int k = (int)(e - (int64_t)b * per), y, x;
    if (k < W) {
      y = 0;
      x = k;
    } else if (k < 2 * W) {
      y = H - 1;
      x = k - W;
    } else {
      k -= 2 * W;
      y = 1 + (k >> 1);
      x = (k & 1) ? W - 1 : 0;
    }
    const int64_t i = (int64_t)b * H * W + (int64_t)y * W + x;
    const float2 pi = in[i], po = out[i];
    const float mi = sqrtf(pi.x * pi.x + pi.y * pi.y), mo = sqrtf(po.x * po.x + po.y * po.y);
    if (mo > 0.f) out[i] = make_float2(po.x * (mi / mo), po.y * (mi / mo));
  }
}

// ---------------------------------------------------------------- launchers

static int grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

}  // namespace nlse

using namespace nlse;

// Compute units of the current device (queried once per process).
static int cu_count() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) ==
                                                 hipSuccess && n > 0)
      cus = n;
    else
      cus = 256;
  }
  return cus;
}

// Waves per convolution workgroup: 8 (two pixel rows each) run four waves per
// SIMD in 128 registers; 4 (four rows each) hold more accumulators per wave
// but only two waves per SIMD.
constexpr int kConvWaves = 8;

// Persistent grid: as many workgroups as the device holds at once (queried
// once per kernel), never more than there are tiles.
template <int CIN, int COUT, int EPI>
static hipError_t launch_conv(const ConvArgs& a, int ntiles, hipStream_t st) {
  constexpr int NW = kConvWaves;
  static int per_cu = 0;
  if (per_cu == 0) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &n, reinterpret_cast<const void*>(&conv3x3_kernel<CIN, COUT, EPI, NW>), 64 * NW, 0) != hipSuccess ||
        n < 1)
      n = 1;
    per_cu = n;
  }
  const dim3 grid((unsigned)std::min(ntiles, per_cu * cu_count()));
  hipLaunchKernelGGL((conv3x3_kernel<CIN, COUT, EPI, NW>), grid, dim3(64 * NW), 0, st, a, ntiles);
  return hipGetLastError();
}

hipError_t sg_pack_input(const void* psi, void* x, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(pack_input_kernel, dim3(grid_for(n)), dim3(256), 0, st, static_cast<const float2*>(psi),
                     static_cast<uint4*>(x), n);
  return hipGetLastError();
}

hipError_t sg_conv(int kind, const SgConv& c, hipStream_t st) {
  ConvArgs a;
  a.in = c.in;
  a.w = c.w;
  a.bias = c.bias;
  a.out = c.out;
  a.x = static_cast<const float2*>(c.x);
  a.pred = static_cast<float2*>(c.pred);
  a.mask = c.mask;
  a.H = c.H;
  a.W = c.W;
  a.project = c.project;
  a.tile_mass = c.tile_mass;
  const int ntiles = c.B * (c.H / 16) * (c.W / 16);
  switch (kind) {
    case kSgFirst: return launch_conv<8, 48, kEpiRelu>(a, ntiles, st);
    case kSgHidden: return launch_conv<48, 48, kEpiRelu>(a, ntiles, st);
    case kSgLast: return launch_conv<48, 16, kEpiLast>(a, ntiles, st);
    case kSgDgradLast: return launch_conv<16, 48, kEpiDgrad>(a, ntiles, st);
    case kSgDgradHidden: return launch_conv<48, 48, kEpiDgrad>(a, ntiles, st);
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t sg_net_forward(const SgNet& c, hipStream_t st) {
  NetArgs a;
  a.x = static_cast<const float2*>(c.x);
  a.pred = static_cast<float2*>(c.pred);
  for (int l = 0; l < 6; ++l) {
    a.w[l] = c.w[l];
    a.bias[l] = c.bias[l];
  }
  a.H = c.H;
  a.W = c.W;
  a.project = c.project;
  a.tile_mass = c.tile_mass;
  const int ntiles = c.B * (c.H / 16) * (c.W / 16);
  // one workgroup per CU (its LDS), persistent over the tiles
  const dim3 grid((unsigned)std::min(ntiles, cu_count()));
  hipLaunchKernelGGL(net_forward_kernel, grid, dim3(kNetThreads), 0, st, a, ntiles);
  return hipGetLastError();
}

hipError_t sg_loss(const void* pred, const void* tgt, uint16_t* dz, double* partial, int nparts, int64_t n,
                   hipStream_t st) {
  hipLaunchKernelGGL(loss_kernel, dim3(nparts), dim3(256), 0, st, static_cast<const float2*>(pred),
                     static_cast<const float2*>(tgt), dz, partial, n, (float)(2.0 / (2.0 * (double)n)));
  return hipGetLastError();
}

hipError_t sg_wgrad(int kind, const uint16_t* a, const uint16_t* dz, float* partial, int nparts, int B, int H, int W,
                    hipStream_t st) {
  WgradArgs A;
  A.a = a;
  A.dz = dz;
  A.partial = partial;
  A.B = B;
  A.H = H;
  A.W = W;
  switch (kind) {
    case kSgFirst: hipLaunchKernelGGL((wgrad_kernel<8, 48>), dim3(nparts), dim3(256), 0, st, A); break;
    case kSgHidden: hipLaunchKernelGGL((wgrad_kernel<48, 48>), dim3(nparts), dim3(256), 0, st, A); break;
    case kSgLast: hipLaunchKernelGGL((wgrad_kernel<48, 16>), dim3(nparts), dim3(256), 0, st, A); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t sg_wgrad_reduce(const float* partial, int nparts, int coutp, int cinp, int cout, int cin, float* gw,
                           float* gb, hipStream_t st) {
  if (cout < 1 || cout > coutp || cin < 1 || cin > cinp || nparts < 1) return hipErrorInvalidValue;
  const int nblk = (9 * cinp + 1 + 63) / 64;
  hipLaunchKernelGGL(wgrad_reduce_kernel, dim3(cout * nblk), dim3(512), 0, st, partial, nparts, coutp, cinp, cout,
                     cin, gw, gb);
  return hipGetLastError();
}

hipError_t sg_prep_weights(const float* w, int cout, int cin, int coutp, int cinp, uint16_t* fwd, uint16_t* bwd,
                           hipStream_t st) {
  const int n = coutp * 9 * cinp;
  hipLaunchKernelGGL(prep_weights_kernel, dim3((n + 255) / 256), dim3(256), 0, st, w, cout, cin, coutp, cinp, fwd,
                     bwd);
  return hipGetLastError();
}

hipError_t sg_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps,
                   float c1, float c2, hipStream_t st) {
  hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n)), dim3(256), 0, st, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t sg_field_mass(const void* psi, int fields, int64_t n, double h2, double* partial, int chunks, double* out,
                         hipStream_t st) {
  hipLaunchKernelGGL(field_mass_partial_kernel, dim3(fields * chunks), dim3(256), 0, st,
                     static_cast<const float2*>(psi), n, chunks, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(field_mass_final_kernel, dim3((fields + 255) / 256), dim3(256), 0, st, partial, fields, chunks,
                     h2, out);
  return hipGetLastError();
}

hipError_t sg_tile_mass_final(const double* tile_mass, int fields, int tiles, double h2, double* out,
                              hipStream_t st) {
  hipLaunchKernelGGL(tile_mass_final_kernel, dim3(fields), dim3(256), 0, st, tile_mass, tiles, h2, out);
  return hipGetLastError();
}

hipError_t sg_msd_project(const void* in, void* out, int B, int H, int W, hipStream_t st) {
  const int64_t n = (int64_t)B * (2 * W + 2 * (H - 2));
  hipLaunchKernelGGL(msd_project_kernel, dim3(grid_for(n)), dim3(256), 0, st, static_cast<const float2*>(in),
                     static_cast<float2*>(out), B, H, W);
  return hipGetLastError();
}
