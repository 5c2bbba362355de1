// Internal interface between the surrogate kernels (surrogate.hip) and the
// C ABI (api_surrogate.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

enum { kSgFirst = 0, kSgHidden = 1, kSgLast = 2, kSgDgradLast = 3, kSgDgradHidden = 4 };

struct SgConv {
  const uint16_t* in;    // BF16 NHWC input
  const uint16_t* w;     // BF16 kernel-layout weights
  const float* bias;     // FP32 bias (forward kinds)
  uint16_t* out;         // BF16 NHWC output (hidden / dgrad kinds)
  const void* x;         // network input field, complex64 (last layer)
  void* pred;            // prediction, complex64 (last layer)
  const uint16_t* mask;  // activation gating the gradient (dgrad kinds)
  int B, H, W;
  int project;           // last layer: MSD projection of the boundary ring
  double* tile_mass;     // last layer, or null: per 16x16 tile, sum of |pred|^2
};

// All six forward layers in one pass per 16x16 tile (inference only: no
// activations are stored).
struct SgNet {
  const void* x;             // network input fields, complex64 [B][H][W]
  void* pred;                // prediction, complex64
  const uint16_t* w[6];      // BF16 forward-layout weights per layer
  const float* bias[6];      // FP32 biases per layer
  int B, H, W;
  int project;               // MSD projection of the boundary ring
  double* tile_mass;         // or null: per 16x16 tile, sum of |pred|^2
};

hipError_t sg_pack_input(const void* psi, void* x, int64_t n, hipStream_t st);
hipError_t sg_net_forward(const SgNet& c, hipStream_t st);
hipError_t sg_conv(int kind, const SgConv& c, hipStream_t st);
hipError_t sg_loss(const void* pred, const void* tgt, uint16_t* dz, double* partial, int nparts, int64_t n,
                   hipStream_t st);
hipError_t sg_wgrad(int kind, const uint16_t* a, const uint16_t* dz, float* partial, int nparts, int B, int H, int W,
                    hipStream_t st);
hipError_t sg_wgrad_reduce(const float* partial, int nparts, int coutp, int cinp, int cout, int cin, float* gw,
                           float* gb, hipStream_t st);
hipError_t sg_prep_weights(const float* w, int cout, int cin, int coutp, int cinp, uint16_t* fwd, uint16_t* bwd,
                           hipStream_t st);
hipError_t sg_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps,
                   float c1, float c2, hipStream_t st);
hipError_t sg_field_mass(const void* psi, int fields, int64_t n, double h2, double* partial, int chunks, double* out,
                         hipStream_t st);
hipError_t sg_msd_project(const void* in, void* out, int B, int H, int W, hipStream_t st);
// out[f] = h2 * (sum of the `tiles` tile sums of field f, in order)
hipError_t sg_tile_mass_final(const double* tile_mass, int fields, int tiles, double h2, double* out,
                              hipStream_t st);
