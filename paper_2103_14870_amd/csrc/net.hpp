// Learned block preconditioner: a small message-passing network on the mesh
// graph, inference and training on the GPU with BF16 MFMA (FP32 accumulate).
//
// Per node i the network predicts a lower-triangular L_i (exponentiated
// diagonal) and the preconditioner block B_i = L_i A_ii^-1 L_i^T: symmetric
// positive definite by construction, and exactly 3x3 block-Jacobi for L = I
// (the zero-initialised head).  The conjugate-gradient solve accepts it only
// at the same FP64 residual as block-Jacobi, which stays the fallback.
//
// Architecture (fixed): node input a_i (8) from the incident edges' features
// (rest length / mean rest length, stretch - 1, damage label), embedding
// 8 -> 64, three residual message-passing layers h <- h + relu(W [h; P h] + b)
// with P the mean over unbroken incident edges (128 -> 64), head 64 -> 6.
// Flat parameter order: W0 (64x8), b0, [W_l (64x128), b_l] x 3, Wh (6x64), bh;
// weights row-major [out][in].
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace gfem {

constexpr int kHid = 64, kNetIn = 8, kNetInPad = 32, kNetLayers = 3, kNetOut = 6;
constexpr int kNetParams = kHid * kNetIn + kHid + kNetLayers * (kHid * 2 * kHid + kHid) + kNetOut * kHid + kNetOut;
constexpr int kNetRows = 64;  // rows per GEMM workgroup; node arrays are padded to a multiple

// offsets of each tensor in the flat parameter vector
constexpr int kOffW0 = 0;
constexpr int kOffB0 = kOffW0 + kHid * kNetIn;
constexpr int kOffL0 = kOffB0 + kHid;  // layer l: W at kOffL0 + l*kLayerSize, b after it
constexpr int kLayerSize = kHid * 2 * kHid + kHid;
constexpr int kOffWh = kOffL0 + kNetLayers * kLayerSize;
constexpr int kOffBh = kOffWh + kNetOut * kHid;

typedef __bf16 bf16;

struct NetParamsDev {
  float* master = nullptr;  // FP32 master weights (kNetParams)
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  bf16* W0 = nullptr;                 // [64][32] (inputs zero-padded)
  bf16* Wl[kNetLayers] = {};          // [64][128]
  bf16* WlT[kNetLayers] = {};         // [128][64]
};

// Per-mesh activations and gradients (node arrays padded to npad rows).
struct NetWork {
  int n = 0, npad = 0, nwg_dw = 0;
  bf16* a = nullptr;                    // [npad][32]
  float* inv_wdeg = nullptr;            // [npad]
  bf16* h[kNetLayers + 1] = {};         // [npad][64]
  bf16* m[kNetLayers] = {};             // [npad][64]
  bf16* z[kNetLayers + 1] = {};         // [npad][64] pre-activations
  float* o = nullptr;                   // [npad][8] head outputs (6 used)
  float* B = nullptr;                   // [6][n] preconditioner blocks (symmetric, SoA)
  float* gh = nullptr;                  // [npad][64]
  bf16* gz = nullptr;                   // [npad][64]
  float* gi = nullptr;                  // [npad][128]
  float* go = nullptr;                  // [npad][8]
  float* part = nullptr;                // weight-gradient partials [nwg_dw][64*128 + 64]
  float* grad = nullptr;                // [kNetParams]
  double* lossp = nullptr;              // [npad / 256 + 1] partial loss sums
};

struct NetInputs {
  int n;
  MatView A;                    // block pattern (graph) of the mesh
  const int32_t* diag_blk;
  const int32_t* blk_edge;
  const d4* X;
  const d4* U;
  const uint8_t* zeta;          // labels of the system being solved
  double inv_mean_len;
  const float* binv;            // block-Jacobi inverse diagonal blocks [6][n]
  const uint8_t* dflag;
};

// Forward pass: node inputs, embedding, three layers, head -> w.B (and w.o).
void net_forward(hipStream_t s, const NetParamsDev& P, NetWork& w, const NetInputs& in);
// Recompute B from the cached head outputs w.o and the current binv.
void net_apply_cached(hipStream_t s, const NetParamsDev& P, NetWork& w, const NetInputs& in);
// Loss and gradient (into w.grad) for the system A dv = b; requires net_forward first.
// inv_norm = 1 / sum of |dv_i|^2 over free nodes.  Loss partials go to w.lossp
// (count returned).
int net_backward(hipStream_t s, const NetParamsDev& P, NetWork& w, const NetInputs& in, const d4* b,
                 const d4* dv, double inv_norm);
// Adam step on the master weights with the gradient in grad, then repack BF16.
void net_adam(hipStream_t s, NetParamsDev& P, const float* grad, int t, float lr);
void net_pack(hipStream_t s, NetParamsDev& P);
// Partial sums of |dv_i|^2 over free nodes (count returned).
int net_dv_norm(hipStream_t s, int n, const d4* dv, const uint8_t* dflag, double* part);

}  // namespace gfem
