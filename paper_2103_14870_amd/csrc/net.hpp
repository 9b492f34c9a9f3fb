// Learned preconditioner: a small message-passing network on the mesh graph
// that predicts the blocks of a factorised sparse approximate inverse
// B = G^T G, inference and training on the GPU with BF16 MFMA (FP32
// accumulate).
//
// G is block lower triangular on the lower block pattern of A (node order):
//   G_ii = L_i C_i,  G_ij = -L_i C_i W_ij A_ij A_jj^-1  (stored blocks j < i),
// C_i the inverse lower Cholesky factor of A_ii, L_i lower triangular with
// exponentiated diagonal, W_ij a 3x3 block.  B is symmetric positive definite
// by construction; L = I, W = 0 is exactly 3x3 block-Jacobi (the zero
// network).  The conjugate-gradient solve accepts it only at the same FP64
// residual as block-Jacobi, which stays the fallback.
//
// Architecture (fixed): node input a_i (8) from the incident edges' features
// f = (rest length / mean rest length, stretch - 1, damage label), embedding
// 8 -> 64, three residual message-passing layers h <- h + relu(W [h; P h] + b)
// with P the mean over unbroken incident edges (128 -> 64), node head 64 -> 24
// (o[0:6] -> L_i, o[6:15] = s_i, o[15:24] = t_i) and the edge term
// W_ij = s_i + t_j + We f_ij + be (row-major 3x3).
// Flat parameter order: W0 (64x8), b0, [W_l (64x128), b_l] x 3, Wh (24x64),
// bh (24), We (9x3), be (9); weights row-major [out][in].
//
// Training minimises Kaporin's condition number of G A G^T, estimated with a
// +-1 probe v: loss = log(v^T G A G^T v / N) - (2/N) log det G, N = 3n.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace gfem {

constexpr int kHid = 64, kNetIn = 8, kNetInPad = 32, kNetLayers = 3, kNetHead = 24, kNetEdgeF = 3;
constexpr int kNetRows = 64;  // rows per GEMM workgroup; node arrays are padded to a multiple

// offsets of each tensor in the flat parameter vector
constexpr int kOffW0 = 0;
constexpr int kOffB0 = kOffW0 + kHid * kNetIn;
constexpr int kOffL0 = kOffB0 + kHid;  // layer l: W at kOffL0 + l*kLayerSize, b after it
constexpr int kLayerSize = kHid * 2 * kHid + kHid;
constexpr int kOffWh = kOffL0 + kNetLayers * kLayerSize;
constexpr int kOffBh = kOffWh + kNetHead * kHid;
constexpr int kOffWe = kOffBh + kNetHead;
constexpr int kOffBe = kOffWe + 9 * kNetEdgeF;
constexpr int kNetParams = kOffBe + 9;
constexpr int kEdgeGrad = 9 * kNetEdgeF + 9;  // We and be gradient entries

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
  float* o = nullptr;                   // [npad][24] head outputs
  float* gh = nullptr;                  // [npad][64]
  bf16* gz = nullptr;                   // [npad][64]
  float* gi = nullptr;                  // [npad][128]
  float* go = nullptr;                  // [npad][24]
  float* part = nullptr;                // weight-gradient partials [nwg_dw][64*128 + 64]
  float* grad = nullptr;                // [kNetParams]
  // factor values: packed BF16 records of FactView for the solve, FP32 SoA
  // for training (gl32, gu32 [9][ne], gd32 [6][n])
  uint4 *glv = nullptr, *guv = nullptr, *gdv = nullptr;
  bf16 *gl8 = nullptr, *gu8 = nullptr;
  float *gl32 = nullptr, *gu32 = nullptr, *gd32 = nullptr;
  // training scratch
  d4* probe = nullptr;                  // [n] +-1 probe v
  d4* u = nullptr;                      // [n] G^T v
  d4* wneg = nullptr;                   // [n] -A u
  d4* zero = nullptr;                   // [n] zeros
  v4<float>* mv = nullptr;              // [n] M_i^T v_i
  v4<float>* sv = nullptr;              // [n] A_ii^-1 w_i
  double* dpart = nullptr;              // partial sums (t, log det), [2][kMaxPart]
  float* epart = nullptr;               // edge-term gradient partials [kMaxPart][kEdgeGrad]
};

struct NetInputs {
  int n;
  MatView A;                    // block pattern and (FP32) values of the system
  const int32_t* diag_blk;
  const int32_t* blk_edge;
  int ne;
  const int32_t* lptr;          // compact strictly lower / upper halves (FactView)
  const int32_t* uptr;
  const int32_t* lcol;
  const int32_t* ucol;
  const int32_t* upos;          // edge -> compact upper index of its block (i, j), i < j
  const d4* X;
  const d4* U;
  const uint8_t* zeta;          // labels of the system being solved
  double inv_mean_len;
  const float* binv;            // block-Jacobi inverse diagonal blocks [6][n]
  const uint8_t* dflag;
};

// Forward pass: node inputs, embedding, three layers, head -> w.o.
// keep_z: also store the pre-activations (the backward pass of training needs them).
void net_forward(hipStream_t s, const NetParamsDev& P, NetWork& w, const NetInputs& in, int Gb, bool keep_z = true);
// Factor values from the head outputs w.o and the current system: packed
// BF16 (fp32 = false) or FP32 SoA into w.gl32/gu32/gd32.
void net_build_factor(hipStream_t s, const NetParamsDev& P, NetWork& w, const NetInputs& in, int Gb, bool fp32);
// Scales each block row of the packed BF16 factor by the inverse Cholesky
// factor of its diagonal block of G A G^T (which becomes I); pairs/ptr list,
// per row, the stored blocks A_ab between its pattern positions a <= b as
// (block index, a, b, 0), position 0 being the row itself and a >= 1 its
// lower slot a - 1.
void net_normalise_factor(hipStream_t s, NetWork& w, const NetInputs& in, int Gb, const int32_t* ptr,
                          const int4* pairs);
// View of the BF16 factor for the solve.
FactView net_factor_view(const NetWork& w, const NetInputs& in);
// Rademacher probe from a counter-based generator (SplitMix64 of seed and index).
void net_probe(hipStream_t s, NetWork& w, uint64_t seed);
// Training quantities for the probe in w.probe after net_forward and an FP32
// factor: u = G^T v (needs -A u in w.wneg afterwards, from the caller's
// residual kernel).
void net_kaporin_u(hipStream_t s, NetWork& w, const NetInputs& in, int Gb);
// After net_kaporin_u and w.wneg = -A u: w.probe = G A G^T v (one power step
// on X) and partials of |w.probe|^2 in dpart[0..G); returns G (<= kMaxPart).
int net_power_apply(hipStream_t s, NetWork& w, const NetInputs& in, int Gb);
// w.probe *= f.
void net_scale_probe(hipStream_t s, NetWork& w, double f);
// After w.wneg = -A u: partials of t = u.A u in dpart[0..G) and of log det G
// in dpart[kMaxPart..kMaxPart+G); returns G.
int net_kaporin_dots(hipStream_t s, const NetParamsDev& P, NetWork& w, const NetInputs& in);
// Gradient of the loss for the given t into w.grad (full backward pass).
void net_kaporin_backward(hipStream_t s, const NetParamsDev& P, NetWork& w, const NetInputs& in, int Gb, double t);
// Adam step on the master weights with the gradient in grad, then repack BF16.
void net_adam(hipStream_t s, NetParamsDev& P, const float* grad, int t, float lr);
void net_pack(hipStream_t s, NetParamsDev& P);

}  // namespace gfem
