// Learned block preconditioner kernels (see net.hpp): node inputs, BF16 MFMA
// GEMMs (v_mfma_f32_16x16x32_bf16, FP32 accumulate) for the embedding, the
// message-passing layers and their backward data pass, LDS-transposed MFMA
// weight gradients, neighbour mean and its transpose as gathers over the
// mesh's block pattern (no atomics), the head with the preconditioner blocks
// and the loss gradient, and Adam.
#include "net.hpp"

namespace gfem {

namespace {

typedef bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kDwWorkgroups = 256;
constexpr int kBuildLanes = 8;  // lanes per block row in the factor and training kernels

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------- inputs

// Node input a_i = [1, mean f0, mean f1, mean f2, mean f1^2, mean |f1|,
// mean (1 - f2) f1, degree / 16] over the incident edges, with edge features
// f0 = rest length / mean rest length, f1 = tanh(current / rest length - 1),
// f2 = damage label; zero-padded to 32.  Also 1 / (number of unbroken
// incident edges) for the neighbour mean.
__global__ __launch_bounds__(256) void k_net_inputs(NetInputs in, int npad, bf16* __restrict__ a,
                                                    float* __restrict__ inv_wdeg) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= npad) return;
  float acc[6] = {0, 0, 0, 0, 0, 0};
  float deg = 0.f, wdeg = 0.f;
  if (i < in.n) {
    const d4 Xi = in.X[i], Ui = in.U[i];
    const int s = in.A.row_ptr[i], e = in.A.row_ptr[i + 1], db = in.diag_blk[i];
    for (int b = s; b < e; ++b) {
      if (b == db) continue;
      const int j = in.A.col[b], ed = in.blk_edge[b];
      const d4 Xj = in.X[j], Uj = in.U[j];
      const double dx = Xj.x - Xi.x, dy = Xj.y - Xi.y, dz = Xj.z - Xi.z;
      const double cx = dx + (Uj.x - Ui.x), cy = dy + (Uj.y - Ui.y), cz = dz + (Uj.z - Ui.z);
      const double L0 = sqrt(dx * dx + dy * dy + dz * dz), L = sqrt(cx * cx + cy * cy + cz * cz);
      const float f0 = (float)(L0 * in.inv_mean_len), f1 = (float)tanh(L / L0 - 1.0);
      const float f2 = in.zeta[ed] ? 1.f : 0.f;
      acc[0] += f0;
      acc[1] += f1;
      acc[2] += f2;
      acc[3] += f1 * f1;
      acc[4] += fabsf(f1);
      acc[5] += (1.f - f2) * f1;
      deg += 1.f;
      wdeg += 1.f - f2;
    }
  }
  const float inv = deg > 0.f ? 1.f / deg : 0.f;
  bf16* ai = a + (size_t)i * kNetInPad;
  ai[0] = (bf16)(i < in.n ? 1.f : 0.f);
#pragma unroll
  for (int c = 0; c < 6; ++c) ai[1 + c] = (bf16)(acc[c] * inv);
  ai[7] = (bf16)(deg / 16.f);
#pragma unroll
  for (int c = 8; c < kNetInPad; ++c) ai[c] = (bf16)0.f;
  inv_wdeg[i] = wdeg > 0.f ? 1.f / wdeg : 0.f;
}

// ---------------------------------------------------------------- GEMM

// Y[rows][NOUT] = [XA | XB] (BF16, row-major, KA + KB columns) times W^T,
// W [NOUT][KA + KB] BF16, FP32 accumulation on the 16x16x32 BF16 MFMA.  One
// wave computes 16 rows x NOUT; a workgroup of four waves 64 rows.
// MFMA operand layout (lane l of 64): A row l%16, k 8*(l/16)..+7; B column
// l%16, same k; D column l%16, rows 4*(l/16)..+3.
// EPI 0: Z = Y + bias, H = relu(Z)          (embedding)
// EPI 1: Z = Y + bias, H = Hin + relu(Z)    (residual message-passing layer)
// EPI 2: F = Y (FP32)                       (backward data pass)
template <int KA, int KB, int NOUT, int EPI>
__global__ __launch_bounds__(256) void k_net_gemm(const bf16* __restrict__ XA, const bf16* __restrict__ XB,
                                                  const bf16* __restrict__ W, const float* __restrict__ bias,
                                                  const bf16* __restrict__ Hin, bf16* __restrict__ Zout,
                                                  bf16* __restrict__ Hout, float* __restrict__ Fout) {
  constexpr int K = KA + KB;
  constexpr int NT = NOUT / 16;
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r0 = blockIdx.x * kNetRows + wv * 16;
  f32x4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int ar = r0 + (l & 15);
  const int kq = 8 * (l >> 4);
#pragma unroll
  for (int kc = 0; kc < K / 32; ++kc) {
    const int k0 = kc * 32 + kq;
    const bf16x8 av = (kc * 32 < KA) ? *reinterpret_cast<const bf16x8*>(XA + (size_t)ar * KA + k0)
                                     : *reinterpret_cast<const bf16x8*>(XB + (size_t)ar * KB + (k0 - KA));
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int col = t * 16 + (l & 15);
      const bf16x8 bv = *reinterpret_cast<const bf16x8*>(W + (size_t)col * K + k0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[t], 0, 0, 0);
    }
  }
  if constexpr (EPI == 2) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = r0 + 4 * (l >> 4) + i, col = t * 16 + (l & 15);
        Fout[(size_t)row * NOUT + col] = acc[t][i];
      }
  } else {
    // The MFMA result layout (lane: 4 rows x NT columns 16 apart) is turned
    // row-major through this wave's slice of LDS, so that the bias, the
    // residual input and both outputs move as 16-byte runs of 8 features.
    static_assert(NOUT == 64, "one 16 x 64 tile per wave");
    __shared__ float tile[4][16][NOUT + 4];
    float(*tw)[NOUT + 4] = tile[wv];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) tw[4 * (l >> 4) + i][t * 16 + (l & 15)] = acc[t][i];
    __syncthreads();
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int rl = l >> 2, c8 = (l & 3) * 16 + half * 8;
      const size_t off = (size_t)(r0 + rl) * NOUT + c8;
      bf16x8 hin;
      if (EPI == 1) hin = *reinterpret_cast<const bf16x8*>(Hin + off);
      bf16x8 zo, ho;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const float zz = tw[rl][c8 + q] + bias[c8 + q];
        zo[q] = (bf16)zz;
        float hr = fmaxf(zz, 0.f);
        if (EPI == 1) hr += (float)hin[q];
        ho[q] = (bf16)hr;
      }
      if (Zout) *reinterpret_cast<bf16x8*>(Zout + off) = zo;
      *reinterpret_cast<bf16x8*>(Hout + off) = ho;
    }
  }
}

// ---------------------------------------------------------------- neighbour mean

// m_i = (1 / number of unbroken incident edges) sum over unbroken edges of h_j.
// Eight lanes per node, eight features (one 16-byte load) per lane.  The
// row's entries are taken four at a time with every load issued before the
// sums (an entry that is absent, the diagonal or a broken edge reads a valid
// stand-in and is skipped), so the gathers overlap; the sums keep the row's
// order.
__global__ __launch_bounds__(256) void k_net_mean(NetInputs in, int npad, const float* __restrict__ inv_wdeg,
                                                  const bf16* __restrict__ h, bf16* __restrict__ m) {
  const int node = blockIdx.x * 32 + (threadIdx.x >> 3), f8 = (threadIdx.x & 7) * 8;
  if (node >= npad) return;
  float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (node < in.n) {
    const int s = in.A.row_ptr[node], e = in.A.row_ptr[node + 1], db = in.diag_blk[node];
    for (int b0 = s; b0 < e; b0 += 4) {
      int col[4], ed[4];
      bool in_row[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int b = b0 + u;
        in_row[u] = b < e && b != db;
        const int bb = b < e ? b : s;
        col[u] = in.A.col[bb];
        ed[u] = in.blk_edge[bb];  // -1 on the diagonal
      }
      bool use[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) use[u] = in_row[u] && in.zeta[ed[u] < 0 ? 0 : ed[u]] == 0;
      bf16x8 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = *reinterpret_cast<const bf16x8*>(h + (size_t)col[u] * kHid + f8);
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (use[u]) {
#pragma unroll
          for (int q = 0; q < 8; ++q) acc[q] += (float)v[u][q];
        }
    }
    const float iw = inv_wdeg[node];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] *= iw;
  }
  bf16x8 out;
#pragma unroll
  for (int q = 0; q < 8; ++q) out[q] = (bf16)acc[q];
  *reinterpret_cast<bf16x8*>(m + (size_t)node * kHid + f8) = out;
}

// Backward through h_l = h_{l-1} + relu(W [h_{l-1}; m]) with m = P h_{l-1}:
// gh <- gh + gi[:, :64] + P^T gi[:, 64:], (P^T g)_j = sum_i w_ij g_i / wdeg_i over
// unbroken edges (a gather over the same symmetric pattern), then
// gz = gh * (zprev > 0) for the layer below.  Eight lanes per node, eight
// features per lane.
__global__ __launch_bounds__(256) void k_net_mean_bwd(NetInputs in, int npad, const float* __restrict__ inv_wdeg,
                                                      const float* __restrict__ gi, float* __restrict__ gh,
                                                      const bf16* __restrict__ zprev, bf16* __restrict__ gz) {
  typedef float f32x8 __attribute__((ext_vector_type(8)));
  const int node = blockIdx.x * 32 + (threadIdx.x >> 3), f8 = (threadIdx.x & 7) * 8;
  if (node >= npad) return;
  f32x8 g = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (node < in.n) {
    g = *reinterpret_cast<const f32x8*>(gh + (size_t)node * kHid + f8) +
        *reinterpret_cast<const f32x8*>(gi + (size_t)node * 2 * kHid + f8);
    const int s = in.A.row_ptr[node], e = in.A.row_ptr[node + 1], db = in.diag_blk[node];
    // four entries at a time, all loads before the sums (as in k_net_mean)
    for (int b0 = s; b0 < e; b0 += 4) {
      int col[4], ed[4];
      bool in_row[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int b = b0 + u;
        in_row[u] = b < e && b != db;
        const int bb = b < e ? b : s;
        col[u] = in.A.col[bb];
        ed[u] = in.blk_edge[bb];  // -1 on the diagonal
      }
      bool use[4];
      float wj[4];
      f32x8 gj[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        use[u] = in_row[u] && in.zeta[ed[u] < 0 ? 0 : ed[u]] == 0;
        wj[u] = inv_wdeg[col[u]];
        gj[u] = *reinterpret_cast<const f32x8*>(gi + (size_t)col[u] * 2 * kHid + kHid + f8);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (use[u]) g += wj[u] * gj[u];
    }
  }
  *reinterpret_cast<f32x8*>(gh + (size_t)node * kHid + f8) = g;
  const bf16x8 zp = *reinterpret_cast<const bf16x8*>(zprev + (size_t)node * kHid + f8);
  bf16x8 out;
#pragma unroll
  for (int q = 0; q < 8; ++q) out[q] = (bf16)((float)zp[q] > 0.f ? g[q] : 0.f);
  *reinterpret_cast<bf16x8*>(gz + (size_t)node * kHid + f8) = out;
}

// ---------------------------------------------------------------- head and factor

// Bounded map b(x) = 2 tanh(x / 2) of the network outputs and its slope.
__device__ __forceinline__ float bnd(float x) { return 2.f * tanhf(0.5f * x); }
__device__ __forceinline__ float bnd_slope(float x) {
  const float t = tanhf(0.5f * x);
  return 1.f - t * t;
}

// L = [[e^b(o0), 0, 0], [b(o3), e^b(o1), 0], [b(o4), b(o5), e^b(o2)]].
__device__ __forceinline__ void lower_from_o(const float* o, float L[3][3]) {
  L[0][0] = expf(bnd(o[0]));
  L[1][1] = expf(bnd(o[1]));
  L[2][2] = expf(bnd(o[2]));
  L[1][0] = bnd(o[3]);
  L[2][0] = bnd(o[4]);
  L[2][1] = bnd(o[5]);
  L[0][1] = L[0][2] = L[1][2] = 0.f;
}

// Row-major 3x3 block of slot b.
__device__ __forceinline__ void load_blk9(const float* __restrict__ val, int nbp, int b, float a[9]) {
#pragma unroll
  for (int c = 0; c < 9; ++c) a[c] = val[(size_t)c * nbp + b];
}

__device__ __forceinline__ void sym_from_binv(const float* binv, int n, int i, float C[3][3]) {
  C[0][0] = binv[i];
  C[1][1] = binv[(size_t)n + i];
  C[2][2] = binv[2 * (size_t)n + i];
  C[0][1] = C[1][0] = binv[3 * (size_t)n + i];
  C[0][2] = C[2][0] = binv[4 * (size_t)n + i];
  C[1][2] = C[2][1] = binv[5 * (size_t)n + i];
}

// C = inverse of the lower Cholesky factor of the SPD block a (FP64 inside),
// and log det C.
__device__ __forceinline__ float inv_chol(const float a[9], float C[3][3]) {
  const double l00 = sqrt((double)a[0]);
  const double l10 = a[3] / l00, l20 = a[6] / l00;
  const double l11 = sqrt((double)a[4] - l10 * l10);
  const double l21 = (a[7] - l20 * l10) / l11;
  const double l22 = sqrt((double)a[8] - l20 * l20 - l21 * l21);
  const double c00 = 1.0 / l00, c11 = 1.0 / l11, c22 = 1.0 / l22;
  const double c10 = -l10 * c00 / l11;
  const double c21 = -l21 * c11 / l22;
  const double c20 = -(l20 * c00 + l21 * c10) / l22;
  C[0][0] = (float)c00;
  C[1][1] = (float)c11;
  C[2][2] = (float)c22;
  C[1][0] = (float)c10;
  C[2][1] = (float)c21;
  C[2][0] = (float)c20;
  C[0][1] = C[0][2] = C[1][2] = 0.f;
  return (float)(log(c00) + log(c11) + log(c22));
}

__device__ __forceinline__ void mat3_mul(const float A[3][3], const float B[3][3], float Cm[3][3]) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) Cm[r][c] = A[r][0] * B[0][c] + A[r][1] * B[1][c] + A[r][2] * B[2][c];
}

// Edge features of the edge between nodes i and j (label of edge e).
__device__ __forceinline__ void edge_feat(const NetInputs& in, int i, int j, int e, float f[3]) {
  const d4 Xi = in.X[i], Xj = in.X[j], Ui = in.U[i], Uj = in.U[j];
  const double dx = Xj.x - Xi.x, dy = Xj.y - Xi.y, dz = Xj.z - Xi.z;
  const double cx = dx + (Uj.x - Ui.x), cy = dy + (Uj.y - Ui.y), cz = dz + (Uj.z - Ui.z);
  const double L0 = sqrt(dx * dx + dy * dy + dz * dz), L = sqrt(cx * cx + cy * cy + cz * cz);
  f[0] = (float)(L0 * in.inv_mean_len);
  f[1] = (float)tanh(L / L0 - 1.0);
  f[2] = in.zeta[e] ? 1.f : 0.f;
}

// M_i = L_i C_i (prescribed nodes: L = I), and log det M_i.
__device__ __forceinline__ float node_factor(const NetInputs& in, const float* __restrict__ o, int i,
                                             float M[3][3], float L[3][3], float C[3][3]) {
  float a[9];
  load_blk9(static_cast<const float*>(in.A.val), in.A.nbp, in.diag_blk[i], a);
  const float ldc = inv_chol(a, C);
  if (in.dflag[i]) {
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) L[r][c] = r == c ? 1.f : 0.f;
  } else {
    lower_from_o(o + (size_t)i * kNetHead, L);
  }
  mat3_mul(L, C, M);
  return in.dflag[i] ? ldc : ldc + bnd(o[(size_t)i * kNetHead]) + bnd(o[(size_t)i * kNetHead + 1]) +
                                 bnd(o[(size_t)i * kNetHead + 2]);
}

// W_b = b(s_i + t_j + We f + be) (row-major 3x3); slope (if given) = b' at the
// pre-activation.
__device__ __forceinline__ void edge_w(const float* __restrict__ o, int i, int j, const float f[3],
                                       const float* __restrict__ We, float W[3][3], float* slope = nullptr) {
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const float raw = o[(size_t)i * kNetHead + 6 + q] + o[(size_t)j * kNetHead + 15 + q] + We[3 * q] * f[0] +
                      We[3 * q + 1] * f[1] + We[3 * q + 2] * f[2] + We[27 + q];
    W[q / 3][q % 3] = bnd(raw);
    if (slope) slope[q] = bnd_slope(raw);
  }
}

// o = Wh h3 + bh for every padded row, one thread per node.
__global__ __launch_bounds__(256) void k_net_head_fwd(int npad, const float* __restrict__ master,
                                                      const bf16* __restrict__ h3, float* __restrict__ o_out) {
  __shared__ float Wh[kNetHead * kHid + kNetHead];
  for (int t = threadIdx.x; t < kNetHead * kHid + kNetHead; t += 256) Wh[t] = master[kOffWh + t];
  __syncthreads();
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= npad) return;
  float h[kHid];
#pragma unroll
  for (int c = 0; c < kHid / 8; ++c) {
    const bf16x8 v = *reinterpret_cast<const bf16x8*>(h3 + (size_t)i * kHid + 8 * c);
#pragma unroll
    for (int q = 0; q < 8; ++q) h[8 * c + q] = (float)v[q];
  }
  for (int k = 0; k < kNetHead; ++k) {
    float acc = Wh[kNetHead * kHid + k];
#pragma unroll
    for (int f = 0; f < kHid; ++f) acc += Wh[k * kHid + f] * h[f];
    o_out[(size_t)i * kNetHead + k] = acc;
  }
}

// Factor values: kBuildLanes lanes per block row; lane 0 writes the diagonal
// block M_i, the lanes walk the row's strictly lower blocks (i, j) and write
// G_ij into the lower arrays and G_ij^T into the upper ones at the mirror
// position.  FP32 (training): SoA gl, gu [9][ne], gd [6][n].  BF16 (solve):
// the packed records of FactView.
struct FactOut {
  float *gl32, *gu32, *gd32;
  uint4 *glv, *guv, *gdv;
  bf16 *gl8, *gu8;
};

template <bool FP32>
__device__ __forceinline__ void store_gblock(const FactOut& out, int ne, int idx, bool lower, const float B[3][3]) {
  if (FP32) {
    float* g = lower ? out.gl32 : out.gu32;
#pragma unroll
    for (int q = 0; q < 9; ++q) g[(size_t)q * ne + idx] = B[q / 3][q % 3];
  } else {
    bf16x8 v;
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = (bf16)B[q / 3][q % 3];
    (lower ? out.glv : out.guv)[idx] = __builtin_bit_cast(uint4, v);
    (lower ? out.gl8 : out.gu8)[idx] = (bf16)B[2][2];
  }
}

template <bool FP32>
__global__ __launch_bounds__(256) void k_fact_build(NetInputs in, const float* __restrict__ o,
                                                    const float* __restrict__ master, FactOut out) {
  __shared__ float We[kEdgeGrad];
  for (int t = threadIdx.x; t < kEdgeGrad; t += 256) We[t] = master[kOffWe + t];
  __syncthreads();
  const int n = in.n, nbp = in.A.nbp, ne = in.ne;
  const int lane = threadIdx.x & (kBuildLanes - 1);
  const float* __restrict__ val = static_cast<const float*>(in.A.val);
  for (int i = blockIdx.x * (256 / kBuildLanes) + threadIdx.x / kBuildLanes; i < n;
       i += gridDim.x * (256 / kBuildLanes)) {
    float M[3][3], L[3][3], C[3][3];
    node_factor(in, o, i, M, L, C);
    if (lane == 0) {
      const float d6[6] = {M[0][0], M[1][0], M[1][1], M[2][0], M[2][1], M[2][2]};
      if (FP32) {
#pragma unroll
        for (int q = 0; q < 6; ++q) out.gd32[(size_t)q * n + i] = d6[q];
      } else {
        bf16x8 v;
#pragma unroll
        for (int q = 0; q < 6; ++q) v[q] = (bf16)d6[q];
        v[6] = v[7] = (bf16)0.f;
        out.gdv[i] = __builtin_bit_cast(uint4, v);
      }
    }
    const int s = in.A.row_ptr[i], d = in.diag_blk[i], l0 = in.lptr[i];
    for (int b = s + lane; b < d; b += kBuildLanes) {
      const int j = in.A.col[b], e = in.blk_edge[b];
      const int li = l0 + (b - s), ui = in.upos[e];
      float f[3], W[3][3], a[9], Dj[3][3], K[3][3], T[3][3], Gb[3][3], Gt[3][3];
      edge_feat(in, i, j, e, f);
      edge_w(o, i, j, f, We, W);
      load_blk9(val, nbp, b, a);
      sym_from_binv(in.binv, n, j, Dj);
      const float Am[3][3] = {{a[0], a[1], a[2]}, {a[3], a[4], a[5]}, {a[6], a[7], a[8]}};
      mat3_mul(Am, Dj, K);
      mat3_mul(W, K, T);
      mat3_mul(M, T, Gb);
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          Gb[r][c] = -Gb[r][c];
          Gt[c][r] = Gb[r][c];
        }
      store_gblock<FP32>(out, ne, li, true, Gb);
      store_gblock<FP32>(out, ne, ui, false, Gt);
    }
  }
}

// ---------------------------------------------------------------- row normalisation of the factor

// Block row i of the packed BF16 factor at pattern position a (0: G_ii, lower
// triangular in the diagonal record; a >= 1: the row's lower slot a - 1).
__device__ __forceinline__ void load_grow_blk(const FactOut& F, int i, int l0, int a, float B[3][3]) {
  if (a == 0) {
    const bf16x8 d = __builtin_bit_cast(bf16x8, F.gdv[i]);
    B[0][0] = (float)d[0]; B[0][1] = 0.f;         B[0][2] = 0.f;
    B[1][0] = (float)d[1]; B[1][1] = (float)d[2]; B[1][2] = 0.f;
    B[2][0] = (float)d[3]; B[2][1] = (float)d[4]; B[2][2] = (float)d[5];
  } else {
    const bf16x8 v = __builtin_bit_cast(bf16x8, F.glv[l0 + a - 1]);
#pragma unroll
    for (int q = 0; q < 8; ++q) B[q / 3][q % 3] = (float)v[q];
    B[2][2] = (float)F.gl8[l0 + a - 1];
  }
}

// Scales every block row of the factor from the left by the inverse lower
// Cholesky factor N_i of its diagonal block of X = G A G^T,
//   X_ii = sum over pattern pairs (a, b) of G_ia A_ab G_ib^T,
// so that X_ii = I.  pairs[ptr[i] .. ptr[i+1]) lists the stored blocks A_ab
// with a <= b among the row's pattern {i, lower neighbours} (a = b once, a < b
// standing for both orders).  kBuildLanes lanes per row; a row's blocks are
// read (for X_ii) and then rewritten by the same lanes, lower records and
// their transposed upper copies; no other row touches them.  A row whose X_ii
// is not positive definite in FP32 is left as it is.
__global__ __launch_bounds__(256) void k_fact_normalise(NetInputs in, const int32_t* __restrict__ ptr,
                                                        const int4* __restrict__ pairs, FactOut F) {
  const int n = in.n, nbp = in.A.nbp;
  const int lane = threadIdx.x & (kBuildLanes - 1);
  const float* __restrict__ val = static_cast<const float*>(in.A.val);
  for (int i = blockIdx.x * (256 / kBuildLanes) + threadIdx.x / kBuildLanes; i < n;
       i += gridDim.x * (256 / kBuildLanes)) {
    const int l0 = in.lptr[i], k = in.lptr[i + 1] - l0;
    float X[3][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
    for (int p = ptr[i] + lane; p < ptr[i + 1]; p += kBuildLanes) {
      const int4 pr = pairs[p];  // (block of A, a, b, unused)
      float Ga[3][3], Gb[3][3], Am[3][3], T[3][3], S[3][3];
      load_grow_blk(F, i, l0, pr.y, Ga);
      load_grow_blk(F, i, l0, pr.z, Gb);
#pragma unroll
      for (int c = 0; c < 9; ++c) Am[c / 3][c % 3] = val[(size_t)c * nbp + pr.x];
      mat3_mul(Ga, Am, T);
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) S[r][c] = T[r][0] * Gb[c][0] + T[r][1] * Gb[c][1] + T[r][2] * Gb[c][2];
      const bool both = pr.y != pr.z;
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) X[r][c] += S[r][c] + (both ? S[c][r] : 0.f);
    }
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int o = kBuildLanes / 2; o > 0; o >>= 1) X[r][c] += __shfl_xor(X[r][c], o, kBuildLanes);
    // every lane of the row holds X_ii: lower Cholesky factor R, N = R^-1
    const float r00s = X[0][0];
    const float r00 = sqrtf(fmaxf(r00s, 0.f)), r10 = X[1][0] / r00, r20 = X[2][0] / r00;
    const float r11s = X[1][1] - r10 * r10;
    const float r11 = sqrtf(fmaxf(r11s, 0.f)), r21 = (X[2][1] - r20 * r10) / r11;
    const float r22s = X[2][2] - r20 * r20 - r21 * r21;
    const bool spd = r00s > 0.f && r11s > 0.f && r22s > 0.f && isfinite(r22s);
    if (!spd) continue;
    const float r22 = sqrtf(r22s);
    const float n00 = 1.f / r00, n11 = 1.f / r11, n22 = 1.f / r22;
    const float n10 = -r10 * n00 * n11, n21 = -r21 * n11 * n22;
    const float n20 = -(r20 * n00 + r21 * n10) * n22;
    const float N[3][3] = {{n00, 0.f, 0.f}, {n10, n11, 0.f}, {n20, n21, n22}};
    for (int a = lane; a <= k; a += kBuildLanes) {
      float B[3][3], NB[3][3];
      load_grow_blk(F, i, l0, a, B);
      mat3_mul(N, B, NB);
      if (a == 0) {
        bf16x8 v;
        v[0] = (bf16)NB[0][0];
        v[1] = (bf16)NB[1][0];
        v[2] = (bf16)NB[1][1];
        v[3] = (bf16)NB[2][0];
        v[4] = (bf16)NB[2][1];
        v[5] = (bf16)NB[2][2];
        v[6] = v[7] = (bf16)0.f;
        F.gdv[i] = __builtin_bit_cast(uint4, v);
      } else {
        float Nt[3][3];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c) Nt[c][r] = NB[r][c];
        const int e = in.blk_edge[in.A.row_ptr[i] + a - 1];
        store_gblock<false>(F, in.ne, l0 + a - 1, true, NB);
        store_gblock<false>(F, in.ne, in.upos[e], false, Nt);
      }
    }
  }
}

// ---------------------------------------------------------------- training (Kaporin probe loss)

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

__global__ __launch_bounds__(256) void k_net_probe_gen(int n, uint64_t seed, d4* __restrict__ v) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const uint64_t base = splitmix64(seed) ^ (3ull * (uint64_t)i);
  d4 r;
  r.x = (splitmix64(base) >> 63) ? -1.0 : 1.0;
  r.y = (splitmix64(base + 1) >> 63) ? -1.0 : 1.0;
  r.z = (splitmix64(base + 2) >> 63) ? -1.0 : 1.0;
  r.w = 0.0;
  v[i] = r;
}

// u = G^T v from the FP32 factor, FP64 accumulation (kBuildLanes lanes per row).
__global__ __launch_bounds__(256) void k_kap_u(NetInputs in, const float* __restrict__ gu,
                                               const float* __restrict__ gd, const d4* __restrict__ v,
                                               d4* __restrict__ u) {
  const int n = in.n, ne = in.ne;
  const int lane = threadIdx.x & (kBuildLanes - 1);
  for (int i = blockIdx.x * (256 / kBuildLanes) + threadIdx.x / kBuildLanes; i < n;
       i += gridDim.x * (256 / kBuildLanes)) {
    double ax = 0, ay = 0, az = 0;
    for (int b = in.uptr[i] + lane; b < in.uptr[i + 1]; b += kBuildLanes) {
      const d4 vj = v[in.ucol[b]];
      float a[9];
      load_blk9(gu, ne, b, a);
      ax += a[0] * vj.x + a[1] * vj.y + a[2] * vj.z;
      ay += a[3] * vj.x + a[4] * vj.y + a[5] * vj.z;
      az += a[6] * vj.x + a[7] * vj.y + a[8] * vj.z;
    }
#pragma unroll
    for (int s = kBuildLanes / 2; s > 0; s >>= 1) {
      ax += __shfl_xor(ax, s, kBuildLanes);
      ay += __shfl_xor(ay, s, kBuildLanes);
      az += __shfl_xor(az, s, kBuildLanes);
    }
    if (lane == 0) {
      const d4 vi = v[i];
      const double g00 = gd[i], g10 = gd[(size_t)n + i], g11 = gd[2 * (size_t)n + i];
      const double g20 = gd[3 * (size_t)n + i], g21 = gd[4 * (size_t)n + i], g22 = gd[5 * (size_t)n + i];
      ax += g00 * vi.x + g10 * vi.y + g20 * vi.z;
      ay += g11 * vi.y + g21 * vi.z;
      az += g22 * vi.z;
      u[i] = d4{ax, ay, az, 0.0};
    }
  }
}

// Per node: partials of t = u.w (w = -wneg) and of log det M_i; m_i = M_i^T v_i
// and s_i = A_ii^-1 w_i for the gradient kernel.
__global__ __launch_bounds__(256) void k_kap_node(NetInputs in, const float* __restrict__ o, const d4* __restrict__ v,
                                                  const d4* __restrict__ u, const d4* __restrict__ wneg,
                                                  v4<float>* __restrict__ mv, v4<float>* __restrict__ sv,
                                                  double* __restrict__ dpart) {
  __shared__ double sh[8];
  const int i = blockIdx.x * 256 + threadIdx.x;
  double t = 0.0, ld = 0.0;
  if (i < in.n) {
    float M[3][3], L[3][3], C[3][3], D[3][3];
    ld = node_factor(in, o, i, M, L, C);
    const d4 vi = v[i], ui = u[i], wi = wneg[i];
    t = -(ui.x * wi.x + ui.y * wi.y + ui.z * wi.z);
    const float v3[3] = {(float)vi.x, (float)vi.y, (float)vi.z};
    const float w3[3] = {(float)-wi.x, (float)-wi.y, (float)-wi.z};
    float m3[3], s3[3];
    sym_from_binv(in.binv, in.n, i, D);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      m3[c] = M[0][c] * v3[0] + M[1][c] * v3[1] + M[2][c] * v3[2];
      s3[c] = D[c][0] * w3[0] + D[c][1] * w3[1] + D[c][2] * w3[2];
    }
    mv[i] = v4<float>{m3[0], m3[1], m3[2], 0.f};
    sv[i] = v4<float>{s3[0], s3[1], s3[2], 0.f};
  }
  t = wsum(t);
  ld = wsum(ld);
  if ((threadIdx.x & 63) == 0) {
    sh[threadIdx.x >> 6] = t;
    sh[4 + (threadIdx.x >> 6)] = ld;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    dpart[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    dpart[kMaxPart + blockIdx.x] = (sh[4] + sh[5]) + (sh[6] + sh[7]);
  }
}

// One power step on X = G A G^T: y = G x with x = -wneg (the caller's residual
// kernel leaves -A G^T v there), FP32 factor, FP64 accumulation
// (kBuildLanes lanes per row), and per-workgroup partials of |y|^2.
__global__ __launch_bounds__(256) void k_kap_gx(NetInputs in, const float* __restrict__ gl,
                                                const float* __restrict__ gd, const d4* __restrict__ wneg,
                                                d4* __restrict__ y, double* __restrict__ part) {
  __shared__ double sh[4];
  const int n = in.n, ne = in.ne;
  const int lane = threadIdx.x & (kBuildLanes - 1);
  double acc = 0.0;
  for (int i = blockIdx.x * (256 / kBuildLanes) + threadIdx.x / kBuildLanes; i < n;
       i += gridDim.x * (256 / kBuildLanes)) {
    double ax = 0, ay = 0, az = 0;
    for (int b = in.lptr[i] + lane; b < in.lptr[i + 1]; b += kBuildLanes) {
      const d4 xj = wneg[in.lcol[b]];
      float a[9];
      load_blk9(gl, ne, b, a);
      ax -= a[0] * xj.x + a[1] * xj.y + a[2] * xj.z;
      ay -= a[3] * xj.x + a[4] * xj.y + a[5] * xj.z;
      az -= a[6] * xj.x + a[7] * xj.y + a[8] * xj.z;
    }
#pragma unroll
    for (int s = kBuildLanes / 2; s > 0; s >>= 1) {
      ax += __shfl_xor(ax, s, kBuildLanes);
      ay += __shfl_xor(ay, s, kBuildLanes);
      az += __shfl_xor(az, s, kBuildLanes);
    }
    if (lane == 0) {
      const d4 xi = wneg[i];
      const double g00 = gd[i], g10 = gd[(size_t)n + i], g11 = gd[2 * (size_t)n + i];
      const double g20 = gd[3 * (size_t)n + i], g21 = gd[4 * (size_t)n + i], g22 = gd[5 * (size_t)n + i];
      ax -= g00 * xi.x;
      ay -= g10 * xi.x + g11 * xi.y;
      az -= g20 * xi.x + g21 * xi.y + g22 * xi.z;
      y[i] = d4{ax, ay, az, 0.0};
      acc += ax * ax + ay * ay + az * az;
    }
  }
  acc = wsum(acc);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ __launch_bounds__(256) void k_scale_d4(int n, double f, d4* __restrict__ v) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const d4 a = v[i];
  v[i] = d4{a.x * f, a.y * f, a.z * f, 0.0};
}

__device__ __forceinline__ float wsumf(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Head-output gradient go (24 per row, zero on padding rows) and per-workgroup
// partials of the edge-term gradient (We, be).  With k_b = A_ij s_j and r_b
// the edge pre-activation (W_b = b(r_b)):
//   dloss/dr_b  = -(2/t) m_i k_b^T * b'(r_b)  (elementwise),
//   go[6:15]_i  = sum over lower slots of row i of dloss/dr_b,
//   go[15:24]_j = sum over lower blocks (i, j) of dloss/dr_b (row j's upper slots),
//   dloss/dL_i  = (2/t) v_i rho_i^T - (2/N) L_i^-T, rho_i = C_i (w_i - sum_b W_b k_b),
//   and through L = L(b(o)) to o[0:6].
__global__ __launch_bounds__(256) void k_kap_grad(NetInputs in, int npad, const float* __restrict__ o,
                                                  const float* __restrict__ master, const d4* __restrict__ v,
                                                  const d4* __restrict__ wneg, const v4<float>* __restrict__ mv,
                                                  const v4<float>* __restrict__ sv, float c2t, float c2n,
                                                  float* __restrict__ go, float* __restrict__ epart) {
  __shared__ float We[kEdgeGrad];
  __shared__ float red[4][kEdgeGrad];
  for (int t = threadIdx.x; t < kEdgeGrad; t += 256) We[t] = master[kOffWe + t];
  __syncthreads();
  const int n = in.n, nbp = in.A.nbp;
  const int lane = threadIdx.x & (kBuildLanes - 1);
  const float* __restrict__ val = static_cast<const float*>(in.A.val);
  float eg[kEdgeGrad];
#pragma unroll
  for (int q = 0; q < kEdgeGrad; ++q) eg[q] = 0.f;
  const int rows_per = 256 / kBuildLanes;
  const int nrow_iter = (npad + gridDim.x * rows_per - 1) / (gridDim.x * rows_per);
  for (int it = 0; it < nrow_iter; ++it) {
    const int i = (it * gridDim.x + blockIdx.x) * rows_per + threadIdx.x / kBuildLanes;
    if (i >= npad) continue;
    if (i >= n) {
      if (lane == 0)
        for (int q = 0; q < kNetHead; ++q) go[(size_t)i * kNetHead + q] = 0.f;
      continue;
    }
    const v4<float> mi = mv[i], si = sv[i];
    float rho3[3] = {0.f, 0.f, 0.f}, gs[9], gt[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) gs[q] = gt[q] = 0.f;
    const int s = in.A.row_ptr[i], d = in.diag_blk[i], e = in.A.row_ptr[i + 1];
    for (int b = s + lane; b < e; b += kBuildLanes) {
      if (b == d) continue;
      const int j = in.A.col[b];
      float a[9];
      load_blk9(val, nbp, b, a);
      if (b < d) {
        const v4<float> sj = sv[j];
        const float k3[3] = {a[0] * sj.x + a[1] * sj.y + a[2] * sj.z, a[3] * sj.x + a[4] * sj.y + a[5] * sj.z,
                             a[6] * sj.x + a[7] * sj.y + a[8] * sj.z};
        float f[3], W[3][3], sl[9];
        edge_feat(in, i, j, in.blk_edge[b], f);
        edge_w(o, i, j, f, We, W, sl);
        const float m3[3] = {mi.x, mi.y, mi.z};
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          rho3[r] += W[r][0] * k3[0] + W[r][1] * k3[1] + W[r][2] * k3[2];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const int q = 3 * r + c;
            const float dw = -c2t * m3[r] * k3[c] * sl[q];
            gs[q] += dw;
            eg[3 * q] += dw * f[0];
            eg[3 * q + 1] += dw * f[1];
            eg[3 * q + 2] += dw * f[2];
            eg[27 + q] += dw;
          }
        }
      } else {
        // upper slot (i, k): lower block (k, i) with k_b = A_ki s_i = A_ik^T s_i
        const v4<float> mk = mv[j];
        const float k3[3] = {a[0] * si.x + a[3] * si.y + a[6] * si.z, a[1] * si.x + a[4] * si.y + a[7] * si.z,
                             a[2] * si.x + a[5] * si.y + a[8] * si.z};
        const float m3[3] = {mk.x, mk.y, mk.z};
        float f[3], W[3][3], sl[9];
        edge_feat(in, j, i, in.blk_edge[b], f);
        edge_w(o, j, i, f, We, W, sl);
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c) gt[3 * r + c] -= c2t * m3[r] * k3[c] * sl[3 * r + c];
      }
    }
#pragma unroll
    for (int sft = kBuildLanes / 2; sft > 0; sft >>= 1) {
#pragma unroll
      for (int r = 0; r < 3; ++r) rho3[r] += __shfl_xor(rho3[r], sft, kBuildLanes);
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        gs[q] += __shfl_xor(gs[q], sft, kBuildLanes);
        gt[q] += __shfl_xor(gt[q], sft, kBuildLanes);
      }
    }
    if (lane == 0) {
      float* gout = go + (size_t)i * kNetHead;
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        gout[6 + q] = gs[q];
        gout[15 + q] = gt[q];
      }
      if (in.dflag[i]) {
        for (int q = 0; q < 6; ++q) gout[q] = 0.f;
      } else {
        float M[3][3], L[3][3], C[3][3];
        node_factor(in, o, i, M, L, C);
        const d4 vi = v[i], wi = wneg[i];
        const float w3[3] = {(float)-wi.x - rho3[0], (float)-wi.y - rho3[1], (float)-wi.z - rho3[2]};
        float rho[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) rho[r] = C[r][0] * w3[0] + C[r][1] * w3[1] + C[r][2] * w3[2];
        const float v3[3] = {(float)vi.x, (float)vi.y, (float)vi.z};
        const float* oi = o + (size_t)i * kNetHead;
        gout[0] = (c2t * v3[0] * rho[0] * L[0][0] - c2n) * bnd_slope(oi[0]);
        gout[1] = (c2t * v3[1] * rho[1] * L[1][1] - c2n) * bnd_slope(oi[1]);
        gout[2] = (c2t * v3[2] * rho[2] * L[2][2] - c2n) * bnd_slope(oi[2]);
        gout[3] = c2t * v3[1] * rho[0] * bnd_slope(oi[3]);
        gout[4] = c2t * v3[2] * rho[0] * bnd_slope(oi[4]);
        gout[5] = c2t * v3[2] * rho[1] * bnd_slope(oi[5]);
      }
    }
  }
  // workgroup partials of the edge-term gradient, fixed order
#pragma unroll
  for (int q = 0; q < kEdgeGrad; ++q) {
    const float r = wsumf(eg[q]);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][q] = r;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < kEdgeGrad; q += 256)
    epart[(size_t)blockIdx.x * kEdgeGrad + q] = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
}

// Sum of nwg per-workgroup partials (record length len, entry src) for 64
// outputs per 256-thread workgroup: the four waves take every fourth partial
// (loads coalesced over the 64 outputs, eight in flight per lane) and the four
// sums are added in order in LDS, so the result does not depend on timing.
__device__ __forceinline__ float reduce_partials64(int nwg, const float* __restrict__ part, size_t len, int src,
                                                   bool act, float* sh) {
  const int o = threadIdx.x & 63, sl = threadIdx.x >> 6;
  float s = 0.f;
  if (act) {
    for (int w0 = sl; w0 < nwg; w0 += 32) {
      float x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int w = w0 + 4 * u;
        x[u] = w < nwg ? part[(size_t)w * len + src] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) s += x[u];
    }
  }
  sh[sl * 64 + o] = s;
  __syncthreads();
  return ((sh[o] + sh[64 + o]) + sh[128 + o]) + sh[192 + o];
}

static_assert(kEdgeGrad <= 64, "one workgroup of 64 outputs reduces the edge-weight gradient");

__global__ __launch_bounds__(256) void k_kap_edge_reduce(int nwg, const float* __restrict__ epart,
                                                         float* __restrict__ grad) {
  __shared__ float sh[256];
  const int q = threadIdx.x & 63;
  const bool act = q < kEdgeGrad;
  const float s = reduce_partials64(nwg, epart, kEdgeGrad, act ? q : 0, act, sh);
  if (act && threadIdx.x < 64) grad[kOffWe + q] = s;
}

// gh3 = Wh^T go and gz3 = gh3 * (z3 > 0), one thread per padded row.
__global__ __launch_bounds__(256) void k_net_head_bwd(int npad, const float* __restrict__ master,
                                                      const float* __restrict__ go, const bf16* __restrict__ z3,
                                                      float* __restrict__ gh, bf16* __restrict__ gz) {
  __shared__ float Wh[kNetHead * kHid];
  for (int t = threadIdx.x; t < kNetHead * kHid; t += 256) Wh[t] = master[kOffWh + t];
  __syncthreads();
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= npad) return;
  float g[kNetHead];
#pragma unroll
  for (int k = 0; k < kNetHead; ++k) g[k] = go[(size_t)i * kNetHead + k];
  for (int f = 0; f < kHid; ++f) {
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < kNetHead; ++k) acc += Wh[k * kHid + f] * g[k];
    gh[(size_t)i * kHid + f] = acc;
    gz[(size_t)i * kHid + f] = (bf16)((float)z3[(size_t)i * kHid + f] > 0.f ? acc : 0.f);
  }
}

// ---------------------------------------------------------------- weight gradients

// dW[o][k] = sum over nodes of gz[node][o] X[node][k] and db[o] = sum gz[node][o]
// for X = [XA | XB]: per workgroup a contiguous node range, 32 nodes at a time
// transposed into LDS, then MFMA with nodes as the reduction dimension (wave
// w owns output rows 16w..16w+15).  Partials [workgroup][64*K + 64].
template <int KA, int KB>
__global__ __launch_bounds__(256) void k_net_dw(int npad, const bf16* __restrict__ gz, const bf16* __restrict__ XA,
                                                const bf16* __restrict__ XB, float* __restrict__ part) {
  constexpr int K = KA + KB;
  constexpr int QT = K / 16;
  __shared__ __attribute__((aligned(16))) bf16 gzT[kHid][32];
  __shared__ __attribute__((aligned(16))) bf16 XT[K][32];
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int G = gridDim.x;
  const int per = ((npad + G - 1) / G + 31) / 32 * 32;
  const int c0 = min(npad, blockIdx.x * per), c1 = min(npad, c0 + per);
  f32x4 acc[QT];
#pragma unroll
  for (int q = 0; q < QT; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
  float dbs = 0.f;
  for (int n0 = c0; n0 < c1; n0 += 32) {
    // gz chunk: 32 nodes x 64 -> 256 loads of 8
    {
      const int node = threadIdx.x >> 3, o8 = (threadIdx.x & 7) * 8;
      const bf16x8 v = *reinterpret_cast<const bf16x8*>(gz + (size_t)(n0 + node) * kHid + o8);
#pragma unroll
      for (int q = 0; q < 8; ++q) gzT[o8 + q][node] = v[q];
    }
    for (int t = threadIdx.x; t < 32 * K / 8; t += 256) {
      const int node = t / (K / 8), k8 = (t % (K / 8)) * 8;
      const bf16x8 v = (k8 < KA) ? *reinterpret_cast<const bf16x8*>(XA + (size_t)(n0 + node) * KA + k8)
                                 : *reinterpret_cast<const bf16x8*>(XB + (size_t)(n0 + node) * KB + (k8 - KA));
#pragma unroll
      for (int q = 0; q < 8; ++q) XT[k8 + q][node] = v[q];
    }
    __syncthreads();
    const bf16x8 av = *reinterpret_cast<const bf16x8*>(&gzT[16 * wv + (l & 15)][8 * (l >> 4)]);
#pragma unroll
    for (int q = 0; q < QT; ++q) {
      const bf16x8 bv = *reinterpret_cast<const bf16x8*>(&XT[16 * q + (l & 15)][8 * (l >> 4)]);
      acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[q], 0, 0, 0);
    }
    if (threadIdx.x < kHid)
      for (int node = 0; node < 32; ++node) dbs += (float)gzT[threadIdx.x][node];
    __syncthreads();
  }
  float* out = part + (size_t)blockIdx.x * (kHid * K + kHid);
#pragma unroll
  for (int q = 0; q < QT; ++q)
#pragma unroll
    for (int i = 0; i < 4; ++i) out[(size_t)(16 * wv + 4 * (l >> 4) + i) * K + 16 * q + (l & 15)] = acc[q][i];
  if (threadIdx.x < kHid) out[kHid * K + threadIdx.x] = dbs;
}

// Sum the partials into the flat gradient (first Kreal columns).
__global__ __launch_bounds__(256) void k_net_dw_reduce(int nwg, int K, int Kreal, const float* __restrict__ part,
                                                       float* __restrict__ grad, int offW, int offb) {
  __shared__ float sh[256];
  const int t = blockIdx.x * 64 + (threadIdx.x & 63);
  const int nW = kHid * Kreal;
  const bool act = t < nW + kHid;
  int src = 0, dst = 0;
  if (t < nW) {
    const int o = t / Kreal, k = t % Kreal;
    src = o * K + k;
    dst = offW + t;
  } else if (act) {
    src = kHid * K + (t - nW);
    dst = offb + (t - nW);
  }
  const float s = reduce_partials64(nwg, part, (size_t)kHid * K + kHid, src, act, sh);
  if (act && threadIdx.x < 64) grad[dst] = s;
}

// dWh[k][f] = sum go[k] h3[f], dbh[k] = sum go[k]: per workgroup a node range,
// outputs strided over the threads; partials [workgroup][24*64 + 24].
constexpr int kHeadGrad = kNetHead * kHid + kNetHead;

__global__ __launch_bounds__(512) void k_net_dhead(int npad, const float* __restrict__ go, const bf16* __restrict__ h3,
                                                   float* __restrict__ part) {
  const int G = gridDim.x;
  const int per = (npad + G - 1) / G;
  const int c0 = min(npad, blockIdx.x * per), c1 = min(npad, c0 + per);
  for (int t = threadIdx.x; t < kHeadGrad; t += 512) {
    const int k = t < kNetHead * kHid ? t / kHid : t - kNetHead * kHid;
    const int f = t < kNetHead * kHid ? t % kHid : -1;
    float s = 0.f;
    for (int i = c0; i < c1; ++i)
      s += go[(size_t)i * kNetHead + k] * (f >= 0 ? (float)h3[(size_t)i * kHid + f] : 1.f);
    part[(size_t)blockIdx.x * kHeadGrad + t] = s;
  }
}

__global__ __launch_bounds__(256) void k_net_dhead_reduce(int nwg, const float* __restrict__ part,
                                                          float* __restrict__ grad) {
  __shared__ float sh[256];
  const int t = blockIdx.x * 64 + (threadIdx.x & 63);
  const bool act = t < kHeadGrad;
  const float s = reduce_partials64(nwg, part, kHeadGrad, act ? t : 0, act, sh);
  if (act && threadIdx.x < 64) grad[kOffWh + t] = s;
}

// ---------------------------------------------------------------- optimiser

__global__ __launch_bounds__(256) void k_net_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                                                  const float* __restrict__ g, float lr, float c1, float c2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= kNetParams) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + 1e-8f);
}

// BF16 copies: W0 [64][32] zero-padded, W_l [64][128] and W_l^T [128][64].
__global__ __launch_bounds__(256) void k_net_pack(const float* __restrict__ w, bf16* __restrict__ W0,
                                                  bf16* __restrict__ W1, bf16* __restrict__ W2, bf16* __restrict__ W3,
                                                  bf16* __restrict__ T1, bf16* __restrict__ T2,
                                                  bf16* __restrict__ T3) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t < kHid * kNetInPad) {
    const int o = t / kNetInPad, k = t % kNetInPad;
    W0[t] = (bf16)(k < kNetIn ? w[kOffW0 + o * kNetIn + k] : 0.f);
  }
  if (t < kHid * 2 * kHid) {
    const int o = t / (2 * kHid), k = t % (2 * kHid);
    bf16* Wd[3] = {W1, W2, W3};
    bf16* Td[3] = {T1, T2, T3};
    for (int l = 0; l < kNetLayers; ++l) {
      const float x = w[kOffL0 + l * kLayerSize + t];
      Wd[l][t] = (bf16)x;
      Td[l][(size_t)k * kHid + o] = (bf16)x;
    }
  }
}

inline int nb256(int n) { return (n + 255) / 256; }

}  // namespace

void net_forward(hipStream_t s, const NetParamsDev& P, NetWork& w, const NetInputs& in, int, bool keep_z) {
  const int np = w.npad;
  k_net_inputs<<<nb256(np), 256, 0, s>>>(in, np, w.a, w.inv_wdeg);
  k_net_gemm<kNetInPad, 0, kHid, 0><<<np / kNetRows, 256, 0, s>>>(w.a, nullptr, P.W0, P.master + kOffB0, nullptr,
                                                                  keep_z ? w.z[0] : nullptr, w.h[0], nullptr);
  for (int l = 0; l < kNetLayers; ++l) {
    k_net_mean<<<np / 32, 256, 0, s>>>(in, np, w.inv_wdeg, w.h[l], w.m[l]);
    k_net_gemm<kHid, kHid, kHid, 1><<<np / kNetRows, 256, 0, s>>>(
        w.h[l], w.m[l], P.Wl[l], P.master + kOffL0 + l * kLayerSize + kHid * 2 * kHid, w.h[l],
        keep_z ? w.z[l + 1] : nullptr, w.h[l + 1], nullptr);
  }
  k_net_head_fwd<<<nb256(np), 256, 0, s>>>(np, P.master, w.h[kNetLayers], w.o);
}

void net_build_factor(hipStream_t s, const NetParamsDev& P, NetWork& w, const NetInputs& in, int Gb, bool fp32) {
  const FactOut out{w.gl32, w.gu32, w.gd32, w.glv, w.guv, w.gdv, w.gl8, w.gu8};
  if (fp32)
    k_fact_build<true><<<Gb, 256, 0, s>>>(in, w.o, P.master, out);
  else
    k_fact_build<false><<<Gb, 256, 0, s>>>(in, w.o, P.master, out);
}

void net_normalise_factor(hipStream_t s, NetWork& w, const NetInputs& in, int Gb, const int32_t* ptr,
                          const int4* pairs) {
  const FactOut out{w.gl32, w.gu32, w.gd32, w.glv, w.guv, w.gdv, w.gl8, w.gu8};
  k_fact_normalise<<<Gb, 256, 0, s>>>(in, ptr, pairs, out);
}

FactView net_factor_view(const NetWork& w, const NetInputs& in) {
  return FactView{in.n, in.ne, in.lptr, in.lcol, in.uptr, in.ucol, w.glv, w.gl8, w.guv, w.gu8, w.gdv};
}

void net_probe(hipStream_t s, NetWork& w, uint64_t seed) { k_net_probe_gen<<<nb256(w.n), 256, 0, s>>>(w.n, seed, w.probe); }

void net_kaporin_u(hipStream_t s, NetWork& w, const NetInputs& in, int Gb) {
  k_kap_u<<<Gb, 256, 0, s>>>(in, w.gu32, w.gd32, w.probe, w.u);
}

int net_power_apply(hipStream_t s, NetWork& w, const NetInputs& in, int Gb) {
  k_kap_gx<<<Gb, 256, 0, s>>>(in, w.gl32, w.gd32, w.wneg, w.probe, w.dpart);
  return Gb;
}

void net_scale_probe(hipStream_t s, NetWork& w, double f) { k_scale_d4<<<nb256(w.n), 256, 0, s>>>(w.n, f, w.probe); }

int net_kaporin_dots(hipStream_t s, const NetParamsDev&, NetWork& w, const NetInputs& in) {
  k_kap_node<<<nb256(in.n), 256, 0, s>>>(in, w.o, w.probe, w.u, w.wneg, w.mv, w.sv, w.dpart);
  return nb256(in.n);
}

void net_kaporin_backward(hipStream_t s, const NetParamsDev& P, NetWork& w, const NetInputs& in, int Gb, double t) {
  const int np = w.npad;
  const double N = 3.0 * in.n;
  k_kap_grad<<<Gb, 256, 0, s>>>(in, np, w.o, P.master, w.probe, w.wneg, w.mv, w.sv, (float)(2.0 / t),
                                (float)(2.0 / N), w.go, w.epart);
  k_kap_edge_reduce<<<1, 256, 0, s>>>(Gb, w.epart, w.grad);
  k_net_dhead<<<kDwWorkgroups, 512, 0, s>>>(np, w.go, w.h[kNetLayers], w.part);
  k_net_dhead_reduce<<<(kHeadGrad + 63) / 64, 256, 0, s>>>(kDwWorkgroups, w.part, w.grad);
  k_net_head_bwd<<<nb256(np), 256, 0, s>>>(np, P.master, w.go, w.z[kNetLayers], w.gh, w.gz);
  for (int l = kNetLayers - 1; l >= 0; --l) {
    // gz holds dloss/dz_{l+1}
    k_net_dw<kHid, kHid><<<kDwWorkgroups, 256, 0, s>>>(np, w.gz, w.h[l], w.m[l], w.part);
    k_net_dw_reduce<<<(kHid * 2 * kHid + kHid + 63) / 64, 256, 0, s>>>(kDwWorkgroups, 2 * kHid, 2 * kHid, w.part,
                                                                       w.grad, kOffL0 + l * kLayerSize,
                                                                       kOffL0 + l * kLayerSize + kHid * 2 * kHid);
    k_net_gemm<kHid, 0, 2 * kHid, 2><<<np / kNetRows, 256, 0, s>>>(w.gz, nullptr, P.WlT[l], nullptr, nullptr,
                                                                   nullptr, nullptr, w.gi);
    k_net_mean_bwd<<<np / 32, 256, 0, s>>>(in, np, w.inv_wdeg, w.gi, w.gh, w.z[l], w.gz);
  }
  k_net_dw<kNetInPad, 0><<<kDwWorkgroups, 256, 0, s>>>(np, w.gz, w.a, nullptr, w.part);
  k_net_dw_reduce<<<(kHid * kNetIn + kHid + 63) / 64, 256, 0, s>>>(kDwWorkgroups, kNetInPad, kNetIn, w.part,
                                                                   w.grad, kOffW0, kOffB0);
}

void net_adam(hipStream_t s, NetParamsDev& P, const float* grad, int t, float lr) {
  const float c1 = 1.f / (1.f - powf(0.9f, (float)t));
  const float c2 = 1.f / (1.f - powf(0.999f, (float)t));
  k_net_adam<<<nb256(kNetParams), 256, 0, s>>>(P.master, P.adam_m, P.adam_v, grad, lr, c1, c2);
  net_pack(s, P);
}

void net_pack(hipStream_t s, NetParamsDev& P) {
  k_net_pack<<<nb256(kHid * 2 * kHid), 256, 0, s>>>(P.master, P.W0, P.Wl[0], P.Wl[1], P.Wl[2], P.WlT[0], P.WlT[1],
                                                     P.WlT[2]);
}

}  // namespace gfem
