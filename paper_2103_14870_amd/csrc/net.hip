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

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------- inputs

// Node input a_i = [1, mean f0, mean f1, mean f2, mean f1^2, mean |f1|,
// mean (1 - f2) f1, degree / 16] over the incident edges, with edge features
// f0 = rest length / mean rest length, f1 = current / rest length - 1,
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
      const float f0 = (float)(L0 * in.inv_mean_len), f1 = (float)(L / L0 - 1.0);
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
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = r0 + 4 * (l >> 4) + i, col = t * 16 + (l & 15);
      const float v = acc[t][i];
      if (EPI == 2) {
        Fout[(size_t)row * NOUT + col] = v;
      } else {
        const float zz = v + bias[col];
        Zout[(size_t)row * NOUT + col] = (bf16)zz;
        float hr = fmaxf(zz, 0.f);
        if (EPI == 1) hr += (float)Hin[(size_t)row * NOUT + col];
        Hout[(size_t)row * NOUT + col] = (bf16)hr;
      }
    }
}

// ---------------------------------------------------------------- neighbour mean

// m_i = (1 / number of unbroken incident edges) sum over unbroken edges of h_j.
// One wave per node, lane = feature.
__global__ __launch_bounds__(256) void k_net_mean(NetInputs in, int npad, const float* __restrict__ inv_wdeg,
                                                  const bf16* __restrict__ h, bf16* __restrict__ m) {
  const int node = blockIdx.x * 4 + (threadIdx.x >> 6), f = threadIdx.x & 63;
  if (node >= npad) return;
  float acc = 0.f;
  if (node < in.n) {
    const int s = in.A.row_ptr[node], e = in.A.row_ptr[node + 1], db = in.diag_blk[node];
    for (int b = s; b < e; ++b) {
      if (b == db) continue;
      if (in.zeta[in.blk_edge[b]]) continue;
      acc += (float)h[(size_t)in.A.col[b] * kHid + f];
    }
    acc *= inv_wdeg[node];
  }
  m[(size_t)node * kHid + f] = (bf16)acc;
}

// Backward through h_l = h_{l-1} + relu(W [h_{l-1}; m]) with m = P h_{l-1}:
// gh <- gh + gi[:, :64] + P^T gi[:, 64:], (P^T g)_j = sum_i w_ij g_i / wdeg_i over
// unbroken edges (a gather over the same symmetric pattern), then
// gz = gh * (zprev > 0) for the layer below.
__global__ __launch_bounds__(256) void k_net_mean_bwd(NetInputs in, int npad, const float* __restrict__ inv_wdeg,
                                                      const float* __restrict__ gi, float* __restrict__ gh,
                                                      const bf16* __restrict__ zprev, bf16* __restrict__ gz) {
  const int node = blockIdx.x * 4 + (threadIdx.x >> 6), f = threadIdx.x & 63;
  if (node >= npad) return;
  float g = 0.f;
  if (node < in.n) {
    g = gh[(size_t)node * kHid + f] + gi[(size_t)node * 2 * kHid + f];
    const int s = in.A.row_ptr[node], e = in.A.row_ptr[node + 1], db = in.diag_blk[node];
    for (int b = s; b < e; ++b) {
      if (b == db) continue;
      if (in.zeta[in.blk_edge[b]]) continue;
      const int j = in.A.col[b];
      g += inv_wdeg[j] * gi[(size_t)j * 2 * kHid + kHid + f];
    }
  }
  gh[(size_t)node * kHid + f] = g;
  gz[(size_t)node * kHid + f] = (bf16)((float)zprev[(size_t)node * kHid + f] > 0.f ? g : 0.f);
}

// ---------------------------------------------------------------- head

__device__ __forceinline__ void lower_from_o(const float* o, float L[3][3]) {
  L[0][0] = expf(o[0]);
  L[1][1] = expf(o[1]);
  L[2][2] = expf(o[2]);
  L[1][0] = o[3];
  L[2][0] = o[4];
  L[2][1] = o[5];
  L[0][1] = L[0][2] = L[1][2] = 0.f;
}

__device__ __forceinline__ void sym_from_binv(const float* binv, int n, int i, float C[3][3]) {
  C[0][0] = binv[i];
  C[1][1] = binv[(size_t)n + i];
  C[2][2] = binv[2 * (size_t)n + i];
  C[0][1] = C[1][0] = binv[3 * (size_t)n + i];
  C[0][2] = C[2][0] = binv[4 * (size_t)n + i];
  C[1][2] = C[2][1] = binv[5 * (size_t)n + i];
}

// B = L C L^T (symmetrised) stored as [6][n] (00, 11, 22, 01, 02, 12).
__device__ __forceinline__ void store_block(float* Bout, int n, int i, const float L[3][3], const float C[3][3]) {
  float LC[3][3], B[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) LC[r][c] = L[r][0] * C[0][c] + L[r][1] * C[1][c] + L[r][2] * C[2][c];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) B[r][c] = LC[r][0] * L[c][0] + LC[r][1] * L[c][1] + LC[r][2] * L[c][2];
  Bout[i] = B[0][0];
  Bout[(size_t)n + i] = B[1][1];
  Bout[2 * (size_t)n + i] = B[2][2];
  Bout[3 * (size_t)n + i] = 0.5f * (B[0][1] + B[1][0]);
  Bout[4 * (size_t)n + i] = 0.5f * (B[0][2] + B[2][0]);
  Bout[5 * (size_t)n + i] = 0.5f * (B[1][2] + B[2][1]);
}

// One thread per node: o = Wh h3 + bh, L(o), B = L A_ii^-1 L^T (prescribed
// nodes keep A_ii^-1).  TRAIN: residual r = B b - dv over free nodes, loss
// partial, go = dloss/do, gh3 = Wh^T go and gz3 = gh3 * (z3 > 0).
template <bool TRAIN>
__global__ __launch_bounds__(256) void k_net_head(NetInputs in, int npad, const float* __restrict__ master,
                                                  const bf16* __restrict__ h3, float* __restrict__ o_out,
                                                  float* __restrict__ Bout, const d4* __restrict__ bvec,
                                                  const d4* __restrict__ dv, double inv_norm,
                                                  const bf16* __restrict__ z3, float* __restrict__ gh,
                                                  bf16* __restrict__ gz, float* __restrict__ go_out,
                                                  double* __restrict__ lossp) {
  __shared__ float Wh[kNetOut * kHid + kNetOut];
  __shared__ double sh[4];
  for (int t = threadIdx.x; t < kNetOut * kHid + kNetOut; t += 256) Wh[t] = master[kOffWh + t];
  __syncthreads();
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int n = in.n;
  double lsum = 0.0;
  if (i < npad) {
    float h[kHid];
#pragma unroll
    for (int c = 0; c < kHid / 8; ++c) {
      const bf16x8 v = *reinterpret_cast<const bf16x8*>(h3 + (size_t)i * kHid + 8 * c);
#pragma unroll
      for (int q = 0; q < 8; ++q) h[8 * c + q] = (float)v[q];
    }
    float o[kNetOut];
#pragma unroll
    for (int k = 0; k < kNetOut; ++k) {
      float acc = Wh[kNetOut * kHid + k];
#pragma unroll
      for (int f = 0; f < kHid; ++f) acc += Wh[k * kHid + f] * h[f];
      o[k] = acc;
    }
#pragma unroll
    for (int k = 0; k < kNetOut; ++k) o_out[(size_t)i * 8 + k] = o[k];
    float go[kNetOut] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (i < n) {
      float L[3][3], C[3][3];
      lower_from_o(o, L);
      sym_from_binv(in.binv, n, i, C);
      const bool fixed = in.dflag[i] != 0;
      if (fixed) {
        float I3[3][3] = {{1.f, 0.f, 0.f}, {0.f, 1.f, 0.f}, {0.f, 0.f, 1.f}};
        store_block(Bout, n, i, I3, C);
      } else {
        store_block(Bout, n, i, L, C);
      }
      if (TRAIN && !fixed) {
        float LC[3][3], B[3][3];
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 3; ++c) LC[r][c] = L[r][0] * C[0][c] + L[r][1] * C[1][c] + L[r][2] * C[2][c];
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 3; ++c) B[r][c] = LC[r][0] * L[c][0] + LC[r][1] * L[c][1] + LC[r][2] * L[c][2];
        const d4 bi = bvec[i], di = dv[i];
        const float bb[3] = {(float)bi.x, (float)bi.y, (float)bi.z};
        float r3[3];
        for (int r = 0; r < 3; ++r)
          r3[r] = B[r][0] * bb[0] + B[r][1] * bb[1] + B[r][2] * bb[2] - (float)(r == 0 ? di.x : (r == 1 ? di.y : di.z));
        lsum = (double)r3[0] * r3[0] + (double)r3[1] * r3[1] + (double)r3[2] * r3[2];
        // dloss/dB = 2 r b^T / D; dloss/dL = (G + G^T) L C
        const float s2 = (float)(2.0 * inv_norm);
        float S[3][3], SL[3][3], GL[3][3];
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 3; ++c) S[r][c] = s2 * (r3[r] * bb[c] + r3[c] * bb[r]);
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 3; ++c) SL[r][c] = S[r][0] * L[0][c] + S[r][1] * L[1][c] + S[r][2] * L[2][c];
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 3; ++c) GL[r][c] = SL[r][0] * C[0][c] + SL[r][1] * C[1][c] + SL[r][2] * C[2][c];
        go[0] = GL[0][0] * L[0][0];
        go[1] = GL[1][1] * L[1][1];
        go[2] = GL[2][2] * L[2][2];
        go[3] = GL[1][0];
        go[4] = GL[2][0];
        go[5] = GL[2][1];
      }
    }
    if (TRAIN) {
#pragma unroll
      for (int k = 0; k < kNetOut; ++k) go_out[(size_t)i * 8 + k] = go[k];
#pragma unroll
      for (int f = 0; f < kHid; ++f) {
        float g = 0.f;
#pragma unroll
        for (int k = 0; k < kNetOut; ++k) g += Wh[k * kHid + f] * go[k];
        gh[(size_t)i * kHid + f] = g;
        gz[(size_t)i * kHid + f] = (bf16)((float)z3[(size_t)i * kHid + f] > 0.f ? g : 0.f);
      }
    }
  }
  if (TRAIN) {
    lsum = wsum(lsum);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = lsum;
    __syncthreads();
    if (threadIdx.x == 0) lossp[blockIdx.x] = ((sh[0] + sh[1]) + (sh[2] + sh[3])) * inv_norm;
  }
}

// B from cached head outputs and the current A_ii^-1.
__global__ __launch_bounds__(256) void k_net_apply(NetInputs in, const float* __restrict__ o_in,
                                                   float* __restrict__ Bout) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= in.n) return;
  float o[kNetOut], L[3][3], C[3][3];
  for (int k = 0; k < kNetOut; ++k) o[k] = o_in[(size_t)i * 8 + k];
  lower_from_o(o, L);
  sym_from_binv(in.binv, in.n, i, C);
  if (in.dflag[i]) {
    float I3[3][3] = {{1.f, 0.f, 0.f}, {0.f, 1.f, 0.f}, {0.f, 0.f, 1.f}};
    store_block(Bout, in.n, i, I3, C);
  } else {
    store_block(Bout, in.n, i, L, C);
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

// Sum the partials in workgroup order into the flat gradient (first Kreal columns).
__global__ __launch_bounds__(256) void k_net_dw_reduce(int nwg, int K, int Kreal, const float* __restrict__ part,
                                                       float* __restrict__ grad, int offW, int offb) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  const int nW = kHid * Kreal;
  if (t >= nW + kHid) return;
  int src;
  int dst;
  if (t < nW) {
    const int o = t / Kreal, k = t % Kreal;
    src = o * K + k;
    dst = offW + t;
  } else {
    src = kHid * K + (t - nW);
    dst = offb + (t - nW);
  }
  float s = 0.f;
  for (int w = 0; w < nwg; ++w) s += part[(size_t)w * (kHid * K + kHid) + src];
  grad[dst] = s;
}

// dWh[k][f] = sum go[k] h3[f], dbh[k] = sum go[k]: per workgroup a node range,
// one output per thread; partials [workgroup][390].
__global__ __launch_bounds__(512) void k_net_dhead(int npad, const float* __restrict__ go, const bf16* __restrict__ h3,
                                                   float* __restrict__ part) {
  constexpr int NO = kNetOut * kHid + kNetOut;
  const int t = threadIdx.x;
  const int G = gridDim.x;
  const int per = (npad + G - 1) / G;
  const int c0 = min(npad, blockIdx.x * per), c1 = min(npad, c0 + per);
  if (t >= NO) return;
  const int k = t < kNetOut * kHid ? t / kHid : t - kNetOut * kHid;
  const int f = t < kNetOut * kHid ? t % kHid : -1;
  float s = 0.f;
  for (int i = c0; i < c1; ++i) s += go[(size_t)i * 8 + k] * (f >= 0 ? (float)h3[(size_t)i * kHid + f] : 1.f);
  part[(size_t)blockIdx.x * NO + t] = s;
}

__global__ __launch_bounds__(512) void k_net_dhead_reduce(int nwg, const float* __restrict__ part,
                                                          float* __restrict__ grad) {
  constexpr int NO = kNetOut * kHid + kNetOut;
  const int t = threadIdx.x;
  if (t >= NO) return;
  float s = 0.f;
  for (int w = 0; w < nwg; ++w) s += part[(size_t)w * NO + t];
  grad[kOffWh + t] = s;
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

__global__ __launch_bounds__(256) void k_net_dvnorm(int n, const d4* __restrict__ dv, const uint8_t* __restrict__ dflag,
                                                    double* __restrict__ part) {
  __shared__ double sh[4];
  const int i = blockIdx.x * 256 + threadIdx.x;
  double s = 0.0;
  if (i < n && !dflag[i]) {
    const d4 d = dv[i];
    s = d.x * d.x + d.y * d.y + d.z * d.z;
  }
  s = wsum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

inline int nb256(int n) { return (n + 255) / 256; }

}  // namespace

void net_forward(hipStream_t s, const NetParamsDev& P, NetWork& w, const NetInputs& in) {
  const int np = w.npad;
  k_net_inputs<<<nb256(np), 256, 0, s>>>(in, np, w.a, w.inv_wdeg);
  k_net_gemm<kNetInPad, 0, kHid, 0><<<np / kNetRows, 256, 0, s>>>(w.a, nullptr, P.W0, P.master + kOffB0, nullptr,
                                                                  w.z[0], w.h[0], nullptr);
  for (int l = 0; l < kNetLayers; ++l) {
    k_net_mean<<<np / 4, 256, 0, s>>>(in, np, w.inv_wdeg, w.h[l], w.m[l]);
    k_net_gemm<kHid, kHid, kHid, 1><<<np / kNetRows, 256, 0, s>>>(
        w.h[l], w.m[l], P.Wl[l], P.master + kOffL0 + l * kLayerSize + kHid * 2 * kHid, w.h[l], w.z[l + 1],
        w.h[l + 1], nullptr);
  }
  k_net_head<false><<<nb256(np), 256, 0, s>>>(in, np, P.master, w.h[kNetLayers], w.o, w.B, nullptr, nullptr, 0.0,
                                              nullptr, nullptr, nullptr, nullptr, nullptr);
}

void net_apply_cached(hipStream_t s, const NetParamsDev&, NetWork& w, const NetInputs& in) {
  k_net_apply<<<nb256(in.n), 256, 0, s>>>(in, w.o, w.B);
}

int net_backward(hipStream_t s, const NetParamsDev& P, NetWork& w, const NetInputs& in, const d4* b, const d4* dv,
                 double inv_norm) {
  const int np = w.npad;
  const int nh = nb256(np);
  k_net_head<true><<<nh, 256, 0, s>>>(in, np, P.master, w.h[kNetLayers], w.o, w.B, b, dv, inv_norm, w.z[kNetLayers],
                                      w.gh, w.gz, w.go, w.lossp);
  k_net_dhead<<<kDwWorkgroups, 512, 0, s>>>(np, w.go, w.h[kNetLayers], w.part);
  k_net_dhead_reduce<<<1, 512, 0, s>>>(kDwWorkgroups, w.part, w.grad);
  for (int l = kNetLayers - 1; l >= 0; --l) {
    // gz holds dloss/dz_{l+1}
    k_net_dw<kHid, kHid><<<kDwWorkgroups, 256, 0, s>>>(np, w.gz, w.h[l], w.m[l], w.part);
    k_net_dw_reduce<<<nb256(kHid * 2 * kHid + kHid), 256, 0, s>>>(kDwWorkgroups, 2 * kHid, 2 * kHid, w.part, w.grad,
                                                                  kOffL0 + l * kLayerSize,
                                                                  kOffL0 + l * kLayerSize + kHid * 2 * kHid);
    k_net_gemm<kHid, 0, 2 * kHid, 2><<<np / kNetRows, 256, 0, s>>>(w.gz, nullptr, P.WlT[l], nullptr, nullptr,
                                                                   nullptr, nullptr, w.gi);
    k_net_mean_bwd<<<np / 4, 256, 0, s>>>(in, np, w.inv_wdeg, w.gi, w.gh, w.z[l], w.gz);
  }
  k_net_dw<kNetInPad, 0><<<kDwWorkgroups, 256, 0, s>>>(np, w.gz, w.a, nullptr, w.part);
  k_net_dw_reduce<<<nb256(kHid * kNetIn + kHid), 256, 0, s>>>(kDwWorkgroups, kNetInPad, kNetIn, w.part, w.grad,
                                                              kOffW0, kOffB0);
  return nh;
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

int net_dv_norm(hipStream_t s, int n, const d4* dv, const uint8_t* dflag, double* part) {
  k_net_dvnorm<<<nb256(n), 256, 0, s>>>(n, dv, dflag, part);
  return nb256(n);
}

}  // namespace gfem
