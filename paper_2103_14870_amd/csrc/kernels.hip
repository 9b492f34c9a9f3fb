// Device kernels of the graph-based FEM step for gfx950 (CDNA4, wave64).
// See kernels.hpp for the data layout.  Citations are to Mandal, Chaudhuri &
// Chaudhuri, "Remeshing-Free Graph-Based Finite Element Method for Ductile
// and Brittle Fracture".
#include "kernels.hpp"

#include <hip/hip_ext.h>

#include <cmath>

namespace gfem {

namespace {

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Deterministic sum over the 256 threads of a workgroup (fixed tree).
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// Per-workgroup event counts: one ballot per wave, one atomic per counter per
// workgroup, into slot (workgroup % kCtrSlots).  Every thread of an
// NT-thread workgroup must call it.
template <int NC, int NT = kThreads>
__device__ __forceinline__ void block_counts(Counters* ctr, int first_field, const bool (&pred)[NC]) {
  __shared__ int sc[NT / 64][NC];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const unsigned long long b = __ballot(pred[c]);
    if (l == 0) sc[w][c] = (int)__popcll(b);
  }
  __syncthreads();
  if (threadIdx.x < NC) {
    int s = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) s += sc[i][threadIdx.x];
    if (s) atomicAdd(&ctr->v[(blockIdx.x % kCtrSlots) * kCtrStride + first_field + threadIdx.x], s);
  }
}

// Workgroups are dispatched round-robin over the 8 XCDs.  Map them so that
// each XCD owns one contiguous slab of rows: its L2 then holds the vector
// entries its rows gather.  G must be a multiple of 8.
__device__ __forceinline__ int xcd_logical(int b, int G) { return (b & 7) * (G >> 3) + (b >> 3); }

// a + beta b per component (fused multiply-add).
template <typename T>
__device__ __forceinline__ v4<T> dir_comb(v4<T> z, T beta, v4<T> p) {
  v4<T> r;
  r.x = fmadd(beta, p.x, z.x);
  r.y = fmadd(beta, p.y, z.y);
  r.z = fmadd(beta, p.z, z.z);
  r.w = 0;
  return r;
}

template <typename T>
__device__ __forceinline__ T sym3_det(T a00, T a11, T a22, T a01, T a02, T a12) {
  return a00 * (a11 * a22 - a12 * a12) - a01 * (a01 * a22 - a12 * a02) + a02 * (a01 * a12 - a11 * a02);
}

// Inverse of a symmetric 3x3 from its adjugate, given its determinant.
template <typename T>
__device__ __forceinline__ void sym3_inv(const T* a, T det, T* o) {
  // a: 00,11,22,01,02,12
  T id = T(1) / det;
  o[0] = (a[1] * a[2] - a[5] * a[5]) * id;
  o[1] = (a[0] * a[2] - a[4] * a[4]) * id;
  o[2] = (a[0] * a[1] - a[3] * a[3]) * id;
  o[3] = (a[4] * a[5] - a[3] * a[2]) * id;
  o[4] = (a[3] * a[5] - a[4] * a[1]) * id;
  o[5] = (a[3] * a[4] - a[0] * a[5]) * id;
}

template <typename T>
__device__ __forceinline__ void sym_full(const T* s, T (*f)[3]) {
  f[0][0] = s[0];
  f[1][1] = s[1];
  f[2][2] = s[2];
  f[0][1] = f[1][0] = s[3];
  f[0][2] = f[2][0] = s[4];
  f[1][2] = f[2][1] = s[5];
}

// 4x4 Gram matrix of the reference barycentric gradients n_a under a
// symmetric 3x3 bilinear form B (n_0 = -(e1+e2+e3), n_i = e_i):
// Gam[a][b] = n_a^T B n_b.  With E_k = dG/ds_k = -(n_a n_b^T + n_b n_a^T)/2
// for local edge k = (a,b), tr(E_k B) = -Gam[a][b].
template <typename T>
__device__ __forceinline__ void gram4(const T* s, T (*g)[4]) {
  T B[3][3];
  sym_full(s, B);
  T rs[3];
  for (int i = 0; i < 3; ++i) rs[i] = B[i][0] + B[i][1] + B[i][2];
  g[0][0] = rs[0] + rs[1] + rs[2];
  for (int i = 0; i < 3; ++i) {
    g[0][i + 1] = g[i + 1][0] = -rs[i];
    for (int j = 0; j < 3; ++j) g[i + 1][j + 1] = B[i][j];
  }
}

// Local edge k joins local nodes EA(k) -> EB(k) (the 12,13,14,23,24,34 order of Eq. 15).
__device__ __forceinline__ constexpr int EA(int k) { return k < 3 ? 0 : (k < 5 ? 1 : 2); }
__device__ __forceinline__ constexpr int EB(int k) { return k < 3 ? k + 1 : (k == 3 ? 2 : 3); }

// ---------------------------------------------------------------- damage

// Counters (new, total broken, near threshold) and the near-threshold edge
// list, shared by the local and the non-local damage passes; every thread of
// the workgroup calls it.  One atomic per wave reserves the wave's entries.
__device__ __forceinline__ void damage_tail(bool act, bool hit, bool was, bool near, int e, Counters* ctr,
                                            int32_t* __restrict__ near_ids) {
  const bool pr[3] = {act && hit && !was, act && (hit || was), act && near};
  block_counts<3>(ctr, kNewBroken, pr);
  const unsigned long long bal = __ballot(act && near);
  if (bal) {
    const int l = threadIdx.x & 63;
    int base = 0;
    if (l == 0) base = atomicAdd(&ctr->near_n, (int)__popcll(bal));
    base = __shfl(base, 0, 64);
    if (act && near) near_ids[base + (int)__popcll(bal & ((1ull << l) - 1ull))] = e;
  }
}

// Per edge: Green normal strain along the rest edge, (s - S) / (2 S) with
// s - S = 2 dX.dU + dU.dU from the displacement (no cancellation of the
// absolute positions); zeta <- zeta OR (strain >= threshold) (Eq. 21; labels
// are irreversible, Sec. 3.3).
__global__ __launch_bounds__(kThreads) void k_damage(int ne, const int2* __restrict__ edges,
                                                     const d4* __restrict__ X, const d4* __restrict__ U,
                                                     const double* __restrict__ S,
                                                     const uint8_t* __restrict__ z_in,
                                                     uint8_t* __restrict__ z_out, double thr,
                                                     Counters* ctr, int32_t* __restrict__ near_ids) {
  int e = blockIdx.x * kThreads + threadIdx.x;
  bool act = e < ne;
  bool hit = false, was = false, near = false;
  if (act) {
    int2 ij = edges[e];
    d4 xi = X[ij.x], xj = X[ij.y], ui = U[ij.x], uj = U[ij.y];
    double dx = xj.x - xi.x, dy = xj.y - xi.y, dz = xj.z - xi.z;
    double ux = uj.x - ui.x, uy = uj.y - ui.y, uz = uj.z - ui.z;
    double ds = 2.0 * (dx * ux + dy * uy + dz * uz) + (ux * ux + uy * uy + uz * uz);
    double eps = ds / (2.0 * S[e]);
    was = z_in[e] != 0;
    hit = eps >= thr;
    near = fabs(eps - thr) < 1e-6;
    z_out[e] = (uint8_t)(was || hit);
  }
  damage_tail(act, hit, was, near, e, ctr, near_ids);
}

// ---------------------------------------------------------------- non-local damage (Eq. 20, R_d > 0)

// Per tet: Green strain E = (H + H^T + H^T H)/2 with H = grad u = Du Dm^-1
// (F = I + H), from the displacement in FP64, so that no absolute positions
// cancel.  F does not depend on the tet's vertex order.
__global__ __launch_bounds__(kThreads) void k_nl_strain(int m, const int4* __restrict__ tets,
                                                        const d4* __restrict__ X, const d4* __restrict__ U,
                                                        Sym6* __restrict__ E) {
  const int t = blockIdx.x * kThreads + threadIdx.x;
  if (t >= m) return;
  const int4 v = tets[t];
  const d4 x0 = X[v.x], x1 = X[v.y], x2 = X[v.z], x3 = X[v.w];
  const d4 u0 = U[v.x], u1 = U[v.y], u2 = U[v.z], u3 = U[v.w];
  // columns i = 1..3: rest edge vectors Dm and displacement differences Du
  const double D[3][3] = {{x1.x - x0.x, x2.x - x0.x, x3.x - x0.x},
                          {x1.y - x0.y, x2.y - x0.y, x3.y - x0.y},
                          {x1.z - x0.z, x2.z - x0.z, x3.z - x0.z}};
  const double W[3][3] = {{u1.x - u0.x, u2.x - u0.x, u3.x - u0.x},
                          {u1.y - u0.y, u2.y - u0.y, u3.y - u0.y},
                          {u1.z - u0.z, u2.z - u0.z, u3.z - u0.z}};
  // Dm^-1 = adj(Dm) / det(Dm)
  double A[3][3];
  A[0][0] = D[1][1] * D[2][2] - D[1][2] * D[2][1];
  A[0][1] = D[0][2] * D[2][1] - D[0][1] * D[2][2];
  A[0][2] = D[0][1] * D[1][2] - D[0][2] * D[1][1];
  A[1][0] = D[1][2] * D[2][0] - D[1][0] * D[2][2];
  A[1][1] = D[0][0] * D[2][2] - D[0][2] * D[2][0];
  A[1][2] = D[0][2] * D[1][0] - D[0][0] * D[1][2];
  A[2][0] = D[1][0] * D[2][1] - D[1][1] * D[2][0];
  A[2][1] = D[0][1] * D[2][0] - D[0][0] * D[2][1];
  A[2][2] = D[0][0] * D[1][1] - D[0][1] * D[1][0];
  const double inv_det = 1.0 / (D[0][0] * A[0][0] + D[0][1] * A[1][0] + D[0][2] * A[2][0]);
  double H[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) H[r][c] = (W[r][0] * A[0][c] + W[r][1] * A[1][c] + W[r][2] * A[2][c]) * inv_det;
  auto e = [&](int a, int b) {
    return 0.5 * (H[a][b] + H[b][a] + H[0][a] * H[0][b] + H[1][a] * H[1][b] + H[2][a] * H[2][b]);
  };
  Sym6 o;
  o.v[0] = e(0, 0);
  o.v[1] = e(1, 1);
  o.v[2] = e(2, 2);
  o.v[3] = e(0, 1);
  o.v[4] = e(0, 2);
  o.v[5] = e(1, 2);
  E[t] = o;
}

// Support-weighted average of the strain tensors (Eq. 20, reading R4): one
// group of LN lanes per tet; the lanes take the tet's support entries in turn
// (consecutive entries, so the index and weight loads coalesce), each keeps
// six partial sums, and a butterfly over the group finishes them in a fixed
// order, so the result is reproducible.
template <int LN>
__global__ __launch_bounds__(kThreads) void k_nl_average(int m, const int64_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ idx,
                                                         const double* __restrict__ w,
                                                         const Sym6* __restrict__ E, Sym6* __restrict__ Eavg) {
  const int lane = threadIdx.x & (LN - 1);
  const int t = (int)(((long)blockIdx.x * kThreads + threadIdx.x) / LN);
  const bool act = t < m;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  if (act) {
    const int64_t j1 = ptr[t + 1];
#pragma unroll 4
    for (int64_t j = ptr[t] + lane; j < j1; j += LN) {
      const Sym6 ej = E[idx[j]];
      const double wj = w[j];
#pragma unroll
      for (int c = 0; c < 6; ++c) acc[c] = fmadd(wj, ej.v[c], acc[c]);
    }
  }
#pragma unroll
  for (int o = LN / 2; o > 0; o >>= 1)
#pragma unroll
    for (int c = 0; c < 6; ++c) acc[c] += __shfl_xor(acc[c], o, LN);
  if (act && lane == 0) {
    Sym6 o;
#pragma unroll
    for (int c = 0; c < 6; ++c) o.v[c] = acc[c];
    Eavg[t] = o;
  }
}

// Per edge: averaged normal strain d^T E* d / d^T d (d the rest edge vector)
// in each tet that contains the edge (slots k*m + t); the edge breaks when
// the largest reaches the threshold (Eq. 21).
__global__ __launch_bounds__(kThreads) void k_nl_damage(int ne, int m, const int2* __restrict__ edges,
                                                        const d4* __restrict__ X,
                                                        const int32_t* __restrict__ edge_ptr,
                                                        const int32_t* __restrict__ edge_slot,
                                                        const Sym6* __restrict__ Eavg,
                                                        const uint8_t* __restrict__ z_in,
                                                        uint8_t* __restrict__ z_out, double thr, Counters* ctr,
                                                        int32_t* __restrict__ near_ids) {
  const int e = blockIdx.x * kThreads + threadIdx.x;
  const bool act = e < ne;
  bool hit = false, was = false, near = false;
  if (act) {
    const int2 ij = edges[e];
    const d4 xi = X[ij.x], xj = X[ij.y];
    const double dx = xj.x - xi.x, dy = xj.y - xi.y, dz = xj.z - xi.z;
    const double inv_dd = 1.0 / (dx * dx + dy * dy + dz * dz);
    for (int i = edge_ptr[e]; i < edge_ptr[e + 1]; ++i) {
      const Sym6 a = Eavg[edge_slot[i] % m];
      const double q = a.v[0] * dx * dx + a.v[1] * dy * dy + a.v[2] * dz * dz +
                       2.0 * (a.v[3] * dx * dy + a.v[4] * dx * dz + a.v[5] * dy * dz);
      const double eps = q * inv_dd;
      hit = hit || eps >= thr;
      near = near || fabs(eps - thr) < 1e-6;
    }
    was = z_in[e] != 0;
    z_out[e] = (uint8_t)(was || hit);
  }
  damage_tail(act, hit, was, near, e, ctr, near_ids);
}

// ---------------------------------------------------------------- plasticity

// Cyclic Jacobi eigen-decomposition of a symmetric 3x3 (FP64): on return a
// is diagonal (the eigenvalues) and the columns of v are the eigenvectors.
__device__ __forceinline__ void jacobi_rot(double (&a)[3][3], double (&v)[3][3], int p, int q) {
  const double apq = a[p][q];
  if (apq == 0.0) return;
  const double th = (a[q][q] - a[p][p]) / (2.0 * apq);
  const double tn = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
  const double c = 1.0 / sqrt(tn * tn + 1.0), s = tn * c;
#pragma unroll
  for (int k = 0; k < 3; ++k) {  // columns p, q
    const double akp = a[k][p], akq = a[k][q];
    a[k][p] = c * akp - s * akq;
    a[k][q] = s * akp + c * akq;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {  // rows p, q
    const double apk = a[p][k], aqk = a[q][k];
    a[p][k] = c * apk - s * aqk;
    a[q][k] = s * apk + c * aqk;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double vkp = v[k][p], vkq = v[k][q];
    v[k][p] = c * vkp - s * vkq;
    v[k][q] = s * vkp + c * vkq;
  }
}

__device__ __forceinline__ void sym_eig3(double (&a)[3][3], double (&v)[3][3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) v[i][j] = i == j ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 12; ++sweep) {
    const double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
    const double dg = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
    if (!(off > 1e-32 * dg)) break;
    jacobi_rot(a, v, 0, 1);
    jacobi_rot(a, v, 0, 2);
    jacobi_rot(a, v, 1, 2);
  }
}

// One thread per tet (ductile workload).  The plastic state is the plastic
// rest shape on the Gram matrix of the tet's edges from node 0,
// Gp = G0 + P (P = 0 before any flow), with det Gp = det G0 (volume-
// preserving flow).  The elastic stretches are the generalised eigenvalues of
// G v = lam Gp v; their Hencky strains h = log(lam)/2 have deviator
// d = h - mean(h).  When |d| exceeds the yield strain, d is scaled back onto
// the yield surface and Gp is replaced by L W diag(lam/lam') W^T L^T
// (Gp = L L^T, L^-1 G L^-T = W diag(lam) W^T): the same eigenvectors, the
// returned elastic stretches lam', the same determinant.  A flat or inverted
// tet (det F < 0.05) keeps its plastic state.  FP64 throughout.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_plastic(int m, const int4* __restrict__ tets,
                                                      const d4* __restrict__ X, const d4* __restrict__ U,
                                                      const T* __restrict__ pl_in, T* __restrict__ pl_out,
                                                      double ey) {
  const int t = blockIdx.x * kThreads + threadIdx.x;
  if (t >= m) return;
  const int4 nd = tets[t];
  const int ids[4] = {nd.x, nd.y, nd.z, nd.w};
  const d4 X0 = X[nd.x], U0 = U[nd.x];
  double Dm[3][3], Ds[3][3];  // [edge from node 0][component]
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const d4 Xk = X[ids[k + 1]], Uk = U[ids[k + 1]];
    Dm[k][0] = Xk.x - X0.x;
    Dm[k][1] = Xk.y - X0.y;
    Dm[k][2] = Xk.z - X0.z;
    Ds[k][0] = Dm[k][0] + (Uk.x - U0.x);
    Ds[k][1] = Dm[k][1] + (Uk.y - U0.y);
    Ds[k][2] = Dm[k][2] + (Uk.z - U0.z);
  }
  double P[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) P[c] = (double)pl_in[(size_t)c * m + t];
  auto det3 = [](const double (&a)[3][3]) {
    return a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) - a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
           a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
  };
  const double J = det3(Ds) / det3(Dm);
  bool flow = J >= 0.05;
  double Pn[6] = {P[0], P[1], P[2], P[3], P[4], P[5]};
  if (flow) {
    constexpr int R[6] = {0, 1, 2, 0, 0, 1}, C[6] = {0, 1, 2, 1, 2, 2};
    double G0[6], G[6], Gp[3][3];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const int i = R[c], j = C[c];
      G0[c] = Dm[i][0] * Dm[j][0] + Dm[i][1] * Dm[j][1] + Dm[i][2] * Dm[j][2];
      G[c] = Ds[i][0] * Ds[j][0] + Ds[i][1] * Ds[j][1] + Ds[i][2] * Ds[j][2];
    }
    double Gf[3][3];
    Gf[0][0] = G[0]; Gf[1][1] = G[1]; Gf[2][2] = G[2];
    Gf[0][1] = Gf[1][0] = G[3]; Gf[0][2] = Gf[2][0] = G[4]; Gf[1][2] = Gf[2][1] = G[5];
    Gp[0][0] = G0[0] + P[0]; Gp[1][1] = G0[1] + P[1]; Gp[2][2] = G0[2] + P[2];
    Gp[0][1] = Gp[1][0] = G0[3] + P[3]; Gp[0][2] = Gp[2][0] = G0[4] + P[4]; Gp[1][2] = Gp[2][1] = G0[5] + P[5];
    // Cholesky Gp = L L^T
    double L[3][3] = {};
    L[0][0] = sqrt(Gp[0][0]);
    L[1][0] = Gp[1][0] / L[0][0];
    L[2][0] = Gp[2][0] / L[0][0];
    L[1][1] = sqrt(Gp[1][1] - L[1][0] * L[1][0]);
    L[2][1] = (Gp[2][1] - L[2][0] * L[1][0]) / L[1][1];
    L[2][2] = sqrt(Gp[2][2] - L[2][0] * L[2][0] - L[2][1] * L[2][1]);
    // Li = L^-1 (lower triangular)
    double Li[3][3] = {};
    Li[0][0] = 1.0 / L[0][0];
    Li[1][1] = 1.0 / L[1][1];
    Li[2][2] = 1.0 / L[2][2];
    Li[1][0] = -L[1][0] * Li[0][0] * Li[1][1];
    Li[2][1] = -L[2][1] * Li[1][1] * Li[2][2];
    Li[2][0] = -(L[2][0] * Li[0][0] + L[2][1] * Li[1][0]) * Li[2][2];
    // S = Li G Li^T
    double T1[3][3], S[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) T1[i][j] = Li[i][0] * Gf[0][j] + Li[i][1] * Gf[1][j] + Li[i][2] * Gf[2][j];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) S[i][j] = T1[i][0] * Li[j][0] + T1[i][1] * Li[j][1] + T1[i][2] * Li[j][2];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i + 1; j < 3; ++j) S[i][j] = S[j][i] = 0.5 * (S[i][j] + S[j][i]);
    double W[3][3];
    sym_eig3(S, W);
    const double lam[3] = {S[0][0], S[1][1], S[2][2]};
    flow = lam[0] > 0.0 && lam[1] > 0.0 && lam[2] > 0.0;
    if (flow) {
      double h[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) h[i] = 0.5 * log(lam[i]);
      const double hm = (h[0] + h[1] + h[2]) / 3.0;
      const double d0 = h[0] - hm, d1 = h[1] - hm, d2 = h[2] - hm;
      const double ndv = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
      flow = ndv > ey;
      if (flow) {
        const double sc = ey / ndv;
        const double hn[3] = {hm + d0 * sc, hm + d1 * sc, hm + d2 * sc};
        double r[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) r[i] = lam[i] / exp(2.0 * hn[i]);
        double LW[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) LW[i][j] = L[i][0] * W[0][j] + L[i][1] * W[1][j] + L[i][2] * W[2][j];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          const int i = R[c], j = C[c];
          Pn[c] = (LW[i][0] * r[0] * LW[j][0] + LW[i][1] * r[1] * LW[j][1] + LW[i][2] * r[2] * LW[j][2]) - G0[c];
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) pl_out[(size_t)c * m + t] = (T)Pn[c];
}

// ---------------------------------------------------------------- element

__constant__ unsigned long long c_disc_lut;  // bit mask set: broken-edge mask disconnects the tet

// Below this |J| the volume term of the energy is evaluated from the
// adjugate of the Gram matrix and the cofactors of the edge matrix in FP64:
// its edge-length form divides by J (one over the volume of a flat tet).
constexpr double kJMin = 0.05;

// One thread per tet.  Kinematics (edge vectors, squared-length changes) in
// FP64, the rest in T.  Writes, per local edge k, the 3x3 stiffness block
// K(i,j) in global orientation (i < j) and the FP64 force weight
// w_k = 2 V chi dPsi/ds_k (Eq. 12).  pl: the plastic rest shapes
// Gp - G0 [6][m] (null: no plasticity).  EN: kEnergyStableNeoHookean
// (Eq. 35) or kEnergyStVK (Eq. 37: with A = Gp^-1, dPsi/ds_k =
// lam/4 (I_C - 3) c_k + mu/2 tr(E_k A dGe A), edge Hessian
// lam/4 c c^T + mu/2 tr(E_k A E_l A), PSD without clamping; no J enters).
template <typename T, int EN>
__global__ __launch_bounds__(kElemTets) void k_element(int m, const int4* __restrict__ tets,
                                                      const int32_t* __restrict__ tet_edge,
                                                      const uint8_t* __restrict__ flip,
                                                      const d4* __restrict__ X, const d4* __restrict__ U,
                                                      const uint8_t* __restrict__ zeta, const T* __restrict__ pl,
                                                      const T* __restrict__ chi_in, T* __restrict__ chi_out,
                                                      ElemConst cst, const int32_t* __restrict__ part_base,
                                                      const int32_t* __restrict__ part_cptr,
                                                      const uint16_t* __restrict__ part_slot,
                                                      Rec<T>* __restrict__ contrib, Counters* ctr) {
  __shared__ Rec<T> lrec[kElemTets * 6];
  const int t0 = blockIdx.x * kElemTets + threadIdx.x;
  const bool act = t0 < m;
  const int t = act ? t0 : m - 1;
  const T mu = (T)cst.mu, lam = (T)cst.lam, am1 = (T)cst.alpha_m1;

  int4 nd = tets[t];
  d4 Xa[4] = {X[nd.x], X[nd.y], X[nd.z], X[nd.w]};
  d4 Ua[4] = {U[nd.x], U[nd.y], U[nd.z], U[nd.w]};

  // Rest and current edge vectors; squared lengths S_k and their change ds_k
  // (Theorem 3.1: the energy is a function of these six lengths).
  T Dr[6][3], dcur[6][3], S[6], ds[6];
  double Dsd[3][3], Dmd[3][3];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int a = EA(k), b = EB(k);
    const double* xa = &Xa[a].x;
    const double* xb = &Xa[b].x;
    const double* ua = &Ua[a].x;
    const double* ub = &Ua[b].x;
    double D[3], dU[3];
    for (int d = 0; d < 3; ++d) {
      D[d] = xb[d] - xa[d];
      dU[d] = ub[d] - ua[d];
    }
    double s0 = D[0] * D[0] + D[1] * D[1] + D[2] * D[2];
    double dsk = 2.0 * (D[0] * dU[0] + D[1] * dU[1] + D[2] * dU[2]) + (dU[0] * dU[0] + dU[1] * dU[1] + dU[2] * dU[2]);
    S[k] = (T)s0;
    ds[k] = (T)dsk;
    for (int d = 0; d < 3; ++d) {
      Dr[k][d] = (T)D[d];
      dcur[k][d] = (T)(D[d] + dU[d]);
    }
    if (k < 3)
      for (int d = 0; d < 3; ++d) {
        Dsd[k][d] = D[d] + dU[d];
        Dmd[k][d] = D[d];
      }
  }
  // Rest Gram matrix G0 = Dm^T Dm (symmetric: 00,11,22,01,02,12) and its inverse.
  T G0[6];
  G0[0] = S[0];
  G0[1] = S[1];
  G0[2] = S[2];
  G0[3] = Dr[0][0] * Dr[1][0] + Dr[0][1] * Dr[1][1] + Dr[0][2] * Dr[1][2];
  G0[4] = Dr[0][0] * Dr[2][0] + Dr[0][1] * Dr[2][1] + Dr[0][2] * Dr[2][2];
  G0[5] = Dr[1][0] * Dr[2][0] + Dr[1][1] * Dr[2][1] + Dr[1][2] * Dr[2][2];
  const T det0 = sym3_det(G0[0], G0[1], G0[2], G0[3], G0[4], G0[5]);
  T G0i[6];
  sym3_inv(G0, det0, G0i);
  // signed volumes in FP64: J = det Ds / det Dm decides the small-J form on
  // both sides of any comparison in the same precision
  auto det3 = [](const double (&a)[3][3]) {
    return a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) - a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
           a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
  };
  const double detDmd = det3(Dmd), detDs = det3(Dsd);
  const double Jd = detDs / detDmd;
  const bool small = fabs(Jd) < kJMin;  // counted for either energy
  const bool cof = EN == kEnergyStableNeoHookean && small;  // volume term in cofactor form
  const T vol = (T)(detDmd / 6.0);

  // Gram change from the squared-length changes by polarisation:
  // dG_ii = ds_0i, dG_ij = (ds_0i + ds_0j - ds_ij) / 2.
  T dG[6];
  dG[0] = ds[0];
  dG[1] = ds[1];
  dG[2] = ds[2];
  dG[3] = T(0.5) * (ds[0] + ds[1] - ds[3]);
  dG[4] = T(0.5) * (ds[0] + ds[2] - ds[4]);
  dG[5] = T(0.5) * (ds[1] + ds[2] - ds[5]);

  // Plastic rest shape Gp = G0 + P: the I_C term is measured from it,
  // the volume term from G0 (volume-preserving flow).
  T Gpi[6], dGe[6];
  if (pl) {
    T Gp[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const T P = pl[(size_t)c * m + t];
      Gp[c] = G0[c] + P;
      dGe[c] = dG[c] - P;
    }
    sym3_inv(Gp, sym3_det(Gp[0], Gp[1], Gp[2], Gp[3], Gp[4], Gp[5]), Gpi);
  } else {
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      Gpi[c] = G0i[c];
      dGe[c] = dG[c];
    }
  }

  // a = I_C - 3 = tr(dGe Gp^-1) without cancellation at the stress-free state
  T Ap[3][3], Be[3][3];
  sym_full(Gpi, Ap);
  sym_full(dGe, Be);
  T aI = 0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) aI += Ap[i][j] * Be[j][i];
  const T IC1 = T(4) + aI;  // I_C + 1
  const T cmu = mu * aI / (T(8) * IC1);

  T GamP[4][4];
  gram4(Gpi, GamP);
  T cc[6], vv[6], g[6];
  double wJ[6];  // FP64 volume-term force weights of a small-J tet
  T J, delta, Jsq;
  T Gam[4][4], GamY[4][4];
  T Ys[6];
  double gJd[4][3];  // dJ/dx_a (small-J tets)
  double adjG[6];    // adjugate of the current Gram matrix, FP64 (small-J tets)
  T Wst[6];          // StVK: A dGe A, A = Gp^-1 (symmetric)
  if constexpr (EN == kEnergyStVK) {
    T Wf[3][3], M1[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) M1[i][j] = Be[i][0] * Ap[0][j] + Be[i][1] * Ap[1][j] + Be[i][2] * Ap[2][j];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Wf[i][j] = Ap[i][0] * M1[0][j] + Ap[i][1] * M1[1][j] + Ap[i][2] * M1[2][j];
    Wst[0] = Wf[0][0];
    Wst[1] = Wf[1][1];
    Wst[2] = Wf[2][2];
    Wst[3] = T(0.5) * (Wf[0][1] + Wf[1][0]);
    Wst[4] = T(0.5) * (Wf[0][2] + Wf[2][0]);
    Wst[5] = T(0.5) * (Wf[1][2] + Wf[2][1]);
    T GamW[4][4];
    gram4(Wst, GamW);
    J = (T)Jd;
    delta = J - T(1);
    Jsq = J * J;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int a = EA(k), b = EB(k);
      cc[k] = -GamP[a][b];
      vv[k] = T(0);
      g[k] = T(0.25) * lam * aI * cc[k] - T(0.5) * mu * GamW[a][b];
      wJ[k] = 0.0;
    }
  } else if (!small) {
    // J^2 - 1 = det(I + G0^-1 dG) - 1 without cancellation at rest
    T A0[3][3], B[3][3], Xm[3][3];
    sym_full(G0i, A0);
    sym_full(dG, B);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Xm[i][j] = A0[i][0] * B[0][j] + A0[i][1] * B[1][j] + A0[i][2] * B[2][j];
    const T a0 = Xm[0][0] + Xm[1][1] + Xm[2][2];
    T trX2 = 0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) trX2 += Xm[i][j] * Xm[j][i];
    const T detX = Xm[0][0] * (Xm[1][1] * Xm[2][2] - Xm[1][2] * Xm[2][1]) -
                   Xm[0][1] * (Xm[1][0] * Xm[2][2] - Xm[1][2] * Xm[2][0]) +
                   Xm[0][2] * (Xm[1][0] * Xm[2][1] - Xm[1][1] * Xm[2][0]);
    const T jm1 = a0 + T(0.5) * (a0 * a0 - trX2) + detX;
    Jsq = T(1) + jm1;
    if (detDs >= 0.0) {
      J = sqrt(Jsq);
      delta = jm1 / (J + T(1));
    } else {
      J = -sqrt(Jsq);
      delta = J - T(1);
    }
    T G[6], Gi[6];
    for (int c = 0; c < 6; ++c) G[c] = G0[c] + dG[c];
    sym3_inv(G, det0 * Jsq, Gi);
    // Y = Gp^-1 - G^-1 = G^-1 dGe Gp^-1 (formed as a product, never as the difference)
    {
      T Gf[3][3], M1[3][3], Y[3][3];
      sym_full(Gi, Gf);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) M1[i][j] = Be[i][0] * Ap[0][j] + Be[i][1] * Ap[1][j] + Be[i][2] * Ap[2][j];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Y[i][j] = Gf[i][0] * M1[0][j] + Gf[i][1] * M1[1][j] + Gf[i][2] * M1[2][j];
      Ys[0] = Y[0][0];
      Ys[1] = Y[1][1];
      Ys[2] = Y[2][2];
      Ys[3] = T(0.5) * (Y[0][1] + Y[1][0]);
      Ys[4] = T(0.5) * (Y[0][2] + Y[2][0]);
      Ys[5] = T(0.5) * (Y[1][2] + Y[2][1]);
    }
    gram4(Gi, Gam);
    gram4(Ys, GamY);
    // Edge-space gradient of Eq. 35 (squared (J - alpha) term, reparametrised
    // Lame constants), rewritten so that the rest-state cancellation happens
    // analytically:  dPsi/ds_k = 3mu/8 t_k + mu a/(8(4+a)) c_k + lam/2 (d(2-alpha)+d^2) v_k
    // with c_k = tr(E_k Gp^-1), v_k = tr(E_k G^-1), t_k = tr(E_k Y) = c_k - v_k.
    const T dj = delta * (T(1) - am1) + delta * delta;  // (J - alpha) J - (1 - alpha)
    const T lamt = T(0.5) * lam * dj;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int a = EA(k), b = EB(k);
      cc[k] = -GamP[a][b];
      vv[k] = -Gam[a][b];
      const T tk = -GamY[a][b];
      g[k] = T(0.375) * mu * tk + cmu * cc[k] + lamt * vv[k];
      wJ[k] = 0.0;
    }
  } else {
    // Small |J|: the I_C term in edge form, the volume term (lam/2)(J - alpha)^2
    // through dJ/ds_k = J tr(E_k G^-1) / 2 = tr(E_k adj G) / (2 J det G0)
    // (force weights, FP64) and dJ/dx (cofactors of the edge matrix, FP64).
    J = (T)Jd;
    delta = J - T(1);
    Jsq = J * J;
    double Gd[6];
    {
      constexpr int R[6] = {0, 1, 2, 0, 0, 1}, C[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
      for (int c = 0; c < 6; ++c)
        Gd[c] = Dsd[R[c]][0] * Dsd[C[c]][0] + Dsd[R[c]][1] * Dsd[C[c]][1] + Dsd[R[c]][2] * Dsd[C[c]][2];
    }
    adjG[0] = Gd[1] * Gd[2] - Gd[5] * Gd[5];
    adjG[1] = Gd[0] * Gd[2] - Gd[4] * Gd[4];
    adjG[2] = Gd[0] * Gd[1] - Gd[3] * Gd[3];
    adjG[3] = Gd[4] * Gd[5] - Gd[3] * Gd[2];
    adjG[4] = Gd[3] * Gd[5] - Gd[4] * Gd[1];
    adjG[5] = Gd[3] * Gd[4] - Gd[0] * Gd[5];
    double GamA[4][4];
    gram4(adjG, GamA);
    // J det G0 = det Ds det Dm; below 1e-12 of det Dm^2 the weights are
    // formed at that floor (their reconstruction of the force loses
    // accuracy as 1e-16 / |J| in FP64)
    const double floor = 1e-12 * detDmd * detDmd;
    const double den = (fabs(detDs * detDmd) > floor) ? detDs * detDmd : (detDs >= 0.0 ? floor : -floor);
    const double cJ = 0.5 * cst.lam * (Jd - (1.0 + cst.alpha_m1));
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int a = EA(k), b = EB(k);
      cc[k] = -GamP[a][b];
      vv[k] = 0;
      g[k] = (T(0.375) * mu + cmu) * cc[k];  // (mu/2)(1 - 1/(I_C+1)) c_k
      wJ[k] = cJ * (-GamA[a][b] / den);
    }
    // dJ/dx_a: (x2'-x0') x (x3'-x0') / det Dm etc., node 0 minus their sum
    const double idm = 1.0 / detDmd;
    gJd[1][0] = (Dsd[1][1] * Dsd[2][2] - Dsd[1][2] * Dsd[2][1]) * idm;
    gJd[1][1] = (Dsd[1][2] * Dsd[2][0] - Dsd[1][0] * Dsd[2][2]) * idm;
    gJd[1][2] = (Dsd[1][0] * Dsd[2][1] - Dsd[1][1] * Dsd[2][0]) * idm;
    gJd[2][0] = (Dsd[2][1] * Dsd[0][2] - Dsd[2][2] * Dsd[0][1]) * idm;
    gJd[2][1] = (Dsd[2][2] * Dsd[0][0] - Dsd[2][0] * Dsd[0][2]) * idm;
    gJd[2][2] = (Dsd[2][0] * Dsd[0][1] - Dsd[2][1] * Dsd[0][0]) * idm;
    gJd[3][0] = (Dsd[0][1] * Dsd[1][2] - Dsd[0][2] * Dsd[1][1]) * idm;
    gJd[3][1] = (Dsd[0][2] * Dsd[1][0] - Dsd[0][0] * Dsd[1][2]) * idm;
    gJd[3][2] = (Dsd[0][0] * Dsd[1][1] - Dsd[0][1] * Dsd[1][0]) * idm;
#pragma unroll
    for (int d = 0; d < 3; ++d) gJd[0][d] = -(gJd[1][d] + gJd[2][d] + gJd[3][d]);
  }

  // Energy fraction chi (Eq. 22-25): 2nd Piola-Kirchhoff stress projected on
  // the rest unit edge directions, sigma' = (1 - zeta) sigma; 0 when the
  // unbroken edges leave the tet in pieces.
  int mask = 0;
#pragma unroll
  for (int k = 0; k < 6; ++k) mask |= (zeta[tet_edge[(size_t)k * m + t]] != 0) << k;
  T chi = T(1);
  if (chi_in) {
    chi = chi_in[t];  // held fixed from an earlier pass (quasi-static Newton iterates)
  } else if (mask) {
    if ((c_disc_lut >> mask) & 1ull) {
      chi = T(0);
    } else {
      // sigma_k = mu (1 - 1/(I_C+1)) p_k + lam (J - alpha) J w_k with
      // p_k = q^T Cp^-1 q = e^T G0 Gp^-1 G0 e / S_k and w_k = q^T C^-1 q
      // (e: reference edge, q: rest unit direction); p_k - w_k =
      // e^T G0 Y G0 e / S_k.  Small |J|: every sigma_k times |J|, with
      // |J| J w_k = sign(J) e^T G0 adj(G) G0 e / (det G0 S_k).
      T G0f[3][3];
      sym_full(G0, G0f);
      auto quad = [&](const T* Ms, T (&Z)[3][3]) {  // Z = G0 M G0
        T Mf[3][3], GM[3][3];
        sym_full(Ms, Mf);
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) GM[i][j] = G0f[i][0] * Mf[0][j] + G0f[i][1] * Mf[1][j] + G0f[i][2] * Mf[2][j];
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) Z[i][j] = GM[i][0] * G0f[0][j] + GM[i][1] * G0f[1][j] + GM[i][2] * G0f[2][j];
      };
      auto edge_quad = [](const T (&Z)[3][3], int k) {  // e_k^T Z e_k
        const int a = EA(k), b = EB(k);
        if (a == 0) return Z[b - 1][b - 1];
        return Z[a - 1][a - 1] + Z[b - 1][b - 1] - (Z[a - 1][b - 1] + Z[b - 1][a - 1]);
      };
      T Zp[3][3];
      const bool plastic = pl != nullptr;
      if (plastic) quad(Gpi, Zp);
      T Zs[3][3];
      T sgnJ = T(1), scl = T(1);
      if constexpr (EN == kEnergyStVK) {
        quad(Wst, Zs);  // G0 A dGe A G0
      } else if (!small) {
        quad(Ys, Zs);
      } else {
        T adjT[6];
        for (int c = 0; c < 6; ++c) adjT[c] = (T)adjG[c];
        quad(adjT, Zs);
        sgnJ = Jd >= 0.0 ? T(1) : T(-1);
        scl = fabs(J);
      }
      const T lamJ = cof ? lam * (J - T(1) - am1) * sgnJ / det0 : T(0);
      T num = 0, den = 0;
      int nub = 0;
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const T pk = plastic ? edge_quad(Zp, k) / S[k] : T(1);
        T sig;
        if constexpr (EN == kEnergyStVK) {
          // q^T S q, S = lam/2 (I_C - 3) Cp^-1 + mu (Cp^-1 C Cp^-1 - Cp^-1)
          sig = T(0.5) * lam * aI * pk + mu * edge_quad(Zs, k) / S[k];
        } else if (!small) {
          const T omw = edge_quad(Zs, k) / S[k];  // p_k - w_k
          const T dj = delta * (T(1) - am1) + delta * delta;
          // mu (1 - 1/(I_C+1)) = 3mu/4 + mu a/(4(4+a)); lam (J-alpha) J = -3mu/4 + lam dj
          sig = T(0.75) * mu * omw + mu * aI / (T(4) * IC1) * pk + lam * dj * (pk - omw);
        } else {
          sig = scl * (T(0.75) * mu + mu * aI / (T(4) * IC1)) * pk + lamJ * edge_quad(Zs, k) / S[k];
        }
        const T as = fabs(sig);
        den += as;
        if (!((mask >> k) & 1)) {
          num += as;
          ++nub;
        }
      }
      chi = (den <= T(1e-12) * (mu + lam) * scl) ? T(nub) / T(6) : num / den;
    }
  }

  {
    const bool pr[2] = {act && chi == T(0), act && small};
    block_counts<2, kElemTets>(ctr, kChiZero, pr);
  }
  if (act && chi_out) chi_out[t] = chi;

  // This tet's six records, staged in LDS (zero when inactive or chi = 0).
  Rec<T>* lr = lrec + 6 * threadIdx.x;
  if (!act || chi == T(0)) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
#pragma unroll
      for (int c = 0; c < 9; ++c) lr[k].b[c] = T(0);
      lr[k].w = 0.0;
    }
  } else {
    // Clamped edge Hessian: H = A1 c c^T + A2 v v^T + A3 M, M_kl = tr(G^-1 E_k G^-1 E_l)
    // = (Gam_ac Gam_bd + Gam_ad Gam_bc)/2; each coefficient clamped at >= 0.
    // Small |J|: only the I_C term (A1); the volume term adds lam dJ dJ^T.
    // StVK: A1 = lam/4, A2 = 0, A3 = mu/2 with M_kl = tr(E_k A E_l A) (Gam of A).
    const T Vc = vol * chi;
    constexpr bool kSt = EN == kEnergyStVK;
    const T A1 = kSt ? T(0.25) * lam : T(0.5) * mu / (IC1 * IC1);
    const T JmA = delta - am1;  // J - alpha
    const T A2 = (kSt || small) ? T(0) : fmax(T(0.25) * lam * (T(2) * J - T(1) - am1) * J, T(0));
    const T A3 = kSt ? T(0.5) * mu : (small ? T(0) : fmax(T(-0.5) * lam * JmA * J, T(0)));
    T H[6][6];
#pragma unroll
    for (int k = 0; k < 6; ++k)
#pragma unroll
      for (int l = k; l < 6; ++l) {
        const int a = EA(k), b = EB(k), c = EA(l), d = EB(l);
        T hkl = A1 * cc[k] * cc[l];
        if (kSt) {
          hkl += A3 * T(0.5) * (GamP[a][c] * GamP[b][d] + GamP[a][d] * GamP[b][c]);
        } else if (!small) {
          const T Mkl = T(0.5) * (Gam[a][c] * Gam[b][d] + Gam[a][d] * Gam[b][c]);
          hkl += A2 * vv[k] * vv[l] + A3 * Mkl;
        }
        H[k][l] = H[l][k] = hkl;
      }

    // Stiffness (Eq. 10, 33): K(a,b) = V chi [ sum_{p at a, q at b} H_pq ds_p/dx_a ds_q/dx_b^T
    //                                          - 2 max(g_ab, 0) I ],  ds_p/dx = +-2 d_p.
    // Node incidence: (edge, sign) with sign +1 when the node is the edge's head.
    constexpr int inc_e[4][3] = {{0, 1, 2}, {0, 3, 4}, {1, 3, 5}, {2, 4, 5}};
    constexpr int inc_s[4][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {1, 1, 1}};
    const uint8_t fl = flip[t];
    const double Vcd = (double)vol * (double)chi;
#pragma unroll
    for (int b = 1; b < 4; ++b) {
      T Tb[6][3];
#pragma unroll
      for (int p = 0; p < 6; ++p)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          T acc = 0;
#pragma unroll
          for (int jq = 0; jq < 3; ++jq) {
            const int q = inc_e[b][jq];
            acc += (T)inc_s[b][jq] * H[p][q] * dcur[q][d];
          }
          Tb[p][d] = acc;
        }
#pragma unroll
      for (int a = 0; a < b; ++a) {
        const int k = (a == 0) ? (b - 1) : (a == 1 ? (b == 2 ? 3 : 4) : 5);
        T Kab[3][3];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            T acc = 0;
#pragma unroll
            for (int jp = 0; jp < 3; ++jp) {
              const int p = inc_e[a][jp];
              acc += (T)inc_s[a][jp] * dcur[p][r] * Tb[p][c];
            }
            Kab[r][c] = T(4) * Vc * acc;
          }
        const T lap = T(2) * Vc * fmax(g[k], T(0));
        Kab[0][0] -= lap;
        Kab[1][1] -= lap;
        Kab[2][2] -= lap;
        if (cof) {
          const T kJ = (T)(Vcd * cst.lam);
#pragma unroll
          for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) Kab[r][c] += kJ * (T)(gJd[a][r] * gJd[b][c]);
        }
        const bool tr = (fl >> k) & 1;
        Rec<T> rec;
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c) rec.b[3 * r + c] = tr ? Kab[c][r] : Kab[r][c];
        rec.w = 2.0 * Vcd * ((double)g[k] + wJ[k]);
        lr[k] = rec;
      }
    }
  }
  __syncthreads();
  // One partial record per edge the workgroup touches: its tets' records
  // summed in the fixed order of the host-built tables.
  const int p1 = part_base[blockIdx.x + 1];
  for (int p = part_base[blockIdx.x] + threadIdx.x; p < p1; p += kElemTets) {
    Rec<T> acc;
#pragma unroll
    for (int c = 0; c < 9; ++c) acc.b[c] = T(0);
    acc.w = 0.0;
    for (int q = part_cptr[p], q1 = part_cptr[p + 1]; q < q1; ++q) {
      const Rec<T>& r = lrec[part_slot[q]];
#pragma unroll
      for (int c = 0; c < 9; ++c) acc.b[c] += r.b[c];
      acc.w += r.w;
    }
    contrib[p] = acc;
  }
}

// ---------------------------------------------------------------- quasi-static Newton (Eq. 36)

// Total energy E = sum_e chi_e V_e Psi_e at the displacement U + step X64,
// chi fixed (Eq. 32 with the energy fraction of Eq. 25 held constant, so
// that -grad E is the restoring force of the Newton system).  FP64 from the
// rest edge vectors and the displacement differences; Psi of Eq. 35 or
// Eq. 37 from I_C = tr(G Gp^-1), J = det Ds / det Dm, II_C = tr((G Gp^-1)^2).
// Grid-stride over the tets; one FP64 partial per workgroup.
template <typename T, int EN>
__global__ __launch_bounds__(kThreads) void k_energy(int m, const int4* __restrict__ tets,
                                                     const d4* __restrict__ X, const d4* __restrict__ U,
                                                     const d4* __restrict__ X64, double step,
                                                     const T* __restrict__ pl, const T* __restrict__ chi_in,
                                                     ElemConst cst, double* __restrict__ part) {
  __shared__ double sh[16];
  double acc = 0.0;
  for (int t = blockIdx.x * kThreads + threadIdx.x; t < m; t += gridDim.x * kThreads) {
    const double chi = (double)chi_in[t];
    if (chi == 0.0) continue;
    const int4 nd = tets[t];
    const int ids[4] = {nd.x, nd.y, nd.z, nd.w};
    const d4 X0 = X[nd.x], U0 = U[nd.x], W0 = X64[nd.x];
    const double u0[3] = {U0.x + step * W0.x, U0.y + step * W0.y, U0.z + step * W0.z};
    double Dm[3][3], Ds[3][3];  // [edge from node 0][component]
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const d4 Xk = X[ids[k + 1]], Uk = U[ids[k + 1]], Wk = X64[ids[k + 1]];
      Dm[k][0] = Xk.x - X0.x;
      Dm[k][1] = Xk.y - X0.y;
      Dm[k][2] = Xk.z - X0.z;
      Ds[k][0] = Dm[k][0] + ((Uk.x + step * Wk.x) - u0[0]);
      Ds[k][1] = Dm[k][1] + ((Uk.y + step * Wk.y) - u0[1]);
      Ds[k][2] = Dm[k][2] + ((Uk.z + step * Wk.z) - u0[2]);
    }
    constexpr int R[6] = {0, 1, 2, 0, 0, 1}, C[6] = {0, 1, 2, 1, 2, 2};
    double G[6], Gp[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const int i = R[c], j = C[c];
      G[c] = Ds[i][0] * Ds[j][0] + Ds[i][1] * Ds[j][1] + Ds[i][2] * Ds[j][2];
      Gp[c] = Dm[i][0] * Dm[j][0] + Dm[i][1] * Dm[j][1] + Dm[i][2] * Dm[j][2] +
              (pl ? (double)pl[(size_t)c * m + t] : 0.0);
    }
    double Gpi[6];
    sym3_inv(Gp, sym3_det(Gp[0], Gp[1], Gp[2], Gp[3], Gp[4], Gp[5]), Gpi);
    double Gf[3][3], Af[3][3], P[3][3];
    sym_full(G, Gf);
    sym_full(Gpi, Af);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) P[i][j] = Gf[i][0] * Af[0][j] + Gf[i][1] * Af[1][j] + Gf[i][2] * Af[2][j];
    const double IC = P[0][0] + P[1][1] + P[2][2];
    auto det3 = [](const double (&a)[3][3]) {
      return a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) - a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
             a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
    };
    const double detDm = det3(Dm);
    double psi;
    if constexpr (EN == kEnergyStVK) {
      double II = 0.0;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) II += P[i][j] * P[j][i];
      psi = cst.lam / 8.0 * (IC - 3.0) * (IC - 3.0) + cst.mu / 4.0 * (II - 2.0 * IC + 3.0);
    } else {
      const double J = det3(Ds) / detDm;
      const double JmA = J - 1.0 - cst.alpha_m1;
      psi = 0.5 * cst.mu * (IC - 3.0) + 0.5 * cst.lam * JmA * JmA - 0.5 * cst.mu * log(IC + 1.0);
    }
    acc += chi * (detDm / 6.0) * psi;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ __launch_bounds__(kThreads) void k_dot(int n, const d4* __restrict__ a, const d4* __restrict__ b,
                                                  double* __restrict__ part) {
  __shared__ double sh[16];
  double acc = 0.0;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
    const d4 x = a[i], y = b[i];
    acc += x.x * y.x + x.y * y.y + x.z * y.z;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ __launch_bounds__(kThreads) void k_axpy(int n, double sc, const d4* __restrict__ x,
                                                   d4* __restrict__ y) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const d4 a = x[i];
  d4 c = y[i];
  c.x += sc * a.x;
  c.y += sc * a.y;
  c.z += sc * a.z;
  y[i] = c;
}

__global__ __launch_bounds__(kThreads) void k_zero_d4(int n, d4* __restrict__ x) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i < n) x[i] = d4{0.0, 0.0, 0.0, 0.0};
}

__global__ __launch_bounds__(kThreads) void k_move_prescribed(int n, const uint8_t* __restrict__ dflag,
                                                              const d4* __restrict__ dvel, double dt,
                                                              d4* __restrict__ U) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n || !dflag[i]) return;
  const d4 v = dvel[i];
  d4 u = U[i];
  u.x += dt * v.x;
  u.y += dt * v.y;
  u.z += dt * v.z;
  U[i] = u;
}

// ---------------------------------------------------------------- visualisation mesh (Sec. 4.1)

// One thread per tet: the node-associated four-split with children placed by
// the unbroken-edge groups of each edge, face and the tet.  FP64.
__global__ __launch_bounds__(kThreads) void k_visual(int t0, int cnt, int m, const int4* __restrict__ tets,
                                                     const uint8_t* __restrict__ swapped,
                                                     const int32_t* __restrict__ tet_edge,
                                                     const uint8_t* __restrict__ zeta, const d4* __restrict__ X,
                                                     const d4* __restrict__ U, double* __restrict__ xyz,
                                                     uint8_t* __restrict__ group) {
  const int r = blockIdx.x * kThreads + threadIdx.x;
  if (r >= cnt) return;
  const int t = t0 + r;
  const int4 nd = tets[t];
  const int ids[4] = {nd.x, nd.y, nd.z, nd.w};
  double Xp[4][3], Up[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const d4 x = X[ids[a]], u = U[ids[a]];
    Xp[a][0] = x.x;
    Xp[a][1] = x.y;
    Xp[a][2] = x.z;
    Up[a][0] = u.x;
    Up[a][1] = u.y;
    Up[a][2] = u.z;
  }
  // unbroken[i][j] between internal corners
  bool ub[4][4] = {};
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const bool u = zeta[tet_edge[(size_t)k * m + t]] == 0;
    ub[EA(k)][EB(k)] = ub[EB(k)][EA(k)] = u;
  }
  // caller corner -> internal corner (an involution)
  const bool sw = swapped[t] != 0;
  const int cmap[4] = {0, 1, sw ? 3 : 2, sw ? 2 : 3};
  double* out = xyz + (size_t)r * 96;
  auto put = [&](int a, int v, const double (&p)[3]) {
#pragma unroll
    for (int d = 0; d < 3; ++d) out[(a * 8 + v) * 3 + d] = p[d];
  };
  for (int a = 0; a < 4; ++a) {
    const int ia = cmap[a];
    int ob[3], j = 0;
    for (int b = 0; b < 4; ++b)
      if (b != a) ob[j++] = cmap[b];
    double p[3];
    for (int d = 0; d < 3; ++d) p[d] = Xp[ia][d] + Up[ia][d];
    put(a, 0, p);
    for (int q = 0; q < 3; ++q) {  // edge points
      const int ib = ob[q];
      const bool join = ub[ia][ib];
      for (int d = 0; d < 3; ++d)
        p[d] = (Xp[ia][d] + Xp[ib][d]) / 2.0 + (join ? (Up[ia][d] + Up[ib][d]) / 2.0 : Up[ia][d]);
      put(a, 1 + q, p);
    }
    const int fp[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (int q = 0; q < 3; ++q) {  // face points
      const int ib = ob[fp[q][0]], ic = ob[fp[q][1]];
      const bool inb = ub[ia][ib] || (ub[ia][ic] && ub[ic][ib]);
      const bool inc = ub[ia][ic] || (ub[ia][ib] && ub[ib][ic]);
      const int cntg = 1 + (int)inb + (int)inc;
      for (int d = 0; d < 3; ++d) {
        const double us = Up[ia][d] + (inb ? Up[ib][d] : 0.0) + (inc ? Up[ic][d] : 0.0);
        p[d] = (Xp[ia][d] + Xp[ib][d] + Xp[ic][d]) / 3.0 + us / cntg;
      }
      put(a, 4 + q, p);
    }
    // tet point: the component of ia in the unbroken-edge graph
    bool in[4] = {false, false, false, false};
    in[ia] = true;
    for (int it = 0; it < 3; ++it)
      for (int i = 0; i < 4; ++i)
        if (in[i])
          for (int k = 0; k < 4; ++k)
            if (ub[i][k]) in[k] = true;
    int cntc = 0, gmin = 4;
    double us[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 4; ++i)
      if (in[i]) {
        ++cntc;
        gmin = min(gmin, cmap[i]);
        for (int d = 0; d < 3; ++d) us[d] += Up[i][d];
      }
    for (int d = 0; d < 3; ++d) p[d] = (Xp[0][d] + Xp[1][d] + Xp[2][d] + Xp[3][d]) / 4.0 + us[d] / cntc;
    put(a, 7, p);
    group[(size_t)r * 4 + a] = (uint8_t)gmin;
  }
}

// ---------------------------------------------------------------- row pass

template <int W>
__device__ __forceinline__ double seg_sum(double v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
  return v;
}

// Assembly by block rows, one row per kRowPassLanes lanes; each lane takes
// off-diagonal blocks (i, j) of the row and forms
//   A_ij = m_ij (1 + dt alpha) I + (dt^2 + dt beta) K_ij
// from the edge's partial records (one per element-pass workgroup that
// touched the edge, summed in ascending order; they hold K(min, max), so row
// i > j takes the transpose: rows i and j sum the same records in the same
// order and A_ji is exactly A_ij^T), writes it to the row's own blocks
// (contiguous), and the lanes then sum:
//   A_ii = (1 + dt alpha) m_i I - sum_j A_ij   (translation invariance of K)
//   f_i  = sum_j w_ij (x_j - x_i)              (Eq. 12: forces along edges)
//   b_i  = dt (m_i g + f_i) - dt alpha (M v)_i - sum_j (A_ij - m_ij (1 + dt alpha) I)(v_j - v_i)
// then Dirichlet elimination (b_f -= A_fc dv_c; rows/columns of c -> identity),
// the block-Jacobi inverse of A_ii, X64 = 0 and the partial |b|^2.
// Lanes per block row in the row pass (22 FP64 partial sums per row are
// reduced across them; 8 lanes cover the ~14 blocks of a row in two rounds).
constexpr int kRowPassLanes = 8;

template <typename T>
__global__ __launch_bounds__(kThreads) void k_row(int n, MatView Am, const int32_t* __restrict__ diag_blk,
                                                  const int32_t* __restrict__ blk_edge,
                                                  const double* __restrict__ edge_mass,
                                                  const int32_t* __restrict__ edge_pptr,
                                                  const int32_t* __restrict__ edge_part,
                                                  const Rec<T>* __restrict__ contrib, double stiff_fac,
                                                  const double* __restrict__ lumped,
                                                  const d4* __restrict__ X, const d4* __restrict__ U,
                                                  const d4* __restrict__ V, const uint8_t* __restrict__ dflag,
                                                  const d4* __restrict__ dvel, RowConst cst, T* __restrict__ val,
                                                  d4* __restrict__ bvec, d4* __restrict__ X64,
                                                  T* __restrict__ binv, d4* __restrict__ f_out,
                                                  double* __restrict__ part_bb) {
  __shared__ double sh[16];
  const int G = gridDim.x;
  const int L = xcd_logical(blockIdx.x, G);
  const int chunk = (n + G - 1) / G;
  const int r0 = L * chunk, r1 = min(n, r0 + chunk);
  const int nbp = Am.nbp;
  const int lane = threadIdx.x & (kRowPassLanes - 1);
  const int grp = threadIdx.x / kRowPassLanes;
  double bb = 0;
  for (int i = r0 + grp; i < r1; i += kThreads / kRowPassLanes) {
    const int s = Am.row_ptr[i], e = Am.row_ptr[i + 1], db = diag_blk[i];
    const d4 Xi = X[i], Ui = U[i], vi = V[i];
    const bool ci = dflag[i] != 0;
    // per-lane partial sums: f(3) kv(3) mv(3) bd(3) As(9) msum(1)
    double acc[22];
#pragma unroll
    for (int c = 0; c < 22; ++c) acc[c] = 0.0;
    for (int b = s + lane; b < e; b += kRowPassLanes) {
      if (b == db) continue;
      const int j = Am.col[b];
      const int ed = blk_edge[b];
      const double me = edge_mass[ed];
      T kb[9];
#pragma unroll
      for (int c = 0; c < 9; ++c) kb[c] = T(0);
      double w = 0.0;
      for (int q = edge_pptr[ed], q1 = edge_pptr[ed + 1]; q < q1; ++q) {
        const Rec<T> r = contrib[edge_part[q]];
#pragma unroll
        for (int c = 0; c < 9; ++c) kb[c] += r.b[c];
        w += r.w;
      }
      const d4 Xj = X[j], Uj = U[j], vj = V[j];
      const double dx[3] = {(Xj.x - Xi.x) + (Uj.x - Ui.x), (Xj.y - Xi.y) + (Uj.y - Ui.y),
                            (Xj.z - Xi.z) + (Uj.z - Ui.z)};
      const double dv[3] = {vj.x - vi.x, vj.y - vi.y, vj.z - vi.z};
      const double md = me * cst.mass_fac;
      double a[9];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const T kv = i < j ? kb[3 * r + c] : kb[3 * c + r];
          a[3 * r + c] = (double)(T)(stiff_fac * (double)kv + (r == c ? md : 0.0));
        }
#pragma unroll
      for (int c = 0; c < 9; ++c) acc[12 + c] += a[c];
      acc[21] += me;
      const double mf = me * cst.mass_fac;
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        acc[r] += w * dx[r];
        double t = 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) t += (a[3 * r + c] - (r == c ? mf : 0.0)) * dv[c];
        acc[3 + r] += t;
      }
      acc[6] += me * vj.x;
      acc[7] += me * vj.y;
      acc[8] += me * vj.z;
      const bool cj = dflag[j] != 0;
      if (cj) {
        const d4 pj = dvel[j];
        const double dvc[3] = {pj.x - vj.x, pj.y - vj.y, pj.z - vj.z};
#pragma unroll
        for (int r = 0; r < 3; ++r) acc[9 + r] += a[3 * r] * dvc[0] + a[3 * r + 1] * dvc[1] + a[3 * r + 2] * dvc[2];
      }
      const bool zero = cj || ci;
#pragma unroll
      for (int c = 0; c < 9; ++c) val[(size_t)c * nbp + b] = zero ? T(0) : (T)a[c];
    }
#pragma unroll
    for (int c = 0; c < 22; ++c) acc[c] = seg_sum<kRowPassLanes>(acc[c]);
    if (lane == 0) {
      const double mi = lumped[i];
      const double mii = mi - acc[21];
      const double mv[3] = {acc[6] + mii * vi.x, acc[7] + mii * vi.y, acc[8] + mii * vi.z};
      double Aii[9];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) Aii[3 * r + c] = (r == c ? cst.mass_fac * mi : 0.0) - acc[12 + 3 * r + c];
      double bi[3];
#pragma unroll
      for (int r = 0; r < 3; ++r)
        bi[r] = cst.dt * (mi * cst.g[r] + acc[r]) - cst.dt * cst.ra * mv[r] - acc[3 + r] - acc[9 + r];
      if (f_out) f_out[i] = d4{acc[0], acc[1], acc[2], 0.0};
      if (ci) {
        const d4 pv = dvel[i];
        bi[0] = pv.x - vi.x;
        bi[1] = pv.y - vi.y;
        bi[2] = pv.z - vi.z;
#pragma unroll
        for (int c = 0; c < 9; ++c) Aii[c] = (c % 4 == 0) ? 1.0 : 0.0;
      }
      // symmetric part of the diagonal block (exactly symmetric up to rounding)
      const double s01 = 0.5 * (Aii[1] + Aii[3]), s02 = 0.5 * (Aii[2] + Aii[6]), s12 = 0.5 * (Aii[5] + Aii[7]);
      Aii[1] = Aii[3] = s01;
      Aii[2] = Aii[6] = s02;
      Aii[5] = Aii[7] = s12;
#pragma unroll
      for (int c = 0; c < 9; ++c) val[(size_t)c * nbp + db] = (T)Aii[c];
      const double sd[6] = {Aii[0], Aii[4], Aii[8], s01, s02, s12};
      const double det = sym3_det(sd[0], sd[1], sd[2], sd[3], sd[4], sd[5]);
      double inv[6];
      sym3_inv(sd, det, inv);
#pragma unroll
      for (int c = 0; c < 6; ++c) binv[(size_t)c * n + i] = (T)inv[c];
      bvec[i] = d4{bi[0], bi[1], bi[2], 0.0};
      X64[i] = d4{0.0, 0.0, 0.0, 0.0};
      bb += bi[0] * bi[0] + bi[1] * bi[1] + bi[2] * bi[2];
    }
  }
  bb = block_sum(bb, sh);
  if (threadIdx.x == 0) part_bb[L] = bb;
}

// ---------------------------------------------------------------- PCG

template <typename T>
__device__ __forceinline__ v4<T> bj_apply(const T* __restrict__ binv, int n, int i, v4<T> r) {
  const T b00 = binv[i], b11 = binv[(size_t)n + i], b22 = binv[2 * (size_t)n + i];
  const T b01 = binv[3 * (size_t)n + i], b02 = binv[4 * (size_t)n + i], b12 = binv[5 * (size_t)n + i];
  v4<T> z;
  z.x = b00 * r.x + b01 * r.y + b02 * r.z;
  z.y = b01 * r.x + b11 * r.y + b12 * r.z;
  z.z = b02 * r.x + b12 * r.y + b22 * r.z;
  z.w = 0;
  return z;
}

// Deterministic sum over an NT-thread workgroup (fixed tree), three values.
template <int NT>
__device__ __forceinline__ void block_sum3n(double& a, double& b, double& c, double* sh) {
  constexpr int NW = NT / 64;
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    sh[threadIdx.x >> 6] = a;
    sh[NW + (threadIdx.x >> 6)] = b;
    sh[2 * NW + (threadIdx.x >> 6)] = c;
  }
  __syncthreads();
  double ra = 0, rb = 0, rc = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    ra += sh[w];
    rb += sh[NW + w];
    rc += sh[2 * NW + w];
  }
  a = ra;
  b = rb;
  c = rc;
}

// Block-Jacobi preconditioned conjugate gradients, two kernels per
// iteration.  Dot products are accumulated in FP64 per workgroup and each
// consumer kernel reduces the producer's partials itself (fixed order, so
// every workgroup computes identical scalars and the run is reproducible).
// Partial layout: part_rz[parity][component][workgroup], component 0 = r.z,
// 1 = r.r; part_pq[workgroup].

template <typename T>
struct Blk {
  T a[9];
};

template <typename T>
__device__ __forceinline__ Blk<T> load_blk(const T* __restrict__ val, int nbp, int b) {
  Blk<T> k;
#pragma unroll
  for (int c = 0; c < 9; ++c) k.a[c] = val[(size_t)c * nbp + b];
  return k;
}

template <typename T>
__device__ __forceinline__ void blk_fma(const Blk<T>& k, const v4<T>& x, T& ax, T& ay, T& az) {
  ax = fmadd(k.a[0], x.x, fmadd(k.a[1], x.y, fmadd(k.a[2], x.z, ax)));
  ay = fmadd(k.a[3], x.x, fmadd(k.a[4], x.y, fmadd(k.a[5], x.z, ay)));
  az = fmadd(k.a[6], x.x, fmadd(k.a[7], x.y, fmadd(k.a[8], x.z, az)));
}

// r = src (rounded to T), z = B r, p_0 = z, x = 0; partials of r.z and r.r;
// resets the control block for the solve.
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_pcg_init(int n, const d4* __restrict__ src, const T* __restrict__ binv,
                                                 v4<T>* __restrict__ r, v4<T>* __restrict__ z,
                                                 v4<T>* __restrict__ p0, v4<T>* __restrict__ x,
                                                 double* __restrict__ part_rz, PcgCtl* ctl) {
  __shared__ double sh[3 * (NT / 64)];
  if (blockIdx.x == 0 && threadIdx.x == 0) *ctl = PcgCtl{0, 0, 0, 0, 0.0};
  const int G = gridDim.x;
  const int L = xcd_logical(blockIdx.x, G);
  const int chunk = (n + G - 1) / G;
  const int r0 = L * chunk, r1 = min(n, r0 + chunk);
  double rz = 0, rr = 0, unused = 0;
  for (int i = r0 + threadIdx.x; i < r1; i += NT) {
    const d4 s = src[i];
    const v4<T> ri{(T)s.x, (T)s.y, (T)s.z, T(0)};
    const v4<T> zi = bj_apply(binv, n, i, ri);
    r[i] = ri;
    z[i] = zi;
    p0[i] = zi;
    x[i] = v4<T>{T(0), T(0), T(0), T(0)};
    rz += (double)ri.x * zi.x + (double)ri.y * zi.y + (double)ri.z * zi.z;
    rr += (double)ri.x * ri.x + (double)ri.y * ri.y + (double)ri.z * ri.z;
  }
  block_sum3n<NT>(rz, rr, unused, sh);
  if (threadIdx.x == 0) {
    part_rz[L] = rz;
    part_rz[kMaxPart + L] = rr;
  }
}

// Iteration k, first kernel: reduce r_k.z_k, r_k.r_k (and r_{k-1}.z_{k-1});
// stop when |r_k|^2 <= rel2 |r_0|^2 (threshold fixed by the k = 0 launch);
// else p_k = z_k + beta_k p_{k-1} (k > 0; for k = 0 p_new already holds
// p_0 = z_0 and is only read), q = A p_k and the partial p_k.q.
// kSpmvLanes lanes share a block row, each with its first two blocks in
// flight; each neighbour's p_k entry is formed on the fly with the same fused
// operation as its owner uses, so all copies agree bitwise.  The first row's
// loads (row bounds, columns, blocks, gathered z and p_{k-1}) are issued before
// the scalar reduction so the two memory latencies overlap.
template <typename T, bool DIR>
struct SpmvSlot {
  bool on;
  Blk<T> k;
  v4<T> z, p;
};

template <typename T, bool DIR>
__device__ __forceinline__ SpmvSlot<T, DIR> spmv_load(const MatView& Am, const T* __restrict__ val, int b, bool on,
                                                      const v4<T>* __restrict__ z, const v4<T>* __restrict__ p_old,
                                                      const v4<T>* __restrict__ p_new) {
  SpmvSlot<T, DIR> s;
  s.on = on;
  if (on) {
    const int j = Am.col[b];
    s.k = load_blk(val, Am.nbp, b);
    if (DIR) {
      s.z = z[j];
      s.p = p_old[j];
    } else {
      s.p = p_new[j];
    }
  }
  return s;
}

template <typename T, bool DIR, int NT>
__global__ __launch_bounds__(NT) void k_pcg_spmv(int k, int Ga, MatView Am, const v4<T>* __restrict__ z,
                                                 const v4<T>* __restrict__ p_old, v4<T>* __restrict__ p_new,
                                                 v4<T>* __restrict__ q, PcgCtl* ctl,
                                                 const double* __restrict__ part_rz,
                                                 double* __restrict__ part_pq, double rel2) {
  __shared__ double sh[3 * (NT / 64)];
  // the control words are read together with the first row's loads (all in
  // bounds); a converged solve returns before anything is written.  At k = 0
  // the threshold is set here, so it is not read.
  const int done = ctl->done;
  const double thr2_prev = k == 0 ? 0.0 : ctl->thr2;
  const int n = Am.n;
  const int G = gridDim.x;
  const int L = xcd_logical(blockIdx.x, G);
  const int chunk = (n + G - 1) / G;
  const int r0 = min(n, L * chunk), r1 = min(n, r0 + chunk);
  constexpr int LN = kSpmvLanes;
  const int lane = threadIdx.x & (LN - 1);
  const int grp = threadIdx.x / LN;
  constexpr int NG = NT / LN;
  const T* __restrict__ val = static_cast<const T*>(Am.val);
  // peeled first row: bounds and first two slots
  int ra = r0 + grp;
  int sa = 0, cnt = 0;
  if (ra < r1) {
    sa = Am.row_ptr[ra];
    cnt = Am.row_ptr[ra + 1] - sa;
  }
  SpmvSlot<T, DIR> fa = spmv_load<T, DIR>(Am, val, sa + lane, lane < cnt, z, p_old, p_new);
  SpmvSlot<T, DIR> fb = spmv_load<T, DIR>(Am, val, sa + lane + LN, lane + LN < cnt, z, p_old, p_new);

  const double* cur = part_rz + (size_t)(k & 1) * 2 * kMaxPart;
  const double* prv = part_rz + (size_t)((k + 1) & 1) * 2 * kMaxPart;
  double rz = 0, rr = 0, rzp = 0;
  for (int i = threadIdx.x; i < Ga; i += NT) {
    rz += cur[i];
    rr += cur[kMaxPart + i];
    if (DIR) rzp += prv[i];
  }
  if (done) return;
  block_sum3n<NT>(rz, rr, rzp, sh);
  double thr2;
  if (k == 0) {
    thr2 = rel2 * rr;
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl->thr2 = thr2;
  } else {
    thr2 = thr2_prev;
  }
  if (!(rr > thr2) || rz == 0.0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl->done = 1;
    return;
  }
  const T beta = DIR ? (T)(rz / rzp) : T(0);
  double dot = 0;
  bool first = true;
  for (; ra < r1; ra += NG) {
    if (!first) {
      sa = Am.row_ptr[ra];
      cnt = Am.row_ptr[ra + 1] - sa;
      fa = spmv_load<T, DIR>(Am, val, sa + lane, lane < cnt, z, p_old, p_new);
      fb = spmv_load<T, DIR>(Am, val, sa + lane + LN, lane + LN < cnt, z, p_old, p_new);
    }
    first = false;
    T ax = 0, ay = 0, az = 0;
    if (fa.on) blk_fma(fa.k, DIR ? dir_comb(fa.z, beta, fa.p) : fa.p, ax, ay, az);
    if (fb.on) blk_fma(fb.k, DIR ? dir_comb(fb.z, beta, fb.p) : fb.p, ax, ay, az);
    for (int o = lane + 2 * LN; o < cnt; o += LN) {
      const SpmvSlot<T, DIR> t = spmv_load<T, DIR>(Am, val, sa + o, true, z, p_old, p_new);
      blk_fma(t.k, DIR ? dir_comb(t.z, beta, t.p) : t.p, ax, ay, az);
    }
#pragma unroll
    for (int o = LN / 2; o > 0; o >>= 1) {
      ax += __shfl_xor(ax, o, LN);
      ay += __shfl_xor(ay, o, LN);
      az += __shfl_xor(az, o, LN);
    }
    if (lane == 0) {
      const v4<T> pa = DIR ? dir_comb(z[ra], beta, p_old[ra]) : p_new[ra];
      if (DIR) p_new[ra] = pa;
      q[ra] = v4<T>{ax, ay, az, T(0)};
      dot += (double)pa.x * ax + (double)pa.y * ay + (double)pa.z * az;
    }
  }
  double u1 = 0, u2 = 0;
  block_sum3n<NT>(dot, u1, u2, sh);
  if (threadIdx.x == 0) part_pq[L] = dot;
}

// Iteration k, second kernel: alpha = r.z / p.q; x += alpha p; r -= alpha q;
// z = B r; partials of r.z and r.r for iteration k+1.  The first row's
// operands are loaded before the reduction so the two latencies overlap.
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_pcg_update(int k, int n, int Gb, const v4<T>* __restrict__ p,
                                                   const v4<T>* __restrict__ q, v4<T>* __restrict__ x,
                                                   v4<T>* __restrict__ r, v4<T>* __restrict__ z,
                                                   const T* __restrict__ binv, PcgCtl* ctl,
                                                   const double* __restrict__ part_pq,
                                                   double* __restrict__ part_rz) {
  __shared__ double sh[3 * (NT / 64)];
  // the control word is read together with the first row's loads (all in
  // bounds); a converged solve returns before anything is written
  const int done = ctl->done;
  const int G = gridDim.x;
  const int L = xcd_logical(blockIdx.x, G);
  const int chunk = (n + G - 1) / G;
  const int r0 = L * chunk, r1 = min(n, r0 + chunk);
  int i = r0 + threadIdx.x;
  v4<T> pi{}, qi{}, xi{}, ri{};
  if (i < r1) {
    pi = p[i];
    qi = q[i];
    xi = x[i];
    ri = r[i];
  }
  const double* cur = part_rz + (size_t)(k & 1) * 2 * kMaxPart;
  double pq = 0, rz = 0, unused = 0;
  for (int t = threadIdx.x; t < Gb; t += NT) pq += part_pq[t];
  for (int t = threadIdx.x; t < G; t += NT) rz += cur[t];
  if (done) return;
  block_sum3n<NT>(pq, rz, unused, sh);
  if (!(pq > 0.0) || !isfinite(pq) || !isfinite(rz)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      ctl->fail = 1;
      ctl->done = 1;
    }
    return;
  }
  const T al = (T)(rz / pq);
  double rzn = 0, rrn = 0;
  for (; i < r1; i += NT) {
    if (i != r0 + (int)threadIdx.x) {
      pi = p[i];
      qi = q[i];
      xi = x[i];
      ri = r[i];
    }
    xi.x = fmadd(al, pi.x, xi.x);
    xi.y = fmadd(al, pi.y, xi.y);
    xi.z = fmadd(al, pi.z, xi.z);
    ri.x = fmadd(-al, qi.x, ri.x);
    ri.y = fmadd(-al, qi.y, ri.y);
    ri.z = fmadd(-al, qi.z, ri.z);
    const v4<T> zi = bj_apply(binv, n, i, ri);
    x[i] = xi;
    r[i] = ri;
    z[i] = zi;
    rzn += (double)ri.x * zi.x + (double)ri.y * zi.y + (double)ri.z * zi.z;
    rrn += (double)ri.x * ri.x + (double)ri.y * ri.y + (double)ri.z * ri.z;
  }
  block_sum3n<NT>(rzn, rrn, unused, sh);
  double* nxt = part_rz + (size_t)((k + 1) & 1) * 2 * kMaxPart;
  if (threadIdx.x == 0) {
    nxt[L] = rzn;
    nxt[kMaxPart + L] = rrn;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl->iters = k + 1;
}

// ---------------------------------------------------------------- factorised preconditioner

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

// One strictly lower (G pass) or upper (G^T pass) block in flight: its 3x3
// values and the gathered operand(s) of its column.
template <typename T>
struct FSlot {
  bool on;
  uint4 g;     // entries 0-7
  __bf16 g8;   // entry 8
  v4<T> a, b;  // gathered operands
};

// MODE 0: G pass of an iteration (a = r_old[j], b = q[j]); 1: G pass at the
// start of a solve (a = src[j] rounded to T); 2: G^T pass (a = y[j]).
template <typename T, int MODE>
__device__ __forceinline__ FSlot<T> fslot_load(const int32_t* __restrict__ colv, const uint4* __restrict__ gv,
                                               const __bf16* __restrict__ g8, int idx, bool on,
                                               const d4* __restrict__ src, const v4<T>* __restrict__ va,
                                               const v4<T>* __restrict__ vb) {
  FSlot<T> s;
  s.on = on;
  if (on) {
    const int j = colv[idx];
    s.g = gv[idx];
    s.g8 = g8[idx];
    if (MODE == 1) {
      const d4 sj = src[j];
      s.a = v4<T>{(T)sj.x, (T)sj.y, (T)sj.z, T(0)};
    } else {
      s.a = va[j];
      if (MODE == 0) s.b = vb[j];
    }
  }
  return s;
}

template <typename T, int MODE>
__device__ __forceinline__ void fslot_apply(const FSlot<T>& s, T al, T& ax, T& ay, T& az) {
  if (!s.on) return;
  v4<T> x = s.a;
  if (MODE == 0) {
    x.x = fmadd(-al, s.b.x, x.x);
    x.y = fmadd(-al, s.b.y, x.y);
    x.z = fmadd(-al, s.b.z, x.z);
  }
  const bf16x8_t g = __builtin_bit_cast(bf16x8_t, s.g);
  ax = fmadd((T)(float)g[0], x.x, fmadd((T)(float)g[1], x.y, fmadd((T)(float)g[2], x.z, ax)));
  ay = fmadd((T)(float)g[3], x.x, fmadd((T)(float)g[4], x.y, fmadd((T)(float)g[5], x.z, ay)));
  az = fmadd((T)(float)g[6], x.x, fmadd((T)(float)g[7], x.y, fmadd((T)(float)s.g8, x.z, az)));
}

template <typename T>
__device__ __forceinline__ T fact_row_sum(T v) {
#pragma unroll
  for (int o = kFactLanes / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kFactLanes);
  return v;
}

// Row-local operands of the G pass (owner lane only).
template <typename T>
struct GOwn {
  v4<T> r, q, p, x;
  uint4 d;
};

// G pass.  INIT: r = src rounded to T (written to r_new), x = 0, partials into
// parity 0.  Otherwise iteration k: alpha from the SpMV's p.q partials and
// this grid's r.z partials of parity k; every neighbour's r_new entry is
// formed on the fly with the same fused operation its owner uses (r_old and
// r_new are distinct buffers, so no row reads a value another workgroup is
// overwriting).  kFactLanes lanes per row, two blocks per lane in flight; the
// first row's loads are issued before the scalar reduction so that the two
// latencies overlap.
template <typename T, bool INIT, int NT>
__global__ __launch_bounds__(NT) void k_pcg_gpass(int k, int npq, FactView F, const d4* __restrict__ src,
                                                  const v4<T>* __restrict__ r_old, v4<T>* __restrict__ r_new,
                                                  const v4<T>* __restrict__ q, const v4<T>* __restrict__ p,
                                                  v4<T>* __restrict__ x, v4<T>* __restrict__ y, PcgCtl* ctl,
                                                  const double* __restrict__ part_pq,
                                                  double* __restrict__ part_rz) {
  constexpr int MODE = INIT ? 1 : 0;
  __shared__ double sh[3 * (NT / 64)];
  if (INIT && blockIdx.x == 0 && threadIdx.x == 0) *ctl = PcgCtl{0, 0, 0, 0, 0.0};
  // the control word is read together with the first row's loads (all in
  // bounds); a converged solve returns before anything is written
  const int done = INIT ? 0 : ctl->done;
  const int n = F.n;
  const int G = gridDim.x;
  const int L = xcd_logical(blockIdx.x, G);
  const int chunk = (n + G - 1) / G;
  const int r0 = min(n, L * chunk), r1 = min(n, r0 + chunk);
  const int lane = threadIdx.x & (kFactLanes - 1);
  const int grp = threadIdx.x / kFactLanes;
  constexpr int NG = NT / kFactLanes;
  int i = r0 + grp;
  int s = 0, e = 0;
  if (i < r1) {
    s = F.lptr[i];
    e = F.lptr[i + 1];
  }
  FSlot<T> fa = fslot_load<T, MODE>(F.lcol, F.glv, F.gl8, s + lane, s + lane < e, src, r_old, q);
  FSlot<T> fb = fslot_load<T, MODE>(F.lcol, F.glv, F.gl8, s + lane + kFactLanes, s + lane + kFactLanes < e, src,
                                    r_old, q);
  GOwn<T> own{};
  auto load_own = [&](int row) {
    if (lane == 0 && row < r1) {
      if (INIT) {
        const d4 si = src[row];
        own.r = v4<T>{(T)si.x, (T)si.y, (T)si.z, T(0)};
      } else {
        own.r = r_old[row];
        own.q = q[row];
        own.p = p[row];
        own.x = x[row];
      }
      own.d = F.gdv[row];
    }
  };
  load_own(i);
  T al = T(0);
  if (!INIT) {
    const double* cur = part_rz + (size_t)(k & 1) * 2 * kMaxPart;
    double pq = 0, rz = 0, unused = 0;
    for (int t = threadIdx.x; t < npq; t += NT) pq += part_pq[t];
    for (int t = threadIdx.x; t < G; t += NT) rz += cur[t];
    if (done) return;
    block_sum3n<NT>(pq, rz, unused, sh);
    if (!(pq > 0.0) || !isfinite(pq) || !isfinite(rz)) {
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->fail = 1;
        ctl->done = 1;
      }
      return;
    }
    al = (T)(rz / pq);
  }
  double yy = 0, rr = 0;
  bool first = true;
  for (; i < r1; i += NG) {
    if (!first) {
      s = F.lptr[i];
      e = F.lptr[i + 1];
      fa = fslot_load<T, MODE>(F.lcol, F.glv, F.gl8, s + lane, s + lane < e, src, r_old, q);
      fb = fslot_load<T, MODE>(F.lcol, F.glv, F.gl8, s + lane + kFactLanes, s + lane + kFactLanes < e, src, r_old,
                               q);
      load_own(i);
    }
    first = false;
    T ax = 0, ay = 0, az = 0;
    fslot_apply<T, MODE>(fa, al, ax, ay, az);
    fslot_apply<T, MODE>(fb, al, ax, ay, az);
    for (int b = s + lane + 2 * kFactLanes; b < e; b += kFactLanes) {
      const FSlot<T> t = fslot_load<T, MODE>(F.lcol, F.glv, F.gl8, b, true, src, r_old, q);
      fslot_apply<T, MODE>(t, al, ax, ay, az);
    }
    ax = fact_row_sum(ax);
    ay = fact_row_sum(ay);
    az = fact_row_sum(az);
    if (lane == 0) {
      v4<T> ri = own.r;
      if (!INIT) {
        ri.x = fmadd(-al, own.q.x, ri.x);
        ri.y = fmadd(-al, own.q.y, ri.y);
        ri.z = fmadd(-al, own.q.z, ri.z);
        v4<T> xi = own.x;
        xi.x = fmadd(al, own.p.x, xi.x);
        xi.y = fmadd(al, own.p.y, xi.y);
        xi.z = fmadd(al, own.p.z, xi.z);
        x[i] = xi;
      } else {
        x[i] = v4<T>{T(0), T(0), T(0), T(0)};
      }
      r_new[i] = ri;
      const bf16x8_t d = __builtin_bit_cast(bf16x8_t, own.d);
      ax = fmadd((T)(float)d[0], ri.x, ax);
      ay = fmadd((T)(float)d[1], ri.x, fmadd((T)(float)d[2], ri.y, ay));
      az = fmadd((T)(float)d[3], ri.x, fmadd((T)(float)d[4], ri.y, fmadd((T)(float)d[5], ri.z, az)));
      y[i] = v4<T>{ax, ay, az, T(0)};
      yy += (double)ax * ax + (double)ay * ay + (double)az * az;
      rr += (double)ri.x * ri.x + (double)ri.y * ri.y + (double)ri.z * ri.z;
    }
  }
  double unused = 0;
  block_sum3n<NT>(yy, rr, unused, sh);
  double* nxt = part_rz + (size_t)(INIT ? 0 : ((k + 1) & 1)) * 2 * kMaxPart;
  if (threadIdx.x == 0) {
    nxt[L] = yy;
    nxt[kMaxPart + L] = rr;
  }
  if (!INIT && blockIdx.x == 0 && threadIdx.x == 0) ctl->iters = k + 1;
}

// G^T pass and direction update.  The G pass's partials (r.z = y.y and r.r
// of parity INIT ? 0 : (k + 1) & 1) are reduced first: stop when
// |r|^2 <= thr2 (thr2 = rel2 |r_0|^2, fixed by the INIT launch), else
// beta = r.z / (previous r.z), z_i = G_ii^T y_i + sum over the upper blocks
// (i, j) of G_ji^T y_j and p_new = z + beta p_old for the workgroup's own rows
// (INIT: p_0 = z).  The SpMV then gathers p alone.
template <typename T, bool INIT, int NT>
__global__ __launch_bounds__(NT) void k_pcg_gtpass(int k, FactView F, const v4<T>* __restrict__ y,
                                                   const v4<T>* __restrict__ p_old, v4<T>* __restrict__ p_new,
                                                   PcgCtl* ctl, const double* __restrict__ part_rz, double rel2) {
  __shared__ double sh[3 * (NT / 64)];
  // the control words are read together with the first row's loads (all in
  // bounds); a converged solve returns before anything is written
  const int done = INIT ? 0 : ctl->done;
  const double thr2_prev = INIT ? 0.0 : ctl->thr2;
  const int n = F.n;
  const int G = gridDim.x;
  const int L = xcd_logical(blockIdx.x, G);
  const int chunk = (n + G - 1) / G;
  const int r0 = min(n, L * chunk), r1 = min(n, r0 + chunk);
  const int lane = threadIdx.x & (kFactLanes - 1);
  const int grp = threadIdx.x / kFactLanes;
  constexpr int NG = NT / kFactLanes;
  // first row's loads before the reduction
  int i = r0 + grp;
  int s = 0, e = 0;
  if (i < r1) {
    s = F.uptr[i];
    e = F.uptr[i + 1];
  }
  FSlot<T> fa = fslot_load<T, 2>(F.ucol, F.guv, F.gu8, s + lane, s + lane < e, nullptr, y, nullptr);
  FSlot<T> fb =
      fslot_load<T, 2>(F.ucol, F.guv, F.gu8, s + lane + kFactLanes, s + lane + kFactLanes < e, nullptr, y, nullptr);
  v4<T> yi{}, po{};
  uint4 dv{};
  auto load_own = [&](int row) {
    if (lane == 0 && row < r1) {
      yi = y[row];
      dv = F.gdv[row];
      if (!INIT) po = p_old[row];
    }
  };
  load_own(i);
  const double* cur = part_rz + (size_t)(INIT ? 0 : ((k + 1) & 1)) * 2 * kMaxPart;
  const double* prv = part_rz + (size_t)(k & 1) * 2 * kMaxPart;
  double rz = 0, rr = 0, rzp = 0;
  for (int t = threadIdx.x; t < G; t += NT) {
    rz += cur[t];
    rr += cur[kMaxPart + t];
    if (!INIT) rzp += prv[t];
  }
  if (done) return;
  block_sum3n<NT>(rz, rr, rzp, sh);
  double thr2;
  if (INIT) {
    thr2 = rel2 * rr;
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl->thr2 = thr2;
  } else {
    thr2 = thr2_prev;
  }
  if (!(rr > thr2) || rz == 0.0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl->done = 1;
    return;
  }
  const T beta = INIT ? T(0) : (T)(rz / rzp);
  bool first = true;
  for (; i < r1; i += NG) {
    if (!first) {
      s = F.uptr[i];
      e = F.uptr[i + 1];
      fa = fslot_load<T, 2>(F.ucol, F.guv, F.gu8, s + lane, s + lane < e, nullptr, y, nullptr);
      fb = fslot_load<T, 2>(F.ucol, F.guv, F.gu8, s + lane + kFactLanes, s + lane + kFactLanes < e, nullptr, y,
                            nullptr);
      load_own(i);
    }
    first = false;
    T ax = 0, ay = 0, az = 0;
    fslot_apply<T, 2>(fa, T(0), ax, ay, az);
    fslot_apply<T, 2>(fb, T(0), ax, ay, az);
    for (int b = s + lane + 2 * kFactLanes; b < e; b += kFactLanes) {
      const FSlot<T> t = fslot_load<T, 2>(F.ucol, F.guv, F.gu8, b, true, nullptr, y, nullptr);
      fslot_apply<T, 2>(t, T(0), ax, ay, az);
    }
    ax = fact_row_sum(ax);
    ay = fact_row_sum(ay);
    az = fact_row_sum(az);
    if (lane == 0) {
      const bf16x8_t d = __builtin_bit_cast(bf16x8_t, dv);
      ax = fmadd((T)(float)d[0], yi.x, fmadd((T)(float)d[1], yi.y, fmadd((T)(float)d[3], yi.z, ax)));
      ay = fmadd((T)(float)d[2], yi.y, fmadd((T)(float)d[4], yi.z, ay));
      az = fmadd((T)(float)d[5], yi.z, az);
      const v4<T> zi{ax, ay, az, T(0)};
      p_new[i] = INIT ? zi : dir_comb(zi, beta, po);
    }
  }
}

// SpMV of the factorised path: q = A p (p formed by the G^T pass), partial
// p.q.  kSpmvLanes lanes per block row, each lane's first two blocks loaded
// before any arithmetic (rows have 14.4 blocks on average), no scalar
// prologue.
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_pcg_spmv_p(MatView Am, const v4<T>* __restrict__ p, v4<T>* __restrict__ q,
                                                   PcgCtl* ctl, double* __restrict__ part_pq) {
  __shared__ double sh[3 * (NT / 64)];
  // the control word is read together with the first row's loads (all in
  // bounds); a converged solve returns before anything is written
  const int done = ctl->done;
  const int n = Am.n;
  const int G = gridDim.x;
  const int L = xcd_logical(blockIdx.x, G);
  const int chunk = (n + G - 1) / G;
  const int r0 = min(n, L * chunk), r1 = min(n, r0 + chunk);
  constexpr int LN = kSpmvLanes;
  const int lane = threadIdx.x & (LN - 1);
  const int grp = threadIdx.x / LN;
  constexpr int NG = NT / LN;
  const T* __restrict__ val = static_cast<const T*>(Am.val);
  int ra = r0 + grp;
  int sa = 0, cnt = 0;
  if (ra < r1) {
    sa = Am.row_ptr[ra];
    cnt = Am.row_ptr[ra + 1] - sa;
  }
  SpmvSlot<T, false> ta = spmv_load<T, false>(Am, val, sa + lane, lane < cnt, nullptr, nullptr, p);
  SpmvSlot<T, false> tb = spmv_load<T, false>(Am, val, sa + lane + LN, lane + LN < cnt, nullptr, nullptr, p);
  if (done) return;
  double dot = 0;
  bool first = true;
  for (; ra < r1; ra += NG) {
    if (!first) {
      sa = Am.row_ptr[ra];
      cnt = Am.row_ptr[ra + 1] - sa;
      ta = spmv_load<T, false>(Am, val, sa + lane, lane < cnt, nullptr, nullptr, p);
      tb = spmv_load<T, false>(Am, val, sa + lane + LN, lane + LN < cnt, nullptr, nullptr, p);
    }
    first = false;
    T ax = 0, ay = 0, az = 0;
    if (ta.on) blk_fma(ta.k, ta.p, ax, ay, az);
    if (tb.on) blk_fma(tb.k, tb.p, ax, ay, az);
    for (int o = lane + 2 * LN; o < cnt; o += LN) {
      const SpmvSlot<T, false> t = spmv_load<T, false>(Am, val, sa + o, true, nullptr, nullptr, p);
      blk_fma(t.k, t.p, ax, ay, az);
    }
#pragma unroll
    for (int o = LN / 2; o > 0; o >>= 1) {
      ax += __shfl_xor(ax, o, LN);
      ay += __shfl_xor(ay, o, LN);
      az += __shfl_xor(az, o, LN);
    }
    if (lane == 0) {
      const v4<T> pa = p[ra];
      q[ra] = v4<T>{ax, ay, az, T(0)};
      dot += (double)pa.x * ax + (double)pa.y * ay + (double)pa.z * az;
    }
  }
  double u1 = 0, u2 = 0;
  block_sum3n<NT>(dot, u1, u2, sh);
  if (threadIdx.x == 0) part_pq[L] = dot;
}

// FP64 residual of the outer (iterative refinement) loop: R = b - A X64 with
// the stored (FP32 or FP64) block values promoted to FP64; partial |R|^2.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_resid(MatView Am, const d4* __restrict__ bvec,
                                                    const d4* __restrict__ X64, d4* __restrict__ R64,
                                                    double* __restrict__ part_rr, const PcgCtl* ctl) {
  __shared__ double sh[16];
  if (ctl && !ctl->done) return;
  const int n = Am.n, nbp = Am.nbp;
  const int G = gridDim.x;
  const int L = xcd_logical(blockIdx.x, G);
  const int chunk = (n + G - 1) / G;
  const int r0 = L * chunk, r1 = min(n, r0 + chunk);
  const int lane = threadIdx.x & (kRowLanes - 1);
  const int grp = threadIdx.x / kRowLanes;
  const T* __restrict__ val = static_cast<const T*>(Am.val);
  double rr = 0;
  for (int row = r0 + grp; row < r1; row += kThreads / kRowLanes) {
    const int s = Am.row_ptr[row], e = Am.row_ptr[row + 1];
    double ax = 0, ay = 0, az = 0;
    for (int b = s + lane; b < e; b += kRowLanes) {
      const int j = Am.col[b];
      const d4 xj = X64[j];
      double a[9];
#pragma unroll
      for (int c = 0; c < 9; ++c) a[c] = (double)val[(size_t)c * nbp + b];
      ax = fmadd(a[0], xj.x, fmadd(a[1], xj.y, fmadd(a[2], xj.z, ax)));
      ay = fmadd(a[3], xj.x, fmadd(a[4], xj.y, fmadd(a[5], xj.z, ay)));
      az = fmadd(a[6], xj.x, fmadd(a[7], xj.y, fmadd(a[8], xj.z, az)));
    }
#pragma unroll
    for (int o = kRowLanes / 2; o > 0; o >>= 1) {
      ax += __shfl_xor(ax, o, kRowLanes);
      ay += __shfl_xor(ay, o, kRowLanes);
      az += __shfl_xor(az, o, kRowLanes);
    }
    if (lane == 0) {
      const d4 bi = bvec[row];
      const d4 ri{bi.x - ax, bi.y - ay, bi.z - az, 0.0};
      R64[row] = ri;
      rr += ri.x * ri.x + ri.y * ri.y + ri.z * ri.z;
    }
  }
  rr = block_sum(rr, sh);
  if (threadIdx.x == 0) part_rr[L] = rr;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_addcorr(int n, const v4<T>* __restrict__ x, d4* __restrict__ X64,
                                                      const PcgCtl* ctl) {
  if (ctl && !ctl->done) return;
  int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const v4<T> xi = x[i];
  d4 X = X64[i];
  X.x += (double)xi.x;
  X.y += (double)xi.y;
  X.z += (double)xi.z;
  X64[i] = X;
}

// v <- v + dv (prescribed nodes: exactly the prescribed velocity); U <- U + dt v.
__global__ __launch_bounds__(kThreads) void k_integrate(int n, const d4* __restrict__ X64, d4* __restrict__ V,
                                                        d4* __restrict__ U, const uint8_t* __restrict__ dflag,
                                                        const d4* __restrict__ dvel, double dt) {
  int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  d4 v = V[i];
  if (dflag[i]) {
    const d4 p = dvel[i];
    v = d4{p.x, p.y, p.z, 0.0};
  } else {
    const d4 d = X64[i];
    v.x += d.x;
    v.y += d.y;
    v.z += d.z;
  }
  V[i] = v;
  d4 u = U[i];
  u.x += dt * v.x;
  u.y += dt * v.y;
  u.z += dt * v.z;
  U[i] = u;
}

inline int blocks_for(long n) { return (int)((n + kThreads - 1) / kThreads); }

}  // namespace

// ---------------------------------------------------------------- launchers

void set_disconnected_lut(unsigned long long lut) {
  (void)hipMemcpyToSymbol(HIP_SYMBOL(c_disc_lut), &lut, sizeof lut);
}

void launch_damage(hipStream_t s, int ne, const int2* edges, const d4* X, const d4* U, const double* S,
                   const uint8_t* z_in, uint8_t* z_out, double thr, Counters* ctr, int32_t* near_ids) {
  if (ne <= 0) return;
  k_damage<<<blocks_for(ne), kThreads, 0, s>>>(ne, edges, X, U, S, z_in, z_out, thr, ctr, near_ids);
}

void launch_damage_nonlocal(hipStream_t s, int m, int ne, const int4* tets, const d4* X, const d4* U,
                            const int64_t* nl_ptr, const int32_t* nl_idx, const double* nl_w, Sym6* E,
                            Sym6* Eavg, const int2* edges, const int32_t* edge_ptr, const int32_t* edge_slot,
                            const uint8_t* z_in, uint8_t* z_out, double thr, Counters* ctr, int32_t* near_ids,
                            int64_t n_entries) {
  if (ne <= 0 || m <= 0) return;
  k_nl_strain<<<blocks_for(m), kThreads, 0, s>>>(m, tets, X, U, E);
  // lanes per tet from the mean support size
  const int64_t per = n_entries / m;
  if (per >= 48)
    k_nl_average<64><<<blocks_for((long)m * 64), kThreads, 0, s>>>(m, nl_ptr, nl_idx, nl_w, E, Eavg);
  else if (per >= 12)
    k_nl_average<16><<<blocks_for((long)m * 16), kThreads, 0, s>>>(m, nl_ptr, nl_idx, nl_w, E, Eavg);
  else
    k_nl_average<4><<<blocks_for((long)m * 4), kThreads, 0, s>>>(m, nl_ptr, nl_idx, nl_w, E, Eavg);
  k_nl_damage<<<blocks_for(ne), kThreads, 0, s>>>(ne, m, edges, X, edge_ptr, edge_slot, Eavg, z_in, z_out, thr,
                                                  ctr, near_ids);
}

template <typename T>
void launch_plastic(hipStream_t s, int m, const int4* tets, const d4* X, const d4* U, const T* pl_in, T* pl_out,
                    double yield) {
  if (m <= 0) return;
  k_plastic<T><<<blocks_for(m), kThreads, 0, s>>>(m, tets, X, U, pl_in, pl_out, yield);
}

template <typename T>
void launch_element(hipStream_t s, int m, const int4* tets, const int32_t* tet_edge, const uint8_t* flip,
                    const d4* X, const d4* U, const uint8_t* zeta, const T* pl, const T* chi_in, T* chi_out,
                    ElemConst c, const int32_t* part_base, const int32_t* part_cptr, const uint16_t* part_slot,
                    Rec<T>* contrib, Counters* ctr) {
  if (m <= 0) return;
  const int G = (m + kElemTets - 1) / kElemTets;
  if (c.energy == kEnergyStVK)
    k_element<T, kEnergyStVK><<<G, kElemTets, 0, s>>>(m, tets, tet_edge, flip, X, U, zeta, pl, chi_in, chi_out, c,
                                                       part_base, part_cptr, part_slot, contrib, ctr);
  else
    k_element<T, kEnergyStableNeoHookean><<<G, kElemTets, 0, s>>>(m, tets, tet_edge, flip, X, U, zeta, pl, chi_in,
                                                                  chi_out, c, part_base, part_cptr, part_slot,
                                                                  contrib, ctr);
}


template <typename T>
void launch_row(hipStream_t s, int n, int G, MatView A, const int32_t* diag_blk, const int32_t* blk_edge,
                const double* edge_mass, const int32_t* edge_pptr, const int32_t* edge_part, const Rec<T>* contrib,
                double stiff_fac, const double* lumped, const d4* X, const d4* U, const d4* V, const uint8_t* dflag,
                const d4* dvel, RowConst c, T* val_mut, d4* b, d4* X64, T* binv, d4* f_out, double* part_bb) {
  k_row<T><<<G, kThreads, 0, s>>>(n, A, diag_blk, blk_edge, edge_mass, edge_pptr, edge_part, contrib, stiff_fac,
                                  lumped, X, U, V, dflag, dvel, c, val_mut, b, X64, binv, f_out, part_bb);
}

// Launch with dispatch-recorded events when given.
template <typename... P, typename... A>
void launch_ev(void (*kernel)(P...), dim3 grid, dim3 block, hipStream_t s, const LaunchEvents& ev, A... args) {
  if (ev.start)
    hipExtLaunchKernelGGL(kernel, grid, block, 0, s, ev.start, ev.stop, 0, static_cast<P>(args)...);
  else
    kernel<<<grid, block, 0, s>>>(static_cast<P>(args)...);
}

template <typename T>
void launch_pcg_init(hipStream_t s, int n, int Ga, const d4* src, const T* binv, v4<T>* r, v4<T>* z, v4<T>* p0,
                     v4<T>* x, double* part_rz, PcgCtl* ctl) {
  k_pcg_init<T, kVecThreads><<<Ga, kVecThreads, 0, s>>>(n, src, binv, r, z, p0, x, part_rz, ctl);
}

template <typename T>
void launch_pcg_spmv(hipStream_t s, int k, int Gb, int Ga, MatView A, const v4<T>* z, const v4<T>* p_old,
                     v4<T>* p_new, v4<T>* q, PcgCtl* ctl, const double* part_rz, double* part_pq, double rel2,
                     LaunchEvents ev) {
  if (k == 0)
    launch_ev(k_pcg_spmv<T, false, kSpmvThreads>, Gb, kSpmvThreads, s, ev, k, Ga, A, z, p_old, p_new, q, ctl,
              part_rz, part_pq, rel2);
  else
    launch_ev(k_pcg_spmv<T, true, kSpmvThreads>, Gb, kSpmvThreads, s, ev, k, Ga, A, z, p_old, p_new, q, ctl, part_rz,
              part_pq, rel2);
}

template <typename T>
void launch_pcg_update(hipStream_t s, int k, int n, int Ga, int Gb, const v4<T>* p, const v4<T>* q, v4<T>* x,
                       v4<T>* r, v4<T>* z, const T* binv, PcgCtl* ctl, const double* part_pq, double* part_rz,
                       LaunchEvents ev) {
  launch_ev(k_pcg_update<T, kVecThreads>, Ga, kVecThreads, s, ev, k, n, Gb, p, q, x, r, z, binv, ctl, part_pq,
            part_rz);
}

template <typename T>
void launch_pcg_fact_init(hipStream_t s, int Gb, FactView F, const d4* src, v4<T>* r0, v4<T>* x, v4<T>* y,
                          v4<T>* p0, PcgCtl* ctl, double* part_rz, double rel2) {
  k_pcg_gpass<T, true, kSpmvThreads><<<Gb, kSpmvThreads, 0, s>>>(0, 0, F, src, nullptr, r0, nullptr, nullptr, x, y,
                                                                ctl, nullptr, part_rz);
  k_pcg_gtpass<T, true, kSpmvThreads><<<Gb, kSpmvThreads, 0, s>>>(0, F, y, nullptr, p0, ctl, part_rz, rel2);
}

template <typename T>
void launch_pcg_spmv_p(hipStream_t s, int Gp, MatView A, const v4<T>* p, v4<T>* q, PcgCtl* ctl, double* part_pq,
                       LaunchEvents ev) {
  launch_ev(k_pcg_spmv_p<T, kSpmvThreads>, Gp, kSpmvThreads, s, ev, A, p, q, ctl, part_pq);
}

template <typename T>
void launch_pcg_gpass(hipStream_t s, int k, int Gb, int npq, FactView F, const v4<T>* r_old, v4<T>* r_new,
                      const v4<T>* q, const v4<T>* p, v4<T>* x, v4<T>* y, PcgCtl* ctl, const double* part_pq,
                      double* part_rz, LaunchEvents ev) {
  launch_ev(k_pcg_gpass<T, false, kSpmvThreads>, Gb, kSpmvThreads, s, ev, k, npq, F, nullptr, r_old, r_new, q, p, x,
            y, ctl, part_pq, part_rz);
}

template <typename T>
void launch_pcg_gtpass(hipStream_t s, int k, int Gb, FactView F, const v4<T>* y, const v4<T>* p_old, v4<T>* p_new,
                       PcgCtl* ctl, const double* part_rz, LaunchEvents ev) {
  launch_ev(k_pcg_gtpass<T, false, kSpmvThreads>, Gb, kSpmvThreads, s, ev, k, F, y, p_old, p_new, ctl, part_rz, 0.0);
}

template void launch_pcg_fact_init<float>(hipStream_t, int, FactView, const d4*, v4<float>*, v4<float>*,
                                          v4<float>*, v4<float>*, PcgCtl*, double*, double);
template void launch_pcg_spmv_p<float>(hipStream_t, int, MatView, const v4<float>*, v4<float>*, PcgCtl*, double*,
                                       LaunchEvents);
template void launch_pcg_gpass<float>(hipStream_t, int, int, int, FactView, const v4<float>*, v4<float>*,
                                      const v4<float>*, const v4<float>*, v4<float>*, v4<float>*, PcgCtl*,
                                      const double*, double*, LaunchEvents);
template void launch_pcg_gtpass<float>(hipStream_t, int, int, FactView, const v4<float>*, const v4<float>*,
                                       v4<float>*, PcgCtl*, const double*, LaunchEvents);

template <typename T>
void launch_resid(hipStream_t s, int Gs, MatView A, const d4* b, const d4* X64, d4* R64, double* part_rr,
                  const PcgCtl* only_if_done) {
  k_resid<T><<<Gs, kThreads, 0, s>>>(A, b, X64, R64, part_rr, only_if_done);
}

template <typename T>
void launch_addcorr(hipStream_t s, int n, int, const v4<T>* x, d4* X64, const PcgCtl* only_if_done) {
  k_addcorr<T><<<blocks_for(n), kThreads, 0, s>>>(n, x, X64, only_if_done);
}

template <typename A, typename B>
__global__ __launch_bounds__(kThreads) void k_convert(const A* __restrict__ in, B* __restrict__ out, size_t count) {
  const size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < count) out[i] = (B)in[i];
}

void launch_convert(hipStream_t s, const float* in, double* out, size_t count) {
  if (count) k_convert<float, double><<<(unsigned)((count + kThreads - 1) / kThreads), kThreads, 0, s>>>(in, out, count);
}

void launch_convert(hipStream_t s, const double* in, float* out, size_t count) {
  if (count) k_convert<double, float><<<(unsigned)((count + kThreads - 1) / kThreads), kThreads, 0, s>>>(in, out, count);
}

void launch_integrate(hipStream_t s, int n, const d4* X64, d4* V, d4* U, const uint8_t* dflag, const d4* dvel,
                      double dt) {
  k_integrate<<<blocks_for(n), kThreads, 0, s>>>(n, X64, V, U, dflag, dvel, dt);
}

template <typename T>
void launch_energy(hipStream_t s, int G, int m, const int4* tets, const d4* X, const d4* U, const d4* X64,
                   double step, const T* pl, const T* chi_in, ElemConst c, double* part) {
  if (c.energy == kEnergyStVK)
    k_energy<T, kEnergyStVK><<<G, kThreads, 0, s>>>(m, tets, X, U, X64, step, pl, chi_in, c, part);
  else
    k_energy<T, kEnergyStableNeoHookean><<<G, kThreads, 0, s>>>(m, tets, X, U, X64, step, pl, chi_in, c, part);
}

void launch_dot(hipStream_t s, int G, int n, const d4* a, const d4* b, double* part) {
  k_dot<<<G, kThreads, 0, s>>>(n, a, b, part);
}

void launch_axpy(hipStream_t s, int n, double sc, const d4* x, d4* y) {
  if (n > 0) k_axpy<<<blocks_for(n), kThreads, 0, s>>>(n, sc, x, y);
}

void launch_zero(hipStream_t s, int n, d4* x) {
  if (n > 0) k_zero_d4<<<blocks_for(n), kThreads, 0, s>>>(n, x);
}

void launch_move_prescribed(hipStream_t s, int n, const uint8_t* dflag, const d4* dvel, double dt, d4* U) {
  if (n > 0) k_move_prescribed<<<blocks_for(n), kThreads, 0, s>>>(n, dflag, dvel, dt, U);
}

void launch_visual(hipStream_t s, int t0, int cnt, int m, const int4* tets, const uint8_t* swapped,
                   const int32_t* tet_edge, const uint8_t* zeta, const d4* X, const d4* U, double* xyz,
                   uint8_t* group) {
  if (cnt > 0) k_visual<<<blocks_for(cnt), kThreads, 0, s>>>(t0, cnt, m, tets, swapped, tet_edge, zeta, X, U, xyz, group);
}

#define GFEM_INST(T)                                                                                         \
  template void launch_plastic<T>(hipStream_t, int, const int4*, const d4*, const d4*, const T*, T*, double); \
  template void launch_energy<T>(hipStream_t, int, int, const int4*, const d4*, const d4*, const d4*, double, \
                                 const T*, const T*, ElemConst, double*);                                    \
  template void launch_element<T>(hipStream_t, int, const int4*, const int32_t*, const uint8_t*, const d4*,  \
                                  const d4*, const uint8_t*, const T*, const T*, T*, ElemConst,              \
                                  const int32_t*, const int32_t*, const uint16_t*, Rec<T>*, Counters*);      \
  template void launch_row<T>(hipStream_t, int, int, MatView, const int32_t*, const int32_t*, const double*, \
                              const int32_t*, const int32_t*, const Rec<T>*, double, const double*,          \
                              const d4*, const d4*, const d4*, const uint8_t*, const d4*, RowConst, T*, d4*, \
                              d4*, T*, d4*, double*);                                                        \
  template void launch_pcg_init<T>(hipStream_t, int, int, const d4*, const T*, v4<T>*, v4<T>*, v4<T>*,      \
                                   v4<T>*, double*, PcgCtl*);                                                \
  template void launch_pcg_spmv<T>(hipStream_t, int, int, int, MatView, const v4<T>*, const v4<T>*, v4<T>*, \
                                   v4<T>*, PcgCtl*, const double*, double*, double, LaunchEvents);          \
  template void launch_pcg_update<T>(hipStream_t, int, int, int, int, const v4<T>*, const v4<T>*, v4<T>*,   \
                                     v4<T>*, v4<T>*, const T*, PcgCtl*, const double*, double*,             \
                                     LaunchEvents);                                                          \
  template void launch_resid<T>(hipStream_t, int, MatView, const d4*, const d4*, d4*, double*,             \
                                const PcgCtl*);                                                              \
  template void launch_addcorr<T>(hipStream_t, int, int, const v4<T>*, d4*, const PcgCtl*);

GFEM_INST(float)
GFEM_INST(double)

}  // namespace gfem
