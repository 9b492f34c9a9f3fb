// Device kernels of the graph-based FEM step (gfx950, wave64).
//
// Data layout in HBM (internal node order):
//   node vectors   : v4<double> / v4<T> records (x, y, z, pad) -> one 32 B or 16 B load per gather
//   tets           : int4 node ids; tet_edge SoA [6][m]; flip bits [m]
//   block matrix   : BSR 3x3, values SoA [9][nbp] (component-major, so the
//                    lanes of a wave read consecutive blocks with unit stride)
//   contributions  : partial records (9 block entries in T + one FP64 force
//                    weight, 48 B in FP32), one per (element-pass workgroup,
//                    edge it touches): each workgroup sums its tets'
//                    contributions per edge in LDS first; the row pass reads
//                    whole records, about two per edge, for each of an
//                    edge's two blocks
// No floating-point atomics anywhere: every sum has a fixed order, so a step
// is bitwise reproducible.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "topo.hpp"

namespace gfem {

template <typename T>
struct alignas(4 * sizeof(T)) v4 {
  T x, y, z, w;
};
using d4 = v4<double>;

constexpr int kThreads = 256;     // 4 waves of 64
constexpr int kMaxPart = 2048;    // max workgroups that leave a reduction partial
constexpr int kRowLanes = 16;     // lanes cooperating on one block row in the row pass and the FP64 residual
#ifndef GFEM_SPMV_THREADS
#define GFEM_SPMV_THREADS 512
#endif
constexpr int kSpmvThreads = GFEM_SPMV_THREADS;  // workgroup size of the PCG SpMV and the G / G^T passes
#ifndef GFEM_SPMV_LANES
#define GFEM_SPMV_LANES 8
#endif
constexpr int kSpmvLanes = GFEM_SPMV_LANES;  // lanes per block row in the two PCG SpMV kernels (two blocks each in flight)
constexpr int kVecThreads = 256;  // workgroup size of the PCG vector kernels

struct PcgCtl {
  int done;   // set once converged or broken down; every later PCG kernel exits at entry
  int fail;   // 1: p.Ap <= 0 (operator not SPD on the Krylov space)
  int iters;  // iterations completed (x holds x_iters)
  int pad;
  double thr2;  // stopping threshold on |r|^2, set by the first SpMV of a solve
};

struct MatView {
  int n, nbp;
  const int32_t* row_ptr;
  const int32_t* col;
  const void* val;  // T[9][nbp]
};

// Event counters, spread over kCtrSlots cache-line-sized slots so that the
// per-workgroup atomics do not contend on one address; the host sums slots.
constexpr int kCtrSlots = 64;
constexpr int kCtrStride = 32;  // ints per slot (128 B)
enum CounterField { kNewBroken = 0, kTotalBroken, kNearThreshold, kChiZero, kDegenerate, kNumCounters };
struct Counters {
  int v[kCtrSlots * kCtrStride];
  int near_n;  // entries appended to the near-threshold edge list by the damage pass
};

// Element energies: the stable neo-Hookean density of Eq. 35 (reparametrised
// Lame constants) or the Saint-Venant Kirchhoff density of Eq. 37 (plain ones).
constexpr int kEnergyStableNeoHookean = 0;
constexpr int kEnergyStVK = 1;

struct ElemConst {
  double mu, lam, alpha_m1;  // Eq. 35: mu', lambda', alpha - 1; Eq. 37: mu, lambda, unused
  int energy;                // kEnergyStableNeoHookean or kEnergyStVK
};

// Per tet edge contribution: the 3x3 stiffness block in global orientation
// and the force weight 2 V chi dPsi/ds_k (FP64: on nearly flat tets the
// weights of the volume term grow as 1/J while their sum along the edges
// stays finite).
template <typename T>
struct alignas(16) Rec {
  T b[9];
  double w;
};

// 64-bit table: bit `mask` set when that broken-edge mask leaves the tet's
// unbroken edges disconnected (chi = 0).  Uploaded once per process.
void set_disconnected_lut(unsigned long long lut);

// Launch helpers (defined in kernels.hip).  All are asynchronous on `s`.
// near_ids (capacity ne): internal ids of the edges with |strain - thr| < 1e-6,
// in no particular order, count in ctr->near_n.
void launch_damage(hipStream_t s, int ne, const int2* edges, const d4* X, const d4* U,
                   const double* S, const uint8_t* z_in, uint8_t* z_out, double thr,
                   Counters* ctr, int32_t* near_ids);

// Non-local damage criterion (Sec. 3.3, Eq. 20, support R_d > 0): per-tet
// Green strain tensors E = (F^T F - I)/2 from the displacement (FP64, entries
// 00,11,22,01,02,12), their weighted averages over each tet's support (CSR
// nl_ptr/nl_idx/nl_w, built once on the host), then per edge the largest
// averaged normal strain q^T E* q (q the rest edge direction) over the tets
// that contain it: zeta <- zeta OR (that strain >= thr); labels, counters and
// the near-threshold list as launch_damage (near: within 1e-6 in any of those
// tets).  E and Eavg are work buffers of m records.
struct alignas(16) Sym6 {
  double v[6];
};
void launch_damage_nonlocal(hipStream_t s, int m, int ne, const int4* tets, const d4* X, const d4* U,
                            const int64_t* nl_ptr, const int32_t* nl_idx, const double* nl_w, Sym6* E,
                            Sym6* Eavg, const int2* edges, const int32_t* edge_ptr, const int32_t* edge_slot,
                            const uint8_t* z_in, uint8_t* z_out, double thr, Counters* ctr, int32_t* near_ids,
                            int64_t n_entries);

// Plastic flow of the ductile workload: pl_in -> pl_out, each [6][m] plastic
// rest-shape offsets Gp - G0 (symmetric 00,11,22,01,02,12).
template <typename T>
void launch_plastic(hipStream_t s, int m, const int4* tets, const d4* X, const d4* U, const T* pl_in, T* pl_out,
                    double yield);

// pl: plastic rest-shape offsets [6][m], or null.  chi_in (nullable): per-tet
// energy fractions to use instead of evaluating Eq. 25; chi_out (nullable):
// receives the fractions used.  kElemTets tets per workgroup; each
// workgroup sums its tets' records per edge in LDS and writes one partial
// record per edge it touches (part_* tables of the topology) into contrib.
template <typename T>
void launch_element(hipStream_t s, int m, const int4* tets, const int32_t* tet_edge,
                    const uint8_t* flip, const d4* X, const d4* U, const uint8_t* zeta,
                    const T* pl, const T* chi_in, T* chi_out, ElemConst c, const int32_t* part_base,
                    const int32_t* part_cptr, const uint16_t* part_slot, Rec<T>* contrib, Counters* ctr);

// Split visualisation mesh (Sec. 4.1) of tets t0 .. t0 + cnt - 1: per tet and
// caller-order corner a the 8 sub-cell vertices (FP64 x, y, z) [corner, edge
// points towards the other corners b1 < b2 < b3, face points (b1,b2), (b1,b3),
// (b2,b3), tet point] into xyz[(t - t0) * 96 ..], and the smallest corner
// index connected to a through unbroken edges into group[(t - t0) * 4 + a].
// A split point's child for a sits at its rest position plus the mean
// displacement of the corners that unbroken edges join to a within that
// edge, face or tet.  swapped[t]: local nodes 2 and 3 were exchanged.
void launch_visual(hipStream_t s, int t0, int cnt, int m, const int4* tets, const uint8_t* swapped,
                   const int32_t* tet_edge, const uint8_t* zeta, const d4* X, const d4* U, double* xyz,
                   uint8_t* group);

// Quasi-static Newton (Eq. 36) helpers.
// Total energy sum_e chi_e V_e Psi_e at the displacement U + s X64 (FP64),
// chi held fixed (chi_in[m]); per-workgroup partials into part[G], G <= kMaxPart.
template <typename T>
void launch_energy(hipStream_t s, int G, int m, const int4* tets, const d4* X, const d4* U, const d4* X64,
                   double step, const T* pl, const T* chi_in, ElemConst c, double* part);
// Partials of a.b over the node records into part[G].
void launch_dot(hipStream_t s, int G, int n, const d4* a, const d4* b, double* part);
// y += s x over the node records (x, y: d4[n]).
void launch_axpy(hipStream_t s, int n, double sc, const d4* x, d4* y);
// x = 0 over the node records (x: d4[n]).
void launch_zero(hipStream_t s, int n, d4* x);
// U += dt * dvel on the prescribed nodes (dflag != 0).
void launch_move_prescribed(hipStream_t s, int n, const uint8_t* dflag, const d4* dvel, double dt, d4* U);

struct RowConst {
  double dt, ra;      // dt, Rayleigh alpha
  double mass_fac;    // 1 + dt * alpha
  double g[3];
};

template <typename T>
void launch_row(hipStream_t s, int n, int G, MatView A, const int32_t* diag_blk,
                const int32_t* blk_edge, const double* edge_mass, const int32_t* edge_pptr,
                const int32_t* edge_part, const Rec<T>* contrib, double stiff_fac,
                const double* lumped, const d4* X, const d4* U, const d4* V,
                const uint8_t* dflag, const d4* dvel, RowConst c, T* val_mut, d4* b,
                d4* X64, T* binv, d4* f_out, double* part_bb);

// Optional start/stop events recorded by the dispatch itself (kernel execution
// time only, as a profiler reports it); null events: plain launch.
struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};

// Ga: workgroups (kVecThreads each) of the vector kernels; Gb: workgroups
// (kSpmvThreads each) of the SpMV.  Both multiples of 8.  rel2: squared relative
// reduction of |r| the solve must reach (threshold = rel2 |r_0|^2).
template <typename T>
void launch_pcg_init(hipStream_t s, int n, int Ga, const d4* src, const T* binv, v4<T>* r, v4<T>* z,
                     v4<T>* p0, v4<T>* x, double* part_rz, PcgCtl* ctl);

template <typename T>
void launch_pcg_spmv(hipStream_t s, int k, int Gb, int Ga, MatView A, const v4<T>* z, const v4<T>* p_old,
                     v4<T>* p_new, v4<T>* q, PcgCtl* ctl, const double* part_rz, double* part_pq,
                     double rel2, LaunchEvents ev = {});

template <typename T>
void launch_pcg_update(hipStream_t s, int k, int n, int Ga, int Gb, const v4<T>* p, const v4<T>* q,
                       v4<T>* x, v4<T>* r, v4<T>* z, const T* binv, PcgCtl* ctl, const double* part_pq,
                       double* part_rz, LaunchEvents ev = {});

// Factorised sparse approximate inverse preconditioner z = G^T G r, G block
// lower triangular on the lower block pattern of A (node order).  BF16 block
// values in compact half-pattern arrays, one 16-byte record (entries 0-7,
// row-major 3x3) plus one BF16 (entry 8) per block, unit stride across blocks:
// glv/gl8 [ne] hold G_ij of the strictly lower blocks in the order of lcol
// (row i: lptr[i] .. lptr[i+1]), guv/gu8 [ne] hold G_ji^T at the mirror
// positions in the order of ucol, and gdv [n] the lower-triangular diagonal
// blocks G_ii (entries 00, 10, 11, 20, 21, 22, then two zero pads).  G r
// streams the lower arrays and G^T y the upper ones, each once.
struct FactView {
  int n, ne;
  const int32_t* lptr;
  const int32_t* lcol;
  const int32_t* uptr;
  const int32_t* ucol;
  const uint4* glv;
  const __bf16* gl8;
  const uint4* guv;
  const __bf16* gu8;
  const uint4* gdv;
};
#ifndef GFEM_FACT_LANES
#define GFEM_FACT_LANES 4
#endif
constexpr int kFactLanes = GFEM_FACT_LANES;  // lanes cooperating on one half row in the G and G^T passes

// Factorised-preconditioner PCG, three kernels per iteration (G and G^T
// passes on Gb workgroups of kSpmvThreads, the SpMV on its own grid of Gp,
// whose p.q partials the G pass reduces):
//   start:  control block reset, r_0 = src (rounded to T), x = 0, y = G r_0,
//           partials y.y (= r.z) and r.r; then threshold thr2 = rel2 |r_0|^2,
//           p_0 = G^T y.
//   k:      SpMV q = A p_k, partial p.q;
//           G pass: alpha = r.z / p.q, x += alpha p_k, r_{k+1} = r_k - alpha q,
//           y = G r_{k+1}, partials for k + 1;
//           G^T pass: stop if |r_{k+1}|^2 <= thr2, else
//           p_{k+1} = G^T y + beta p_k.
template <typename T>
void launch_pcg_fact_init(hipStream_t s, int Gb, FactView F, const d4* src, v4<T>* r0, v4<T>* x, v4<T>* y,
                          v4<T>* p0, PcgCtl* ctl, double* part_rz, double rel2);
template <typename T>
void launch_pcg_spmv_p(hipStream_t s, int Gp, MatView A, const v4<T>* p, v4<T>* q, PcgCtl* ctl, double* part_pq,
                       LaunchEvents ev = {});
template <typename T>
void launch_pcg_gpass(hipStream_t s, int k, int Gb, int npq, FactView F, const v4<T>* r_old, v4<T>* r_new,
                      const v4<T>* q, const v4<T>* p, v4<T>* x, v4<T>* y, PcgCtl* ctl, const double* part_pq,
                      double* part_rz, LaunchEvents ev = {});
template <typename T>
void launch_pcg_gtpass(hipStream_t s, int k, int Gb, FactView F, const v4<T>* y, const v4<T>* p_old,
                       v4<T>* p_new, PcgCtl* ctl, const double* part_rz, LaunchEvents ev = {});

// only_if_done (nullable): the kernel does nothing unless that PCG control
// block reports convergence, so it can be queued behind a launch chunk.
template <typename T>
void launch_resid(hipStream_t s, int Gs, MatView A, const d4* b, const d4* X64, d4* R64,
                  double* part_rr, const PcgCtl* only_if_done = nullptr);

template <typename T>
void launch_addcorr(hipStream_t s, int n, int G, const v4<T>* x, d4* X64, const PcgCtl* only_if_done = nullptr);

// Elementwise precision conversion of count values.
void launch_convert(hipStream_t s, const float* in, double* out, size_t count);
void launch_convert(hipStream_t s, const double* in, float* out, size_t count);

void launch_integrate(hipStream_t s, int n, const d4* X64, d4* V, d4* U, const uint8_t* dflag,
                      const d4* dvel, double dt);

}  // namespace gfem
