// C ABI of the graph-based FEM fracture library (include/gfem.h): device
// buffers, the per-step kernel sequence and the iterative-refinement PCG
// driver.  Citations are to Mandal, Chaudhuri & Chaudhuri, "Remeshing-Free
// Graph-Based Finite Element Method for Ductile and Brittle Fracture".
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <memory>
#include <mutex>
#include <new>
#include <random>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/gfem.h"
#include "kernels.hpp"
#include "net.hpp"
#include "topo.hpp"

using gfem::d4;
using gfem::v4;

namespace {

thread_local std::string g_err;

gf_status fail(gf_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

struct HipError {
  hipError_t e;
  const char* what;
};

inline void hchk(hipError_t e, const char* what) {
  if (e != hipSuccess) throw HipError{e, what};
}

struct Alloc {
  std::vector<void*> ptrs;
  template <typename P>
  P* get(size_t count) {
    void* p = nullptr;
    size_t bytes = std::max<size_t>(count * sizeof(P), 256);
    if (hipMalloc(&p, bytes) != hipSuccess) throw std::bad_alloc();
    hchk(hipMemset(p, 0, bytes), "hipMemset");
    ptrs.push_back(p);
    return static_cast<P*>(p);
  }
  ~Alloc() {
    for (void* p : ptrs) (void)hipFree(p);
  }
};

// Disconnected-mask table, built here by union-find over the tet's six edges
// (independently of any other implementation).
unsigned long long disconnected_lut() {
  unsigned long long lut = 0;
  for (int mask = 0; mask < 64; ++mask) {
    int parent[4] = {0, 1, 2, 3};
    auto find = [&](int a) {
      while (parent[a] != a) a = parent[a];
      return a;
    };
    for (int k = 0; k < 6; ++k)
      if (!((mask >> k) & 1)) parent[find(gfem::kEdgeA[k])] = find(gfem::kEdgeB[k]);
    int roots = 0;
    for (int a = 0; a < 4; ++a) roots += find(a) == a;
    if (roots > 1) lut |= 1ull << mask;
  }
  return lut;
}

struct TimeRec {
  int cat;
  int solve;  // PCG solve index, -1 outside PCG
  int k;      // iteration index inside the solve
  hipEvent_t a, b;
};

int round_up8(int x) { return (x + 7) / 8 * 8; }

// Grid cap of the PCG SpMV and G / G^T passes (their FP64 partials are
// reduced by every workgroup of the consumer kernel).  Measured on the
// 619,830-tet ellipsoid (threads per workgroup x cap, learned steps/s):
// 256 x 1024: 282, 512 x 512: 295, 1024 x 256: 290, 512 x 1024: 260,
// 512 x 256: 269, 384 x 512: 282, 768 x 256: 284 -- half the partials of
// 256 x 1024 at the same four waves per SIMD.
// Launch chunks of a PCG solve: the first covers the previous step's count for
// the same outer pass plus GFEM_CHUNK_MARGIN iterations, further ones
// GFEM_CHUNK_NEXT iterations each.
#ifndef GFEM_CHUNK_MARGIN
#define GFEM_CHUNK_MARGIN 0
#endif
#ifndef GFEM_CHUNK_NEXT
#define GFEM_CHUNK_NEXT 3
#endif

#ifndef GFEM_PCG_MAX_WG
#define GFEM_PCG_MAX_WG 512
#endif
constexpr int kPcgMaxWorkgroups = GFEM_PCG_MAX_WG;
// Below the cap, the grid gives each workgroup about this many block rows: on
// the 23,409-node notched beam 96 rows (248 workgroups) beat 46 (512, the cap):
// 233-235 against 214-215 learned steps/s uncracked, 227-236 against 207-210
// with 30 % pre-broken edges; 183 rows (128 workgroups) lose (186-205).  The
// 111,912-node ellipsoid stays at the cap either way.
#ifndef GFEM_PCG_ROWS_PER_WG
#define GFEM_PCG_ROWS_PER_WG 96
#endif
constexpr int kPcgRowsPerWorkgroup = GFEM_PCG_ROWS_PER_WG;

// Each inner (working-precision) PCG solve aims at this fraction of the
// outer FP64 tolerance relative to its right-hand side.  It must stay below 1
// (the last pass then ends below the tolerance); measured on the 619,830-tet
// ellipsoid (learned steps/s, two outer passes at every value): 0.5: 312,
// 0.7: 321, 0.8: 324, 0.9: 327.5 -- the second pass starts from the FP64
// residual either way, so the first one need not go further; 0.8 keeps a
// margin for the drift of the FP32 recursive residual.
#ifndef GFEM_INNER_TOL
#define GFEM_INNER_TOL 0.8
#endif
static_assert(GFEM_INNER_TOL > 0.0 && GFEM_INNER_TOL < 1.0, "inner tolerance factor in (0, 1)");
// First pass of a split-precision solve: its target relative to the outer
// tolerance.  It may lie above 1, since a second pass (at GFEM_INNER_TOL)
// follows anyway: the FP32 recursive residual of the first pass drifts from
// the FP64 one by about the tolerance, so iterations below that level do not
// lower the true residual.  Measured on the 619,830-tet ellipsoid (learned
// steps/s, with 0.8 for the last pass): 0.8: 342.7, 1.2: 348.1, 2.0: 341.7,
// 4.0: 342.4; 1.2 also gains 2-5 % on the notched beams.
#ifndef GFEM_INNER_TOL_FIRST
#define GFEM_INNER_TOL_FIRST 1.2
#endif
constexpr double kInnerTol = GFEM_INNER_TOL;

}  // namespace

struct gf_net {
  int dev = 0;
  Alloc al;
  gfem::NetParamsDev P;
  std::vector<float> host;  // master weights (host copy, kept in sync)
  int adam_t = 0;
  uint64_t seed = 0;
  int power_steps = 0;  // power steps on X = G A G^T applied to the training probe
};

struct gf_mesh {
  gfem::Topology topo;
  gf_params p{};
  bool split = false;
  bool plastic = false;
  int dev = 0;
  hipStream_t own = nullptr, stream = nullptr;
  int n = 0, m = 0, ne = 0, nb = 0, nbp = 0, Gv = 8, Gs = 8, Ga = 8, Gb = 8, Gp = 8, Gn = 8;
  double mu = 0, lam = 0, alpha_m1 = 0;
  Alloc al;
  // node data
  d4 *X = nullptr, *U = nullptr, *V = nullptr, *dvel = nullptr, *b = nullptr, *X64 = nullptr, *R64 = nullptr,
     *fbuf = nullptr;
  uint8_t* dflag = nullptr;
  double* lumped = nullptr;
  // tets
  int4* tets = nullptr;
  int32_t* tet_edge = nullptr;
  uint8_t* flip = nullptr;
  void* pl[2] = {nullptr, nullptr};
  int plcur = 0;
  void* contrib = nullptr;
  // edges
  int2* edges = nullptr;
  double *edge_S = nullptr, *edge_mass = nullptr;
  uint8_t* zeta[2] = {nullptr, nullptr};
  int zcur = 0;
  int32_t* near_ids = nullptr;  // near-threshold edges of the last damage pass (internal ids)
  // non-local damage criterion (R_d > 0): support CSR and two strain buffers
  int64_t* nl_ptr = nullptr;
  int32_t* nl_idx = nullptr;
  double* nl_w = nullptr;
  gfem::Sym6 *nl_E = nullptr, *nl_Eavg = nullptr;
  size_t nl_entries = 0;
  // quasi-static load steps: zero node vector, chi held fixed, displacement at the step's start
  d4 *qs_zero = nullptr, *qs_U0 = nullptr;
  void* qs_chi = nullptr;
  // split visualisation mesh (built on first use, in chunks of tets)
  uint8_t* tet_swapped = nullptr;
  double* vis_xyz = nullptr;
  uint8_t* vis_group = nullptr;
  int32_t *edge_ptr = nullptr, *edge_slot = nullptr;
  // workgroup-staged assembly tables (topo.hpp) and the number of partial records
  int32_t *part_base = nullptr, *part_cptr = nullptr, *edge_pptr = nullptr, *edge_part = nullptr;
  uint16_t* part_slot = nullptr;
  int np = 0;
  // block matrix
  int32_t *row_ptr = nullptr, *col = nullptr, *diag_blk = nullptr, *blk_edge = nullptr;
  int32_t *lptr = nullptr, *lcol = nullptr, *uptr = nullptr, *ucol = nullptr, *upos = nullptr;
  void* val = nullptr;
  void* binv = nullptr;
  // PCG
  void *vr = nullptr, *vz = nullptr, *vp[2] = {nullptr, nullptr}, *vq = nullptr, *vx = nullptr;
  void *vr2 = nullptr, *vy = nullptr;  // second residual buffer and G r (factorised preconditioner)
  // FP64 copies of the precision-typed buffers of a split-precision mesh, for
  // steps re-run in FP64 (allocated on first use; swapped in for that step)
  struct PrecBufs {
    void *val, *contrib, *binv, *pl[2], *vr, *vz, *vp[2], *vq, *vx, *vr2, *vy;
  };
  bool esc_ready = false;
  PrecBufs esc{};
  PrecBufs cur() const { return PrecBufs{val, contrib, binv, {pl[0], pl[1]}, vr, vz, {vp[0], vp[1]}, vq, vx, vr2, vy}; }
  void use(const PrecBufs& b) {
    val = b.val; contrib = b.contrib; binv = b.binv; pl[0] = b.pl[0]; pl[1] = b.pl[1];
    vr = b.vr; vz = b.vz; vp[0] = b.vp[0]; vp[1] = b.vp[1]; vq = b.vq; vx = b.vx; vr2 = b.vr2; vy = b.vy;
  }
  double *part_a = nullptr, *part_rz = nullptr, *part_pq = nullptr, *part_r = nullptr;
  gfem::PcgCtl* ctl = nullptr;
  gfem::Counters* ctr = nullptr;
  // host side
  double* h_part = nullptr;          // pinned, 2 x kMaxPart
  gfem::PcgCtl* h_ctl = nullptr;     // pinned
  gfem::Counters* h_ctr = nullptr;   // pinned
  std::vector<uint8_t> h_dflag;
  std::vector<d4> h_dvel;
  int step_index = 0;
  // inner iterations of each outer solve of the last step, per solve kind
  // (0 working precision block-Jacobi, 1 learned factor, 2 FP64 re-run)
  int last_solve_iters[3][4] = {};
  int last_learned_iters = 0;  // inner iterations of the last accepted learned solve
  int learned_skip = 0;        // steps left that use block-Jacobi directly after a rejected learned solve
  int learned_backoff = 4;     // length of the next such pause (doubles per rejection, up to 64)
  bool timing = false;
  bool force_fp64 = false;  // test hook: re-run every split step in FP64
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<TimeRec> recs;
  std::vector<int> solve_iters;
  // learned preconditioner
  gf_net* net = nullptr;
  int precond = GF_PC_BLOCK_JACOBI;
  bool netw_ready = false, net_train_ready = false, net_cached = false;
  bool fact_norm = false;                 // row normalisation of the learned factor
  int32_t* norm_ptr = nullptr;            // per-row pattern pairs for it (built on first use)
  int4* norm_pairs = nullptr;
  int net_age = 0;
  double inv_mean_len = 1.0;
  gfem::NetWork netw;

  ~gf_mesh() {
    if (stream) (void)hipStreamSynchronize(stream);
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    if (h_part) (void)hipHostFree(h_part);
    if (h_ctl) (void)hipHostFree(h_ctl);
    if (h_ctr) (void)hipHostFree(h_ctr);
    if (own) (void)hipStreamDestroy(own);
  }

  gfem::MatView mat() const { return gfem::MatView{n, nbp, row_ptr, col, val}; }

  hipEvent_t ev() {
    if (ev_used == ev_pool.size()) {
      hipEvent_t e;
      hchk(hipEventCreate(&e), "hipEventCreate");
      ev_pool.push_back(e);
    }
    return ev_pool[ev_used++];
  }
  // Timing with events recorded by the dispatch itself (kernel execution only):
  // launch(LaunchEvents) receives the events, or null events when timing is off.
  template <typename F>
  void timed_ev(int cat, int solve, int k, F&& launch) {
    if (!timing) {
      launch(gfem::LaunchEvents{});
      return;
    }
    TimeRec r{cat, solve, k, ev(), ev()};
    launch(gfem::LaunchEvents{r.a, r.b});
    recs.push_back(r);
  }
  // Records events around one launch when timing is on.
  template <typename F>
  void timed(int cat, int solve, int k, F&& launch) {
    if (!timing) {
      launch();
      return;
    }
    TimeRec r{cat, solve, k, ev(), ev()};
    hchk(hipEventRecord(r.a, stream), "hipEventRecord");
    launch();
    hchk(hipEventRecord(r.b, stream), "hipEventRecord");
    recs.push_back(r);
  }
  void flush_times(gf_step_stats* st) {
    if (!timing) return;
    for (const TimeRec& r : recs) {
      if (r.solve >= 0 && (r.solve >= (int)solve_iters.size() || r.k >= solve_iters[r.solve])) continue;
      float ms = 0;
      hchk(hipEventElapsedTime(&ms, r.a, r.b), "hipEventElapsedTime");
      if (st) {
        st->kernel_us[r.cat] += 1000.0 * ms;
        st->n_launch[r.cat] += 1;
      }
    }
    recs.clear();
    ev_used = 0;
    solve_iters.clear();
  }
  void sync() { hchk(hipStreamSynchronize(stream), "hipStreamSynchronize"); }
  void check_launch() { hchk(hipGetLastError(), "kernel launch"); }
};

namespace {

using gfem::kMaxPart;
constexpr int kMaxPowerSteps = 64;

// Upload host vector to a fresh device buffer.
template <typename P>
P* upload(gf_mesh* M, const std::vector<P>& h) {
  P* d = M->al.get<P>(h.size());
  if (!h.empty()) hchk(hipMemcpy(d, h.data(), h.size() * sizeof(P), hipMemcpyHostToDevice), "hipMemcpy H2D");
  return d;
}

template <typename T>
void alloc_precision(gf_mesh* M) {
  const int n = M->n, m = M->m;
  M->val = M->al.get<T>((size_t)9 * M->nbp);
  M->contrib = M->al.get<gfem::Rec<T>>((size_t)M->np);
  M->binv = M->al.get<T>((size_t)6 * n);
  if (M->plastic) {
    M->pl[0] = M->al.get<T>((size_t)6 * m);
    M->pl[1] = M->al.get<T>((size_t)6 * m);
  }
  M->vr = M->al.get<v4<T>>(n);
  M->vz = M->al.get<v4<T>>(n);
  M->vp[0] = M->al.get<v4<T>>(n);
  M->vp[1] = M->al.get<v4<T>>(n);
  M->vq = M->al.get<v4<T>>(n);
  M->vx = M->al.get<v4<T>>(n);
  M->vr2 = M->al.get<v4<T>>(n);
  M->vy = M->al.get<v4<T>>(n);
}

// Damage pass at the current displacement: counters reset, labels of the
// current buffer OR-ed with the new breaks into the spare one (Eq. 20-21,
// local or non-local support), near-threshold edges listed.
void damage_pass(gf_mesh* M) {
  hipStream_t s = M->stream;
  const int zi = M->zcur, zo = 1 - M->zcur;
  hchk(hipMemsetAsync(M->ctr, 0, sizeof(gfem::Counters), s), "hipMemsetAsync");
  if (M->nl_ptr)
    gfem::launch_damage_nonlocal(s, M->m, M->ne, M->tets, M->X, M->U, M->nl_ptr, M->nl_idx, M->nl_w, M->nl_E,
                                 M->nl_Eavg, M->edges, M->edge_ptr, M->edge_slot, M->zeta[zi], M->zeta[zo],
                                 M->p.damage_strain, M->ctr, M->near_ids, (int64_t)M->nl_entries);
  else
    gfem::launch_damage(s, M->ne, M->edges, M->X, M->U, M->edge_S, M->zeta[zi], M->zeta[zo], M->p.damage_strain,
                        M->ctr, M->near_ids);
}

// What one assembly does (defaults: a timestep's system).
struct AsmOpt {
  bool damage = true;      // damage pass into the spare label buffer (counters reset first)
  bool flow = true;        // plastic flow at the current state into the spare plastic buffer
  bool next_state = true;  // the element pass reads the spare (updated) labels and plastic state
  const void* chi_in = nullptr;  // per-tet chi held fixed (T[m]) instead of Eq. 25
  void* chi_out = nullptr;       // receives the chi used (T[m])
  bool quasi_static = false;     // zero velocities and prescribed velocities, no damping or gravity
  const d4* zero = nullptr;      // quasi-static: a zero node vector (n records)
  d4* f_out = nullptr;           // restoring forces, when wanted
};

// Damage (into the spare label buffer), element pass (+ plastic flow into the
// spare plastic buffer) and row pass (assembly): the system of the next step.
template <typename T>
void assemble(gf_mesh* M, const AsmOpt& o) {
  hipStream_t s = M->stream;
  const bool flow = o.flow;
  d4* f_out = o.f_out;
  const int zi = M->zcur, zo = 1 - M->zcur;
  if (o.damage) M->timed(0, -1, 0, [&] { damage_pass(M); });
  gfem::ElemConst ec{M->mu, M->lam, M->alpha_m1, M->p.energy};
  const T* pl = nullptr;
  if (M->plastic) {
    if (flow) {
      // plastic flow at x_n into the spare buffer, which the element pass reads
      M->timed(1, -1, 0, [&] {
        gfem::launch_plastic<T>(s, M->m, M->tets, M->X, M->U, static_cast<const T*>(M->pl[M->plcur]),
                                static_cast<T*>(M->pl[1 - M->plcur]), M->p.yield_strain);
      });
    }
    pl = static_cast<const T*>(M->pl[o.next_state ? 1 - M->plcur : M->plcur]);
  }
  M->timed(1, -1, 0, [&] {
    gfem::launch_element<T>(s, M->m, M->tets, M->tet_edge, M->flip, M->X, M->U, M->zeta[o.next_state ? zo : zi], pl,
                            static_cast<const T*>(o.chi_in), static_cast<T*>(o.chi_out), ec, M->part_base,
                            M->part_cptr, M->part_slot, static_cast<gfem::Rec<T>*>(M->contrib), M->ctr);
  });
  const double dt = M->p.dt;
  const double ra = o.quasi_static ? 0.0 : M->p.rayleigh_alpha;
  const double mass_fac = 1.0 + dt * ra;
  const double stiff_fac = dt * dt + (o.quasi_static ? 0.0 : dt * M->p.rayleigh_beta);
  gfem::RowConst rc{dt, ra, mass_fac, {M->p.gravity[0], M->p.gravity[1], M->p.gravity[2]}};
  if (o.quasi_static) rc.g[0] = rc.g[1] = rc.g[2] = 0.0;
  const d4* V = o.quasi_static ? o.zero : M->V;
  const d4* dvel = o.quasi_static ? o.zero : M->dvel;
  M->timed(2, -1, 0, [&] {
    gfem::launch_row<T>(s, M->n, M->Gs, M->mat(), M->diag_blk, M->blk_edge, M->edge_mass, M->edge_pptr,
                        M->edge_part, static_cast<const gfem::Rec<T>*>(M->contrib), stiff_fac, M->lumped, M->X, M->U,
                        V, M->dflag, dvel, rc,
                        static_cast<T*>(M->val), M->b, M->X64, static_cast<T*>(M->binv), f_out, M->part_a);
  });
  M->check_launch();
}

double read_partials(gf_mesh* M, const double* dpart, int count) {
  double s = 0;
  for (int c0 = 0; c0 < count; c0 += kMaxPart) {
    const int c = std::min(kMaxPart, count - c0);
    hchk(hipMemcpyAsync(M->h_part, dpart + c0, sizeof(double) * c, hipMemcpyDeviceToHost, M->stream), "D2H");
    M->sync();
    for (int i = 0; i < c; ++i) s += M->h_part[i];
  }
  return s;
}

struct SolveResult {
  bool ok;
  int inner, outer;
  double rel;
};

// Mixed-precision iterative refinement around block-Jacobi PCG.  Outer loop
// in FP64: R = b - A X64 until |R| <= tol |b|; inner PCG on A d = R with T
// vectors, FP64 dot products, device-side scalars and early exit, launched in
// chunks so the host only synchronises once per chunk.
template <typename T>
SolveResult solve(gf_mesh* M, const void* precond_blocks, const gfem::FactView* F = nullptr, int max_inner = 0,
                  int kind = 0) {
  hipStream_t s = M->stream;
  const double tol = M->p.cg_rel_tol;
  SolveResult res{false, 0, 0, 0.0};
  const double floor_rel = M->split ? 1e-7 : 0.0;
  double bb = -1.0, rr = -1.0;  // |b|^2 is read back with the first chunk
  double rr_prev = 0.0;
  const d4* src = M->b;
  int budget = std::max(1, (int)M->p.cg_max_iter);
  if (max_inner > 0) budget = std::min(budget, max_inner);
  const gfem::MatView A = M->mat();
  v4<T>* r = static_cast<v4<T>*>(M->vr);
  v4<T>* z = static_cast<v4<T>*>(M->vz);
  v4<T>* q = static_cast<v4<T>*>(M->vq);
  v4<T>* x = static_cast<v4<T>*>(M->vx);
  v4<T>* pb[2] = {static_cast<v4<T>*>(M->vp[0]), static_cast<v4<T>*>(M->vp[1])};
  v4<T>* rb[2] = {r, static_cast<v4<T>*>(M->vr2)};
  v4<T>* y = static_cast<v4<T>*>(M->vy);
  const T* binv = static_cast<const T*>(precond_blocks);
  // factorised preconditioner (split precision only): the G pass replaces the
  // vector update and writes Gb partials, which the SpMV then reduces
  constexpr bool kFloat = std::is_same<T, float>::value;
  const bool fact = kFloat && F != nullptr;
  const int nrz = fact ? M->Gb : M->Ga;
  for (int outer = 0;; ++outer) {
    if (outer > 0) {
      res.rel = bb > 0 ? std::sqrt(rr / bb) : 0.0;
      if (res.rel <= tol || bb == 0.0) {
        res.ok = std::isfinite(bb);
        break;
      }
      if (outer >= 30 || res.inner >= budget || !std::isfinite(rr)) break;
    }
    const double first = M->split ? (double)GFEM_INNER_TOL_FIRST : kInnerTol;
    const double rel_in = outer == 0 ? std::max(first * tol, floor_rel)
                                     : std::max(kInnerTol * tol * std::sqrt(bb / rr), floor_rel);
    const int solve_id = (int)M->solve_iters.size();
    // (the control block is reset by the solve's first kernel)
    M->timed(5, -1, 0, [&] {
      if constexpr (kFloat) {
        if (fact) {
          gfem::launch_pcg_fact_init<float>(s, M->Gb, *F, src, rb[0], x, y, pb[0], M->ctl, M->part_rz,
                                            rel_in * rel_in);
          return;
        }
      }
      gfem::launch_pcg_init<T>(s, M->n, M->Ga, src, binv, r, z, pb[0], x, M->part_rz, M->ctl);
    });
    const int left = budget - res.inner;
    int k = 0;
    // The first chunk covers the iteration count of the same outer solve in the
    // previous step; further chunks are short.  A launch after convergence
    // exits at entry but still costs the dispatch latency (~9 us per kernel on
    // MI355X, ~30 us per iteration), about as much as one extra host
    // synchronisation, so the prediction carries no margin.
    const int slot = std::min(outer, 3);
    int* hist = M->last_solve_iters[kind];
    int chunk = hist[slot] > 0 ? hist[slot] + GFEM_CHUNK_MARGIN : (outer == 0 ? 16 : 8);
    chunk = std::max(1, std::min(chunk, left));
    int iters = 0;
    bool failed = false, converged_flag = false;
    while (true) {
      const int kend = std::min(k + chunk, left);
      for (; k < kend; ++k) {
        if constexpr (kFloat) {
          if (fact) {
            M->timed_ev(4, solve_id, k, [&](gfem::LaunchEvents e) {
              gfem::launch_pcg_spmv_p<float>(s, M->Gp, A, pb[k & 1], q, M->ctl, M->part_pq, e);
            });
            M->timed_ev(5, solve_id, k, [&](gfem::LaunchEvents e) {
              gfem::launch_pcg_gpass<float>(s, k, M->Gb, M->Gp, *F, rb[k & 1], rb[(k + 1) & 1], q, pb[k & 1], x, y,
                                            M->ctl, M->part_pq, M->part_rz, e);
            });
            M->timed_ev(8, solve_id, k, [&](gfem::LaunchEvents e) {
              gfem::launch_pcg_gtpass<float>(s, k, M->Gb, *F, y, pb[k & 1], pb[(k + 1) & 1], M->ctl, M->part_rz, e);
            });
            continue;
          }
        }
        M->timed_ev(4, solve_id, k, [&](gfem::LaunchEvents e) {
          gfem::launch_pcg_spmv<T>(s, k, M->Gb, nrz, A, z, pb[(k + 1) & 1], pb[k & 1], q, M->ctl, M->part_rz,
                                   M->part_pq, rel_in * rel_in, e);
        });
        M->timed_ev(5, solve_id, k, [&](gfem::LaunchEvents e) {
          gfem::launch_pcg_update<T>(s, k, M->n, M->Ga, M->Gb, pb[k & 1], q, x, r, z, binv, M->ctl, M->part_pq,
                                     M->part_rz, e);
        });
      }
      // queued behind the chunk, effective only once the solve has converged:
      // the FP64 correction dv += x and the FP64 residual, read back with the
      // control block by the same synchronisation
      M->timed(6, -1, 0, [&] { gfem::launch_addcorr<T>(s, M->n, M->Gv, x, M->X64, M->ctl); });
      M->timed(6, -1, 0, [&] { gfem::launch_resid<T>(s, M->Gs, A, M->b, M->X64, M->R64, M->part_r, M->ctl); });
      M->check_launch();
      hchk(hipMemcpyAsync(M->h_ctl, M->ctl, sizeof(gfem::PcgCtl), hipMemcpyDeviceToHost, s), "D2H");
      if (bb < 0.0)
        hchk(hipMemcpyAsync(M->h_part, M->part_a, sizeof(double) * M->Gs, hipMemcpyDeviceToHost, s), "D2H");
      hchk(hipMemcpyAsync(M->h_part + kMaxPart, M->part_r, sizeof(double) * M->Gs, hipMemcpyDeviceToHost, s),
           "D2H");
      M->sync();
      if (bb < 0.0) {
        bb = 0.0;
        for (int i = 0; i < M->Gs; ++i) bb += M->h_part[i];
        rr = bb;
      }
      iters = M->h_ctl->iters;
      failed = M->h_ctl->fail != 0;
      converged_flag = M->h_ctl->done != 0;
      if (converged_flag || k >= left || bb == 0.0) break;
      chunk = GFEM_CHUNK_NEXT;
    }
    M->solve_iters.push_back(iters);
    hist[slot] = iters;
    res.inner += iters;
    res.outer = outer + 1;
    if (bb == 0.0) {  // b = 0: dv = 0 (X64 was zeroed by the row pass)
      res.ok = true;
      res.rel = 0.0;
      break;
    }
    if (converged_flag) {
      // correction and residual were applied behind the last chunk
      rr = 0;
      for (int i = 0; i < M->Gs; ++i) rr += M->h_part[kMaxPart + i];
    } else {
      // iteration budget exhausted without the flag: apply what was reached
      if (iters > 0) M->timed(6, -1, 0, [&] { gfem::launch_addcorr<T>(s, M->n, M->Gv, x, M->X64); });
      M->timed(6, -1, 0, [&] { gfem::launch_resid<T>(s, M->Gs, A, M->b, M->X64, M->R64, M->part_r); });
      M->check_launch();
      rr = read_partials(M, M->part_r, M->Gs);
    }
    src = M->R64;
    // an outer correction that grows the FP64 residual means the inner solve
    // broke down on the working-precision operator: give up on this solve
    if (rr > 100.0 * (outer == 0 ? bb : rr_prev)) break;
    rr_prev = rr;
    if (failed && iters == 0) {
      res.rel = std::sqrt(rr / bb);
      res.ok = res.rel <= tol;
      break;
    }
  }
  if (res.outer > 0 && !res.ok && bb > 0) res.rel = std::sqrt(rr / bb);
  return res;
}

void ensure_netw(gf_mesh* M) {
  if (M->netw_ready) return;
  gfem::NetWork& w = M->netw;
  w.n = M->n;
  w.npad = (M->n + gfem::kNetRows - 1) / gfem::kNetRows * gfem::kNetRows;
  w.nwg_dw = 256;
  const size_t np = w.npad;
  w.a = M->al.get<gfem::bf16>(np * gfem::kNetInPad);
  w.inv_wdeg = M->al.get<float>(np);
  for (auto& h : w.h) h = M->al.get<gfem::bf16>(np * gfem::kHid);
  for (auto& m : w.m) m = M->al.get<gfem::bf16>(np * gfem::kHid);
  for (auto& z : w.z) z = M->al.get<gfem::bf16>(np * gfem::kHid);
  w.o = M->al.get<float>(np * gfem::kNetHead);
  w.glv = M->al.get<uint4>(M->ne);
  w.guv = M->al.get<uint4>(M->ne);
  w.gl8 = M->al.get<gfem::bf16>(M->ne);
  w.gu8 = M->al.get<gfem::bf16>(M->ne);
  w.gdv = M->al.get<uint4>(M->n);
  double sum = 0;
  for (int e = 0; e < M->ne; ++e) sum += std::sqrt(M->topo.edge_S[e]);
  M->inv_mean_len = M->ne > 0 ? M->ne / sum : 1.0;
  M->netw_ready = true;
}

// Buffers used only by training and the evaluation hook.
void ensure_net_train(gf_mesh* M) {
  ensure_netw(M);
  if (M->net_train_ready) return;
  gfem::NetWork& w = M->netw;
  const size_t np = w.npad;
  w.gh = M->al.get<float>(np * gfem::kHid);
  w.gz = M->al.get<gfem::bf16>(np * gfem::kHid);
  w.gi = M->al.get<float>(np * 2 * gfem::kHid);
  w.go = M->al.get<float>(np * gfem::kNetHead);
  w.part = M->al.get<float>((size_t)w.nwg_dw * (gfem::kHid * 2 * gfem::kHid + gfem::kHid));
  w.grad = M->al.get<float>(gfem::kNetParams);
  w.gl32 = M->al.get<float>((size_t)9 * M->ne);
  w.gu32 = M->al.get<float>((size_t)9 * M->ne);
  w.gd32 = M->al.get<float>((size_t)6 * M->n);
  w.probe = M->al.get<d4>(M->n);
  w.u = M->al.get<d4>(M->n);
  w.wneg = M->al.get<d4>(M->n);
  w.zero = M->al.get<d4>(M->n);  // zero-filled by the allocator
  w.mv = M->al.get<v4<float>>(M->n);
  w.sv = M->al.get<v4<float>>(M->n);
  w.dpart = M->al.get<double>(2 * kMaxPart);
  w.epart = M->al.get<float>((size_t)kMaxPart * gfem::kEdgeGrad);
  M->net_train_ready = true;
}

gfem::NetInputs net_inputs(gf_mesh* M, const uint8_t* zeta) {
  return gfem::NetInputs{M->n,    M->mat(), M->diag_blk, M->blk_edge, M->ne,           M->lptr,
                         M->uptr, M->lcol,  M->ucol,     M->upos,     M->X,            M->U,
                         zeta,    M->inv_mean_len, static_cast<const float*>(M->binv), M->dflag};
}

// Stored blocks A_ab between the factor pattern positions a <= b of every row
// (position 0 the row itself, a >= 1 its lower slot a - 1), for the row
// normalisation: (block index, a, b, 0).
void ensure_norm_pairs(gf_mesh* M) {
  if (M->norm_ptr) return;
  const gfem::Topology& T = M->topo;
  std::vector<int32_t> ptr(M->n + 1, 0);
  std::vector<int4> pairs;
  std::vector<int32_t> P;
  for (int i = 0; i < M->n; ++i) {
    P.assign(1, i);
    for (int l = T.lptr[i]; l < T.lptr[i + 1]; ++l) P.push_back(T.lcol[l]);
    for (int a = 0; a < (int)P.size(); ++a) {
      const int32_t* c0 = T.col.data() + T.row_ptr[P[a]];
      const int32_t* c1 = T.col.data() + T.row_ptr[P[a] + 1];
      for (int b = a; b < (int)P.size(); ++b) {
        const int32_t* hit = std::lower_bound(c0, c1, P[b]);
        if (hit != c1 && *hit == P[b]) pairs.push_back(int4{(int)(hit - T.col.data()), a, b, 0});
      }
    }
    ptr[i + 1] = (int32_t)pairs.size();
  }
  M->norm_ptr = upload(M, ptr);
  M->norm_pairs = upload(M, pairs);
}

// Factor of the learned path for the assembled step: the network runs every
// net_every_n_steps steps; in between its cached head outputs are combined
// with the current system.
void learned_precond(gf_mesh* M) {
  ensure_netw(M);
  if (M->fact_norm) ensure_norm_pairs(M);
  const gfem::NetInputs in = net_inputs(M, M->zeta[1 - M->zcur]);
  const int every = std::max(1, (int)M->p.net_every_n_steps);
  M->timed(3, -1, 0, [&] {
    const bool fresh = !M->net_cached || M->net_age >= every;
    if (fresh) {
      gfem::net_forward(M->stream, M->net->P, M->netw, in, M->Gn, false);
      M->net_cached = true;
      M->net_age = 0;
    }
    gfem::net_build_factor(M->stream, M->net->P, M->netw, in, M->Gn, false);
    // a row normalisation from an earlier A does not fit the current rows:
    // it is computed for every factor
    if (M->fact_norm) gfem::net_normalise_factor(M->stream, M->netw, in, M->Gn, M->norm_ptr, M->norm_pairs);
  });
  ++M->net_age;
  M->check_launch();
}

// FP64 copies of the precision-typed buffers of a split-precision mesh.
void ensure_esc(gf_mesh* M) {
  if (M->esc_ready) return;
  const size_t n = M->n, m = M->m;
  gf_mesh::PrecBufs& b = M->esc;
  b.val = M->al.get<double>(9 * (size_t)M->nbp);
  b.contrib = M->al.get<gfem::Rec<double>>((size_t)M->np);
  b.binv = M->al.get<double>(6 * n);
  b.pl[0] = M->plastic ? M->al.get<double>(6 * m) : nullptr;
  b.pl[1] = M->plastic ? M->al.get<double>(6 * m) : nullptr;
  b.vr = M->al.get<d4>(n);
  b.vz = M->al.get<d4>(n);
  b.vp[0] = M->al.get<d4>(n);
  b.vp[1] = M->al.get<d4>(n);
  b.vq = M->al.get<d4>(n);
  b.vx = M->al.get<d4>(n);
  b.vr2 = M->al.get<d4>(n);
  b.vy = M->al.get<d4>(n);
  M->esc_ready = true;
}

// Re-run the assembled step of a split-precision mesh in FP64 (element pass,
// block values and block-Jacobi PCG): used when the FP32 operator cannot be
// solved, which happens once near-flat tets make the rounding of their
// stiffness exceed the mass term.  Nothing is committed here.
SolveResult fp64_rerun(gf_mesh* M) {
  ensure_esc(M);
  const gf_mesh::PrecBufs keep = M->cur();
  const size_t np = 6 * (size_t)M->m;
  if (M->plastic)
    gfem::launch_convert(M->stream, static_cast<const float*>(keep.pl[M->plcur]),
                         static_cast<double*>(M->esc.pl[M->plcur]), np);
  M->use(M->esc);
  M->split = false;
  SolveResult r{false, 0, 0, 0.0};
  try {
    assemble<double>(M, AsmOpt{});
    r = solve<double>(M, M->binv, nullptr, 0, 2);
  } catch (...) {
    M->use(keep);
    M->split = true;
    throw;
  }
  M->use(keep);
  M->split = true;
  if (r.ok && M->plastic)
    gfem::launch_convert(M->stream, static_cast<const double*>(M->esc.pl[1 - M->plcur]),
                         static_cast<float*>(keep.pl[1 - M->plcur]), np);
  M->check_launch();
  return r;
}

template <typename T>
gf_status step_impl(gf_mesh* M, int n_steps, gf_step_stats* st) {
  for (int i = 0; i < n_steps; ++i) {
    assemble<T>(M, AsmOpt{});
    hchk(hipMemcpyAsync(M->h_ctr, M->ctr, sizeof(gfem::Counters), hipMemcpyDeviceToHost, M->stream), "D2H");
    SolveResult r;
    int fallback = 0;
    if (M->precond == GF_PC_LEARNED && M->learned_skip == 0) {
      // network factor B = G^T G; block-Jacobi re-solve if not accepted.  The
      // learned attempt may spend at most 3x (+100) the iterations of the last
      // accepted learned solve, so a poor factor costs a bounded detour; after
      // a rejection the next steps use block-Jacobi directly (back-off).
      learned_precond(M);
      const gfem::FactView F = gfem::net_factor_view(M->netw, net_inputs(M, M->zeta[1 - M->zcur]));
      const int cap = M->last_learned_iters > 0 ? 3 * M->last_learned_iters + 100 : 0;
      r = solve<T>(M, M->binv, &F, cap, 1);
      if (r.ok) {
        M->last_learned_iters = r.inner;
        M->learned_backoff = 4;
      } else {
        fallback = 1;
        M->learned_skip = M->learned_backoff;
        M->learned_backoff = std::min(2 * M->learned_backoff, 64);
        hchk(hipMemsetAsync(M->X64, 0, sizeof(d4) * M->n, M->stream), "hipMemsetAsync");
        const int prev_inner = r.inner, prev_outer = r.outer;
        r = solve<T>(M, M->binv);
        r.inner += prev_inner;
        r.outer += prev_outer;
      }
    } else {
      if (M->precond == GF_PC_LEARNED) {
        fallback = 1;
        --M->learned_skip;
      }
      r = solve<T>(M, M->binv);
    }
    int escalated = 0;
    if constexpr (std::is_same<T, float>::value) {
      if (!r.ok || M->force_fp64) {
        escalated = 1;
        const int prev_inner = r.inner, prev_outer = r.outer;
        r = fp64_rerun(M);
        r.inner += prev_inner;
        r.outer += prev_outer;
      }
    }
    int cnt[gfem::kNumCounters] = {0, 0, 0, 0, 0};
    for (int sl = 0; sl < gfem::kCtrSlots; ++sl)
      for (int c = 0; c < gfem::kNumCounters; ++c) cnt[c] += M->h_ctr->v[sl * gfem::kCtrStride + c];
    if (st) {
      st->used_fallback += fallback;
      st->fp64_steps += escalated;
      st->inner_iters += r.inner;
      st->outer_iters += r.outer;
      st->rel_residual = r.rel;
      st->new_broken += cnt[gfem::kNewBroken];
      st->total_broken = cnt[gfem::kTotalBroken];
      st->near_threshold += cnt[gfem::kNearThreshold];
      st->chi_zero_tets = cnt[gfem::kChiZero];
      st->degenerate_tets = cnt[gfem::kDegenerate];
    }
    if (!r.ok) {
      M->flush_times(st);
      char buf[160];
      snprintf(buf, sizeof buf, "step %d: PCG reached rel. residual %.3e > tol %.3e after %d iterations",
               M->step_index, r.rel, M->p.cg_rel_tol, r.inner);
      return fail(GF_ENOTCONVERGED, buf);
    }
    M->timed(7, -1, 0, [&] { gfem::launch_integrate(M->stream, M->n, M->X64, M->V, M->U, M->dflag, M->dvel, M->p.dt); });
    M->check_launch();
    M->zcur = 1 - M->zcur;
    if (M->plastic) M->plcur = 1 - M->plcur;
    ++M->step_index;
    // the integration stays queued: the next step's kernels follow it on the
    // stream, and every call that reads device state synchronises first
    // (timing reads its events, so it waits here)
    if (M->timing) M->sync();
    M->flush_times(st);
    if (st) st->steps_done += 1;
  }
  return GF_OK;
}

// Scratch of a quasi-static load step: a zero node vector, the displacement
// at the step's start (restored on failure) and the frozen chi (T[m]).
struct QsBufs {
  d4* zero;
  d4* U0;
  void* chi;
};

// The mesh's own scratch (allocated on first use).
QsBufs qs_owned(gf_mesh* M) {
  if (!M->qs_zero) {
    M->qs_zero = M->al.get<d4>(M->n);  // zero-filled by the allocator, never written
    M->qs_U0 = M->al.get<d4>(M->n);
    M->qs_chi = M->split ? (void*)M->al.get<float>(M->m) : (void*)M->al.get<double>(M->m);
  }
  return QsBufs{M->qs_zero, M->qs_U0, M->qs_chi};
}

// Allocation-free variant: the scratch lives in a file-scope device array of
// fixed size (per device, kept until the process ends).  Host code uses the
// address hipGetSymbolAddress returns for the current device, never the
// array's name.  Every call on a device shares it: calls that overlap on one
// device race.
constexpr int kNoAllocMaxNodes = 1 << 16;
constexpr int kNoAllocMaxTets = 393216;
constexpr size_t kNoAllocZero = 0;
constexpr size_t kNoAllocU0 = sizeof(d4) * (size_t)kNoAllocMaxNodes;
constexpr size_t kNoAllocChi = 2 * sizeof(d4) * (size_t)kNoAllocMaxNodes;
constexpr size_t kNoAllocBytes = kNoAllocChi + sizeof(double) * (size_t)kNoAllocMaxTets;  // 7 MiB
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
void* scratch_address(int dev) {
  if (dev < 0 || dev >= kMaxDevices) throw std::runtime_error("device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hchk(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress");
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

// Quasi-static load steps (Eq. 36; Sec. 4.3 names Newton with a line search):
// damage and plastic flow at the previous equilibrium; prescribed nodes move
// by dt times their prescribed velocity; chi evaluated at that first iterate
// and held fixed; Newton systems (M/dt^2 + K*) dx = f* (the backward-Euler
// operator at zero velocity, dx = dt dv; the mass term regularises detached
// fragments and vanishes as dt grows); backtracking Armijo line search on
// E = sum chi V Psi (FP64); stop at |f| <= rtol |f_0|.  A failed load step
// restores the displacement and commits nothing.
template <typename T>
gf_status qs_step_impl(gf_mesh* M, const QsBufs& B, int n_steps, double rtol, int max_newton, double armijo,
                       gf_qs_stats* st) {
  hipStream_t s = M->stream;
  const double dt = M->p.dt;
  const int Ge = std::min(gfem::kMaxPart, std::max(8, (M->m + gfem::kThreads - 1) / gfem::kThreads));
  const int Gd = std::min(gfem::kMaxPart, std::max(8, (M->n + gfem::kThreads - 1) / gfem::kThreads));
  const gfem::ElemConst ec{M->mu, M->lam, M->alpha_m1, M->p.energy};
  constexpr double kMinStep = 1.0 / (1 << 20);
  for (int step = 0; step < n_steps; ++step) {
    hchk(hipMemcpyAsync(B.U0, M->U, sizeof(d4) * M->n, hipMemcpyDeviceToDevice, s), "D2D");
    // 1. damage and plastic flow at x_n
    damage_pass(M);
    const T* pl = nullptr;
    if (M->plastic) {
      gfem::launch_plastic<T>(s, M->m, M->tets, M->X, M->U, static_cast<const T*>(M->pl[M->plcur]),
                              static_cast<T*>(M->pl[1 - M->plcur]), M->p.yield_strain);
      pl = static_cast<const T*>(M->pl[1 - M->plcur]);
    }
    // 2. the prescribed nodes move
    gfem::launch_move_prescribed(s, M->n, M->dflag, M->dvel, dt, M->U);
    M->check_launch();
    hchk(hipMemcpyAsync(M->h_ctr, M->ctr, sizeof(gfem::Counters), hipMemcpyDeviceToHost, s), "D2H");
    // 3. first iterate: chi evaluated and stored
    AsmOpt o;
    o.damage = o.flow = false;
    o.next_state = true;
    o.quasi_static = true;
    o.zero = B.zero;
    o.chi_out = B.chi;
    assemble<T>(M, o);
    o.chi_out = nullptr;
    o.chi_in = B.chi;
    double f0 = -1.0, fn = 0.0;
    int iters = 0, halvings = 0, inner = 0;
    bool ok = false;
    double energy = 0.0;
    for (int it = 0;; ++it) {
      // |b| = dt |f| on the free nodes (prescribed rows carry dv_c = 0)
      fn = std::sqrt(read_partials(M, M->part_a, M->Gs)) / dt;
      if (f0 < 0.0) f0 = fn;
      if (!std::isfinite(fn)) break;
      if (fn == 0.0 || fn <= rtol * f0) {
        ok = true;
        break;
      }
      if (it >= max_newton) break;
      const SolveResult r = solve<T>(M, M->binv);
      inner += r.inner;
      if (!r.ok) break;
      // slope f.dx = b.dv (dx = dt dv, b = dt f)
      gfem::launch_dot(s, Gd, M->n, M->b, M->X64, M->part_r);
      M->check_launch();
      const double slope = read_partials(M, M->part_r, Gd);
      gfem::launch_energy<T>(s, Ge, M->m, M->tets, M->X, M->U, M->X64, 0.0, pl, static_cast<const T*>(B.chi),
                             ec, M->part_r);
      M->check_launch();
      const double E0 = read_partials(M, M->part_r, Ge);
      double alpha = 1.0, E1 = E0;
      while (true) {
        gfem::launch_energy<T>(s, Ge, M->m, M->tets, M->X, M->U, M->X64, alpha * dt, pl,
                               static_cast<const T*>(B.chi), ec, M->part_r);
        M->check_launch();
        E1 = read_partials(M, M->part_r, Ge);
        if (E1 <= E0 - armijo * alpha * slope || std::fabs(E1 - E0) <= 1e-14 * std::fabs(E0)) break;
        alpha *= 0.5;
        ++halvings;
        if (alpha < kMinStep) break;
      }
      if (alpha < kMinStep) break;
      gfem::launch_axpy(s, M->n, alpha * dt, M->X64, M->U);
      energy = E1;
      iters = it + 1;
      assemble<T>(M, o);
    }
    M->recs.clear();
    M->ev_used = 0;
    M->solve_iters.clear();
    if (st) {
      st->newton_iters += iters;
      st->line_search_halvings += halvings;
      st->inner_iters += inner;
      st->force_residual = fn;
      st->force_initial = f0;
      st->energy = energy;
      int cnt[gfem::kNumCounters] = {0, 0, 0, 0, 0};
      for (int sl = 0; sl < gfem::kCtrSlots; ++sl)
        for (int c = 0; c < gfem::kNumCounters; ++c) cnt[c] += M->h_ctr->v[sl * gfem::kCtrStride + c];
      st->new_broken += cnt[gfem::kNewBroken];
      st->total_broken = cnt[gfem::kTotalBroken];
    }
    if (!ok) {
      hchk(hipMemcpyAsync(M->U, B.U0, sizeof(d4) * M->n, hipMemcpyDeviceToDevice, s), "D2D");
      M->sync();
      char buf[200];
      snprintf(buf, sizeof buf,
               "quasi-static step %d: no equilibrium (|f| %.3e of %.3e after %d Newton iterations, %d halvings)",
               M->step_index, fn, f0, iters, halvings);
      return fail(GF_ENOTCONVERGED, buf);
    }
    hchk(hipMemsetAsync(M->V, 0, sizeof(d4) * M->n, s), "hipMemsetAsync");
    M->zcur = 1 - M->zcur;
    if (M->plastic) M->plcur = 1 - M->plcur;
    ++M->step_index;
    M->sync();
    if (st) st->steps_done += 1;
  }
  return GF_OK;
}

gf_status guard(gf_mesh* m, const char* what) {
  if (!m) return fail(GF_EINVAL, std::string(what) + ": null mesh");
  return GF_OK;
}

#define GF_TRY(...)                                                                      \
  try {                                                                                  \
    __VA_ARGS__                                                                          \
  } catch (const HipError& e) {                                                          \
    return fail(GF_EDEVICE, std::string(e.what) + ": " + hipGetErrorString(e.e));        \
  } catch (const std::bad_alloc&) {                                                      \
    return fail(GF_ENOMEM, "allocation failed");                                         \
  } catch (const std::exception& e) {                                                    \
    return fail(GF_EINVAL, e.what());                                                    \
  }

}  // namespace

extern "C" {

const char* gf_last_error(void) { return g_err.c_str(); }

gf_status gf_mesh_create(const double* rest_xyz, int32_t n_nodes, const int32_t* tets, int32_t n_tets,
                         const gf_params* params, gf_mesh** out) {
  g_err.clear();
  if (!rest_xyz || !tets || !params || !out) return fail(GF_EINVAL, "gf_mesh_create: null argument");
  *out = nullptr;
  const gf_params& p = *params;
  if (!(p.youngs > 0) || !(p.poisson > -1.0 && p.poisson < 0.5) || !(p.density > 0) || !(p.dt > 0) ||
      !(p.cg_rel_tol > 0) || p.cg_max_iter <= 0 || (p.precision != GF_PREC_FP64 && p.precision != GF_PREC_SPLIT) ||
      (p.precond != GF_PC_BLOCK_JACOBI && p.precond != GF_PC_LEARNED) || !std::isfinite(p.damage_strain) ||
      !(p.damage_radius >= 0.0) || !std::isfinite(p.damage_radius) ||
      (p.energy != GF_ENERGY_STABLE_NEO_HOOKEAN && p.energy != GF_ENERGY_STVK) ||
      (p.reorder != GF_REORDER_NONE && p.reorder != GF_REORDER_RCM))
    return fail(GF_EINVAL, "gf_mesh_create: invalid parameters");
  if (p.precond == GF_PC_LEARNED && p.precision != GF_PREC_SPLIT)
    return fail(GF_EINVAL, "gf_mesh_create: the learned preconditioner needs the split precision mode");
  std::unique_ptr<gf_mesh> holder;
  GF_TRY({
    // Host-side validation and topology first: errors in the input are
    // reported the same way with or without a device.
    std::unique_ptr<gfem::Topology> topo(new gfem::Topology());
    bool degen = false;
    std::string err =
        gfem::build_topology(rest_xyz, n_nodes, tets, n_tets, p.density, topo.get(), &degen, p.reorder);
    if (!err.empty()) return fail(degen ? GF_EDEGENERATE : GF_EINVAL, "gf_mesh_create: " + err);
    // support of the non-local criterion (Eq. 20), also host-side
    std::vector<int64_t> nl_ptr;
    std::vector<int32_t> nl_idx;
    std::vector<double> nl_w;
    if (p.damage_radius > 0.0) {
      // at most 2^31 entries (12 B each: 24 GiB of the 288 GiB of HBM)
      err = gfem::build_nonlocal_support(*topo, p.damage_radius, (size_t)1 << 31, &nl_ptr, &nl_idx, &nl_w);
      if (!err.empty()) return fail(GF_EINVAL, "gf_mesh_create: " + err);
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(GF_EDEVICE, "no HIP device");
    int dev = 0;
    hchk(hipGetDevice(&dev), "hipGetDevice");
    hipDeviceProp_t prop;
    hchk(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
      return fail(GF_EDEVICE, std::string("device is ") + prop.gcnArchName + ", library built for gfx950");
    holder.reset(new gf_mesh());
    gf_mesh* M = holder.get();
    M->dev = dev;
    M->p = p;
    M->split = p.precision == GF_PREC_SPLIT;
    M->plastic = p.yield_strain > 0;
    M->precond = p.precond;
    M->topo = std::move(*topo);
    const gfem::Topology& T = M->topo;
    M->n = T.n;
    M->m = T.m;
    M->ne = T.ne;
    M->nb = T.nb;
    M->nbp = (T.nb + 63) / 64 * 64;
    M->Gv = std::min(kMaxPart, std::max(8, round_up8((T.n + gfem::kThreads - 1) / gfem::kThreads)));
    M->Gs = std::min(kMaxPart, std::max(8, round_up8((T.n * gfem::kRowLanes + gfem::kThreads - 1) / gfem::kThreads)));
    // PCG SpMV and G / G^T grid: about kPcgRowsPerWorkgroup block rows per
    // workgroup, capped at kPcgMaxWorkgroups (two 512-thread workgroups per
    // CU) so the consumer kernels reduce few partials.
    M->Gb = std::min(kPcgMaxWorkgroups, std::max(8, round_up8((T.n + kPcgRowsPerWorkgroup - 1) / kPcgRowsPerWorkgroup)));
    M->Ga = std::min(kMaxPart, std::max(8, round_up8((T.n + gfem::kVecThreads - 1) / gfem::kVecThreads)));
    // SpMV of the factorised path: the same cap (its partials are reduced by
    // every workgroup of the G pass, so more of them cost more than they save)
    M->Gp = M->Gb;
    // network and factor kernels: 256-thread workgroups, one 16-lane group per row, at most 1024
    M->Gn = std::min(1024, std::max(8, round_up8((T.n * gfem::kRowLanes + 255) / 256)));
    const double E = p.youngs, nu = p.poisson;
    const double mu0 = E / (2 * (1 + nu)), lam0 = E * nu / ((1 + nu) * (1 - 2 * nu));
    if (p.energy == GF_ENERGY_STVK) {
      M->mu = mu0;  // Eq. 37 with the plain Lame constants
      M->lam = lam0;
      M->alpha_m1 = 0.0;
    } else {
      M->mu = 4.0 * mu0 / 3.0;             // Smith et al. reparametrisation of Eq. 35
      M->lam = lam0 + 5.0 * mu0 / 6.0;
      M->alpha_m1 = 0.75 * M->mu / M->lam;  // alpha - 1 = mu/lam - mu/(4 lam)
    }
    hchk(hipStreamCreate(&M->own), "hipStreamCreate");
    M->stream = M->own;
    gfem::set_disconnected_lut(disconnected_lut());

    std::vector<d4> hX(T.n);
    for (int i = 0; i < T.n; ++i) hX[i] = d4{T.X[3 * i], T.X[3 * i + 1], T.X[3 * i + 2], 0.0};
    M->X = upload(M, hX);
    M->U = M->al.get<d4>(T.n);
    M->V = M->al.get<d4>(T.n);
    M->dvel = M->al.get<d4>(T.n);
    M->b = M->al.get<d4>(T.n);
    M->X64 = M->al.get<d4>(T.n);
    M->R64 = M->al.get<d4>(T.n);
    M->fbuf = M->al.get<d4>(T.n);
    M->dflag = M->al.get<uint8_t>(T.n);
    M->lumped = upload(M, T.lumped);
    std::vector<int4> ht(T.m);
    for (int t = 0; t < T.m; ++t) ht[t] = int4{T.tets[4 * t], T.tets[4 * t + 1], T.tets[4 * t + 2], T.tets[4 * t + 3]};
    M->tets = upload(M, ht);
    M->tet_edge = upload(M, T.tet_edge);
    M->flip = upload(M, T.tet_flip);
    std::vector<int2> he(T.ne);
    for (int e = 0; e < T.ne; ++e) he[e] = int2{T.edges[2 * e], T.edges[2 * e + 1]};
    M->edges = upload(M, he);
    M->edge_S = upload(M, T.edge_S);
    M->edge_mass = upload(M, T.edge_mass);
    M->zeta[0] = M->al.get<uint8_t>(T.ne);
    M->zeta[1] = M->al.get<uint8_t>(T.ne);
    M->near_ids = M->al.get<int32_t>(T.ne);
    if (!nl_ptr.empty()) {
      M->nl_ptr = upload(M, nl_ptr);
      M->nl_idx = upload(M, nl_idx);
      M->nl_w = upload(M, nl_w);
      M->nl_E = M->al.get<gfem::Sym6>(T.m);
      M->nl_Eavg = M->al.get<gfem::Sym6>(T.m);
      M->nl_entries = nl_idx.size();
    }
    M->edge_ptr = upload(M, T.edge_ptr);
    M->edge_slot = upload(M, T.edge_slot);
    M->part_base = upload(M, T.part_base);
    M->part_cptr = upload(M, T.part_cptr);
    M->part_slot = upload(M, T.part_slot);
    M->edge_pptr = upload(M, T.edge_pptr);
    M->edge_part = upload(M, T.edge_part);
    M->np = (int)T.edge_part.size();
    M->row_ptr = upload(M, T.row_ptr);
    M->col = upload(M, T.col);
    M->diag_blk = upload(M, T.diag_blk);
    M->blk_edge = upload(M, T.blk_edge);
    M->lptr = upload(M, T.lptr);
    M->lcol = upload(M, T.lcol);
    M->uptr = upload(M, T.uptr);
    M->ucol = upload(M, T.ucol);
    M->upos = upload(M, T.upos);
    if (M->split)
      alloc_precision<float>(M);
    else
      alloc_precision<double>(M);
    M->part_a = M->al.get<double>(kMaxPart);
    M->part_rz = M->al.get<double>(4 * kMaxPart);
    M->part_pq = M->al.get<double>(kMaxPart);
    M->part_r = M->al.get<double>(kMaxPart);
    M->ctl = M->al.get<gfem::PcgCtl>(1);
    M->ctr = M->al.get<gfem::Counters>(1);
    hchk(hipHostMalloc((void**)&M->h_part, sizeof(double) * 2 * kMaxPart, hipHostMallocDefault), "hipHostMalloc");
    hchk(hipHostMalloc((void**)&M->h_ctl, sizeof(gfem::PcgCtl), hipHostMallocDefault), "hipHostMalloc");
    hchk(hipHostMalloc((void**)&M->h_ctr, sizeof(gfem::Counters), hipHostMallocDefault), "hipHostMalloc");
    M->h_dflag.assign(T.n, 0);
    M->h_dvel.assign(T.n, d4{0, 0, 0, 0});
    hchk(hipDeviceSynchronize(), "hipDeviceSynchronize");
    *out = holder.release();
    return GF_OK;
  })
}

gf_status gf_mesh_destroy(gf_mesh* m) {
  if (!m) return GF_OK;
  delete m;
  return GF_OK;
}

gf_status gf_set_stream(gf_mesh* m, void* hip_stream) {
  if (gf_status s = guard(m, "gf_set_stream")) return s;
  GF_TRY({
    m->sync();
    m->stream = hip_stream ? static_cast<hipStream_t>(hip_stream) : m->own;
    return GF_OK;
  })
}

gf_status gf_get_sizes(const gf_mesh* m, int32_t* n_nodes, int32_t* n_tets, int32_t* n_edges, int32_t* n_blocks) {
  if (!m) return fail(GF_EINVAL, "gf_get_sizes: null mesh");
  if (n_nodes) *n_nodes = m->n;
  if (n_tets) *n_tets = m->m;
  if (n_edges) *n_edges = m->ne;
  if (n_blocks) *n_blocks = m->nb;
  return GF_OK;
}

gf_status gf_get_edges(const gf_mesh* m, int32_t* ij_out) {
  if (!m || !ij_out) return fail(GF_EINVAL, "gf_get_edges: null argument");
  const gfem::Topology& T = m->topo;
  for (int c = 0; c < T.ne; ++c) {
    int e = T.edge_internal[c];
    int a = T.perm_old[T.edges[2 * e]], b = T.perm_old[T.edges[2 * e + 1]];
    ij_out[2 * c] = std::min(a, b);
    ij_out[2 * c + 1] = std::max(a, b);
  }
  return GF_OK;
}

gf_status gf_set_dirichlet(gf_mesh* m, const int32_t* nodes, int32_t n, const double* vel) {
  if (gf_status s = guard(m, "gf_set_dirichlet")) return s;
  if (n < 0 || (n > 0 && (!nodes || !vel))) return fail(GF_EINVAL, "gf_set_dirichlet: bad arguments");
  std::vector<uint8_t> fl(m->n, 0);
  std::vector<d4> dv(m->n, d4{0, 0, 0, 0});
  for (int i = 0; i < n; ++i) {
    int id = nodes[i];
    if (id < 0 || id >= m->n) return fail(GF_EINVAL, "gf_set_dirichlet: node id out of range");
    int k = m->topo.perm_new[id];
    if (fl[k]) return fail(GF_EINVAL, "gf_set_dirichlet: repeated node");
    for (int d = 0; d < 3; ++d)
      if (!std::isfinite(vel[3 * i + d])) return fail(GF_EINVAL, "gf_set_dirichlet: non-finite velocity");
    fl[k] = 1;
    dv[k] = d4{vel[3 * i], vel[3 * i + 1], vel[3 * i + 2], 0.0};
  }
  GF_TRY({
    m->sync();
    hchk(hipMemcpy(m->dflag, fl.data(), m->n, hipMemcpyHostToDevice), "H2D");
    hchk(hipMemcpy(m->dvel, dv.data(), sizeof(d4) * m->n, hipMemcpyHostToDevice), "H2D");
    m->h_dflag = fl;
    m->h_dvel = dv;
    return GF_OK;
  })
}

gf_status gf_set_edge_damage(gf_mesh* m, const uint8_t* zeta) {
  if (gf_status s = guard(m, "gf_set_edge_damage")) return s;
  if (!zeta) return fail(GF_EINVAL, "gf_set_edge_damage: null labels");
  GF_TRY({
    m->sync();
    std::vector<uint8_t> cur(m->ne);
    hchk(hipMemcpy(cur.data(), m->zeta[m->zcur], m->ne, hipMemcpyDeviceToHost), "D2H");
    for (int c = 0; c < m->ne; ++c)
      if (zeta[c]) cur[m->topo.edge_internal[c]] = 1;
    hchk(hipMemcpy(m->zeta[m->zcur], cur.data(), m->ne, hipMemcpyHostToDevice), "H2D");
    return GF_OK;
  })
}

gf_status gf_step(gf_mesh* m, int32_t n_steps, gf_step_stats* stats) {
  if (gf_status s = guard(m, "gf_step")) return s;
  if (n_steps < 0) return fail(GF_EINVAL, "gf_step: negative step count");
  if (stats) std::memset(stats, 0, sizeof *stats);
  if (m->precond == GF_PC_LEARNED && !m->net)
    return fail(GF_ESTATE, "gf_step: learned preconditioner selected but no network attached");
  GF_TRY({
    return m->split ? step_impl<float>(m, n_steps, stats) : step_impl<double>(m, n_steps, stats);
  })
}

static gf_status get_node_vec(const gf_mesh* m, const d4* src, bool add_rest, double* out, const char* who) {
  if (!m || !out) return fail(GF_EINVAL, std::string(who) + ": null argument");
  GF_TRY({
    std::vector<d4> h(m->n);
    hchk(hipStreamSynchronize(m->stream), "sync");
    hchk(hipMemcpy(h.data(), src, sizeof(d4) * m->n, hipMemcpyDeviceToHost), "D2H");
    for (int c = 0; c < m->n; ++c) {
      const int i = m->topo.perm_new[c];
      const double* X = &m->topo.X[3 * (size_t)i];
      out[3 * (size_t)c] = h[i].x + (add_rest ? X[0] : 0.0);
      out[3 * (size_t)c + 1] = h[i].y + (add_rest ? X[1] : 0.0);
      out[3 * (size_t)c + 2] = h[i].z + (add_rest ? X[2] : 0.0);
    }
    return GF_OK;
  })
}

gf_status gf_get_positions(const gf_mesh* m, double* xyz_out) {
  return get_node_vec(m, m ? m->U : nullptr, true, xyz_out, "gf_get_positions");
}

gf_status gf_get_velocities(const gf_mesh* m, double* vel_out) {
  return get_node_vec(m, m ? m->V : nullptr, false, vel_out, "gf_get_velocities");
}

gf_status gf_get_edge_damage(const gf_mesh* m, uint8_t* zeta_out) {
  if (!m || !zeta_out) return fail(GF_EINVAL, "gf_get_edge_damage: null argument");
  GF_TRY({
    std::vector<uint8_t> h(m->ne);
    hchk(hipStreamSynchronize(m->stream), "sync");
    hchk(hipMemcpy(h.data(), m->zeta[m->zcur], m->ne, hipMemcpyDeviceToHost), "D2H");
    for (int c = 0; c < m->ne; ++c) zeta_out[c] = h[m->topo.edge_internal[c]] ? 1 : 0;
    return GF_OK;
  })
}

static gf_status qs_check(gf_mesh* m, int32_t n_steps, double newton_rel_tol, int32_t max_newton, double armijo,
                          gf_qs_stats* stats, const char* who) {
  if (gf_status s = guard(m, who)) return s;
  if (stats) std::memset(stats, 0, sizeof *stats);
  if (n_steps < 0 || !(newton_rel_tol > 0.0 && newton_rel_tol < 1.0) || max_newton < 0 ||
      !(armijo > 0.0 && armijo < 1.0))
    return fail(GF_EINVAL, std::string(who) + ": bad arguments");
  if (m->p.gravity[0] != 0.0 || m->p.gravity[1] != 0.0 || m->p.gravity[2] != 0.0)
    return fail(GF_EINVAL, std::string(who) + ": the quasi-static problem has no gravity (set it to zero)");
  return GF_OK;
}

gf_status gf_quasi_static_step(gf_mesh* m, int32_t n_steps, double newton_rel_tol, int32_t max_newton,
                               double armijo, gf_qs_stats* stats) {
  if (gf_status s = qs_check(m, n_steps, newton_rel_tol, max_newton, armijo, stats, "gf_quasi_static_step"))
    return s;
  GF_TRY({
    const QsBufs B = qs_owned(m);
    return m->split ? qs_step_impl<float>(m, B, n_steps, newton_rel_tol, max_newton, armijo, stats)
                    : qs_step_impl<double>(m, B, n_steps, newton_rel_tol, max_newton, armijo, stats);
  })
}

gf_status gf_quasi_static_step_noalloc(gf_mesh* m, int32_t n_steps, double newton_rel_tol, int32_t max_newton,
                                       double armijo, gf_qs_stats* stats) {
  const char* who = "gf_quasi_static_step_noalloc";
  if (gf_status s = qs_check(m, n_steps, newton_rel_tol, max_newton, armijo, stats, who)) return s;
  if (m->n > kNoAllocMaxNodes || m->m > kNoAllocMaxTets) {
    char buf[200];
    snprintf(buf, sizeof buf, "%s: mesh of %d nodes / %d tets exceeds the fixed scratch (at most %d nodes, %d tets)",
             who, m->n, m->m, kNoAllocMaxNodes, kNoAllocMaxTets);
    return fail(GF_EINVAL, buf);
  }
  GF_TRY({
    int dev = -1;
    hchk(hipGetDevice(&dev), "hipGetDevice");
    if (dev != m->dev) return fail(GF_EINVAL, std::string(who) + ": the mesh's device is not the current device");
    unsigned char* base = static_cast<unsigned char*>(scratch_address(dev));
    const QsBufs B{reinterpret_cast<d4*>(base + kNoAllocZero), reinterpret_cast<d4*>(base + kNoAllocU0),
                   base + kNoAllocChi};
    // the array keeps the last call's contents: the zero vector is cleared here
    gfem::launch_zero(m->stream, m->n, B.zero);
    m->check_launch();
    return m->split ? qs_step_impl<float>(m, B, n_steps, newton_rel_tol, max_newton, armijo, stats)
                    : qs_step_impl<double>(m, B, n_steps, newton_rel_tol, max_newton, armijo, stats);
  })
}

gf_status gf_get_visual_mesh(gf_mesh* m, double* subcell_xyz_out, uint8_t* group_out) {
  if (gf_status s = guard(m, "gf_get_visual_mesh")) return s;
  GF_TRY({
    constexpr int kChunk = 1 << 16;
    if (!m->vis_xyz) {
      m->tet_swapped = upload(m, m->topo.tet_swapped);
      m->vis_xyz = m->al.get<double>((size_t)96 * kChunk);
      m->vis_group = m->al.get<uint8_t>((size_t)4 * kChunk);
    }
    for (int t0 = 0; t0 < m->m; t0 += kChunk) {
      const int cnt = std::min(kChunk, m->m - t0);
      gfem::launch_visual(m->stream, t0, cnt, m->m, m->tets, m->tet_swapped, m->tet_edge, m->zeta[m->zcur], m->X,
                          m->U, m->vis_xyz, m->vis_group);
      m->check_launch();
      if (subcell_xyz_out)
        hchk(hipMemcpyAsync(subcell_xyz_out + (size_t)96 * t0, m->vis_xyz, sizeof(double) * 96 * (size_t)cnt,
                            hipMemcpyDeviceToHost, m->stream),
             "D2H");
      if (group_out)
        hchk(hipMemcpyAsync(group_out + (size_t)4 * t0, m->vis_group, 4 * (size_t)cnt, hipMemcpyDeviceToHost,
                            m->stream),
             "D2H");
      m->sync();
    }
    return GF_OK;
  })
}

gf_status gf_get_near_threshold_edges(const gf_mesh* m, int32_t* ids_out, int32_t capacity, int32_t* n_out) {
  if (!m || !n_out || capacity < 0 || (capacity > 0 && !ids_out))
    return fail(GF_EINVAL, "gf_get_near_threshold_edges: bad argument");
  GF_TRY({
    gfem::Counters c;
    hchk(hipStreamSynchronize(m->stream), "sync");
    hchk(hipMemcpy(&c.near_n, &m->ctr->near_n, sizeof(int), hipMemcpyDeviceToHost), "D2H");
    const int n = std::min(std::max(c.near_n, 0), m->ne);
    std::vector<int32_t> h(n);
    if (n) hchk(hipMemcpy(h.data(), m->near_ids, sizeof(int32_t) * n, hipMemcpyDeviceToHost), "D2H");
    // internal -> canonical edge ids, ascending
    std::vector<int32_t> inv(m->ne);
    for (int c2 = 0; c2 < m->ne; ++c2) inv[m->topo.edge_internal[c2]] = c2;
    for (int32_t& e : h) e = inv[e];
    std::sort(h.begin(), h.end());
    for (int i = 0; i < std::min(n, (int)capacity); ++i) ids_out[i] = h[i];
    *n_out = n;
    return GF_OK;
  })
}

gf_status gf_eval_forces(gf_mesh* m, double* f_out) {
  if (gf_status s = guard(m, "gf_eval_forces")) return s;
  if (!f_out) return fail(GF_EINVAL, "gf_eval_forces: null output");
  GF_TRY({
    AsmOpt o;
    o.flow = o.next_state = false;
    o.f_out = m->fbuf;
    if (m->split)
      assemble<float>(m, o);
    else
      assemble<double>(m, o);
    m->sync();
    m->recs.clear();
    m->ev_used = 0;
    return get_node_vec(m, m->fbuf, false, f_out, "gf_eval_forces");
  })
}

gf_status gf_get_system(gf_mesh* m, int32_t* bi_out, int32_t* bj_out, double* vals_out, double* rhs_out) {
  if (gf_status s = guard(m, "gf_get_system")) return s;
  GF_TRY({
    if (m->split)
      assemble<float>(m, AsmOpt{});
    else
      assemble<double>(m, AsmOpt{});
    m->sync();
    m->recs.clear();
    m->ev_used = 0;
    const gfem::Topology& T = m->topo;
    if (vals_out) {
      std::vector<double> hv((size_t)9 * m->nbp);
      if (m->split) {
        std::vector<float> hf((size_t)9 * m->nbp);
        hchk(hipMemcpy(hf.data(), m->val, sizeof(float) * hf.size(), hipMemcpyDeviceToHost), "D2H");
        for (size_t i = 0; i < hf.size(); ++i) hv[i] = hf[i];
      } else {
        hchk(hipMemcpy(hv.data(), m->val, sizeof(double) * hv.size(), hipMemcpyDeviceToHost), "D2H");
      }
      for (int bk = 0; bk < m->nb; ++bk)
        for (int c = 0; c < 9; ++c) vals_out[9 * (size_t)bk + c] = hv[(size_t)c * m->nbp + bk];
    }
    if (bi_out || bj_out)
      for (int i = 0; i < m->n; ++i)
        for (int bk = T.row_ptr[i]; bk < T.row_ptr[i + 1]; ++bk) {
          if (bi_out) bi_out[bk] = T.perm_old[i];
          if (bj_out) bj_out[bk] = T.perm_old[T.col[bk]];
        }
    if (rhs_out) return get_node_vec(m, m->b, false, rhs_out, "gf_get_system");
    return GF_OK;
  })
}

namespace {
struct StateHeader {
  uint32_t magic, version;
  int32_t n, ne, m, step, plastic, split;
};
constexpr uint32_t kMagic = 0x4d454647;  // "GFEM"

size_t state_bytes(const gf_mesh* m) {
  return sizeof(StateHeader) + sizeof(double) * 6 * (size_t)m->n + (size_t)m->ne +
         (m->plastic ? sizeof(double) * 6 * (size_t)m->m : 0);
}
}  // namespace

// Checkpoint blob: header | U (n*3 f64, caller order) | V (n*3 f64) |
// zeta (n_edges u8, canonical order) | plastic Gram offset (6*n_tets f64, SoA).
gf_status gf_get_state(const gf_mesh* m, void* buf, size_t* bytes) {
  if (!m || !bytes) return fail(GF_EINVAL, "gf_get_state: null argument");
  const size_t need = state_bytes(m);
  if (!buf) {
    *bytes = need;
    return GF_OK;
  }
  if (*bytes < need) return fail(GF_EINVAL, "gf_get_state: buffer too small");
  char* o = static_cast<char*>(buf);
  StateHeader h{kMagic, 2, m->n, m->ne, m->m, m->step_index, m->plastic, m->split};
  std::memcpy(o, &h, sizeof h);
  o += sizeof h;
  if (gf_status s = get_node_vec(m, m->U, false, reinterpret_cast<double*>(o), "gf_get_state")) return s;
  o += sizeof(double) * 3 * m->n;
  if (gf_status s = get_node_vec(m, m->V, false, reinterpret_cast<double*>(o), "gf_get_state")) return s;
  o += sizeof(double) * 3 * m->n;
  if (gf_status s = gf_get_edge_damage(m, reinterpret_cast<uint8_t*>(o))) return s;
  o += m->ne;
  GF_TRY({
    if (m->plastic) {
      std::vector<double> d((size_t)6 * m->m);
      if (m->split) {
        std::vector<float> f((size_t)6 * m->m);
        hchk(hipMemcpy(f.data(), m->pl[m->plcur], sizeof(float) * f.size(), hipMemcpyDeviceToHost), "D2H");
        std::copy(f.begin(), f.end(), d.begin());
      } else {
        hchk(hipMemcpy(d.data(), m->pl[m->plcur], sizeof(double) * d.size(), hipMemcpyDeviceToHost), "D2H");
      }
      std::memcpy(o, d.data(), sizeof(double) * d.size());
    }
    *bytes = need;
    return GF_OK;
  })
}

gf_status gf_set_state(gf_mesh* m, const void* buf, size_t bytes) {
  if (!m || !buf) return fail(GF_EINVAL, "gf_set_state: null argument");
  StateHeader h;
  if (bytes < sizeof h) return fail(GF_EINVAL, "gf_set_state: buffer too small");
  std::memcpy(&h, buf, sizeof h);
  if (h.magic != kMagic || h.version != 2 || h.n != m->n || h.ne != m->ne || h.m != m->m ||
      h.plastic != (int)m->plastic || h.split != (int)m->split || bytes < state_bytes(m))
    return fail(GF_EINVAL, "gf_set_state: state does not match this mesh");
  const char* o = static_cast<const char*>(buf) + sizeof h;
  std::vector<d4> U(m->n), V(m->n);
  for (int c = 0; c < m->n; ++c) {
    double u[3], v[3];
    std::memcpy(u, o + sizeof(double) * 3 * c, sizeof u);
    std::memcpy(v, o + sizeof(double) * 3 * ((size_t)m->n + c), sizeof v);
    for (int d = 0; d < 3; ++d)
      if (!std::isfinite(u[d]) || !std::isfinite(v[d])) return fail(GF_EINVAL, "gf_set_state: non-finite state");
    const int i = m->topo.perm_new[c];
    U[i] = d4{u[0], u[1], u[2], 0.0};
    V[i] = d4{v[0], v[1], v[2], 0.0};
  }
  o += sizeof(double) * 6 * m->n;
  std::vector<uint8_t> z(m->ne);
  for (int c = 0; c < m->ne; ++c) z[m->topo.edge_internal[c]] = o[c] ? 1 : 0;
  o += m->ne;
  GF_TRY({
    m->sync();
    hchk(hipMemcpy(m->U, U.data(), sizeof(d4) * m->n, hipMemcpyHostToDevice), "H2D");
    hchk(hipMemcpy(m->V, V.data(), sizeof(d4) * m->n, hipMemcpyHostToDevice), "H2D");
    hchk(hipMemcpy(m->zeta[m->zcur], z.data(), m->ne, hipMemcpyHostToDevice), "H2D");
    if (m->plastic) {
      std::vector<double> d((size_t)6 * m->m);
      std::memcpy(d.data(), o, sizeof(double) * d.size());
      if (m->split) {
        std::vector<float> f(d.begin(), d.end());
        hchk(hipMemcpy(m->pl[m->plcur], f.data(), sizeof(float) * f.size(), hipMemcpyHostToDevice), "H2D");
      } else {
        hchk(hipMemcpy(m->pl[m->plcur], d.data(), sizeof(double) * d.size(), hipMemcpyHostToDevice), "H2D");
      }
    }
    m->step_index = h.step;
    // a restored state starts a fresh solver history: the network runs on the
    // next learned step, and the learned back-off, attempt cap and launch
    // chunk predictions are cleared
    m->net_cached = false;
    m->last_learned_iters = 0;
    m->learned_skip = 0;
    m->learned_backoff = 4;
    std::memset(m->last_solve_iters, 0, sizeof m->last_solve_iters);
    return GF_OK;
  })
}

gf_status gf_set_fp64_rerun(gf_mesh* m, int32_t always) {
  if (gf_status s = guard(m, "gf_set_fp64_rerun")) return s;
  if (always && !m->split) return fail(GF_EINVAL, "gf_set_fp64_rerun: needs the split precision mode");
  m->force_fp64 = always != 0;
  return GF_OK;
}

gf_status gf_set_timing(gf_mesh* m, int32_t on) {
  if (gf_status s = guard(m, "gf_set_timing")) return s;
  m->timing = on != 0;
  return GF_OK;
}

gf_status gf_bench_spmv(gf_mesh* m, int32_t reps, double* us_per_launch, double* bytes_per_launch) {
  if (gf_status s = guard(m, "gf_bench_spmv")) return s;
  if (reps <= 0 || !us_per_launch) return fail(GF_EINVAL, "gf_bench_spmv: bad arguments");
  GF_TRY({
    const size_t vb = m->split ? 12 : 24, ab = m->split ? 4 : 8;
    // algorithmic bytes of one SpMV launch (iteration k > 0): 3x3 values +
    // column index per block; z and p_{k-1} read once, p_k and q written and
    // row_ptr per block row
    if (bytes_per_launch) *bytes_per_launch = (double)m->nb * (9 * ab + 4) + (double)m->n * (4 * vb + 4);
    hipStream_t s = m->stream;
    std::vector<hipEvent_t> evs(2 * (size_t)reps);
    for (auto& e : evs) hchk(hipEventCreate(&e), "hipEventCreate");
    auto run = [&](auto tag) {
      using T = decltype(tag);
      v4<T>* pb[2] = {static_cast<v4<T>*>(m->vp[0]), static_cast<v4<T>*>(m->vp[1])};
      v4<T>* z = static_cast<v4<T>*>(m->vz);
      v4<T>* q = static_cast<v4<T>*>(m->vq);
      const T* binv = static_cast<const T*>(m->binv);
      hchk(hipMemsetAsync(m->ctl, 0, sizeof(gfem::PcgCtl), s), "hipMemsetAsync");
      gfem::launch_pcg_init<T>(s, m->n, m->Ga, m->b, binv, static_cast<v4<T>*>(m->vr), z, pb[0],
                               static_cast<v4<T>*>(m->vx), m->part_rz, m->ctl);
      gfem::launch_pcg_spmv<T>(s, 0, m->Gb, m->Ga, m->mat(), z, pb[1], pb[0], q, m->ctl, m->part_rz, m->part_pq,
                               -1.0);  // negative threshold: never converges
      gfem::launch_pcg_update<T>(s, 0, m->n, m->Ga, m->Gb, pb[0], q, static_cast<v4<T>*>(m->vx),
                                 static_cast<v4<T>*>(m->vr), z, binv, m->ctl, m->part_pq, m->part_rz);
      for (int i = 0; i < reps; ++i)
        gfem::launch_pcg_spmv<T>(s, 1, m->Gb, m->Ga, m->mat(), z, pb[0], pb[1], q, m->ctl, m->part_rz, m->part_pq,
                                 -1.0, gfem::LaunchEvents{evs[2 * i], evs[2 * i + 1]});
    };
    if (m->split)
      run(float{});
    else
      run(double{});
    m->check_launch();
    m->sync();
    double total_ms = 0;
    for (int i = 0; i < reps; ++i) {
      float ms = 0;
      hchk(hipEventElapsedTime(&ms, evs[2 * i], evs[2 * i + 1]), "hipEventElapsedTime");
      total_ms += ms;
    }
    for (auto& e : evs) (void)hipEventDestroy(e);
    *us_per_launch = 1000.0 * total_ms / reps;
    return GF_OK;
  })
}

// ---------------------------------------------------------------- learned preconditioner

gf_status gf_net_num_params(int32_t* n) {
  if (!n) return fail(GF_EINVAL, "gf_net_num_params: null output");
  *n = gfem::kNetParams;
  return GF_OK;
}

gf_status gf_net_create(uint64_t seed, gf_net** out) {
  if (!out) return fail(GF_EINVAL, "gf_net_create: null output");
  *out = nullptr;
  std::unique_ptr<gf_net> holder;
  GF_TRY({
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(GF_EDEVICE, "no HIP device");
    holder.reset(new gf_net());
    gf_net* net = holder.get();
    net->seed = seed;
    hchk(hipGetDevice(&net->dev), "hipGetDevice");
    gfem::NetParamsDev& P = net->P;
    P.master = net->al.get<float>(gfem::kNetParams);
    P.adam_m = net->al.get<float>(gfem::kNetParams);
    P.adam_v = net->al.get<float>(gfem::kNetParams);
    P.W0 = net->al.get<gfem::bf16>(gfem::kHid * gfem::kNetInPad);
    for (int l = 0; l < gfem::kNetLayers; ++l) {
      P.Wl[l] = net->al.get<gfem::bf16>(gfem::kHid * 2 * gfem::kHid);
      P.WlT[l] = net->al.get<gfem::bf16>(gfem::kHid * 2 * gfem::kHid);
    }
    // He-style initial layers, zero biases and zero head (block-Jacobi at start)
    net->host.assign(gfem::kNetParams, 0.f);
    std::mt19937_64 rng(seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    for (int i = 0; i < gfem::kHid * gfem::kNetIn; ++i)
      net->host[gfem::kOffW0 + i] = (float)(nd(rng) * std::sqrt(2.0 / gfem::kNetIn));
    for (int l = 0; l < gfem::kNetLayers; ++l)
      for (int i = 0; i < gfem::kHid * 2 * gfem::kHid; ++i)
        net->host[gfem::kOffL0 + l * gfem::kLayerSize + i] = (float)(nd(rng) * std::sqrt(2.0 / (2 * gfem::kHid)));
    hchk(hipMemcpy(P.master, net->host.data(), sizeof(float) * gfem::kNetParams, hipMemcpyHostToDevice), "H2D");
    gfem::net_pack(nullptr, P);
    hchk(hipGetLastError(), "kernel launch");
    hchk(hipDeviceSynchronize(), "hipDeviceSynchronize");
    *out = holder.release();
    return GF_OK;
  })
}

gf_status gf_net_destroy(gf_net* net) {
  if (net) {
    (void)hipDeviceSynchronize();
    delete net;
  }
  return GF_OK;
}

namespace {
// Weight blob: header (magic "GFNW", format version, parameter count, element
// type 0 = FP32) followed by the FP32 master weights in the documented order.
struct NetBlobHeader {
  uint32_t magic, version, n_params, dtype;
};
constexpr uint32_t kNetMagic = 0x574e4647;  // "GFNW"
constexpr uint32_t kNetBlobVersion = 1;
constexpr size_t kNetBlobBytes = sizeof(NetBlobHeader) + sizeof(float) * (size_t)gfem::kNetParams;

// Host-only validation of a weight blob; on success *w points at its weights.
gf_status check_net_blob(const void* blob, size_t bytes, const float** w, const char* who) {
  if (!blob) return fail(GF_EINVAL, std::string(who) + ": null blob");
  if (bytes < sizeof(NetBlobHeader)) return fail(GF_EINVAL, std::string(who) + ": blob shorter than its header");
  NetBlobHeader h;
  std::memcpy(&h, blob, sizeof h);
  if (h.magic != kNetMagic) return fail(GF_EINVAL, std::string(who) + ": not a weight blob (bad magic)");
  if (h.version != kNetBlobVersion) return fail(GF_EINVAL, std::string(who) + ": unsupported blob version");
  if (h.dtype != 0) return fail(GF_EINVAL, std::string(who) + ": unsupported weight type");
  if (h.n_params != (uint32_t)gfem::kNetParams)
    return fail(GF_EINVAL, std::string(who) + ": parameter count does not match this network");
  if (bytes != kNetBlobBytes) return fail(GF_EINVAL, std::string(who) + ": blob size does not match its header");
  const float* p = reinterpret_cast<const float*>(static_cast<const char*>(blob) + sizeof h);
  for (int i = 0; i < gfem::kNetParams; ++i) {
    float v;
    std::memcpy(&v, p + i, sizeof v);
    if (!std::isfinite(v)) return fail(GF_EINVAL, std::string(who) + ": non-finite weight");
  }
  if (w) *w = p;
  return GF_OK;
}
}  // namespace

gf_status gf_net_check_weights(const void* blob, size_t bytes) {
  g_err.clear();
  return check_net_blob(blob, bytes, nullptr, "gf_net_check_weights");
}

gf_status gf_net_get_weights(const gf_net* net, void* blob, size_t* bytes) {
  if (!net || !bytes) return fail(GF_EINVAL, "gf_net_get_weights: null argument");
  if (!blob) {
    *bytes = kNetBlobBytes;
    return GF_OK;
  }
  if (*bytes < kNetBlobBytes) return fail(GF_EINVAL, "gf_net_get_weights: buffer too small");
  const NetBlobHeader h{kNetMagic, kNetBlobVersion, (uint32_t)gfem::kNetParams, 0};
  std::memcpy(blob, &h, sizeof h);
  std::memcpy(static_cast<char*>(blob) + sizeof h, net->host.data(), sizeof(float) * gfem::kNetParams);
  *bytes = kNetBlobBytes;
  return GF_OK;
}

gf_status gf_net_set_weights(gf_net* net, const void* blob, size_t bytes) {
  if (!net) return fail(GF_EINVAL, "gf_net_set_weights: null network");
  const float* w = nullptr;
  if (gf_status st = check_net_blob(blob, bytes, &w, "gf_net_set_weights")) return st;
  GF_TRY({
    hchk(hipDeviceSynchronize(), "hipDeviceSynchronize");
    std::vector<float> hw(gfem::kNetParams);
    std::memcpy(hw.data(), w, sizeof(float) * gfem::kNetParams);
    net->host = hw;
    hchk(hipMemcpy(net->P.master, hw.data(), sizeof(float) * gfem::kNetParams, hipMemcpyHostToDevice), "H2D");
    hchk(hipMemset(net->P.adam_m, 0, sizeof(float) * gfem::kNetParams), "hipMemset");
    hchk(hipMemset(net->P.adam_v, 0, sizeof(float) * gfem::kNetParams), "hipMemset");
    net->adam_t = 0;
    gfem::net_pack(nullptr, net->P);
    hchk(hipGetLastError(), "kernel launch");
    hchk(hipDeviceSynchronize(), "hipDeviceSynchronize");
    return GF_OK;
  })
}

gf_status gf_set_precond_net(gf_mesh* m, gf_net* net) {
  if (gf_status s = guard(m, "gf_set_precond_net")) return s;
  if (net && !m->split) return fail(GF_EINVAL, "gf_set_precond_net: needs the split precision mode");
  if (net && net->dev != m->dev) return fail(GF_EINVAL, "gf_set_precond_net: network on another device");
  m->net = net;
  m->net_cached = false;
  return GF_OK;
}

gf_status gf_set_precond(gf_mesh* m, int32_t precond) {
  if (gf_status s = guard(m, "gf_set_precond")) return s;
  if (precond != GF_PC_BLOCK_JACOBI && precond != GF_PC_LEARNED) return fail(GF_EINVAL, "gf_set_precond: bad value");
  if (precond == GF_PC_LEARNED && !m->split) return fail(GF_EINVAL, "gf_set_precond: needs the split precision mode");
  m->precond = precond;
  m->net_cached = false;
  return GF_OK;
}

static gf_status net_train_eval(gf_net* net, gf_mesh* m, bool train, double lr, const double* probe,
                                double* loss_out, float* gdiag_out, float* glower_out, float* grad_out,
                                const char* who) {
  if (!net || !m) return fail(GF_EINVAL, std::string(who) + ": null argument");
  if (!m->split) return fail(GF_EINVAL, std::string(who) + ": needs the split precision mode");
  if (net->dev != m->dev) return fail(GF_EINVAL, std::string(who) + ": network on another device");
  if (train && !(lr > 0.0 && std::isfinite(lr))) return fail(GF_EINVAL, std::string(who) + ": bad learning rate");
  if ((size_t)m->n > (size_t)256 * kMaxPart) return fail(GF_EINVAL, std::string(who) + ": mesh too large");
  if (probe)
    for (size_t i = 0; i < 3 * (size_t)m->n; ++i)
      if (!std::isfinite(probe[i])) return fail(GF_EINVAL, std::string(who) + ": non-finite probe");
  GF_TRY({
    hipStream_t s = m->stream;
    ensure_net_train(m);
    assemble<float>(m, AsmOpt{});
    m->recs.clear();
    m->ev_used = 0;
    m->solve_iters.clear();
    const gfem::NetInputs in = net_inputs(m, m->zeta[1 - m->zcur]);
    gfem::NetWork& w = m->netw;
    gfem::net_forward(s, net->P, w, in, m->Gn);
    gfem::net_build_factor(s, net->P, w, in, m->Gn, true);
    std::vector<d4> hv;
    if (probe) {
      hv.resize(m->n);
      for (int c = 0; c < m->n; ++c)
        hv[m->topo.perm_new[c]] = d4{probe[3 * (size_t)c], probe[3 * (size_t)c + 1], probe[3 * (size_t)c + 2], 0.0};
      hchk(hipMemcpyAsync(w.probe, hv.data(), sizeof(d4) * m->n, hipMemcpyHostToDevice, s), "H2D");
    } else {
      gfem::net_probe(s, w, net->seed * 0x9E3779B97F4A7C15ull + (uint64_t)net->adam_t + 1);
    }
    // power-weighted probe: v <- X v rescaled to |v|^2 = N, X = G A G^T, so
    // that t / N below is the Rayleigh quotient of X^k v
    const double Nd = 3.0 * m->n;
    for (int k = 0; k < net->power_steps; ++k) {
      gfem::net_kaporin_u(s, w, in, m->Gn);
      gfem::launch_resid<float>(s, m->Gs, m->mat(), w.zero, w.u, w.wneg, m->part_a);
      const int G = gfem::net_power_apply(s, w, in, m->Gn);
      m->check_launch();
      const double yy = read_partials(m, w.dpart, G);
      if (!(yy > 0.0) || !std::isfinite(yy))
        return fail(GF_ESTATE, std::string(who) + ": power step of the probe is not positive and finite");
      gfem::net_scale_probe(s, w, std::sqrt(Nd / yy));
    }
    gfem::net_kaporin_u(s, w, in, m->Gn);
    gfem::launch_resid<float>(s, m->Gs, m->mat(), w.zero, w.u, w.wneg, m->part_a);
    const int G = gfem::net_kaporin_dots(s, net->P, w, in);
    m->check_launch();
    const double t = read_partials(m, w.dpart, G);
    const double ld = read_partials(m, w.dpart + kMaxPart, G);
    const double N = 3.0 * m->n;
    if (!(t > 0.0) || !std::isfinite(t) || !std::isfinite(ld))
      return fail(GF_ESTATE, std::string(who) + ": probe energy of the factor is not positive and finite");
    const double loss = std::log(t / N) - 2.0 * ld / N;
    gfem::net_kaporin_backward(s, net->P, w, in, m->Gn, t);
    m->check_launch();
    if (train) {
      ++net->adam_t;
      gfem::net_adam(s, net->P, w.grad, net->adam_t, (float)lr);
      m->check_launch();
      hchk(hipMemcpyAsync(net->host.data(), net->P.master, sizeof(float) * gfem::kNetParams, hipMemcpyDeviceToHost,
                          s),
           "D2H");
    }
    if (grad_out)
      hchk(hipMemcpyAsync(grad_out, w.grad, sizeof(float) * gfem::kNetParams, hipMemcpyDeviceToHost, s), "D2H");
    std::vector<float> hd, hl;
    if (gdiag_out) {
      hd.resize((size_t)6 * m->n);
      hchk(hipMemcpyAsync(hd.data(), w.gd32, sizeof(float) * hd.size(), hipMemcpyDeviceToHost, s), "D2H");
    }
    if (glower_out) {
      hl.resize((size_t)9 * m->ne);
      hchk(hipMemcpyAsync(hl.data(), w.gl32, sizeof(float) * hl.size(), hipMemcpyDeviceToHost, s), "D2H");
    }
    m->sync();
    if (gdiag_out)
      for (int c = 0; c < m->n; ++c) {
        const size_t i = m->topo.perm_new[c];
        const size_t nn = m->n;
        float* o = gdiag_out + 9 * (size_t)c;
        o[0] = hd[i];
        o[1] = o[2] = o[5] = 0.f;
        o[3] = hd[nn + i];
        o[4] = hd[2 * nn + i];
        o[6] = hd[3 * nn + i];
        o[7] = hd[4 * nn + i];
        o[8] = hd[5 * nn + i];
      }
    if (glower_out)
      for (int c = 0; c < m->ne; ++c) {
        const int li = m->topo.lpos[m->topo.edge_internal[c]];
        for (int q = 0; q < 9; ++q) glower_out[9 * (size_t)c + q] = hl[(size_t)q * m->ne + li];
      }
    if (loss_out) *loss_out = loss;
    m->net_cached = false;
    return GF_OK;
  })
}

gf_status gf_set_precond_normalise(gf_mesh* m, int32_t on) {
  if (gf_status s = guard(m, "gf_set_precond_normalise")) return s;
  m->fact_norm = on != 0;
  return GF_OK;
}

gf_status gf_net_set_power_steps(gf_net* net, int32_t k) {
  if (!net) return fail(GF_EINVAL, "gf_net_set_power_steps: null network");
  if (k < 0 || k > kMaxPowerSteps) return fail(GF_EINVAL, "gf_net_set_power_steps: k outside [0, 64]");
  net->power_steps = k;
  return GF_OK;
}

gf_status gf_net_train_step(gf_net* net, gf_mesh* m, double lr, double* loss_out) {
  return net_train_eval(net, m, true, lr, nullptr, loss_out, nullptr, nullptr, nullptr, "gf_net_train_step");
}

gf_status gf_net_eval(gf_net* net, gf_mesh* m, const double* probe, double* loss_out, float* gdiag_out,
                      float* glower_out, float* grad_out) {
  return net_train_eval(net, m, false, 0.0, probe, loss_out, gdiag_out, glower_out, grad_out, "gf_net_eval");
}

}  // extern "C"
