/*
 * gfem.h -- C ABI of the MI355X (gfx950) graph-based FEM fracture library.
 *
 * Method: Mandal, Chaudhuri & Chaudhuri, "Remeshing-Free Graph-Based Finite
 * Element Method for Ductile and Brittle Fracture".  One timestep is
 * Algorithm 1 (Sec. 4.3) without collisions and visualisation:
 *   1. per-edge damage update and relabel (Sec. 3.3, Eq. 20-21, local support),
 *   2. per-tet energy fraction chi (Sec. 3.4, Eq. 22-25),
 *   3. element pass: stable neo-Hookean energy (Sec. 5.1, Eq. 35) or
 *      Saint-Venant Kirchhoff energy (Sec. 5.2, Eq. 37) written in
 *      the six squared edge lengths (Sec. 3.5, Theorem 3.1), nodal forces
 *      along the edges (Sec. 3.2, Eq. 12), tangent stiffness (Eq. 10), both
 *      scaled by chi (Sec. 3.6, Eq. 32-34), scattered into a block-sparse
 *      system whose pattern never changes (Sec. 1),
 *   4. one linearised backward-Euler step (Sec. 4.3) solved by preconditioned
 *      conjugate gradients, x += dt v.
 *
 * Conventions (all entry points):
 *   - Every function returns a gf_status; nothing throws across the ABI.  On
 *     error, gf_last_error() returns a thread-local message that stays valid
 *     until the next call on the same thread.
 *   - Pointers named *_out are caller-allocated HOST buffers of the stated
 *     size; inputs are host buffers that are copied (the caller keeps
 *     ownership).  No device pointer crosses this boundary except the
 *     optional HIP stream of gf_set_stream.
 *   - Node ids are the caller's 0-based ids; edges are in canonical order
 *     (i < j, lexicographic in caller node ids) as returned by gf_get_edges.
 *   - Not thread-safe per mesh: calls on one gf_mesh must be serialised.
 */
#ifndef GFEM_H
#define GFEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gf_mesh gf_mesh; /* opaque; owned by the library from create to destroy */

typedef enum {
  GF_OK = 0,
  GF_EINVAL = -1,         /* bad argument: null pointer, size or index out of range */
  GF_EDEGENERATE = -2,    /* a tet with |volume| <= 1e-14 h^3 */
  GF_ENOMEM = -3,         /* host or device allocation failed */
  GF_EDEVICE = -4,        /* a HIP runtime call failed, or no gfx950 device */
  GF_ENOTCONVERGED = -5,  /* PCG missed the tolerance; the step was not committed */
  GF_ESTATE = -6          /* call not valid in the current state (e.g. no weights loaded) */
} gf_status;

typedef enum { GF_PREC_FP64 = 0, GF_PREC_SPLIT = 1 } gf_precision;
typedef enum { GF_PC_BLOCK_JACOBI = 0, GF_PC_LEARNED = 1 } gf_precond;
/* Element energy: the stable neo-Hookean density of the quasi-static runs
 * (Sec. 5.1, Eq. 35, with the Lame constants reparametrised so that the
 * small-strain response has the given E and nu) or the Saint-Venant Kirchhoff
 * density of the dynamic runs (Sec. 5.2, Eq. 37, plain Lame constants), both
 * written in the six squared edge lengths (Sec. 3.5, Theorem 3.1). */
typedef enum { GF_ENERGY_STABLE_NEO_HOOKEAN = 0, GF_ENERGY_STVK = 1 } gf_energy;
/* Internal node numbering (invisible to the caller, who always uses its own
 * ids): the caller's order, or reverse Cuthill-McKee on the tet graph (narrow
 * band, so the gathers of neighbouring rows stay close in memory for any
 * input order).  The learned factor is block lower triangular in internal
 * order, so its blocks depend on this choice. */
typedef enum { GF_REORDER_NONE = 0, GF_REORDER_RCM = 1 } gf_reorder;

/* Material, integrator and solver parameters (copied at create). */
typedef struct {
  double youngs;          /* E [Pa]: small-strain Young's modulus */
  double poisson;         /* nu in (-1, 0.5) */
  double density;         /* rho [kg/m^3]: consistent mass of Eq. 5 */
  double damage_strain;   /* an edge breaks when its Green normal strain >= this (Eq. 21) */
  double damage_radius;   /* R_d of Eq. 20 [m]: 0 = local criterion (each edge's own strain);
                             > 0 = non-local: the strain tensors of the tets whose rest
                             centroids lie within R_d are averaged with the weights
                             (1 - (r/R_d)^2)^2 normalised to 1, and an edge breaks when the
                             averaged normal strain along it reaches damage_strain in any tet
                             that contains it (the support is built once, at create) */
  double yield_strain;    /* ductile yield on |dev E_elastic|_F; <= 0 disables plasticity */
  double dt;              /* timestep [s] */
  double rayleigh_alpha;  /* damping b = alpha M + beta K* (Sec. 3.1, Sec. 3.6) */
  double rayleigh_beta;
  double gravity[3];      /* body acceleration [m/s^2] (Eq. 6 with t = rho g) */
  double cg_rel_tol;      /* accept a solve at FP64 |b - A dv|_2 <= tol |b|_2 */
  int32_t cg_max_iter;    /* total inner PCG iterations allowed per step */
  int32_t precision;      /* gf_precision: FP64 everything, or FP32 element/SpMV + FP64 dots/residual */
  int32_t precond;        /* gf_precond */
  int32_t net_every_n_steps; /* learned preconditioner: run the network every n steps (>= 1) */
  int32_t energy;         /* gf_energy */
  int32_t reorder;        /* gf_reorder */
} gf_params;

/* Per-call statistics (summed over the steps of one gf_step call, except
 * rel_residual and total_broken which describe the last step). */
typedef struct {
  int32_t steps_done;       /* committed steps */
  int32_t inner_iters;      /* PCG iterations */
  int32_t outer_iters;      /* FP64 residual recomputations (iterative refinement) */
  int32_t used_fallback;    /* learned preconditioner selected but the step solved with
                               block-Jacobi: a rejected learned solve (re-solved), or one of
                               the following back-off steps (4, doubling to 64 per rejection) */
  int32_t new_broken;       /* edges newly labelled broken */
  int32_t total_broken;     /* broken edges after the last step */
  int32_t near_threshold;   /* edge evaluations with |strain - threshold| < 1e-6 */
  int32_t chi_zero_tets;    /* tets with chi = 0 (disconnected) in the last step */
  int32_t degenerate_tets;  /* tets with |J| < 0.05 in the last step */
  int32_t fp64_steps;       /* split precision only: steps whose FP32 operator could not be
                               solved and that were re-run in FP64 (element pass, blocks, PCG) */
  int32_t n_launch[9];      /* kernel launches per timing category (timing on) */
  double rel_residual;      /* final FP64 |b - A dv| / |b| of the last step */
  double kernel_us[9];      /* device time per category (timing on), microseconds:
                               0 damage, 1 element (+plasticity), 2 assembly (edge + row),
                               3 preconditioner set-up (network, factor), 4 SpMV (PCG),
                               5 PCG vector updates (with the G pass of the factorised
                               preconditioner), 6 FP64 residual / refinement, 7 integrate,
                               8 G^T pass of the factorised preconditioner */
} gf_step_stats;

/* Create a mesh.  rest_xyz: n_nodes*3 doubles (caller order); tets:
 * n_tets*4 node ids in any orientation (reoriented inside by swapping local
 * nodes 2 and 3 when the signed volume is negative).  Builds the edge list
 * (the induced graph of Sec. 1 and 3.1), the fixed block-sparse pattern
 * (one 3x3 block per node and two per edge), the consistent mass (Eq. 5)
 * and all device buffers.  Selects HIP device 0 unless one is current.
 * Returns GF_EINVAL for bad sizes/ids, GF_EDEGENERATE for a flat tet. */
gf_status gf_mesh_create(const double* rest_xyz, int32_t n_nodes, const int32_t* tets,
                         int32_t n_tets, const gf_params* params, gf_mesh** out);
gf_status gf_mesh_destroy(gf_mesh* m);

/* Run all device work on this HIP stream (hipStream_t passed as void*;
 * NULL = the library's own stream). The caller keeps ownership. */
gf_status gf_set_stream(gf_mesh* m, void* hip_stream);

/* Sizes: any output pointer may be NULL. n_blocks = stored 3x3 blocks. */
gf_status gf_get_sizes(const gf_mesh* m, int32_t* n_nodes, int32_t* n_tets, int32_t* n_edges,
                       int32_t* n_blocks);

/* Canonical edge list: ij_out holds n_edges*2 node ids, i < j, lexicographic. */
gf_status gf_get_edges(const gf_mesh* m, int32_t* ij_out);

/* Prescribed velocities (the fixed or moved points of the experiments of
 * Sec. 5.1, and Algorithm 1's external conditions applied before the system is
 * built): nodes[n] (caller ids, distinct), vel[n*3] m/s.  These nodes move at
 * exactly that velocity every step: their rows and columns are eliminated
 * from the backward-Euler system (right-hand side b_f -= A_fc dv_c, identity
 * rows, b_c = dv_c).  Replaces any previous set; n = 0 clears it.  GF_EINVAL
 * for an id out of range, a repeated id or a non-finite velocity (the set is
 * then unchanged). */
gf_status gf_set_dirichlet(gf_mesh* m, const int32_t* nodes, int32_t n, const double* vel);

/* OR labels into the damage variable zeta (Eq. 21): zeta[n_edges] in
 * canonical edge order, nonzero = broken.  Labels never revert. */
gf_status gf_set_edge_damage(gf_mesh* m, const uint8_t* zeta);

/* Advance n_steps timesteps.  Each step is committed only when its solve
 * reaches the FP64 tolerance; otherwise the call stops, leaves positions,
 * velocities, damage and plastic state as they were before that step and
 * returns GF_ENOTCONVERGED.  stats may be NULL.  The last step's integration
 * may still be running on the library's stream when the call returns; every
 * call that reads or replaces device state waits for it, and a device fault
 * in it is reported by the next such call. */
gf_status gf_step(gf_mesh* m, int32_t n_steps, gf_step_stats* stats);

/* Statistics of gf_quasi_static_step (summed over its load steps, except
 * the last four fields, which describe the last one). */
typedef struct {
  int32_t steps_done;            /* committed load steps */
  int32_t newton_iters;          /* Newton iterations (linear solves) */
  int32_t line_search_halvings;  /* step halvings of the line search */
  int32_t inner_iters;           /* PCG iterations over all Newton solves */
  int32_t new_broken;            /* edges newly labelled broken */
  int32_t total_broken;          /* broken edges after the last load step */
  double force_initial;          /* |f| on the free nodes at the first iterate of the last load step */
  double force_residual;         /* |f| at its last iterate */
  double energy;                 /* total energy sum chi V Psi there */
} gf_qs_stats;

/* Quasi-static load steps: equilibrium of Eq. 36, sum chi k u = sum chi f,
 * by Newton's method with a backtracking line search on the total energy
 * (Sec. 4.3, Sec. 5.1).  Per load step: damage (and plastic flow) at the
 * previous equilibrium; the prescribed nodes of gf_set_dirichlet move by dt
 * times their prescribed velocity; chi is evaluated at that first iterate and
 * held fixed, so the energy E = sum chi V Psi is the potential of the forces;
 * each Newton system is (M/dt^2 + K*) dx = f* on the free nodes (the backward-
 * Euler operator at zero velocity: the mass term regularises detached
 * fragments and vanishes as dt grows), solved by block-Jacobi PCG to
 * cg_rel_tol; the step length is the largest of 1, 1/2, 1/4, ... (down to
 * 2^-20) with E(x + a dx) <= E(x) - armijo a f.dx, a change of E below FP64
 * resolution (1e-14 |E|) being accepted; iteration stops at
 * |f| <= newton_rel_tol |f_0|, f_0 the force of the first iterate.  Velocities
 * are zero after a load step.  newton_rel_tol and armijo in (0, 1);
 * max_newton >= 0.  Returns GF_ENOTCONVERGED (displacement restored, nothing
 * committed) when a load step has no equilibrium within max_newton Newton
 * iterations, the line search fails or a linear solve misses its tolerance;
 * GF_EINVAL for bad arguments or a nonzero gravity (the quasi-static
 * experiments of Sec. 5.1 have none).  stats may be NULL. */
gf_status gf_quasi_static_step(gf_mesh* m, int32_t n_steps, double newton_rel_tol, int32_t max_newton,
                               double armijo, gf_qs_stats* stats);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation): gf_quasi_static_step
 * with its per-call scratch (a zero node vector, the displacement at the load
 * step's start and the frozen chi) in a fixed device array of the library
 * (7 MiB per device, held until the process ends) instead of buffers the
 * library allocates on first use; same arguments, kernels and results.  Calls
 * no hipMalloc/hipFree.  Meshes of at most 65,536 nodes and 393,216 tets
 * (GF_EINVAL beyond, nothing done); the mesh's device must be current.  All
 * calls on one device share the array: calls that overlap on a device race
 * and must be serialised by the caller. */
gf_status gf_quasi_static_step_noalloc(gf_mesh* m, int32_t n_steps, double newton_rel_tol, int32_t max_newton,
                                       double armijo, gf_qs_stats* stats);

/* Current positions x = X + u after the last committed step (Algorithm 1's
 * update x += dt v of Sec. 4.3), n_nodes*3 doubles, caller order, into a
 * caller-owned buffer.  Waits for the library's stream. */
gf_status gf_get_positions(const gf_mesh* m, double* xyz_out);
/* Current velocities, n_nodes*3 doubles, caller order. */
gf_status gf_get_velocities(const gf_mesh* m, double* vel_out);
/* Damage labels zeta of Eq. 21 after the last committed step (1 = broken,
 * irreversible, Sec. 3.3), n_edges bytes (0/1), canonical edge order, into a
 * caller-owned buffer.  Waits for the library's stream. */
gf_status gf_get_edge_damage(const gf_mesh* m, uint8_t* zeta_out);

/* Split visualisation mesh of the current state (Sec. 4.1): the computational
 * mesh is never remeshed; for rendering, each tet is split into one sub-cell
 * per corner (the node-associated four-split: the corner, the centroids of
 * its three edges, of its three faces and of the tet).  A split point has one
 * child per group of the tet's corners that its unbroken edges connect within
 * that edge, face or tet, placed at the point's rest position plus the mean
 * displacement of the group: a broken edge gives each parent its own child;
 * unbroken, the children coincide.  Outputs (caller-owned host buffers, each
 * may be NULL), tets in caller order, corners in the caller's local order a:
 *   subcell_xyz_out[n_tets*4*8*3] doubles: per tet and corner a the vertices
 *     [corner a, edge points towards the other corners b1 < b2 < b3, face
 *     points (b1,b2), (b1,b3), (b2,b3), tet point], each x, y, z;
 *   group_out[n_tets*4]: the smallest local corner index joined to a by
 *     unbroken edges of the tet (sub-cells of one group render as one piece;
 *     faces between groups are crack surfaces).
 * Off the timestep path; uses the library's stream and waits for it. */
gf_status gf_get_visual_mesh(gf_mesh* m, double* subcell_xyz_out, uint8_t* group_out);

/* Edges whose Green strain was within 1e-6 of the damage threshold in the
 * last damage pass (Eq. 21: labels there depend on rounding, so they are
 * reported rather than graded): canonical edge ids, ascending.  At most
 * `capacity` ids are written to the caller-owned ids_out (may be NULL when
 * capacity is 0); *n_out receives the total count.  The last damage pass is
 * the one of the last gf_step attempt (committed or not), gf_eval_forces or
 * gf_get_system. */
gf_status gf_get_near_threshold_edges(const gf_mesh* m, int32_t* ids_out, int32_t capacity, int32_t* n_out);

/* Test hook: restoring force f* = sum_e chi_e f_e (Eq. 12, 32) at the current
 * state and labels, n_nodes*3 doubles, caller order. */
gf_status gf_eval_forces(gf_mesh* m, double* f_out);

/* Test hook: assemble (without solving or committing) the system of the
 * next step at the current state and copy it out in COO block form:
 * bi_out/bj_out[n_blocks] caller node ids, vals_out[n_blocks*9] row-major 3x3
 * blocks, rhs_out[n_nodes*3].  Dirichlet rows/columns are eliminated as in
 * the solve.  Any output may be NULL. */
gf_status gf_get_system(gf_mesh* m, int32_t* bi_out, int32_t* bj_out, double* vals_out,
                        double* rhs_out);

/* Checkpoint: the step is Markov in (displacement, velocity, damage, plastic
 * state, step index).  gf_get_state with buf == NULL reports the size.
 * gf_set_state also clears the solver history (the network's cached outputs,
 * the learned back-off and attempt cap, the launch chunk predictions), so a
 * restored state is solved as from a fresh mesh. */
gf_status gf_get_state(const gf_mesh* m, void* buf, size_t* bytes);
gf_status gf_set_state(gf_mesh* m, const void* buf, size_t bytes);

/* Test hook (split precision only): always = 1 re-runs every step in FP64
 * (element pass, blocks, block-Jacobi PCG into FP64 buffers; the committed
 * state stays split), the path taken automatically when a step's FP32
 * operator cannot be solved; always = 0 restores the automatic choice. */
gf_status gf_set_fp64_rerun(gf_mesh* m, int32_t always);

/* Per-kernel device timing with HIP events on the library's stream
 * (fills gf_step_stats.kernel_us / n_launch); the PCG kernels' events are
 * recorded by their dispatches, so they time kernel execution only.  Off by
 * default. */
gf_status gf_set_timing(gf_mesh* m, int32_t on);

/* Time `reps` launches of the PCG SpMV kernel alone on the current operator
 * (after at least one step or gf_get_system) with HIP events recorded by each
 * dispatch (kernel execution only); returns the mean duration in microseconds
 * and the algorithmic bytes per launch. */
gf_status gf_bench_spmv(gf_mesh* m, int32_t reps, double* us_per_launch, double* bytes_per_launch);

/* ---------------------------------------------------------------------------
 * Learned preconditioner (an addition to the paper, whose solver is plain
 * conjugate gradients).  A message-passing network on the mesh graph maps edge
 * features (rest length, current length, damage label) to the 3x3 blocks of a
 * factorised sparse approximate inverse B = G^T G, with G block lower
 * triangular on the lower block pattern of A in node order:
 *   G_ii = L_i C_i,   G_ij = -L_i C_i W_ij A_ij A_jj^-1   (j < i, i-j an edge),
 * C_i the inverse lower Cholesky factor of A_ii, L_i lower triangular with
 * exponentiated diagonal (per node) and W_ij a 3x3 block (per edge).  B is
 * symmetric positive definite by construction; the zero network gives 3x3
 * block-Jacobi.  Inference and training run on the GPU in BF16 with FP32
 * accumulation; the solve stores G in BF16.  A learned solve is accepted only
 * at the same FP64 residual; otherwise the step is re-solved with block-Jacobi
 * (gf_step_stats.used_fallback).  Only the split precision mode supports it.
 * ------------------------------------------------------------------------- */
typedef struct gf_net gf_net; /* opaque, owned by the library from create to destroy */

/* Create a network on the current device: He-initialised hidden layers, zero
 * head and edge term (so it starts as block-Jacobi).  Deterministic in seed,
 * which also seeds the training probes. */
gf_status gf_net_create(uint64_t seed, gf_net** out);
gf_status gf_net_destroy(gf_net* net);
/* Number of FP32 parameters (same for every network). */
gf_status gf_net_num_params(int32_t* n);
/* Weights travel as a self-describing blob of exactly 16 + 4 * n_params bytes:
 * a header of four little-endian uint32 (magic 0x574e4647 "GFNW", format
 * version 1, parameter count = gf_net_num_params, element type 0 = FP32)
 * followed by the FP32 master weights in this order: W0 (64x8), b0 (64), then
 * for each of 3 layers W (64x128, columns 0-63 act on h, 64-127 on the
 * neighbour mean), b (64), then the node head Wh (24x64), bh (24) (outputs 0-5:
 * L_i, 6-14: s_i, 15-23: t_i) and the edge term We (9x3), be (9), with
 * W_ij = s_i + t_j + We f_ij + be (row-major 3x3); matrices row-major [out][in].
 *
 * gf_net_check_weights: host-only validation of a blob (no device needed).
 * Returns GF_EINVAL when the blob is null, shorter than its header, has
 * another magic, version, element type or parameter count, when bytes differs
 * from 16 + 4 * n_params, or when a weight is not finite.
 * gf_net_get_weights: blob == NULL stores the size in *bytes; otherwise
 * *bytes is the capacity of the caller-owned buffer (GF_EINVAL if too
 * small) and receives the size written.
 * gf_net_set_weights: copies a blob that passes gf_net_check_weights (the
 * network is unchanged otherwise) and resets the optimiser. */
gf_status gf_net_check_weights(const void* blob, size_t bytes);
gf_status gf_net_get_weights(const gf_net* net, void* blob, size_t* bytes);
gf_status gf_net_set_weights(gf_net* net, const void* blob, size_t bytes);
/* Attach (borrowed: must outlive its use) or detach (NULL) the network used by
 * GF_PC_LEARNED steps, and select the preconditioner of the following steps. */
gf_status gf_set_precond_net(gf_mesh* m, gf_net* net);
gf_status gf_set_precond(gf_mesh* m, int32_t precond);
/* Row normalisation of the learned factor (off by default): after each factor
 * build every block row G_i is scaled from the left by the inverse lower
 * Cholesky factor of its diagonal block of G A G^T, so that block becomes I;
 * a row whose block is not positive definite in FP32 is left unscaled.  It
 * caps the large eigenvalues that strongly anisotropic rows of heavily damaged
 * states give G A G^T, at the cost of one more pass per step (~85 us at 620k
 * tets: the blocks of A between every pair of a row's pattern nodes are
 * gathered); the network's per-node scaling L_i has no effect while it is on.
 * on: 0 or 1. */
gf_status gf_set_precond_normalise(gf_mesh* m, int32_t on);
/* One training step on the system of the mesh's next timestep at its current
 * state (assembled, not solved, not committed).  Loss: Kaporin's condition
 * number of X = G A G^T estimated with a +-1 probe v (drawn from a
 * counter-based generator seeded by the network's seed and step count),
 *   loss = log(v^T X v / N) - (2/N) log det G,   N = 3 n_nodes,
 * which is log K / N up to the constant log det A / N; gradient by the
 * network's backward pass, one Adam step (lr).  loss_out may be NULL.
 * With k power steps (gf_net_set_power_steps) the probe is first replaced by
 * X^k v rescaled to |v|^2 = N, so the first term is the Rayleigh quotient of
 * X^k v: k = 0 weighs the spectrum by its mean (Kaporin), large k by its
 * largest eigenvalue.  The gradient treats the power-stepped probe as fixed. */
gf_status gf_net_set_power_steps(gf_net* net, int32_t k); /* 0 <= k <= 64; default 0 */
gf_status gf_net_train_step(gf_net* net, gf_mesh* m, double lr, double* loss_out);
/* Same system, no update.  probe: n_nodes*3 doubles in caller order (NULL: the
 * generator's next probe).  Outputs (each may be NULL): the loss; the diagonal
 * factor blocks G_ii (n_nodes*9 floats, caller order, row-major); the lower
 * blocks G_ji of every edge (i, j), i < j (n_edges*9 floats, canonical edge
 * order, row-major); the weight gradient (gf_net_num_params floats).  Test hook. */
gf_status gf_net_eval(gf_net* net, gf_mesh* m, const double* probe, double* loss_out, float* gdiag_out,
                      float* glower_out, float* grad_out);

/* Thread-local message of the last failing call ("" if none). */
const char* gf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GFEM_H */
