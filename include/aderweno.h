/*
 * aderweno.h -- C ABI of the MI355X (gfx950) implementation of the cell-centred
 * direct ALE ADER-WENO finite volume scheme with time-accurate local time
 * stepping (LTS) for the 2D Euler equations on moving triangular meshes
 * (Boscheri, Dumbser, Zanotti, arXiv:1408.3719).
 *
 * Problem statement (paper Sec. 2.1, eqs. PDE, trian, xietaTransf,
 * eqn.cellaverage): a conforming triangulation whose elements carry cell
 * averages Q = (rho, rho u, rho v, rho E) of the Euler equations (Sec. 3,
 * eqs. eulerTerms, eqn.eos); the mesh moves with the local fluid velocity
 * (V = v, Sec. 3) and every element advances with its own time step.
 *
 * Conventions
 *   - Ownership: the library owns the context and its host copy of the
 *     topology.  The caller owns the device workspace and every *_dev buffer
 *     (FP64, contiguous); the library never frees caller memory.
 *   - Streams: all device work is queued on the HIP stream given at
 *     creation.  Calls that return host values synchronise that stream.
 *   - Errors: every int-returning call returns 0 on success or a negative
 *     ADER_E_* code; ader_last_error() then holds a message.  Nothing throws
 *     across the ABI.  After a stepping error the device state is undefined;
 *     restore a saved state with ader_upload_state_xy.
 *   - Threads: one context per host thread.
 *   - Call order: ader_create -> ader_upload_mesh -> ader_workspace_size ->
 *     ader_bind_workspace -> ader_upload_state -> ader_step_* ...;
 *     out-of-order calls return ADER_E_ORDER.
 */
#ifndef ADERWENO_H
#define ADERWENO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ADER_OK = 0,
  ADER_E_ARG = -1,      /* invalid argument (null pointer, size, range)              */
  ADER_E_MESH = -2,     /* clockwise/degenerate triangle, non-manifold, bad boundary */
  ADER_E_STATE = -3,    /* rho <= 0, p <= 0 or NaN after an update                   */
  ADER_E_GEOM = -4,     /* element inverted by the mesh motion                        */
  ADER_E_GCL = -5,      /* space-time volume not closed (geometric conservation law) */
  ADER_E_DEADLOCK = -6, /* no element satisfies the update criterion                  */
  ADER_E_HIP = -7,      /* HIP runtime error                                          */
  ADER_E_ORDER = -8     /* call out of sequence                                       */
};

/* Numerical fluxes (ader_config.flux).
 *  RUSANOV: eq. eqn.rusanov with the largest |eigenvalue| of eq. A_n^V.
 *  OSHER:   eq. eqn.osher on the straight-line path of eq. eqn.path, the path
 *           integral of |A| = R |Lambda| R^-1 by 3-point Gauss-Legendre in s.
 *  HLL:     two-wave HLL flux with the ALE signal speeds u.N + N_t -/+ c |N_xy|
 *           bounded over both states (not in the paper). */
enum { ADER_FLUX_RUSANOV = 0, ADER_FLUX_OSHER = 1, ADER_FLUX_HLL = 2 };

/* Boundary tags of ader_upload_mesh.  A transmissive edge takes as outer
 * state the inner element's predicted cell mean at each flux point's time
 * (a ghost copy of the element); a slip wall takes the mirror image of the
 * inner state, and its nodes slide along the wall. */
enum { ADER_BC_TRANSMISSIVE = 1, ADER_BC_SLIP = 2 };

typedef struct ader_ctx ader_ctx;

/* Scheme parameters (paper Sec. 2.2 after eq. Sigma, eq. eqn.timestep). */
typedef struct {
  int32_t M;             /* polynomial degree 1..3; order of accuracy M+1              */
  int32_t flux;          /* ADER_FLUX_*: numerical flux on the space-time patches       */
  double gamma;          /* ratio of specific heats (eq. eqn.eos)                      */
  double cfl;            /* CFL number of eq. eqn.timestep, (0, 0.5]                   */
  int32_t lts_levels;    /* L in 1..8: dyadic levels used by ader_step_lts;
                            0: free local steps (see ader_step_lts)                    */
  int32_t n_picard;      /* Picard sweeps of the predictor; 0 -> M+1                   */
  int32_t mesh_velocity; /* 0 = Lagrangian (V = v), 1 = Eulerian (V = 0)               */
  double weno_eps;       /* epsilon of the WENO weights (paper: 1e-14)                 */
  double weno_r;         /* exponent r (paper: 8; only 8 is supported)                 */
  double weno_lambda;    /* central-stencil linear weight lambda_1 (paper: 1e5)        */
  double lts_step_fraction; /* theta in (0, 1]: with L >= 2 dyadic levels the nominal
                            finest step of a macro step is theta times the smallest
                            CFL step at its start (0 -> the default 0.95, which
                            leaves room for the CFL step's usual decrease within a
                            macro step); L = 1 ignores it                          */
} ader_config;

typedef struct {
  int64_t element_updates; /* sum over cycles of the active-set size                   */
  int64_t cycles;          /* cycles run (a cycle = one pass of the update criterion)  */
  int64_t macro_steps;     /* macro steps completed (free steps: one per target time)  */
  int64_t cfl_overshoots;  /* element steps longer than their CFL bound (a step of one
                              tick, 2^-30 of the macro step, still too long)          */
  double max_gcl_residual; /* max |closure of the space-time volume| / (|T|+|T'|)      */
  double t;                /* common time of all elements (they meet at macro steps);
                              with several instances the earliest instance time        */
  double delta;            /* tick length of the last macro step (of instance 0)       */
  int64_t predictor_evals; /* element predictors computed                              */
  int64_t patches;         /* space-time patches integrated                            */
  int64_t node_moves;      /* node motions                                             */
  int64_t extra_cycles;    /* cycles beyond 2^(L-1) per macro step, run because some
                              element's CFL step fell below the nominal finest step
                              during the macro step (spare finer levels)             */
  int64_t long_macro_steps;/* macro steps that needed such extra cycles              */
  int64_t replay_overrides;/* under schedule replay: replayed steps that differ from
                              the level rule's own choice                            */
} ader_stats;

/* Create a context.  hip_stream: a hipStream_t (NULL = default stream).
 * Allocates host memory only; no device call is made. */
int ader_create(const ader_config* cfg, void* hip_stream, ader_ctx** out);

/* Mesh topology and initial node positions (paper eqs. trian, xietaTransf).
 * node_xy: host [n_nodes][2]; tri: host [n_elems][3], counter-clockwise;
 * bedge: host [n_bedges][3] = (node a, node b, tag) for every boundary edge,
 * oriented with the interior on the left of a->b.  Builds, on the host, the
 * edges, node rings, the 7 WENO stencils of n_e = (M+1)(M+2) elements and
 * the symmetric scheduling stencils (eqs. stencil, eqn.WENOstencil and the
 * discussion after eqn.WENOupdate).  No device call.  ADER_E_MESH on a
 * clockwise or degenerate triangle, a non-manifold edge, a boundary list
 * that does not match the mesh, or a mesh too small for the central stencil.
 * ADER_E_ARG on an empty mesh or n_elems * n_e * 8 >= 2^31 (32-bit indices of
 * the stencil rows: 13.4 M triangles at M = 3, 22 M at M = 2). */
int ader_upload_mesh(ader_ctx* ctx, int32_t n_nodes, const double* node_xy,
                     int32_t n_elems, const int32_t* tri,
                     int32_t n_bedges, const int32_t* bedge);

/* Device bytes needed for state, topology and scratch of this mesh. */
int ader_workspace_size(const ader_ctx* ctx, size_t* bytes);

/* Batch of independent simulations (optional; default one instance): the
 * mesh of ader_upload_mesh is n_instances meshes concatenated, instance k
 * owning elements [elem_first[k], elem_first[k+1]) (elem_first has
 * n_instances+1 entries, elem_first[0] = 0, elem_first[n_instances] =
 * n_elems).  Instances share no node (else ADER_E_MESH).  Each keeps its own
 * time and its own macro-step tick length (the smallest CFL step of its own
 * elements); all step through the same macro-step structure in the same
 * kernel launches, and each stops at t_target.  Call after ader_upload_mesh,
 * before ader_workspace_size. */
int ader_set_instances(ader_ctx* ctx, int32_t n_instances, const int32_t* elem_first);

/* Hand the library a caller-owned device buffer of at least
 * ader_workspace_size bytes (256-byte aligned).  It must outlive the context.
 * Copies the topology and tables to it (synchronises the stream). */
int ader_bind_workspace(ader_ctx* ctx, void* dev_ptr, size_t bytes);

/* Initial cell averages, device [4][n_elems] SoA (rho, rho u, rho v, rho E),
 * at time t0, on the mesh of ader_upload_mesh (node positions are reset to
 * that mesh).  Runs the pre-processing of the paper (Sec. 2.6): first
 * reconstruction without projection and first CFL time step of every
 * element.  ADER_E_STATE on rho <= 0 or p <= 0. */
int ader_upload_state(ader_ctx* ctx, const double* Q_dev, double t0);

/* The same with the node positions too: node_xy_dev, device [n_nodes][2]
 * (the layout of ader_download_state), or NULL for the mesh of
 * ader_upload_mesh.  Restores a state of a Lagrangian run on a moved mesh
 * (topology, stencils and slip-wall normals stay those of the uploaded mesh,
 * paper Sec. 2.2: fixed stencils).  ADER_E_GEOM when an element is inverted
 * or degenerate at those positions. */
int ader_upload_state_xy(ader_ctx* ctx, const double* Q_dev, const double* node_xy_dev, double t0);

/* Global time stepping up to t_target (at most max_steps steps; <= 0 means
 * no limit): one level, every element updates in every step. */
int ader_step_gts(ader_ctx* ctx, double t_target, int32_t max_steps, ader_stats* st);

/* Local time stepping up to t_target in at most max_macro_steps macro steps
 * (<= 0: no limit), paper Sec. 2.6 with dyadic steps.  A macro step spans
 * 2^(L-1) times the smallest CFL step (eq. eqn.timestep) at its start, cut into
 * 2^30 integer ticks of length delta (clamped so it ends at t_target at the
 * latest); each element steps the largest power of two of ticks within its
 * CFL step, aligned to its current tick, under the update criterion of eq.
 * eqn.WENOupdate over its scheduling stencil; all elements meet again at the
 * end of the macro step.  Steps below the nominal finest one (2^(31-L) ticks)
 * are taken only by elements whose CFL step fell below it during the macro
 * step; the macro step then needs cycles beyond its 2^(L-1) (stats:
 * extra_cycles), so no step exceeds its element's CFL bound.
 * lts_levels == 0 (free local steps, Sec. 2.3 with each element at its own CFL
 * step of eq. eqn.timestep): the whole interval to t_target is one macro step
 * of 2^30 ticks of length (t_target - t) / 2^30; an element steps
 * floor(dt_CFL / delta) ticks, at most to the end of the interval (at least
 * one: counted as a CFL overshoot, so t_target - t must stay well below 2^30
 * CFL steps).  Cycles run in batches of 16 with a host check after each;
 * `cycles` counts the launched ones.  Results match the oracle's reading. */
int ader_step_lts(ader_ctx* ctx, double t_target, int32_t max_macro_steps, ader_stats* st);

/* Current time of the first n instances into host memory (synchronises). */
int ader_instance_times(ader_ctx* ctx, int32_t n, double* T_host);

/* Launch choices that leave every result bit-identical: elements per
 * workgroup of the scheduler (0: built-in rule), workgroups per CU of the
 * reconstruction and predictor launches over the active list (0: one grid
 * covering every element), and workgroups per CU of the node and patch
 * launches that sweep every node and edge (0: one grid over all of them;
 * else a persistent grid whose workgroups stride them). */
typedef struct {
  int32_t sched_chunk;        /* 0 or 32..1024 */
  int32_t list_wg_per_cu;     /* 0 or 1..64    */
  double ms_per_macro_step;   /* ader_autotune: time of the chosen setting     */
  int32_t sweep_wg_per_cu;    /* 0 or 1..64    */
  int32_t reserved;           /* 0             */
} ader_tune;

/* Set the launch choices explicitly. */
int ader_set_tune(ader_ctx* ctx, const ader_tune* tune);

/* Autotuner: from a snapshot of the current device state, times
 * `trial_macro_steps` LTS macro steps (levels of the configuration, 3 under
 * free steps; no target time) for each candidate setting, one coordinate at a
 * time (scheduler chunk in {rule, 64, 128, 256, 512, 1024}, then workgroups
 * per CU of the list launches in {all, 4, 8, 16, 32}, then of the node and
 * edge sweeps in {all, 4, 8, 16}), keeps the fastest, and restores the state,
 * so the simulation does not advance.  Allocates a device copy of the workspace for the duration
 * (hipMalloc).  The choice is written to *chosen when not null. */
int ader_autotune(ader_ctx* ctx, int32_t trial_macro_steps, ader_tune* chosen);

/* Schedule replay for parity tests (Sec. 2.6: which step each element takes).
 * step_ptr: host [n_elems + 1], step_ptr[0] = 0, non-decreasing, step_ptr[n_elems]
 * = n_steps; steps: host [n_steps]; element i takes, in order, the steps (in
 * ticks) steps[step_ptr[i] .. step_ptr[i+1]) at its step decisions (at each
 * macro-step start and after each update that leaves it short of the
 * macro-step end) instead of the level rule's, e.g. the steps another
 * implementation took, so that a decision taken in floating point on both
 * sides (a CFL step at a level boundary, a free step's floor) cannot flip.
 * The library copies the tables into device memory it allocates (hipMalloc)
 * and owns; positions restart at zero here and at ader_upload_state.
 * stats.replay_overrides counts replayed steps that differ from the rule's.
 * A missing entry or a step that would leave the macro step fails the next
 * stepping call with ADER_E_ARG.  step_ptr == NULL switches replay off.
 * Synchronises the stream. */
int ader_set_schedule_replay(ader_ctx* ctx, const int32_t* step_ptr, const int32_t* steps, int64_t n_steps);

/* Tick-length replay: macro step m (counted from the last state upload)
 * takes deltas[m] as its tick length instead of the one computed from the
 * smallest CFL step (still clamped so that the macro step does not pass the
 * target time); with ader_set_schedule_replay this fixes the whole schedule,
 * e.g. to take differences of runs from perturbed data.  deltas: host
 * array of n positive tick lengths (copied); n = 0 turns it off.  One
 * instance only (ADER_E_ARG otherwise).  A run past the last entry stops with
 * ADER_E_ARG. */
int ader_set_delta_replay(ader_ctx* ctx, const double* deltas, int32_t n);

/* Schedule record: from this call on, every step an element takes (its level
 * rule's, or the replayed one) is appended to that element's record, at most
 * steps_per_element of them, and the tick length of each macro step (counted
 * from the last state upload) is kept, at most macro_steps of them; a run
 * that exceeds a capacity stops with ADER_E_ARG.  steps_per_element = 0 turns
 * it off.  One instance only.  ader_get_schedule_record copies the record to
 * host memory: step_ptr [n_elems + 1] (CSR offsets, always written), steps
 * [steps_cap] and deltas [deltas_cap] (either may be NULL: then only the
 * counts *n_steps and *n_deltas are returned), in the layout that
 * ader_set_schedule_replay and ader_set_delta_replay take.  Synchronises. */
int ader_set_schedule_record(ader_ctx* ctx, int32_t steps_per_element, int32_t macro_steps);
int ader_get_schedule_record(ader_ctx* ctx, int32_t* step_ptr, int32_t* steps, int64_t steps_cap, double* deltas,
                             int32_t deltas_cap, int64_t* n_steps, int32_t* n_deltas);

/* Launch mode of ader_step_gts / ader_step_lts.  on != 0 (the default): each
 * macro step (levels and predictors, its 2^(L-1) cycles, the unfinished count
 * and the macro-step end) is one HIP graph, captured on a private stream of
 * the context at the first step with a given number of levels and replayed on
 * the context's stream (the target time is read from device memory, so one
 * graph serves every target); one host synchronisation per macro step, more
 * only when extra cycles are needed (two cycles per captured batch). on == 0:
 * the same kernels are launched one by one.  Results are identical.  While
 * profiling is on, kernels are always launched one by one. */
int ader_set_graphs(ader_ctx* ctx, int32_t on);

/* ---- Adjoint of one global time step (reverse mode) ----------------------
 * The step map Q^n -> Q^{n+1} of global time stepping of length dt from the
 * current state, on a fixed mesh (mesh_velocity = 1: the mesh ODE of eq.
 * ODEmesh with V = 0, so |T'| = |T|) with the Rusanov or HLL flux: WENO
 * reconstruction with the neighbours' real averages (eqs. intConsRec ..
 * eqn.weno), space-time predictor (eq. CGfinal), fluxes over the space-time
 * faces of the edges with (M+1)^2 Gauss points (eqs. eqn.rusanov,
 * eqn.STint) and the update of eq. PDEfinal.  ader_adjoint_gts_step writes
 * Qbar = (dQ^{n+1}/dQ^n)^T Qbar_next with dt held fixed (the dependence of
 * the CFL step of eq. eqn.timestep on the state is not differentiated);
 * subgradients: the larger Rusanov signal speed, and the bounding HLL speeds,
 * are taken from the left state on ties, d|x|/dx = 0 at 0.  ADER_E_ARG with
 * the Osher flux.  It does not change the simulation state.
 *   Q_dev: device [4][n_elems] SoA averages Q^n to differentiate at, or NULL
 *     for the context's current averages (then every element must be at one
 *     common time);
 *   Qbar_next_dev, Qbar_dev: device [4][n_elems] SoA (same layout as Q),
 *     not overlapping;
 *   work_dev: caller device memory of at least ader_adjoint_workspace_size
 *     bytes, 256-byte aligned, used as scratch by the call only.
 * Preconditions: a single instance, state uploaded (the fixed geometry), and
 * with Q_dev == NULL every element at one common time (after
 * ader_upload_state or a completed stepping call; not after the test hooks)
 * -> else ADER_E_ARG / ADER_E_ORDER.  Queued on the
 * context's stream; no synchronisation.  The step that
 * ader_step_gts(ctx, t + dt, 1, ...) takes from the same state is the one
 * differentiated when dt is at most the smallest CFL step. */
int ader_adjoint_workspace_size(const ader_ctx* ctx, size_t* bytes);
int ader_adjoint_gts_step(ader_ctx* ctx, double dt, const double* Q_dev, const double* Qbar_next_dev,
                          double* Qbar_dev, void* work_dev, size_t work_bytes);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the step
 * adjoint of ader_adjoint_gts_step, same arguments and preconditions, with its
 * scratch in a fixed device array of ADER_STATIC_SCRATCH_BYTES that the
 * library holds on every GPU it runs on until the process ends (its address
 * on the context's GPU is looked up once, by ader_bind_workspace).  Calls no
 * allocating routine.  ADER_E_ARG when ader_adjoint_workspace_size exceeds
 * ADER_STATIC_SCRATCH_BYTES (M = 2 fits ~26k triangles).  Every call on one
 * GPU uses the same array, which keeps the last call's contents (nothing in it
 * is read before the call writes it): calls that overlap on one GPU, from
 * any stream or context, race and must be serialised by the caller. */
#define ADER_STATIC_SCRATCH_BYTES ((size_t)256 << 20)
int ader_adjoint_gts_step_static(ader_ctx* ctx, double dt, const double* Q_dev,
                                 const double* Qbar_next_dev, double* Qbar_dev);

/* ---- Adjoint of one global step on the moving (Lagrangian) mesh ----------
 * The step map (Q^n, X^n) -> (Q^{n+1}, X^{n+1}) of global time stepping of
 * length dt with the mesh moving with the fluid (mesh_velocity = 0, V = v in
 * eq. ODEmesh) and the Rusanov or HLL flux: reconstruction on the current geometry
 * (eqs. intConsRec .. eqn.weno), predictor of the PDE and the mesh ODE (eqs.
 * CGfinal, VCG, newVertPos), node solver with mass weights rho |T| and the
 * velocities averaged over the step (eqs. eqnNScs, eqn.NScs.weights,
 * NodesVel, eqn.newVertex), fluxes over the bilinear space-time patches of
 * the moving edges (eqs. eqn.spacetimenodes, G_ij, eqn.STint) and the update
 * with the new areas (eq. PDEfinal).  Writes Qbar = (dQ^{n+1}/dQ^n)^T Qbar_next
 * + (dX^{n+1}/dQ^n)^T Xbar_next and Xbar likewise with respect to X^n, dt held
 * fixed; subgradients as for ader_adjoint_gts_step.  Optionally also the
 * forward result.  It does not change the simulation state.
 *   Q_dev: device [4][n_elems] SoA averages Q^n, or NULL for the context's;
 *   X_dev: device [n_nodes][2] node positions X^n, or NULL for the context's
 *     (NULL for either: every element must be at one common time);
 *   Qbar_next_dev, Qbar_dev: device [4][n_elems] SoA;
 *   Xbar_next_dev, Xbar_dev: device [n_nodes][2];
 *   Q_next_dev ([4][n_elems]), X_next_dev ([n_nodes][2]): device buffers for
 *     (Q^{n+1}, X^{n+1}), or NULL;
 *   work_dev: caller device memory of at least
 *     ader_adjoint_lagrangian_workspace_size bytes, 256-byte aligned, scratch
 *     of the call only.  No output may overlap an input.
 * Slip walls: the outer state is the mirrored inner one (its dependence on the
 * patch normal included) and wall nodes slide or stay pinned as in the
 * forward step.  ADER_E_ARG for a fixed mesh, the Osher flux, a batch of
 * instances, a workspace too small; ADER_E_ORDER before a state upload.
 * Queued on the context's stream; no synchronisation.  With dt at most the
 * smallest CFL step, the step that ader_step_gts(ctx, t + dt, 1, ...) takes
 * from the same state is the one differentiated. */
int ader_adjoint_lagrangian_workspace_size(const ader_ctx* ctx, size_t* bytes);
int ader_adjoint_lagrangian_step(ader_ctx* ctx, double dt, const double* Q_dev, const double* X_dev,
                                 const double* Qbar_next_dev, const double* Xbar_next_dev, double* Qbar_dev,
                                 double* Xbar_dev, double* Q_next_dev, double* X_next_dev, void* work_dev,
                                 size_t work_bytes);

/* ---- Gradient through macro steps of the local time stepping -------------
 * Dyadic LTS (Sec. 2.6; lts_levels >= 1) or free local steps (lts_levels = 0:
 * one macro step to t_end) on the mesh moving with the fluid (mesh_velocity = 0)
 * or on a fixed mesh (mesh_velocity = 1: V = 0 in eq. ODEmesh, the node
 * positions still differentiated through the geometry) with the Rusanov or
 * HLL flux, differentiated with its schedule held fixed:
 * the tick length of every macro step and every element's sequence of steps
 * are those the forward run takes (with ader_set_schedule_replay, the
 * replayed ones), so the update sets and the moved nodes and swept edges of
 * every cycle are fixed; the averages and node positions are differentiated
 * through the pre-processing reconstruction, the virtual projection of the
 * stencils in space and time (eqs. eqn.virtGeom, eqn.virtCellaverage), the
 * predictor with the mesh ODE (eqs. CGfinal, VCG, newVertPos), the node
 * solver over each node's own interval (eqs. eqn.dtau, NodesVel, eqnNScs,
 * eqn.NScs.weights, eqn.newVertex), the swept patches with corners at
 * different times (eqs. eqn.spacetimenodes, eqn.STint), the memory variables
 * (eq. eqn.Qm2) and the updates (eq. PDEfinal).  From the uploaded state
 * (Q_0, X_0) (no step may have been taken since ader_upload_state*), runs up
 * to n_macro macro steps towards t_end (fewer when t_end is reached first:
 * *n_done) and writes Qbar0 = (dQ_end/dQ_0)^T Qbar + (dX_end/dQ_0)^T Xbar and
 * Xbar0 likewise with respect to X_0; subgradients as for
 * ader_adjoint_gts_step.  The context ends at the state after the macro steps,
 * as ader_step_lts would leave it.
 *   Qbar_dev, Qbar0_dev: device [4][n_elems] SoA; Xbar_dev, Xbar0_dev:
 *   device [n_nodes][2]; no output may overlap an input.
 * Memory (allocated by the library and freed before returning): for the last
 * keep_macro_steps macro steps (-1: as many as 60% of the free device memory
 * holds, counting 2^(L-1) + 3 states each) the forward keeps the state the
 * reverse sweep reads (ticks, element records, traces, reconstructions, node
 * positions and ticks; about 1.5 KB per element at M = 2) after the
 * macro-step start and after every cycle; every earlier macro step keeps its
 * full state at the start only and is replayed cycle by cycle when the sweep
 * reaches it (one more forward pass over those steps).  Scratch of about
 * 1.2 KB per element at M = 2.  Synchronises.
 * ADER_E_ARG for the Osher flux, a batch of instances or n_macro < 1; ADER_E_ORDER before a state upload or after a step; the
 * forward run's own errors as ader_step_lts. */
int ader_adjoint_lts(ader_ctx* ctx, int32_t n_macro, int32_t keep_macro_steps, double t_end, const double* Qbar_dev,
                     const double* Xbar_dev, double* Qbar0_dev, double* Xbar0_dev, int32_t* n_done);

/* ---- Measurement: the predictor's derivative contraction -----------------
 * Not a step of the scheme: runs, in one timed launch on the context's
 * stream, `iters` rounds of the space-time predictor's spatial-derivative
 * contraction (D_xi and D_eta of eq. CGfinal's nodal basis applied to ten
 * fields at the six nodes of each of n_elems elements, fed back as
 * q <- q/2 + (d_xi q + d_eta q)/20) in the lane layout of the step's predictor,
 * on the vector ALUs (use_mfma = 0) or on the matrix cores (use_mfma = 1,
 * v_mfma_f64_16x16x4f64 over ten elements per wavefront), so that the two can
 * be timed and profiled against each other.  F_dev, out_dev: device
 * [n_elems][10][6] (element, field, node), not overlapping; ms: the launch's
 * duration (HIP events; synchronises the stream).  Needs M = 2 and a bound
 * workspace (the tables), else ADER_E_ARG / ADER_E_ORDER. */
int ader_probe_contraction(ader_ctx* ctx, int32_t use_mfma, int64_t n_elems, int32_t iters, const double* F_dev,
                           double* out_dev, float* ms);

/* Current state into caller device buffers (any may be NULL):
 * Q_dev [4][n_elems] SoA, node_xy_dev [n_nodes][2], elem_t_dev [n_elems]. */
int ader_download_state(ader_ctx* ctx, double* Q_dev, double* node_xy_dev, double* elem_t_dev);

/* Cumulative statistics since ader_upload_state (synchronises). */
int ader_get_stats(ader_ctx* ctx, ader_stats* st);

/* ---- Test hooks: raw access to internal arrays ----------------------------
 * ader_debug_dump copies the array `what` to host memory; ader_debug_inject
 * overwrites it from host memory.  `bytes` must equal the array size returned
 * by ader_debug_size.  Topology arrays (ADER_DBG_TOPO_*, ADER_DBG_TAB_*) live
 * on the host and are available right after ader_upload_mesh with no device.
 * Layouts (NE elements, NV nodes, NF edges, nb = (M+1)(M+2)/2, T = M+1, nG = M+1):
 *   Q [4][NE]  A [NE]  XE [6][NE] (x0 y0 x1 y1 x2 y2)  TICK, STEP [NE] int32
 *   DTCFL [NE]  QM [4][NE]  HM [3][NE]  WNOD [nb][4][NE]  AVG [T][4][NE]
 *   TRACE [3][nG][T][4][NE]  VVEL [3][T][2][NE]  X [2][NV]  NTICK [NV] int32
 *   SCAL [4] double: T, delta, N (as double), t_end
 *   TOPO_EDGES [NF][6] int32: a, b, L, R, local edge in L, in R (-1)
 *   TOPO_STENCILS [NE][7][n_e] int32 (-1 rows: dropped sector stencil)
 *   TOPO_SCHED_PTR [NE+1] int32, TOPO_SCHED_IDX [nnz] int32
 *   TOPO_TSTEN_PTR [NE+1] int32, TOPO_TSTEN_IDX [nnz] int32: for each element j
 *     the stencil rows that name it, as (i * n_e + c) * 8 + s (row c >= 1 of
 *     stencil s of element i), ascending (the adjoint's gather lists)
 *   TAB_* host tables: see ader_debug_size. */
enum {
  ADER_DBG_Q = 0, ADER_DBG_A, ADER_DBG_XE, ADER_DBG_TICK, ADER_DBG_STEP, ADER_DBG_DTCFL,
  ADER_DBG_QM, ADER_DBG_HM, ADER_DBG_WNOD, ADER_DBG_AVG, ADER_DBG_TRACE, ADER_DBG_VVEL,
  ADER_DBG_X, ADER_DBG_NTICK, ADER_DBG_SCAL,
  ADER_DBG_TOPO_EDGES = 32, ADER_DBG_TOPO_STENCILS, ADER_DBG_TOPO_SCHED_PTR,
  ADER_DBG_TOPO_SCHED_IDX, ADER_DBG_TOPO_TSTEN_PTR, ADER_DBG_TOPO_TSTEN_IDX,
  ADER_DBG_TAB_DXI = 48, ADER_DBG_TAB_DETA, ADER_DBG_TAB_AMEAN, ADER_DBG_TAB_EDGE,
  ADER_DBG_TAB_AT, ADER_DBG_TAB_BT, ADER_DBG_TAB_DT, ADER_DBG_TAB_PSIC, ADER_DBG_TAB_SIGMA,
  ADER_DBG_TAB_GAUSS
};
int ader_debug_size(const ader_ctx* ctx, int32_t what, size_t* bytes);
int ader_debug_dump(ader_ctx* ctx, int32_t what, void* host, size_t bytes);
int ader_debug_inject(ader_ctx* ctx, int32_t what, const void* host, size_t bytes);

/* Test hook: run `n` cycles of the current macro step (no macro boundary
 * handling), or begin a macro step (levels and predictors) toward t_end with
 * `levels` dyadic levels (0: free steps, 2^30 ticks). */
int ader_debug_cycles(ader_ctx* ctx, int32_t n);
int ader_debug_macro_begin(ader_ctx* ctx, double t_end, int32_t levels);

/* Per-kernel timing for benchmarks: a stage of one kernel launch is timed by
 * start and stop events attached to that launch (the kernel's own execution);
 * a stage of several launches (macro-step boundary, status, adjoint) by HIP
 * events recorded before and after it on the context's stream.  ader_set_profiling(ctx, 1) clears the
 * totals and starts recording, 0 stops.  ader_kernel_times synchronises and
 * writes, for each kernel id k < n (ADER_K_*), the summed milliseconds and
 * the number of launches since profiling was switched on. */
enum {
  ADER_K_SCHED = 0,   /* update criterion and active-list compaction            */
  ADER_K_NODE,        /* node solver and node motion                            */
  ADER_K_PATCH,       /* space-time patch fluxes                                */
  ADER_K_UPDATE,      /* memory variables and conservative update               */
  ADER_K_RECON,       /* virtual projection, WENO, CFL step and level           */
  ADER_K_PREDICT,     /* space-time predictor                                   */
  ADER_K_MACRO,       /* macro-step boundary: min CFL step, levels              */
  ADER_K_STATUS,      /* unfinished-element count                               */
  ADER_K_ADJOINT,     /* ader_adjoint_gts_step (all its kernels)                */
  ADER_K_COUNT
};
int ader_set_profiling(ader_ctx* ctx, int32_t on);
int ader_kernel_times(ader_ctx* ctx, int32_t n, double* total_ms, int64_t* launches);

/* Message of the last error on this context (never NULL). */
const char* ader_last_error(const ader_ctx* ctx);

/* Free the context (not the caller's workspace). */
void ader_destroy(ader_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* ADERWENO_H */
