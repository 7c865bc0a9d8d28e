// Shared host/device definitions of the aderweno library.
#pragma once
#include <cstddef>
#include <cstdint>

namespace aw {

constexpr int MAXM = 3;
constexpr int MAXNB = 10;   // (M+1)(M+2)/2
constexpr int MAXT = 4;     // time nodes M+1
constexpr int MAXG = 4;     // Gauss points per patch direction, M+1
constexpr int MAXRQ = 7;    // points of the reconstruction triangle rule
constexpr int NSTEN = 7;    // 1 central + 3 primary + 3 reverse sector stencils

// Reference-element tables (built on the host, read by every kernel through
// the scalar cache).  Index conventions:
//   monomial k <-> xi^monoA[k] eta^monoB[k], ordered by total degree;
//   lattice node m = (i/M, j/M), i+j <= M, ordered by j then i;
//   psi_0 = 1, every other psi_l has zero mean on the reference triangle.
struct Tables {
  int M, nb, nt, nG, ne, nrq;
  int vtx[3];                       // lattice index of the reference vertices
  int monoA[MAXNB], monoB[MAXNB];
  double psiC[MAXNB][MAXNB];        // psi_l = sum_k psiC[l][k] mono_k
  double Sigma[MAXNB][MAXNB];       // oscillation indicator matrix
  double psiNodes[MAXNB][MAXNB];    // psi_l at lattice node m: [m][l]
  double Dxi[MAXNB][MAXNB];         // d/dxi of the nodal interpolant at node m': [m'][m]
  double Deta[MAXNB][MAXNB];
  double amean[MAXNB];              // mean over T_e of the nodal basis function m
  double edge[3][MAXG][MAXNB];      // nodal basis at Gauss point g of reference edge e
  double At[MAXT][MAXT];            // rows r = 0..M-1 <-> time nodes 1..M
  double Bt[MAXT];
  double Dt[MAXT][MAXT];            // d/dtau of the time interpolant at node q': [q'][q]
  double lag[MAXT][MAXT + 1];       // l_q(tau) = sum_k lag[q][k] tau^k
  double Lint[MAXT][MAXT + 2];      // int_0^tau l_q = sum_k Lint[q][k] tau^k
  double gchi[MAXG], gw[MAXG];      // Gauss-Legendre on [0,1]
  double rqw[MAXRQ];                // triangle rule, exact to degree M (barycentric)
  double rqb[MAXRQ][3];
  double osh_s[3], osh_w[3];        // Gauss-Legendre on [0,1] for the Osher path integral
};

struct Params {
  double gamma, cfl, eps, lambda, gcl_tol;
  int npic;
  int lagrangian;
  int flux;         // ADER_FLUX_*
};

// One simulation of a batch: independent meshes are concatenated (no shared
// node), each with its own time and tick length; an unbatched run is one
// instance. All instances step through the same macro-step structure.
struct Inst {
  double T;                        // common time at the start of the macro step
  double delta;                    // tick length of the macro step (0 while closed)
  unsigned long long min_dt_bits;  // min CFL step over its elements (as ordered bits)
  int open;                        // 1 while short of the target time
  int pad;
};

// Device-resident scalars of the running simulation.
struct Scal {
  double t_end;     // target time of the current call (set before a run, read by the kernels)
  int N;            // ticks per macro step
  int n_open;       // instances short of the target time
  // n_active and n_live share one 8-byte word (little-endian, n_active low):
  // one 64-bit atomic reserves space in both lists
  alignas(8) int n_active;  // active elements of the current cycle
  int n_live;       // active elements that stay short of tick N (they need a new predictor)
  int n_unfinished; // elements that have not reached tick N
  int err;          // sticky error bits (ERR_*)
  int cycle;        // stamp of the current cycle (advanced by the cycle's first kernel)
  int pad;
  unsigned long long max_gcl_bits;  // max relative GCL residual
  unsigned long long updates;
  unsigned long long overshoots;
  unsigned long long n_pred;    // predictor evaluations
  unsigned long long n_patch;   // space-time patches integrated
  unsigned long long n_node;    // node moves
  unsigned long long replay_overrides;   // replayed steps that differ from the level rule's
  int macro_index;  // macro steps ended since the state upload
  int pad2;
};

static_assert(offsetof(Scal, n_live) == offsetof(Scal, n_active) + sizeof(int) &&
                  offsetof(Scal, n_active) % 8 == 0,
              "n_active and n_live must form one aligned 8-byte word");

enum : int { ERR_GEOM = 1, ERR_STATE = 2, ERR_GCL = 4, ERR_PRED = 8, ERR_DT = 16, ERR_REPLAY = 32, ERR_RECORD = 64 };

// Ticks per macro step. Free local time steps: the interval to the target
// time is one macro step of FREE_TICKS ticks; every element steps
// floor(dt_CFL / delta) ticks. Dyadic levels: a macro step of L levels spans
// 2^(L-1) smallest CFL steps and is cut into the same number of ticks, so the
// nominal finest step is 2^(31-L) ticks and the powers of two below it are
// spare levels for elements whose CFL step falls below it during the macro
// step (no step exceeds its element's CFL step).
constexpr int FREE_TICKS = 1 << 30;
constexpr int MACRO_TICKS = FREE_TICKS;

// Per-element storage.  Data that other elements gather (vertices, average,
// area, the predictor's time-node averages and vertex velocities) sits in one
// contiguous record per element, so a neighbour costs a few cache lines
// instead of one line per field; edge traces are contiguous per element too.
//   record: [0,6) vertices x0 y0 x1 y1 x2 y2 | [6,10) Q | 10 area |
//           [11, 11+4T) averages at time node t (t*4+v) |
//           [11+4T, 11+10T) vertex velocities ((k*T+t)*2+c)
//   trace:  ((e*nG+g)*T+t)*4+v        wnod: m*4+v
constexpr int rec_off_xe() { return 0; }
constexpr int rec_off_q() { return 6; }
constexpr int rec_off_a() { return 10; }
constexpr int rec_off_avg() { return 11; }
constexpr int rec_off_vv(int M) { return 11 + 4 * (M + 1); }
constexpr int round16(int n) { return (n + 15) / 16 * 16; }
constexpr int rec_stride(int M) { return round16(11 + 10 * (M + 1)); }
constexpr int trace_stride(int M) { return round16(3 * (M + 1) * (M + 1) * 4); }
constexpr int wnod_stride(int M) { return (M + 1) * (M + 2) / 2 * 4; }

constexpr int MEM_W = 8;   // doubles per memory-variable slot (G, N, one pad)

struct TickStep {   // tick in the macro step and step length in ticks (0: finished)
  int tick, step;
};

// Pointers into the caller's workspace.
struct Dev {
  int NE, NV, NF, M, K;
  // launch choices (host side; 0 = built-in default): elements per scheduler
  // workgroup, and workgroups per CU of the list-driven reconstruction and
  // predictor launches (0: one workgroup per slice of the whole element range)
  int sched_chunk, list_wg_per_cu, n_cu;
  // workgroups per CU of the node and patch launches, which sweep every node
  // and edge (0: one grid over all of them; else a persistent grid striding them)
  int sweep_wg_per_cu;
  int free_steps;   // 1: free local steps (one macro step of FREE_TICKS to the target)
  Scal* scal;
  Inst* inst;                        // [K]
  const int *e_inst, *v_inst;        // instance of each element [NE] and node [NV]
  const Tables* tab;
  // elements
  double* rec;        // [NE][rec_stride]
  double* trace;      // [NE][trace_stride]
  double* wnod;       // [NE][wnod_stride]
  TickStep* ts;       // [NE]
  double* dtcfl;      // [NE]
  // memory variables per (element, local edge), accumulated by the swept
  // patches of that edge since the element's last update: flux (4) and
  // space-time normal integral (3), MEM_W doubles per slot, [NE][3][MEM_W]
  double* mem;
  int *act_stamp, *act_list;
  int* live_list;     // the active elements that stay short of tick N after the update
  const int *tri, *elem_edges, *neigh, *sten, *sched_ptr, *sched_idx;   // SoA [k][NE]
  const int *tsten_ptr, *tsten_idx;   // stencil rows naming each element (adjoint gather)
  // nodes
  double *X, *Xnew;   // [2][NV]
  int *ntick, *ntick_new, *node_stamp;
  const int *ring_ptr, *ring_ent;   // ring entry = element * 4 + local vertex
  const double* wall_n;             // [2][NV] slip-wall normal (0 off walls)
  const int* wall_pin;              // node held fixed (two walls meet)
  // edges
  const int *e_a, *e_b, *e_L, *e_R, *e_el, *e_er, *e_bc;
  // schedule replay (null when off): element i takes, in order, the steps
  // replay_steps[replay_ptr[i] .. replay_ptr[i+1]); replay_pos[i] counts them
  const int *replay_ptr, *replay_steps;
  int* replay_pos;
  // tick-length replay (null when off; one instance): macro step m takes
  // replay_delta[m] (clamped to the target time as the computed one)
  const double* replay_delta;
  int replay_delta_n;
  // schedule record (null when off): element i's k-th step at
  // rec_steps[i * rec_cap + k], rec_pos[i] of them; macro step m's tick length
  // at rec_delta[m] (m < rec_delta_cap; one instance)
  int* rec_steps;
  int* rec_pos;
  int rec_cap;
  double* rec_delta;
  int rec_delta_cap;
};

// Buffers of the reverse-mode step (adjoint.hip), carved from the caller's
// adjoint workspace; nodal space-time data are element-minor ([slot][NE]).
struct AdjWork {
  const double* q;           // [4][NE] averages at the step start (the caller's, or a copy)
  double* qcopy;             // [4][NE] copy of the context's averages
  const double* qbar_next;   // [4][NE] adjoint of the averages after the step
  double* qbar;              // [4][NE] adjoint of the averages before the step
  double* wnod;              // [NE][wnod_stride] reconstruction at the step start
  double* trace;             // [NE][trace_stride] predictor edge traces
  double* tbar;              // [NE][trace_stride] their adjoints
  double* wbar;              // [NE][wnod_stride] adjoint of the reconstruction
  double* sweeps;            // [npic][nb*(M+1)*4][NE] predictor iterate before each sweep
  double* lsq;               // [slot][NE][8] per stencil lane: R factor, solution, weight,
                             // indicator and least-squares rows of the forward pass
  double* rowbar;            // [NE][ne][8][4] adjoint of each stencil row's right-hand side
                             // ([NE][ne][8][10] with the vertex adjoints after it, moving mesh)
  double* avg;               // [NE][M+1][4] predictor cell means at the time nodes
  double* abar;              // [NF][M+1][4] their adjoints, a slot per transmissive edge
                             // (row 0: the element's own terms), summed by the gather
  // element vertices the least squares is built on: [NE][geo_stride] from
  // geo, or the context's records when geo is null
  const double* geo;
  int geo_stride;
  double* xeb;               // [NE][6] adjoint of the element's vertices (gather adds rows)
};

// Scratch and arguments of the adjoint of a global step with the mesh moving
// with the fluid (adjoint.hip). a.q / a.qbar_next / a.qbar are the averages,
// their adjoint after and before the step; the least squares runs on xe.
struct LagWork {
  AdjWork a;
  const double* x;           // [NV][2] node positions at the step start
  const double* xbar_next;   // [NV][2] adjoint of the positions after the step
  double* xbar;              // [NV][2] adjoint of the positions before the step
  double* qnext;             // [4][NE] averages after the step, or null
  double* xnext;             // [NV][2] positions after the step, or null
  double* xcopy;             // [NV][2] copy of the context's positions
  double* xe;                // [NE][6] element vertices
  double* area;              // [NE] areas at the step start
  double* an;                // [NE] areas after the step
  double* xn;                // [NV][2] positions after the step
  double* vraw;              // [NV][2] ring-mean velocity before the wall constraint
  double* den;               // [NV] ring mass
  double* keep;              // [npic+1][M+1][4][NE][nb] predictor iterates
  double* vvel;              // [NE][3][M+1][2] predicted vertex velocities
  double* gslot;             // [NE][3][4] inflow-positive patch flux per (element, edge)
  double* xs;                // [NF][8] adjoint of the patch corners (a, b old; a, b new)
  double* xnbe;              // [NE][6] adjoint of the element's new vertices (area)
  double* nslot;             // [NE][3][3] per (element, vertex): adjoint of the time-averaged
                             // vertex velocity (2) and of the ring mass (1)
  double* qdir;              // [4][NE] adjoint of the averages not through the reconstruction
};

// A saved copy of the simulation state as the adjoint of the local time
// stepping reads it: element records, traces, reconstructions, ticks and
// steps, node positions and node ticks.
struct LtsView {
  const double* rec;      // [NE][rec_stride]
  const double* trace;    // [NE][trace_stride]
  const double* wnod;     // [NE][wnod_stride]
  const TickStep* ts;     // [NE]
  const double* X;        // [2][NV]
  const int* ntick;       // [NV]
};

// Adjoint state and scratch of the reverse sweep through the cycles of a
// macro step of the local time stepping (adjoint.hip). The adjoints are those
// of the stored state: averages qb, areas ab, element vertices g.a.xeb, the
// reconstruction g.a.wbar, the predictor's traces g.a.tbar, cell means avb and
// vertex velocities vvb, the memory variables mb (one per element: the update
// sums its three edge slots), node positions xb. s0 / s1: the state before /
// after the cycle being reversed.
struct LtsWork {
  LagWork g;          // g.a.lsq, g.a.rowbar, g.a.wnod (recomputed reconstruction), g.keep,
                      // g.xs [NF][8] patch corners, g.xnbe [NE][6] new vertices, g.nslot [NE][3][3]
  double* qb;         // [NE][4]
  double* ab;         // [NE]
  double* mb;         // [NE][4]
  double* avb;        // [NE][M+1][4]
  double* vvb;        // [NE][3][M+1][2]
  double* xb;         // [NV][2]
  double* abar_e;     // [NF][M+1][4] means' adjoint from a transmissive patch
  int* eflag;         // [NE] bit 0: updated in the cycle; bit 1: takes a new predictor
  int* nflag;         // [NV] moved in the cycle
  int* act_list;      // [NE]
  int* going_list;    // [NE]
  int* edge_list;     // [NF] edges swept in the cycle
  int* counts;        // [3] lengths of the three lists
  double delta;       // tick length of the macro step
  LtsView s0, s1;
};

// Device address of the library's fixed adjoint scratch on the current GPU
// and its size (adjoint.hip); looked up once per device.
int static_scratch(void** ptr, size_t* bytes);
// Bytes of the adjoint workspace (each buffer 256-byte aligned).
size_t adjoint_work_bytes(int M, int NE, int NF, int npic);
size_t lagadj_work_bytes(int M, int NE, int NV, int NF, int npic);
void lagadj_carve(int M, int NE, int NV, int NF, int npic, char* base, LagWork& w);
int launch_adjoint_lagrangian(const Dev& d, const Params& p, int M, const LagWork& w, double dt,
                              bool q_from_context, bool x_from_context, void* stream);
// Carve the buffers from base (qbar_next, qbar left to the caller).
void adjoint_carve(int M, int NE, int NF, int npic, char* base, AdjWork& w);
// The reverse-mode step: qbar = (dQ^{n+1}/dQ^n)^T qbar_next for one global
// step of length dt on a fixed mesh (adjoint.hip).
int launch_adjoint_gts(const Dev& d, const Params& p, int M, const AdjWork& w, double dt,
                       bool state_from_context, void* stream);
// Reverse mode of the local time stepping (adjoint.hip), schedule frozen.
// Bytes of the scratch (each buffer 256-byte aligned) and its carving.
size_t lts_work_bytes(int M, int NE, int NV, int NF, int npic);
void lts_carve(int M, int NE, int NV, int NF, int npic, char* base, LtsWork& w);
// The adjoint state from (Qbar [4][NE], Xbar [NV][2]) with every other part zero.
int launch_lts_init(const Dev& d, const LtsWork& w, const double* Qbar, const double* Xbar, void* stream);
// Reverse of one cycle from the states before (w.s0) and after (w.s1) it.
int launch_lts_cycle_rev(const Dev& d, const Params& p, int M, const LtsWork& w, void* stream);
// Reverse of the predictors of every element at a macro-step start (w.s1: the
// state after the start), then the element vertices' and areas' adjoints
// folded into the node positions'.
int launch_lts_macro_begin_rev(const Dev& d, const Params& p, int M, const LtsWork& w, void* stream);
// Reverse of the pre-processing reconstruction (real neighbours, w.s1: the
// state after upload), folded into the node positions' adjoints.
int launch_lts_initial_rev(const Dev& d, const Params& p, int M, const LtsWork& w, void* stream);
// (Qbar [4][NE], Xbar [NV][2]) from the adjoint state.
int launch_lts_out(const Dev& d, const LtsWork& w, double* Qbar, double* Xbar, void* stream);

// The derivative-contraction measurement (probe.hip): one launch, M = 2
// tables, F and out [n][10][6]; blocks <= 0: one block per 40 elements.
int probe_contraction(const Tables* tab, int use_mfma, long n, int iters, const double* F, double* out,
                      void* stream, int blocks);

// Kernel launchers (kernels.hip).  All launch on `stream`, return a
// hipError_t as int.
int launch_init_geometry(const Dev& d, void* stream);
int launch_reconstruct(const Dev& d, const Params& p, int M, int use_list, int set_level,
                       void* stream);
int launch_predict(const Dev& d, const Params& p, int M, int use_list, void* stream);
int launch_macro_begin(const Dev& d, int N, int nominal, double fraction, void* stream);
int launch_set_target(const Dev& d, double t_end, void* stream);
int launch_cycle_begin(const Dev& d, void* stream);
int launch_sched(const Dev& d, void* stream);
// Start and stop events (hipEvent_t) for the next grid launch of this host
// thread: its timestamps are the kernel's own start and end.
void set_next_launch_events(void* start, void* stop);
bool next_launch_events_pending();
int launch_node(const Dev& d, const Params& p, int M, void* stream);
int launch_patch(const Dev& d, const Params& p, int M, void* stream);
int launch_update(const Dev& d, const Params& p, void* stream);
int launch_status(const Dev& d, void* stream);
int launch_macro_end(const Dev& d, int only_if_done, void* stream);
int launch_open(const Dev& d, void* stream);
int launch_download_xy(const Dev& d, double* out, void* stream);
int launch_upload_xy(const Dev& d, const double* in, void* stream);
int launch_download_q(const Dev& d, double* out, void* stream);
int launch_upload_q(const Dev& d, const double* in, void* stream);
int launch_elem_times(const Dev& d, double* out, void* stream);
int launch_check_state(const Dev& d, double gamma, void* stream);

}  // namespace aw
