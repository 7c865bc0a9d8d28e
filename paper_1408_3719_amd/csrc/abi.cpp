// C ABI of the aderweno library: context, workspace, upload/download and the
// host side of the time stepping loops.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/aderweno.h"
#include "common.h"
#include "host.h"

struct ader_ctx {
  ader_config cfg{};
  aw::Params prm{};
  hipStream_t stream = nullptr;
  bool has_mesh = false, bound = false, has_state = false;
  bool synced = false;   // every element at one common time (no macro step in progress)
  aw::Topology topo;
  aw::Tables tab{};
  char* ws = nullptr;
  size_t ws_bytes = 0;
  aw::Dev dev{};
  std::string err;
  int64_t cycles = 0, macro_steps = 0;
  // batch: element ranges [inst_first[k], inst_first[k+1]) of the instances
  std::vector<int> inst_first, e_inst, v_inst;
  // each macro step as one HIP graph (captured on a private stream, replayed on
  // the caller's), rebuilt when the number of levels or the launch settings change
  bool graphs = true;
  hipStream_t cap = nullptr;
  hipGraphExec_t gexec = nullptr;
  int g_nominal = 0;
  hipGraphExec_t gcyc = nullptr;    // FREE_BATCH cycles and the status count
  hipGraphExec_t gextra = nullptr;  // EXTRA_BATCH cycles and the status count
  int64_t extra_cycles = 0, long_macro_steps = 0;   // beyond 2^(L-1) cycles
  // schedule replay tables (device memory owned by the context)
  int* replay_buf = nullptr;
  double* delta_buf = nullptr;     // tick-length replay
  int* rec_buf = nullptr;          // schedule record: steps, then positions
  double* rec_delta_buf = nullptr; // schedule record: tick lengths
  // the library's fixed adjoint scratch on this context's GPU (ader_bind_workspace)
  void* static_work = nullptr;
  size_t static_bytes = 0;
  // profiling
  bool prof = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[ADER_K_COUNT];
  double kms[ADER_K_COUNT] = {};
  int64_t klaunch[ADER_K_COUNT] = {};
};

namespace {

int fail(ader_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

int hip_fail(ader_ctx* c, int e, const char* where) {
  return fail(c, ADER_E_HIP, std::string(where) + ": " + hipGetErrorString(hipError_t(e)));
}

#define HIPCHK(ctx, expr)                                          \
  do {                                                             \
    hipError_t _e = (expr);                                        \
    if (_e != hipSuccess) return hip_fail(ctx, int(_e), #expr);    \
  } while (0)

#define LCHK(ctx, expr)                                            \
  do {                                                             \
    int _e = (expr);                                               \
    if (_e != 0) return hip_fail(ctx, _e, #expr);                  \
  } while (0)

struct Layout {
  size_t total = 0;
  size_t take(size_t bytes) {
    size_t off = total;
    total += (bytes + 255) & ~size_t(255);
    return off;
  }
};

// Workspace carving; when base == nullptr only the size is computed.
size_t carve(ader_ctx* c, char* base) {
  const aw::Topology& t = c->topo;
  const int M = c->cfg.M;
  const int nb = (M + 1) * (M + 2) / 2, ne = 2 * nb;
  const size_t NE = t.NE, NV = t.NV, NF = t.NF, D = sizeof(double), I = sizeof(int);
  Layout L;
  aw::Dev& d = c->dev;
  auto pd = [&](size_t n) { size_t o = L.take(n * D); return base ? (double*)(base + o) : nullptr; };
  auto pi = [&](size_t n) { size_t o = L.take(n * I); return base ? (int*)(base + o) : nullptr; };
  size_t o_scal = L.take(sizeof(aw::Scal));
  size_t o_tab = L.take(sizeof(aw::Tables));
  size_t o_ts = L.take(NE * sizeof(aw::TickStep));
  const size_t K = c->inst_first.size() - 1;
  size_t o_inst = L.take(K * sizeof(aw::Inst));
  d.NE = t.NE;
  d.NV = t.NV;
  d.NF = t.NF;
  d.M = M;
  d.K = int(K);
  d.inst = base ? (aw::Inst*)(base + o_inst) : nullptr;
  d.e_inst = pi(NE);
  d.v_inst = pi(NV);
  d.scal = base ? (aw::Scal*)(base + o_scal) : nullptr;
  d.tab = base ? (const aw::Tables*)(base + o_tab) : nullptr;
  d.ts = base ? (aw::TickStep*)(base + o_ts) : nullptr;
  d.rec = pd(NE * aw::rec_stride(M));
  d.trace = pd(NE * aw::trace_stride(M));
  d.wnod = pd(NE * aw::wnod_stride(M));
  d.dtcfl = pd(NE);
  d.mem = pd(NE * 3 * aw::MEM_W);
  d.act_stamp = pi(NE);
  d.act_list = pi(NE);
  d.live_list = pi(NE);
  d.tri = pi(3 * NE);
  d.elem_edges = pi(3 * NE);
  d.neigh = pi(3 * NE);
  d.sten = pi(size_t(aw::NSTEN) * ne * NE);
  d.sched_ptr = pi(NE + 1);
  d.sched_idx = pi(t.sched_idx.size());
  d.tsten_ptr = pi(NE + 1);
  d.tsten_idx = pi(t.tsten_idx.size());
  d.X = pd(2 * NV);
  d.Xnew = pd(2 * NV);
  d.ntick = pi(NV);
  d.ntick_new = pi(NV);
  d.node_stamp = pi(NV);
  d.ring_ptr = pi(NV + 1);
  d.ring_ent = pi(t.ring_ent.size());
  d.wall_n = pd(2 * NV);
  d.wall_pin = pi(NV);
  d.e_a = pi(NF);
  d.e_b = pi(NF);
  d.e_L = pi(NF);
  d.e_R = pi(NF);
  d.e_el = pi(NF);
  d.e_er = pi(NF);
  d.e_bc = pi(NF);
  return L.total;
}

template <class T>
std::vector<T> to_soa(const std::vector<T>& aos, size_t n, size_t f) {
  std::vector<T> out(aos.size());
  for (size_t i = 0; i < n; ++i)
    for (size_t k = 0; k < f; ++k) out[k * n + i] = aos[i * f + k];
  return out;
}

int h2d(ader_ctx* c, const void* dst, const void* src, size_t bytes) {
  HIPCHK(c, hipMemcpyAsync(const_cast<void*>(dst), src, bytes, hipMemcpyHostToDevice, c->stream));
  return 0;
}

// Fold finished event pairs into the per-kernel totals (stream synchronised).
void flush_events(ader_ctx* c) {
  for (int k = 0; k < ADER_K_COUNT; ++k) {
    for (auto& p : c->ev[k]) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, p.first, p.second) == hipSuccess) c->kms[k] += ms;
      c->klaunch[k]++;
      (void)hipEventDestroy(p.first);
      (void)hipEventDestroy(p.second);
    }
    c->ev[k].clear();
  }
}

// Under profiling, a stage of one grid launch is timed by that kernel's own
// start and end (events attached to the launch); a stage of several launches
// by events recorded before and after it on the stream.
template <class F>
int timed(ader_ctx* c, int k, hipStream_t st, F launch) {
  if (!c->prof) return launch();
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return int(hipErrorOutOfMemory);
  const bool one = k != ADER_K_MACRO && k != ADER_K_STATUS && k != ADER_K_ADJOINT;
  if (one)
    aw::set_next_launch_events(a, b);
  else
    (void)hipEventRecord(a, st);
  const int r = launch();
  if (!one) {
    (void)hipEventRecord(b, st);
  } else if (aw::next_launch_events_pending()) {   // no grid launch took them
    aw::set_next_launch_events(nullptr, nullptr);
    (void)hipEventRecord(a, st);
    (void)hipEventRecord(b, st);
  }
  c->ev[k].push_back({a, b});
  return r;
}

int read_scal(ader_ctx* c, aw::Scal& s) {
  HIPCHK(c, hipMemcpyAsync(&s, c->dev.scal, sizeof(s), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->prof) flush_events(c);
  return 0;
}

int check_err(ader_ctx* c, const aw::Scal& s) {
  if (s.err & aw::ERR_GEOM) return fail(c, ADER_E_GEOM, "an element was inverted by the mesh motion");
  if (s.err & aw::ERR_GCL) return fail(c, ADER_E_GCL, "space-time control volume not closed (GCL residual above tolerance)");
  if (s.err & aw::ERR_STATE) return fail(c, ADER_E_STATE, "non-physical state (rho <= 0, p <= 0 or NaN)");
  if (s.err & aw::ERR_PRED) return fail(c, ADER_E_STATE, "a predictor was read outside its time slab");
  if (s.err & aw::ERR_DT) return fail(c, ADER_E_STATE, "time step is not positive");
  if (s.err & aw::ERR_REPLAY)
    return fail(c, ADER_E_ARG, "schedule replay: an element ran out of recorded steps, a step leaves its macro step, "
                               "or the tick lengths ran out");
  if (s.err & aw::ERR_RECORD) return fail(c, ADER_E_ARG, "schedule record: capacity exceeded");
  return 0;
}

// Queue n cycles on stream st: update criterion and list, node motion, patch
// fluxes, update, reconstruction and time step, predictor.
int issue_cycles(ader_ctx* c, int n, hipStream_t st) {
  const aw::Dev& d = c->dev;
  const aw::Params& p = c->prm;
  const int M = c->cfg.M;
  void* s = st;
  for (int k = 0; k < n; ++k) {
    LCHK(c, timed(c, ADER_K_SCHED, st, [&] {
      int r = aw::launch_cycle_begin(d, s);
      return r ? r : aw::launch_sched(d, s);
    }));
    LCHK(c, timed(c, ADER_K_NODE, st, [&] { return aw::launch_node(d, p, M, s); }));
    LCHK(c, timed(c, ADER_K_PATCH, st, [&] { return aw::launch_patch(d, p, M, s); }));
    LCHK(c, timed(c, ADER_K_UPDATE, st, [&] { return aw::launch_update(d, p, s); }));
    LCHK(c, timed(c, ADER_K_RECON, st, [&] { return aw::launch_reconstruct(d, p, M, 1, 1, s); }));
    LCHK(c, timed(c, ADER_K_PREDICT, st, [&] { return aw::launch_predict(d, p, M, 1, s); }));
  }
  return 0;
}

// Tick lengths and levels of the open instances (flagged by launch_open for
// the target time on the device beforehand), predictors. nominal = 2^(L-1)
// for L dyadic levels, 0 for free steps.
int issue_macro_begin(ader_ctx* c, int nominal, hipStream_t st) {
  const double frac = nominal <= 1 ? 1.0 : c->cfg.lts_step_fraction > 0.0 ? c->cfg.lts_step_fraction : 0.95;
  LCHK(c, timed(c, ADER_K_MACRO, st,
                [&] { return aw::launch_macro_begin(c->dev, aw::MACRO_TICKS, nominal, frac, st); }));
  LCHK(c, timed(c, ADER_K_PREDICT, st, [&] { return aw::launch_predict(c->dev, c->prm, c->cfg.M, 0, st); }));
  return 0;
}

// One macro step of L dyadic levels: levels and predictors, 2^(L-1) cycles
// (enough unless some element took a step below the nominal finest one), the
// count of elements short of the macro-step end, the macro-step end when that
// count is zero, and the count of instances still short of the target time.
// Nothing here depends on the target time, which the kernels read from the
// device (launch_set_target), so one captured graph serves every target.
int issue_macro(ader_ctx* c, int nominal, hipStream_t st) {
  int r;
  if ((r = issue_macro_begin(c, nominal, st))) return r;
  if ((r = issue_cycles(c, nominal, st))) return r;
  LCHK(c, timed(c, ADER_K_STATUS, st, [&] { return aw::launch_status(c->dev, st); }));
  LCHK(c, aw::launch_macro_end(c->dev, 1, st));
  LCHK(c, aw::launch_open(c->dev, st));
  return 0;
}

// Cycles per host check of the free-step run, and of the cycles a dyadic
// macro step needs beyond 2^(L-1) when elements took spare finer steps.
constexpr int FREE_BATCH = 16;
constexpr int EXTRA_BATCH = 2;

// n cycles, then the count of elements short of tick N.
int issue_cycle_batch(ader_ctx* c, int n, hipStream_t st) {
  int r;
  if ((r = issue_cycles(c, n, st))) return r;
  LCHK(c, timed(c, ADER_K_STATUS, st, [&] { return aw::launch_status(c->dev, st); }));
  return 0;
}

// Capture what `issue` queues into one executable graph.
template <class F>
int capture(ader_ctx* c, hipGraphExec_t* out, F issue) {
  if (*out) {
    HIPCHK(c, hipGraphExecDestroy(*out));
    *out = nullptr;
  }
  if (!c->cap) HIPCHK(c, hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
  HIPCHK(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
  const int r = issue(c->cap);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(c->cap, &g);
  if (r || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return r ? r : hip_fail(c, int(e), "hipStreamEndCapture");
  }
  const hipError_t ei = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) {
    *out = nullptr;
    return hip_fail(c, int(ei), "hipGraphInstantiate");
  }
  return 0;
}

// Drop the captured graphs (launch settings or the step mode changed).
void drop_graphs(ader_ctx* c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->gcyc) (void)hipGraphExecDestroy(c->gcyc);
  if (c->gextra) (void)hipGraphExecDestroy(c->gextra);
  c->gexec = nullptr;
  c->gcyc = nullptr;
  c->gextra = nullptr;
}

int ensure_graph(ader_ctx* c, int nominal) {
  if (c->gexec && c->g_nominal == nominal) return 0;
  int r = capture(c, &c->gexec, [&](hipStream_t s) { return issue_macro(c, nominal, s); });
  if (r) return r;
  c->g_nominal = nominal;
  return 0;
}

// The step mode the kernels see: free steps change how levels are chosen and
// how tick lengths are set. Captured graphs hold the mode they were made with.
void set_free(ader_ctx* c, bool free_steps) {
  if (c->dev.free_steps != int(free_steps)) drop_graphs(c);
  c->dev.free_steps = free_steps;
}

// Macro steps of L dyadic levels until t_target; returns 0 or an error code.
// One host synchronisation per macro step of 2^(L-1) cycles; when some element
// has not reached the macro-step end by then (it took spare finer steps), more
// cycles in captured batches of EXTRA_BATCH with a status read after each.
int run_macro(ader_ctx* c, double t_target, int max_macro, int levels) {
  if (!c->has_state) return fail(c, ADER_E_ORDER, "no state uploaded");
  if (!std::isfinite(t_target)) return fail(c, ADER_E_ARG, "t_target is not finite");
  c->synced = false;
  set_free(c, false);
  const int nominal = 1 << (levels - 1);
  const bool graph = c->graphs && !c->prof;
  aw::Scal s;
  int r;
  LCHK(c, aw::launch_set_target(c->dev, t_target, c->stream));
  LCHK(c, aw::launch_open(c->dev, c->stream));
  if ((r = read_scal(c, s))) return r;
  for (int k = 0; max_macro <= 0 || k < max_macro; ++k) {
    if ((r = check_err(c, s))) return r;
    if (s.n_open == 0) break;      // every instance has reached t_target
    if (graph) {
      if ((r = ensure_graph(c, nominal))) return r;
      HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
    } else if ((r = issue_macro(c, nominal, c->stream))) {
      return r;
    }
    c->cycles += nominal;
    if ((r = read_scal(c, s))) return r;
    if ((r = check_err(c, s))) return r;
    if (s.n_unfinished != 0) {
      long long last = (long long)s.updates;
      for (;;) {
        if (graph) {
          if (!c->gextra &&
              (r = capture(c, &c->gextra, [&](hipStream_t st) { return issue_cycle_batch(c, EXTRA_BATCH, st); })))
            return r;
          HIPCHK(c, hipGraphLaunch(c->gextra, c->stream));
        } else if ((r = issue_cycle_batch(c, EXTRA_BATCH, c->stream))) {
          return r;
        }
        c->cycles += EXTRA_BATCH;
        c->extra_cycles += EXTRA_BATCH;
        if ((r = read_scal(c, s))) return r;
        if ((r = check_err(c, s))) return r;
        if (s.n_unfinished == 0) break;
        if ((long long)s.updates == last) return fail(c, ADER_E_DEADLOCK, "no element satisfies the update criterion");
        last = (long long)s.updates;
      }
      LCHK(c, aw::launch_macro_end(c->dev, 0, c->stream));
      LCHK(c, aw::launch_open(c->dev, c->stream));
      if ((r = read_scal(c, s))) return r;
      c->long_macro_steps++;
    }
    c->macro_steps++;
  }
  c->synced = true;
  return 0;
}

// Free local steps: the interval to t_target is one macro step of FREE_TICKS
// ticks, run in batches of FREE_BATCH cycles with a status read after each
// until every element has reached the end of the interval.
int run_free(ader_ctx* c, double t_target, int max_macro) {
  if (!c->has_state) return fail(c, ADER_E_ORDER, "no state uploaded");
  if (!std::isfinite(t_target)) return fail(c, ADER_E_ARG, "t_target is not finite");
  c->synced = false;
  set_free(c, true);
  const bool graph = c->graphs && !c->prof;
  aw::Scal s;
  int r;
  LCHK(c, aw::launch_set_target(c->dev, t_target, c->stream));
  LCHK(c, aw::launch_open(c->dev, c->stream));
  if ((r = read_scal(c, s))) return r;
  for (int k = 0; max_macro <= 0 || k < max_macro; ++k) {
    if ((r = check_err(c, s))) return r;
    if (s.n_open == 0) break;
    if ((r = issue_macro_begin(c, 0, c->stream))) return r;
    long long last = -1;
    for (;;) {
      if (graph) {
        if (!c->gcyc &&
            (r = capture(c, &c->gcyc, [&](hipStream_t st) { return issue_cycle_batch(c, FREE_BATCH, st); })))
          return r;
        HIPCHK(c, hipGraphLaunch(c->gcyc, c->stream));
      } else if ((r = issue_cycle_batch(c, FREE_BATCH, c->stream))) {
        return r;
      }
      c->cycles += FREE_BATCH;
      if ((r = read_scal(c, s))) return r;
      if ((r = check_err(c, s))) return r;
      if (s.n_unfinished == 0) break;
      if ((long long)s.updates == last) return fail(c, ADER_E_DEADLOCK, "no element satisfies the update criterion");
      last = (long long)s.updates;
    }
    LCHK(c, aw::launch_macro_end(c->dev, 0, c->stream));
    LCHK(c, aw::launch_open(c->dev, c->stream));
    if ((r = read_scal(c, s))) return r;
    c->macro_steps++;
  }
  c->synced = true;
  return 0;
}

int read_insts(ader_ctx* c, std::vector<aw::Inst>& in) {
  in.resize(c->dev.K);
  HIPCHK(c, hipMemcpyAsync(in.data(), c->dev.inst, in.size() * sizeof(aw::Inst), hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return 0;
}

// t: the earliest instance time (the common time of all elements when there
// is one instance); delta: the tick length of instance 0.
void fill_stats(ader_ctx* c, const aw::Scal& s, const std::vector<aw::Inst>& in, ader_stats* st) {
  st->element_updates = s.updates;
  st->cycles = c->cycles;
  st->macro_steps = c->macro_steps;
  st->cfl_overshoots = s.overshoots;
  unsigned long long b = s.max_gcl_bits;
  double g;
  std::memcpy(&g, &b, sizeof(g));
  st->max_gcl_residual = g;
  double tmin = in[0].T;
  for (const auto& x : in) tmin = std::fmin(tmin, x.T);
  st->t = tmin;
  st->delta = in[0].delta;
  st->predictor_evals = (int64_t)s.n_pred;
  st->patches = (int64_t)s.n_patch;
  st->node_moves = (int64_t)s.n_node;
  st->extra_cycles = c->extra_cycles;
  st->long_macro_steps = c->long_macro_steps;
  st->replay_overrides = (int64_t)s.replay_overrides;
}

struct Arr {
  void* dev = nullptr;          // device array
  const void* host = nullptr;   // host array (topology and tables)
  size_t bytes = 0;
};

Arr lookup(ader_ctx* c, int what) {
  Arr a;
  const aw::Topology& t = c->topo;
  const int M = c->cfg.M;
  const size_t nb = (M + 1) * (M + 2) / 2, nt = M + 1, nG = M + 1;
  const size_t NE = t.NE, NV = t.NV, D = sizeof(double), I = sizeof(int);
  const aw::Dev& d = c->dev;
  switch (what) {
    case ADER_DBG_Q: a.bytes = 4 * NE * D; break;
    case ADER_DBG_A: a.bytes = NE * D; break;
    case ADER_DBG_XE: a.bytes = 6 * NE * D; break;
    case ADER_DBG_TICK: a.bytes = NE * I; break;
    case ADER_DBG_STEP: a.bytes = NE * I; break;
    case ADER_DBG_DTCFL: a.dev = d.dtcfl; a.bytes = NE * D; break;
    case ADER_DBG_QM: a.bytes = 4 * NE * D; break;
    case ADER_DBG_HM: a.bytes = 3 * NE * D; break;
    case ADER_DBG_WNOD: a.bytes = nb * 4 * NE * D; break;
    case ADER_DBG_AVG: a.bytes = nt * 4 * NE * D; break;
    case ADER_DBG_TRACE: a.bytes = 3 * nG * nt * 4 * NE * D; break;
    case ADER_DBG_VVEL: a.bytes = 3 * nt * 2 * NE * D; break;
    case ADER_DBG_X: a.dev = d.X; a.bytes = 2 * NV * D; break;
    case ADER_DBG_NTICK: a.dev = d.ntick; a.bytes = NV * I; break;
    case ADER_DBG_SCAL: a.bytes = 4 * D; break;
    case ADER_DBG_TOPO_EDGES: a.bytes = size_t(t.NF) * 6 * I; break;
    case ADER_DBG_TOPO_STENCILS: a.host = t.sten.data(); a.bytes = t.sten.size() * I; break;
    case ADER_DBG_TOPO_SCHED_PTR: a.host = t.sched_ptr.data(); a.bytes = t.sched_ptr.size() * I; break;
    case ADER_DBG_TOPO_SCHED_IDX: a.host = t.sched_idx.data(); a.bytes = t.sched_idx.size() * I; break;
    case ADER_DBG_TOPO_TSTEN_PTR: a.host = t.tsten_ptr.data(); a.bytes = t.tsten_ptr.size() * I; break;
    case ADER_DBG_TOPO_TSTEN_IDX: a.host = t.tsten_idx.data(); a.bytes = t.tsten_idx.size() * I; break;
    case ADER_DBG_TAB_DXI: a.bytes = nb * nb * D; break;
    case ADER_DBG_TAB_DETA: a.bytes = nb * nb * D; break;
    case ADER_DBG_TAB_AMEAN: a.bytes = nb * D; break;
    case ADER_DBG_TAB_EDGE: a.bytes = 3 * nG * nb * D; break;
    case ADER_DBG_TAB_AT: a.bytes = M * nt * D; break;
    case ADER_DBG_TAB_BT: a.bytes = M * D; break;
    case ADER_DBG_TAB_DT: a.bytes = nt * nt * D; break;
    case ADER_DBG_TAB_PSIC: a.bytes = nb * nb * D; break;
    case ADER_DBG_TAB_SIGMA: a.bytes = nb * nb * D; break;
    case ADER_DBG_TAB_GAUSS: a.bytes = 2 * nG * D; break;
    default: break;
  }
  return a;
}

// Element arrays kept per element on the device (records, traces, nodal
// reconstruction, tick/step): field f of element i in the documented
// field-major layout [f][NE] maps to (buffer, stride, offset f').
struct Packed {
  void* dev = nullptr;
  size_t stride = 0;                     // doubles (or ints) per element
  std::vector<size_t> off;               // device offset of documented field f
  bool ints = false;
};

Packed packed(ader_ctx* c, int what) {
  Packed p;
  const int M = c->cfg.M;
  const int nb = (M + 1) * (M + 2) / 2, T = M + 1, nG = M + 1;
  const aw::Dev& d = c->dev;
  auto rec = [&](int first, int count) {
    p.dev = d.rec;
    p.stride = aw::rec_stride(M);
    for (int k = 0; k < count; ++k) p.off.push_back(first + k);
  };
  switch (what) {
    case ADER_DBG_Q: rec(aw::rec_off_q(), 4); break;
    case ADER_DBG_A: rec(aw::rec_off_a(), 1); break;
    case ADER_DBG_XE: rec(aw::rec_off_xe(), 6); break;
    case ADER_DBG_AVG: rec(aw::rec_off_avg(), 4 * T); break;
    case ADER_DBG_VVEL: rec(aw::rec_off_vv(M), 6 * T); break;
    case ADER_DBG_TRACE:
      p.dev = d.trace;
      p.stride = aw::trace_stride(M);
      for (int k = 0; k < 3 * nG * T * 4; ++k) p.off.push_back(k);
      break;
    case ADER_DBG_WNOD:
      p.dev = d.wnod;
      p.stride = aw::wnod_stride(M);
      for (int k = 0; k < nb * 4; ++k) p.off.push_back(k);
      break;
    case ADER_DBG_TICK:
    case ADER_DBG_STEP:
      p.dev = d.ts;
      p.stride = 2;
      p.off.push_back(what == ADER_DBG_TICK ? 0 : 1);
      p.ints = true;
      break;
    default: break;
  }
  return p;
}

int packed_io(ader_ctx* c, int what, void* host, const void* in, size_t bytes) {
  Packed p = packed(c, what);
  const size_t NE = c->topo.NE, es = p.ints ? sizeof(int) : sizeof(double);
  std::vector<char> buf(NE * p.stride * es);
  HIPCHK(c, hipMemcpyAsync(buf.data(), p.dev, buf.size(), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const size_t nf = p.off.size();
  if (bytes != nf * NE * es) return fail(c, ADER_E_ARG, "size mismatch");
  for (size_t f = 0; f < nf; ++f)
    for (size_t i = 0; i < NE; ++i) {
      char* dev_el = buf.data() + (i * p.stride + p.off[f]) * es;
      if (host)
        std::memcpy((char*)host + (f * NE + i) * es, dev_el, es);
      else
        std::memcpy(dev_el, (const char*)in + (f * NE + i) * es, es);
    }
  if (!host) {
    HIPCHK(c, hipMemcpyAsync(p.dev, buf.data(), buf.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return 0;
}

// host tables and edges packed densely
std::vector<char> host_pack(ader_ctx* c, int what) {
  const aw::Tables& T = c->tab;
  const int nb = T.nb, nt = T.nt, nG = T.nG, M = T.M;
  std::vector<double> v;
  switch (what) {
    case ADER_DBG_TAB_DXI:
      for (int a = 0; a < nb; ++a) for (int b = 0; b < nb; ++b) v.push_back(T.Dxi[a][b]);
      break;
    case ADER_DBG_TAB_DETA:
      for (int a = 0; a < nb; ++a) for (int b = 0; b < nb; ++b) v.push_back(T.Deta[a][b]);
      break;
    case ADER_DBG_TAB_AMEAN:
      for (int a = 0; a < nb; ++a) v.push_back(T.amean[a]);
      break;
    case ADER_DBG_TAB_EDGE:
      for (int e = 0; e < 3; ++e) for (int g = 0; g < nG; ++g) for (int m = 0; m < nb; ++m) v.push_back(T.edge[e][g][m]);
      break;
    case ADER_DBG_TAB_AT:
      for (int r = 0; r < M; ++r) for (int q = 0; q < nt; ++q) v.push_back(T.At[r][q]);
      break;
    case ADER_DBG_TAB_BT:
      for (int r = 0; r < M; ++r) v.push_back(T.Bt[r]);
      break;
    case ADER_DBG_TAB_DT:
      for (int a = 0; a < nt; ++a) for (int b = 0; b < nt; ++b) v.push_back(T.Dt[a][b]);
      break;
    case ADER_DBG_TAB_PSIC:
      for (int a = 0; a < nb; ++a) for (int b = 0; b < nb; ++b) v.push_back(T.psiC[a][b]);
      break;
    case ADER_DBG_TAB_SIGMA:
      for (int a = 0; a < nb; ++a) for (int b = 0; b < nb; ++b) v.push_back(T.Sigma[a][b]);
      break;
    case ADER_DBG_TAB_GAUSS:
      for (int g = 0; g < nG; ++g) v.push_back(T.gchi[g]);
      for (int g = 0; g < nG; ++g) v.push_back(T.gw[g]);
      break;
    case ADER_DBG_TOPO_EDGES: {
      std::vector<char> out(size_t(c->topo.NF) * 6 * sizeof(int));
      int* p = (int*)out.data();
      const aw::Topology& t = c->topo;
      for (int e = 0; e < t.NF; ++e) {
        p[6 * e] = t.e_a[e];
        p[6 * e + 1] = t.e_b[e];
        p[6 * e + 2] = t.e_L[e];
        p[6 * e + 3] = t.e_R[e];
        p[6 * e + 4] = t.e_el[e];
        p[6 * e + 5] = t.e_er[e];
      }
      return out;
    }
    default: break;
  }
  std::vector<char> out(v.size() * sizeof(double));
  std::memcpy(out.data(), v.data(), out.size());
  return out;
}

}  // namespace

extern "C" {

int ader_create(const ader_config* cfg, void* hip_stream, ader_ctx** out) {
  if (!cfg || !out) return ADER_E_ARG;
  *out = nullptr;
  if (cfg->M < 1 || cfg->M > 3) return ADER_E_ARG;
  if (cfg->flux < ADER_FLUX_RUSANOV || cfg->flux > ADER_FLUX_HLL) return ADER_E_ARG;
  if (!(cfg->cfl > 0.0 && cfg->cfl <= 1.0)) return ADER_E_ARG;
  if (!(cfg->gamma > 1.0)) return ADER_E_ARG;
  if (cfg->lts_levels < 0 || cfg->lts_levels > 8) return ADER_E_ARG;
  if (cfg->weno_r != 8.0) return ADER_E_ARG;
  if (cfg->mesh_velocity != 0 && cfg->mesh_velocity != 1) return ADER_E_ARG;
  if (!(cfg->lts_step_fraction >= 0.0 && cfg->lts_step_fraction <= 1.0)) return ADER_E_ARG;
  ader_ctx* c = new (std::nothrow) ader_ctx();
  if (!c) return ADER_E_ARG;
  c->cfg = *cfg;
  c->stream = (hipStream_t)hip_stream;
  c->prm.gamma = cfg->gamma;
  c->prm.cfl = cfg->cfl;
  c->prm.eps = cfg->weno_eps;
  c->prm.lambda = cfg->weno_lambda;
  c->prm.gcl_tol = 1e-12;
  c->prm.npic = cfg->n_picard > 0 ? cfg->n_picard : cfg->M + 1;
  c->prm.lagrangian = cfg->mesh_velocity == 0;
  c->prm.flux = cfg->flux;
  try {
    aw::build_tables(cfg->M, c->tab);
  } catch (const std::exception& e) {
    delete c;
    return ADER_E_ARG;
  }
  *out = c;
  return ADER_OK;
}

int ader_upload_mesh(ader_ctx* c, int32_t n_nodes, const double* node_xy, int32_t n_elems,
                     const int32_t* tri, int32_t n_bedges, const int32_t* bedge) {
  if (!c) return ADER_E_ARG;
  if (n_nodes <= 0 || n_elems <= 0 || n_bedges < 0 || !node_xy || !tri || (n_bedges > 0 && !bedge))
    return fail(c, ADER_E_ARG, "invalid mesh arguments");
  if (c->bound) return fail(c, ADER_E_ORDER, "mesh already bound to a workspace");
  {
    // 32-bit indices of stencil rows ((element * ne + row) * 8 + lane)
    const long long ne = (long long)(c->cfg.M + 1) * (c->cfg.M + 2);
    if ((long long)n_elems * ne * 8 >= (1LL << 31))
      return fail(c, ADER_E_ARG, "mesh too large: n_elems * (M+1)(M+2) * 8 must stay below 2^31");
  }
  try {
    aw::build_topology(c->cfg.M, n_nodes, node_xy, n_elems, tri, n_bedges, bedge, c->topo);
  } catch (const std::exception& e) {
    c->has_mesh = false;
    return fail(c, ADER_E_MESH, e.what());
  }
  c->has_mesh = true;
  // one instance until ader_set_instances says otherwise
  c->inst_first = {0, n_elems};
  c->e_inst.assign(n_elems, 0);
  c->v_inst.assign(n_nodes, 0);
  return ADER_OK;
}

int ader_set_instances(ader_ctx* c, int32_t n_instances, const int32_t* elem_first) {
  if (!c || n_instances < 1 || !elem_first) return ADER_E_ARG;
  if (!c->has_mesh) return fail(c, ADER_E_ORDER, "no mesh uploaded");
  if (c->bound) return fail(c, ADER_E_ORDER, "mesh already bound to a workspace");
  const aw::Topology& t = c->topo;
  if (elem_first[0] != 0 || elem_first[n_instances] != t.NE)
    return fail(c, ADER_E_ARG, "instance ranges must start at 0 and end at n_elems");
  for (int k = 0; k < n_instances; ++k)
    if (elem_first[k + 1] <= elem_first[k]) return fail(c, ADER_E_ARG, "empty or decreasing instance range");
  std::vector<int> ei(t.NE), vi(t.NV, -1);
  for (int k = 0; k < n_instances; ++k)
    for (int i = elem_first[k]; i < elem_first[k + 1]; ++i) {
      ei[i] = k;
      for (int j = 0; j < 3; ++j) {
        int& v = vi[t.tri[3 * i + j]];
        if (v >= 0 && v != k) return fail(c, ADER_E_MESH, "instances share a node");
        v = k;
      }
    }
  for (int& v : vi) v = v < 0 ? 0 : v;
  c->inst_first.assign(elem_first, elem_first + n_instances + 1);
  c->e_inst = std::move(ei);
  c->v_inst = std::move(vi);
  return ADER_OK;
}

int ader_workspace_size(const ader_ctx* cc, size_t* bytes) {
  ader_ctx* c = const_cast<ader_ctx*>(cc);
  if (!c || !bytes) return ADER_E_ARG;
  if (!c->has_mesh) return fail(c, ADER_E_ORDER, "no mesh uploaded");
  aw::Dev keep = c->dev;
  *bytes = carve(c, nullptr);
  c->dev = keep;
  return ADER_OK;
}

int ader_bind_workspace(ader_ctx* c, void* dev_ptr, size_t bytes) {
  if (!c || !dev_ptr) return ADER_E_ARG;
  if (!c->has_mesh) return fail(c, ADER_E_ORDER, "no mesh uploaded");
  if ((reinterpret_cast<uintptr_t>(dev_ptr) & 255) != 0) return fail(c, ADER_E_ARG, "workspace not 256-byte aligned");
  size_t need = carve(c, nullptr);
  if (bytes < need) return fail(c, ADER_E_ARG, "workspace too small");
  c->ws = (char*)dev_ptr;
  c->ws_bytes = need;
  carve(c, c->ws);
  {
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
      c->dev.n_cu = ncu;
  }
  const aw::Topology& t = c->topo;
  aw::Dev& d = c->dev;
  const size_t NE = t.NE, NV = t.NV, NF = t.NF;
  // staging vectors must outlive the asynchronous copies: keep them until the sync
  std::vector<int> tri = to_soa(t.tri, NE, 3), ee = to_soa(t.elem_edges, NE, 3), nb = to_soa(t.neigh, NE, 3);
  std::vector<int> st = to_soa(t.sten, NE, size_t(aw::NSTEN) * t.ne);
  std::vector<double> wn = to_soa(t.wall_n, NV, 2);
  int r;
  if ((r = h2d(c, d.tab, &c->tab, sizeof(aw::Tables)))) return r;
  if ((r = h2d(c, d.e_inst, c->e_inst.data(), NE * sizeof(int)))) return r;
  if ((r = h2d(c, d.v_inst, c->v_inst.data(), NV * sizeof(int)))) return r;
  std::vector<aw::Inst> in0(d.K);
  if ((r = h2d(c, d.inst, in0.data(), in0.size() * sizeof(aw::Inst)))) return r;
  if ((r = h2d(c, d.tri, tri.data(), tri.size() * sizeof(int)))) return r;
  if ((r = h2d(c, d.elem_edges, ee.data(), ee.size() * sizeof(int)))) return r;
  if ((r = h2d(c, d.neigh, nb.data(), nb.size() * sizeof(int)))) return r;
  if ((r = h2d(c, d.sten, st.data(), st.size() * sizeof(int)))) return r;
  if ((r = h2d(c, d.sched_ptr, t.sched_ptr.data(), t.sched_ptr.size() * sizeof(int)))) return r;
  if ((r = h2d(c, d.sched_idx, t.sched_idx.data(), t.sched_idx.size() * sizeof(int)))) return r;
  if ((r = h2d(c, d.tsten_ptr, t.tsten_ptr.data(), t.tsten_ptr.size() * sizeof(int)))) return r;
  if ((r = h2d(c, d.tsten_idx, t.tsten_idx.data(), t.tsten_idx.size() * sizeof(int)))) return r;
  if ((r = h2d(c, d.ring_ptr, t.ring_ptr.data(), t.ring_ptr.size() * sizeof(int)))) return r;
  if ((r = h2d(c, d.ring_ent, t.ring_ent.data(), t.ring_ent.size() * sizeof(int)))) return r;

  if ((r = h2d(c, d.wall_n, wn.data(), wn.size() * sizeof(double)))) return r;
  if ((r = h2d(c, d.wall_pin, t.wall_pin.data(), NV * sizeof(int)))) return r;
  if ((r = h2d(c, d.e_a, t.e_a.data(), NF * sizeof(int)))) return r;
  if ((r = h2d(c, d.e_b, t.e_b.data(), NF * sizeof(int)))) return r;
  if ((r = h2d(c, d.e_L, t.e_L.data(), NF * sizeof(int)))) return r;
  if ((r = h2d(c, d.e_R, t.e_R.data(), NF * sizeof(int)))) return r;
  if ((r = h2d(c, d.e_el, t.e_el.data(), NF * sizeof(int)))) return r;
  if ((r = h2d(c, d.e_er, t.e_er.data(), NF * sizeof(int)))) return r;
  if ((r = h2d(c, d.e_bc, t.e_bc.data(), NF * sizeof(int)))) return r;
  aw::Scal s{};
  s.N = 1;
  if ((r = h2d(c, d.scal, &s, sizeof(s)))) return r;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  // the fixed adjoint scratch of this GPU (device address looked up once per device)
  if ((r = aw::static_scratch(&c->static_work, &c->static_bytes))) return hip_fail(c, r, "hipGetSymbolAddress");
  c->bound = true;
  return ADER_OK;
}

int ader_upload_state(ader_ctx* c, const double* Q_dev, double t0) {
  return ader_upload_state_xy(c, Q_dev, nullptr, t0);
}

int ader_upload_state_xy(ader_ctx* c, const double* Q_dev, const double* node_xy_dev, double t0) {
  if (!c || !Q_dev) return ADER_E_ARG;
  if (!c->bound) return fail(c, ADER_E_ORDER, "no workspace bound");
  const aw::Topology& t = c->topo;
  aw::Dev& d = c->dev;
  c->has_state = false;
  c->synced = false;
  int r;
  std::vector<double> xy;
  if (node_xy_dev) {
    LCHK(c, aw::launch_upload_xy(d, node_xy_dev, c->stream));
  } else {
    xy = to_soa(t.xy, t.NV, 2);
    if ((r = h2d(c, d.X, xy.data(), xy.size() * sizeof(double)))) return r;
  }
  aw::Scal s{};
  s.N = 1;
  if ((r = h2d(c, d.scal, &s, sizeof(s)))) return r;
  std::vector<aw::Inst> in(d.K);
  for (auto& x : in) x.T = t0;
  if ((r = h2d(c, d.inst, in.data(), in.size() * sizeof(aw::Inst)))) return r;
  c->cycles = 0;
  c->macro_steps = 0;
  c->extra_cycles = 0;
  c->long_macro_steps = 0;
  LCHK(c, aw::launch_init_geometry(d, c->stream));
  if (node_xy_dev) {
    // caller positions: refuse inverted elements before any kernel uses them
    aw::Scal g;
    if ((r = read_scal(c, g))) return r;
    if (g.err & aw::ERR_GEOM) return fail(c, ADER_E_GEOM, "node positions give an inverted or degenerate element");
  }
  LCHK(c, aw::launch_upload_q(d, Q_dev, c->stream));
  LCHK(c, aw::launch_check_state(d, c->prm.gamma, c->stream));
  LCHK(c, aw::launch_reconstruct(d, c->prm, c->cfg.M, 0, 0, c->stream));
  aw::Scal back;
  if ((r = read_scal(c, back))) return r;
  if (back.err) return fail(c, ADER_E_STATE, "initial state has rho <= 0 or p <= 0");
  c->has_state = true;
  c->synced = true;
  return ADER_OK;
}

int ader_step_gts(ader_ctx* c, double t_target, int32_t max_steps, ader_stats* st) {
  if (!c) return ADER_E_ARG;
  int r = run_macro(c, t_target, max_steps, 1);
  if (r) return r;
  return st ? ader_get_stats(c, st) : ADER_OK;
}

int ader_step_lts(ader_ctx* c, double t_target, int32_t max_macro_steps, ader_stats* st) {
  if (!c) return ADER_E_ARG;
  int r = c->cfg.lts_levels == 0 ? run_free(c, t_target, max_macro_steps)
                                 : run_macro(c, t_target, max_macro_steps, c->cfg.lts_levels);
  if (r) return r;
  return st ? ader_get_stats(c, st) : ADER_OK;
}

int ader_download_state(ader_ctx* c, double* Q_dev, double* node_xy_dev, double* elem_t_dev) {
  if (!c) return ADER_E_ARG;
  if (!c->has_state) return fail(c, ADER_E_ORDER, "no state uploaded");
  const aw::Dev& d = c->dev;
  if (Q_dev) LCHK(c, aw::launch_download_q(d, Q_dev, c->stream));
  if (node_xy_dev) LCHK(c, aw::launch_download_xy(d, node_xy_dev, c->stream));
  if (elem_t_dev) LCHK(c, aw::launch_elem_times(d, elem_t_dev, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return ADER_OK;
}

int ader_get_stats(ader_ctx* c, ader_stats* st) {
  if (!c || !st) return ADER_E_ARG;
  if (!c->bound) return fail(c, ADER_E_ORDER, "no workspace bound");
  aw::Scal s;
  std::vector<aw::Inst> in;
  int r = read_scal(c, s);
  if (r || (r = read_insts(c, in))) return r;
  fill_stats(c, s, in, st);
  return ADER_OK;
}

int ader_debug_size(const ader_ctx* cc, int32_t what, size_t* bytes) {
  ader_ctx* c = const_cast<ader_ctx*>(cc);
  if (!c || !bytes) return ADER_E_ARG;
  if (!c->has_mesh) return fail(c, ADER_E_ORDER, "no mesh uploaded");
  Arr a = lookup(c, what);
  if (a.bytes == 0) return fail(c, ADER_E_ARG, "unknown array");
  *bytes = a.bytes;
  return ADER_OK;
}

int ader_debug_dump(ader_ctx* c, int32_t what, void* host, size_t bytes) {
  if (!c || !host) return ADER_E_ARG;
  if (!c->has_mesh) return fail(c, ADER_E_ORDER, "no mesh uploaded");
  Arr a = lookup(c, what);
  if (a.bytes == 0 || bytes != a.bytes) return fail(c, ADER_E_ARG, "size mismatch");
  if (what >= ADER_DBG_TOPO_EDGES) {
    if (a.host) {
      std::memcpy(host, a.host, bytes);
    } else {
      std::vector<char> p = host_pack(c, what);
      if (p.size() != bytes) return fail(c, ADER_E_ARG, "size mismatch");
      std::memcpy(host, p.data(), bytes);
    }
    return ADER_OK;
  }
  if (!c->bound) return fail(c, ADER_E_ORDER, "no workspace bound");
  if (what == ADER_DBG_SCAL) {
    aw::Scal s;
    std::vector<aw::Inst> in;
    int r = read_scal(c, s);
    if (r || (r = read_insts(c, in))) return r;
    double v[4] = {in[0].T, in[0].delta, double(s.N), s.t_end};
    std::memcpy(host, v, sizeof(v));
    return ADER_OK;
  }
  if (what == ADER_DBG_QM || what == ADER_DBG_HM) {
    // memory variables: the sum of the element's three edge slots
    const size_t NE = c->topo.NE, W = aw::MEM_W;
    std::vector<double> m(NE * 3 * W);
    HIPCHK(c, hipMemcpyAsync(m.data(), c->dev.mem, m.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const int nf = what == ADER_DBG_QM ? 4 : 3, f0 = what == ADER_DBG_QM ? 0 : 4;
    double* out = static_cast<double*>(host);
    for (int f = 0; f < nf; ++f)
      for (size_t i = 0; i < NE; ++i)
        out[f * NE + i] = (m[(i * 3 + 0) * W + f0 + f] + m[(i * 3 + 1) * W + f0 + f]) + m[(i * 3 + 2) * W + f0 + f];
    return ADER_OK;
  }
  if (!a.dev) return packed_io(c, what, host, nullptr, bytes);
  HIPCHK(c, hipMemcpyAsync(host, a.dev, bytes, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return ADER_OK;
}

int ader_debug_inject(ader_ctx* c, int32_t what, const void* host, size_t bytes) {
  if (!c || !host) return ADER_E_ARG;
  if (!c->bound) return fail(c, ADER_E_ORDER, "no workspace bound");
  if (what >= ADER_DBG_TOPO_EDGES) return fail(c, ADER_E_ARG, "topology and tables are read-only");
  if (what == ADER_DBG_QM || what == ADER_DBG_HM)
    return fail(c, ADER_E_ARG, "memory variables are kept per element edge and cannot be injected");
  Arr a = lookup(c, what);
  if (a.bytes == 0 || bytes != a.bytes) return fail(c, ADER_E_ARG, "size mismatch");
  if (what == ADER_DBG_SCAL) {
    aw::Scal s;
    std::vector<aw::Inst> in;
    int r = read_scal(c, s);
    if (r || (r = read_insts(c, in))) return r;
    double v[4];
    std::memcpy(v, host, sizeof(v));
    in[0].T = v[0];
    in[0].delta = v[1];
    s.N = int(v[2]);
    s.t_end = v[3];
    if ((r = h2d(c, c->dev.scal, &s, sizeof(s)))) return r;
    if ((r = h2d(c, c->dev.inst, in.data(), sizeof(aw::Inst)))) return r;
  } else if (!a.dev) {
    int r = packed_io(c, what, nullptr, host, bytes);
    if (r) return r;
  } else {
    HIPCHK(c, hipMemcpyAsync(a.dev, host, bytes, hipMemcpyHostToDevice, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->has_state = true;
  c->synced = false;
  return ADER_OK;
}

int ader_debug_cycles(ader_ctx* c, int32_t n) {
  if (!c || n < 0) return ADER_E_ARG;
  if (!c->has_state) return fail(c, ADER_E_ORDER, "no state uploaded");
  c->synced = false;
  int r = issue_cycles(c, n, c->stream);
  if (r) return r;
  c->cycles += n;
  aw::Scal s;
  if ((r = read_scal(c, s))) return r;
  return check_err(c, s);
}

int ader_debug_macro_begin(ader_ctx* c, double t_end, int32_t levels) {
  if (!c || levels < 0 || levels > 8) return ADER_E_ARG;
  if (!c->has_state) return fail(c, ADER_E_ORDER, "no state uploaded");
  set_free(c, levels == 0);
  c->synced = false;
  LCHK(c, aw::launch_set_target(c->dev, t_end, c->stream));
  LCHK(c, aw::launch_open(c->dev, c->stream));
  int r = issue_macro_begin(c, levels == 0 ? 0 : 1 << (levels - 1), c->stream);
  if (r) return r;
  aw::Scal s;
  if ((r = read_scal(c, s))) return r;
  return check_err(c, s);
}

int ader_set_profiling(ader_ctx* c, int32_t on) {
  if (!c) return ADER_E_ARG;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  flush_events(c);
  for (int k = 0; k < ADER_K_COUNT; ++k) {
    c->kms[k] = 0.0;
    c->klaunch[k] = 0;
  }
  c->prof = on != 0;
  return ADER_OK;
}

int ader_instance_times(ader_ctx* c, int32_t n, double* T_host) {
  if (!c || n < 0 || (n > 0 && !T_host)) return ADER_E_ARG;
  if (!c->bound) return fail(c, ADER_E_ORDER, "no workspace bound");
  std::vector<aw::Inst> in;
  int r = read_insts(c, in);
  if (r) return r;
  for (int k = 0; k < n && k < int(in.size()); ++k) T_host[k] = in[k].T;
  return ADER_OK;
}

int ader_set_tune(ader_ctx* c, const ader_tune* t) {
  if (!c || !t) return ADER_E_ARG;
  if (t->sched_chunk != 0 && (t->sched_chunk < 32 || t->sched_chunk > 1024)) return ADER_E_ARG;
  if (t->list_wg_per_cu < 0 || t->list_wg_per_cu > 64) return ADER_E_ARG;
  if (t->sweep_wg_per_cu < 0 || t->sweep_wg_per_cu > 64) return ADER_E_ARG;
  c->dev.sched_chunk = t->sched_chunk;
  c->dev.list_wg_per_cu = t->list_wg_per_cu;
  c->dev.sweep_wg_per_cu = t->sweep_wg_per_cu;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  drop_graphs(c);
  return ADER_OK;
}

int ader_autotune(ader_ctx* c, int32_t trials, ader_tune* chosen) {
  if (!c || trials < 1) return ADER_E_ARG;
  if (!c->has_state) return fail(c, ADER_E_ORDER, "no state uploaded");
  const bool prof = c->prof;
  const int64_t cycles = c->cycles, macro = c->macro_steps;
  set_free(c, false);
  void* snap = nullptr;
  HIPCHK(c, hipMalloc(&snap, c->ws_bytes));
  c->prof = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int r = 0;
  auto cleanup = [&] {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(snap);
    c->prof = prof;
    c->cycles = cycles;
    c->macro_steps = macro;
  };
  auto restore = [&]() -> int {
    HIPCHK(c, hipMemcpyAsync(c->ws, snap, c->ws_bytes, hipMemcpyDeviceToDevice, c->stream));
    return 0;
  };
  // time `trials` macro steps of the current setting from the snapshot
  auto trial = [&](double& ms) -> int {
    int rr;
    if ((rr = restore())) return rr;
    const double far = 1e300;
    // free steps are tuned on 3 dyadic levels: the settings only group work
    const int nominal = c->cfg.lts_levels > 0 ? 1 << (c->cfg.lts_levels - 1) : 4;
    LCHK(c, aw::launch_set_target(c->dev, far, c->stream));
    LCHK(c, aw::launch_open(c->dev, c->stream));
    HIPCHK(c, hipEventRecord(e0, c->stream));
    for (int k = 0; k < trials; ++k)
      if ((rr = issue_macro(c, nominal, c->stream))) return rr;
    HIPCHK(c, hipEventRecord(e1, c->stream));
    HIPCHK(c, hipEventSynchronize(e1));
    float f = 0.f;
    HIPCHK(c, hipEventElapsedTime(&f, e0, e1));
    ms = double(f) / trials;
    return 0;
  };
  do {
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
      r = fail(c, ADER_E_HIP, "hipEventCreate");
      break;
    }
    hipError_t he = hipMemcpyAsync(snap, c->ws, c->ws_bytes, hipMemcpyDeviceToDevice, c->stream);
    if (he != hipSuccess) {
      r = hip_fail(c, int(he), "snapshot copy");
      break;
    }
    const int chunks[] = {0, 64, 128, 256, 512, 1024};
    const int wgs[] = {0, 4, 8, 16, 32};
    const int sweeps[] = {0, 4, 8, 16};
    double best = 1e300, ms = 0.0;
    int bc = c->dev.sched_chunk, bw = c->dev.list_wg_per_cu, bs = c->dev.sweep_wg_per_cu;
    for (int ch : chunks) {
      c->dev.sched_chunk = ch;
      c->dev.list_wg_per_cu = bw;
      c->dev.sweep_wg_per_cu = bs;
      if ((r = trial(ms))) break;
      if (ms < best) best = ms, bc = ch;
    }
    if (r) break;
    for (int w : wgs) {
      c->dev.sched_chunk = bc;
      c->dev.list_wg_per_cu = w;
      if ((r = trial(ms))) break;
      if (ms < best) best = ms, bw = w;
    }
    if (r) break;
    for (int w : sweeps) {
      c->dev.list_wg_per_cu = bw;
      c->dev.sweep_wg_per_cu = w;
      if ((r = trial(ms))) break;
      if (ms < best) best = ms, bs = w;
    }
    if (r) break;
    c->dev.sched_chunk = bc;
    c->dev.list_wg_per_cu = bw;
    c->dev.sweep_wg_per_cu = bs;
    if ((r = restore())) break;
    if ((he = hipStreamSynchronize(c->stream)) != hipSuccess) {
      r = hip_fail(c, int(he), "hipStreamSynchronize");
      break;
    }
    drop_graphs(c);
    if (chosen) {
      chosen->sched_chunk = bc;
      chosen->list_wg_per_cu = bw;
      chosen->sweep_wg_per_cu = bs;
      chosen->reserved = 0;
      chosen->ms_per_macro_step = best;
    }
  } while (false);
  (void)hipStreamSynchronize(c->stream);
  cleanup();
  return r;
}

int ader_adjoint_workspace_size(const ader_ctx* c, size_t* bytes) {
  if (!c || !bytes) return ADER_E_ARG;
  if (!c->has_mesh) return ADER_E_ORDER;
  *bytes = aw::adjoint_work_bytes(c->cfg.M, c->topo.NE, c->topo.NF, c->prm.npic);
  return ADER_OK;
}

}  // extern "C"

namespace {

// Checks shared by both adjoint entry points.
int adjoint_check(ader_ctx* c, double dt, const double* Q_dev) {
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, ADER_E_ARG, "dt must be positive and finite");
  if (c->cfg.mesh_velocity != 1) return fail(c, ADER_E_ARG, "the adjoint needs a fixed mesh (mesh_velocity = 1)");
  if (c->cfg.flux == ADER_FLUX_OSHER) return fail(c, ADER_E_ARG, "the adjoint covers the Rusanov and HLL fluxes");
  if (c->dev.K != 1) return fail(c, ADER_E_ARG, "the adjoint runs on a single instance");
  if (!c->has_state) return fail(c, ADER_E_ORDER, "no state uploaded");
  if (!Q_dev && !c->synced)
    return fail(c, ADER_E_ORDER, "elements are not at a common time (macro step in progress)");
  return 0;
}

aw::AdjWork adjoint_buffers(ader_ctx* c, const double* Q_dev, const double* Qbar_next_dev, double* Qbar_dev,
                            char* work) {
  aw::AdjWork w{};
  w.qbar_next = Qbar_next_dev;
  w.qbar = Qbar_dev;
  aw::adjoint_carve(c->cfg.M, c->topo.NE, c->topo.NF, c->prm.npic, work, w);
  w.q = Q_dev ? Q_dev : w.qcopy;
  return w;
}

}  // namespace

extern "C" {

int ader_adjoint_gts_step(ader_ctx* c, double dt, const double* Q_dev, const double* Qbar_next_dev,
                          double* Qbar_dev, void* work_dev, size_t work_bytes) {
  if (!c || !Qbar_next_dev || !Qbar_dev || !work_dev) return ADER_E_ARG;
  int r = adjoint_check(c, dt, Q_dev);
  if (r) return r;
  const size_t need = aw::adjoint_work_bytes(c->cfg.M, c->topo.NE, c->topo.NF, c->prm.npic);
  if (work_bytes < need) return fail(c, ADER_E_ARG, "adjoint workspace too small");
  if ((reinterpret_cast<uintptr_t>(work_dev) & 255) != 0)
    return fail(c, ADER_E_ARG, "adjoint workspace must be 256-byte aligned");
  const aw::AdjWork w = adjoint_buffers(c, Q_dev, Qbar_next_dev, Qbar_dev, static_cast<char*>(work_dev));
  LCHK(c, timed(c, ADER_K_ADJOINT, c->stream, [&] {
    return aw::launch_adjoint_gts(c->dev, c->prm, c->cfg.M, w, dt, Q_dev == nullptr, c->stream);
  }));
  return ADER_OK;
}

int ader_adjoint_gts_step_static(ader_ctx* c, double dt, const double* Q_dev, const double* Qbar_next_dev,
                                 double* Qbar_dev) {
  if (!c || !Qbar_next_dev || !Qbar_dev) return ADER_E_ARG;
  int r = adjoint_check(c, dt, Q_dev);
  if (r) return r;
  if (!c->static_work) return fail(c, ADER_E_ORDER, "no workspace bound (the fixed scratch is set up there)");
  const size_t need = aw::adjoint_work_bytes(c->cfg.M, c->topo.NE, c->topo.NF, c->prm.npic);
  if (need > c->static_bytes)
    return fail(c, ADER_E_ARG, "mesh too large for the fixed adjoint scratch: needs " + std::to_string(need) +
                                   " bytes, ADER_STATIC_SCRATCH_BYTES is " + std::to_string(c->static_bytes));
  const aw::AdjWork w = adjoint_buffers(c, Q_dev, Qbar_next_dev, Qbar_dev, static_cast<char*>(c->static_work));
  LCHK(c, aw::launch_adjoint_gts(c->dev, c->prm, c->cfg.M, w, dt, Q_dev == nullptr, c->stream));
  return ADER_OK;
}

int ader_adjoint_lagrangian_workspace_size(const ader_ctx* c, size_t* bytes) {
  if (!c || !bytes) return ADER_E_ARG;
  if (!c->has_mesh) return ADER_E_ORDER;
  *bytes = aw::lagadj_work_bytes(c->cfg.M, c->topo.NE, c->topo.NV, c->topo.NF, c->prm.npic);
  return ADER_OK;
}

int ader_adjoint_lagrangian_step(ader_ctx* c, double dt, const double* Q_dev, const double* X_dev,
                                 const double* Qbar_next_dev, const double* Xbar_next_dev, double* Qbar_dev,
                                 double* Xbar_dev, double* Q_next_dev, double* X_next_dev, void* work_dev,
                                 size_t work_bytes) {
  if (!c || !Qbar_next_dev || !Xbar_next_dev || !Qbar_dev || !Xbar_dev || !work_dev) return ADER_E_ARG;
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, ADER_E_ARG, "dt must be positive and finite");
  if (c->cfg.mesh_velocity != 0)
    return fail(c, ADER_E_ARG, "the moving-mesh adjoint needs the Lagrangian mesh (mesh_velocity = 0)");
  if (c->cfg.flux == ADER_FLUX_OSHER)
    return fail(c, ADER_E_ARG, "the moving-mesh adjoint covers the Rusanov and HLL fluxes");
  if (c->dev.K != 1) return fail(c, ADER_E_ARG, "the adjoint runs on a single instance");
  if (!c->has_state) return fail(c, ADER_E_ORDER, "no state uploaded");
  if ((!Q_dev || !X_dev) && !c->synced)
    return fail(c, ADER_E_ORDER, "elements are not at a common time (macro step in progress)");
  const size_t need = aw::lagadj_work_bytes(c->cfg.M, c->topo.NE, c->topo.NV, c->topo.NF, c->prm.npic);
  if (work_bytes < need) return fail(c, ADER_E_ARG, "adjoint workspace too small");
  if ((reinterpret_cast<uintptr_t>(work_dev) & 255) != 0)
    return fail(c, ADER_E_ARG, "adjoint workspace must be 256-byte aligned");
  aw::LagWork w{};
  aw::lagadj_carve(c->cfg.M, c->topo.NE, c->topo.NV, c->topo.NF, c->prm.npic, static_cast<char*>(work_dev), w);
  w.a.q = Q_dev;
  w.a.qbar_next = Qbar_next_dev;
  w.a.qbar = Qbar_dev;
  w.x = X_dev;
  w.xbar_next = Xbar_next_dev;
  w.xbar = Xbar_dev;
  w.qnext = Q_next_dev;
  w.xnext = X_next_dev;
  LCHK(c, timed(c, ADER_K_ADJOINT, c->stream, [&] {
    return aw::launch_adjoint_lagrangian(c->dev, c->prm, c->cfg.M, w, dt, Q_dev == nullptr, X_dev == nullptr,
                                         c->stream);
  }));
  return ADER_OK;
}

}  // extern "C"

namespace {
// The arrays of the simulation state that a time step changes, in a fixed
// order: the saved copies of the LTS adjoint hold them one after another,
// each 256-byte aligned.
std::vector<std::pair<void*, size_t>> state_arrays(const ader_ctx* c) {
  const aw::Dev& d = c->dev;
  const size_t NE = d.NE, NV = d.NV, M = d.M, D = sizeof(double), I = sizeof(int);
  std::vector<std::pair<void*, size_t>> a = {{d.scal, sizeof(aw::Scal)},
                                             {d.inst, size_t(d.K) * sizeof(aw::Inst)},
                                             {d.ts, NE * sizeof(aw::TickStep)},
                                             {d.rec, NE * aw::rec_stride(int(M)) * D},
                                             {d.trace, NE * aw::trace_stride(int(M)) * D},
                                             {d.wnod, NE * aw::wnod_stride(int(M)) * D},
                                             {d.dtcfl, NE * D},
                                             {d.mem, NE * 3 * aw::MEM_W * D},
                                             {d.act_stamp, NE * I},
                                             {d.act_list, NE * I},
                                             {d.live_list, NE * I},
                                             {d.X, 2 * NV * D},
                                             {d.Xnew, 2 * NV * D},
                                             {d.ntick, NV * I},
                                             {d.ntick_new, NV * I},
                                             {d.node_stamp, NV * I}};
  if (d.replay_pos) a.push_back({d.replay_pos, NE * I});
  if (d.rec_pos) a.push_back({d.rec_pos, NE * I});
  return a;
}

size_t al256(size_t n) { return (n + 255) & ~size_t(255); }

size_t state_bytes(const ader_ctx* c) {
  size_t n = 0;
  for (const auto& a : state_arrays(c)) n += al256(a.second);
  return n;
}

int state_copy(ader_ctx* c, char* saved, bool save) {
  size_t off = 0;
  for (const auto& a : state_arrays(c)) {
    if (save)
      HIPCHK(c, hipMemcpyAsync(saved + off, a.first, a.second, hipMemcpyDeviceToDevice, c->stream));
    else
      HIPCHK(c, hipMemcpyAsync(a.first, saved + off, a.second, hipMemcpyDeviceToDevice, c->stream));
    off += al256(a.second);
  }
  return 0;
}

// The parts of the state that the adjoint kernels read (ticks and steps,
// element records, traces, reconstructions, node positions and ticks): a
// view snapshot holds them one after another, each 256-byte aligned.
std::vector<std::pair<void*, size_t>> view_arrays(const ader_ctx* c) {
  const auto a = state_arrays(c);
  return {a[2], a[3], a[4], a[5], a[11], a[13]};
}

size_t view_bytes(const ader_ctx* c) {
  size_t n = 0;
  for (const auto& a : view_arrays(c)) n += al256(a.second);
  return n;
}

int view_save(ader_ctx* c, char* dst) {
  size_t off = 0;
  for (const auto& a : view_arrays(c)) {
    HIPCHK(c, hipMemcpyAsync(dst + off, a.first, a.second, hipMemcpyDeviceToDevice, c->stream));
    off += al256(a.second);
  }
  return 0;
}

aw::LtsView view_at(const ader_ctx* c, const char* saved) {
  std::vector<const char*> at;
  size_t off = 0;
  for (const auto& a : view_arrays(c)) {
    at.push_back(saved + off);
    off += al256(a.second);
  }
  aw::LtsView v;
  v.ts = (const aw::TickStep*)at[0];
  v.rec = (const double*)at[1];
  v.trace = (const double*)at[2];
  v.wnod = (const double*)at[3];
  v.X = (const double*)at[4];
  v.ntick = (const int*)at[5];
  return v;
}

// Device memory handed out in order from large chunks (freed together).
struct Pool {
  std::vector<char*> chunks;
  size_t chunk = 0, used = 0;
  int take(ader_ctx* c, size_t bytes, char** out) {
    bytes = al256(bytes);
    if (chunks.empty() || used + bytes > chunk) {
      const size_t n = bytes > chunk ? bytes : chunk;
      char* p = nullptr;
      HIPCHK(c, hipMalloc((void**)&p, n));
      chunks.push_back(p);
      chunk = n > chunk ? n : chunk;
      used = 0;
    }
    *out = chunks.back() + used;
    used += bytes;
    return 0;
  }
  void release() {
    for (char* p : chunks) (void)hipFree(p);
    chunks.clear();
  }
};

// One macro step cycle by cycle: after(k) runs after the macro-step start
// (k = 0) and after each cycle k (the cycle count read back each time);
// *ran = 0 when every instance had already reached t_end. Leaves the context
// as run_macro does.
template <class F>
int macro_by_cycles(ader_ctx* c, double t_end, int nominal, F after, int* ran, double* delta) {
  const aw::Dev& d = c->dev;
  aw::Scal s;
  int r;
  *ran = 0;
  c->synced = false;
  set_free(c, nominal == 0);
  LCHK(c, aw::launch_set_target(d, t_end, c->stream));
  LCHK(c, aw::launch_open(d, c->stream));
  if ((r = read_scal(c, s))) return r;
  if ((r = check_err(c, s))) return r;
  if (s.n_open == 0) {
    c->synced = true;
    return 0;
  }
  if ((r = issue_macro_begin(c, nominal, c->stream))) return r;
  aw::Inst in0;
  HIPCHK(c, hipMemcpyAsync(&in0, d.inst, sizeof(in0), hipMemcpyDeviceToHost, c->stream));
  if ((r = after(0))) return r;
  // the first 2^(L-1) cycles without a host check (as run_macro), then one
  // cycle per check; free steps: FREE_BATCH cycles per check (as run_free)
  int k = 0;
  for (;;) {
    const int batch = nominal == 0 ? FREE_BATCH : (k == 0 ? nominal : 1);
    for (int b = 0; b < batch; ++b) {
      if ((r = issue_cycles(c, 1, c->stream))) return r;
      if (b == batch - 1) LCHK(c, aw::launch_status(d, c->stream));
      if ((r = after(k + 1))) return r;
      ++k;
    }
    if ((r = read_scal(c, s))) return r;
    if ((r = check_err(c, s))) return r;
    if (s.n_unfinished == 0) break;
    if (k > (1 << 20)) return fail(c, ADER_E_DEADLOCK, "no element satisfies the update criterion");
  }
  LCHK(c, aw::launch_macro_end(d, 0, c->stream));
  LCHK(c, aw::launch_open(d, c->stream));
  if ((r = read_scal(c, s))) return r;
  c->cycles += k;
  if (nominal > 0 && k > nominal) {
    c->extra_cycles += k - nominal;
    c->long_macro_steps++;
  }
  c->macro_steps++;
  c->synced = true;
  *delta = in0.delta;
  *ran = 1;
  return 0;
}

// Forward over up to n_macro macro steps, then the reverse sweep. The last
// macro steps (as many as a budget of 60% of the free device memory allows)
// run cycle by cycle with the state after the macro-step start and after
// every cycle kept; each earlier one runs as in ader_step_lts with the full
// state saved at its start, and is replayed cycle by cycle when the sweep
// reaches it. Per macro step (last first): the cycles in reverse, then the
// start's predictors; finally the pre-processing reconstruction. The context
// ends at the forward's end state.
int adjoint_lts_run(ader_ctx* c, int n_macro, int keep_req, double t_end, const double* Qbar, const double* Xbar,
                    double* Qbar0, double* Xbar0, int* n_done, Pool& pool, std::vector<char*>& bufs) {
  const aw::Dev& d = c->dev;
  const int M = c->cfg.M, L = c->cfg.lts_levels, nominal = L > 0 ? 1 << (L - 1) : 0;
  const size_t sb = state_bytes(c), vb = view_bytes(c);
  auto take = [&](char** out, size_t bytes) -> int {
    HIPCHK(c, hipMalloc((void**)out, bytes));
    bufs.push_back(*out);
    return 0;
  };
  int r;
  char* wb = nullptr;
  const size_t wbytes = aw::lts_work_bytes(M, d.NE, d.NV, d.NF, c->prm.npic);
  if ((r = take(&wb, wbytes))) return r;
  aw::LtsWork w;
  aw::lts_carve(M, d.NE, d.NV, d.NF, c->prm.npic, wb, w);
  char* v0 = nullptr;   // the uploaded state
  if ((r = take(&v0, vb))) return r;
  if ((r = view_save(c, v0))) return r;
  size_t free_b = 0, total_b = 0;
  HIPCHK(c, hipMemGetInfo(&free_b, &total_b));
  const size_t per_macro = size_t(nominal > 0 ? nominal + 3 : 4 * FREE_BATCH) * vb;
  const long fits = long(std::min<size_t>(size_t(n_macro), size_t(0.6 * double(free_b)) / per_macro));
  const long kept = keep_req < 0 ? fits : std::min<long>(keep_req, n_macro);
  pool.chunk = std::max<size_t>(vb, size_t(64) * vb);
  std::vector<std::vector<char*>> views(n_macro);   // kept macro steps: start, then each cycle
  std::vector<char*> start(n_macro, nullptr);       // replayed macro steps: full state at the start
  std::vector<double> delta(n_macro, 0.0);
  int done = 0;
  for (int m = 0; m < n_macro; ++m) {
    int ran = 0;
    if (m >= n_macro - kept) {
      auto keep = [&](int k) -> int {
        char* p = nullptr;
        int e = pool.take(c, vb, &p);
        if (e) return e;
        views[m].push_back(p);
        (void)k;
        return view_save(c, p);
      };
      if ((r = macro_by_cycles(c, t_end, nominal, keep, &ran, &delta[m]))) return r;
    } else {
      if ((r = take(&start[m], sb))) return r;
      if ((r = state_copy(c, start[m], true))) return r;
      const int64_t before = c->macro_steps;
      if ((r = L > 0 ? run_macro(c, t_end, 1, L) : run_free(c, t_end, 1))) return r;
      ran = c->macro_steps != before;
    }
    if (!ran) break;
    ++done;
  }
  char* end_state = nullptr;
  if (done > 0 && start[0]) {   // a replay will change the state: keep the end state
    if ((r = take(&end_state, sb))) return r;
    if ((r = state_copy(c, end_state, true))) return r;
  }
  LCHK(c, aw::launch_lts_init(d, w, Qbar, Xbar, c->stream));
  std::vector<char*> replay;   // views of a replayed macro step (buffers reused)
  std::vector<char*> cur;
  for (int m = done - 1; m >= 0; --m) {
    std::vector<char*>* vs = &views[m];
    if (start[m]) {
      if ((r = state_copy(c, start[m], false))) return r;
      size_t n = 0;
      auto keep = [&](int k) -> int {
        if (replay.size() < n + 1) {
          char* p = nullptr;
          int e = take(&p, vb);
          if (e) return e;
          replay.push_back(p);
        }
        (void)k;
        return view_save(c, replay[n++]);
      };
      int ran = 0;
      const int64_t steps = c->macro_steps, cycles = c->cycles, extra = c->extra_cycles,
                    longm = c->long_macro_steps;
      if ((r = macro_by_cycles(c, t_end, nominal, keep, &ran, &delta[m]))) return r;
      c->macro_steps = steps;
      c->cycles = cycles;
      c->extra_cycles = extra;
      c->long_macro_steps = longm;
      if (!ran) return fail(c, ADER_E_STATE, "LTS adjoint: a replayed macro step did not run");
      cur.assign(replay.begin(), replay.begin() + n);
      vs = &cur;
    }
    const int nc = int(vs->size()) - 1;
    w.delta = delta[m];
    for (int k = nc - 1; k >= 0; --k) {
      w.s0 = view_at(c, (*vs)[k]);
      w.s1 = view_at(c, (*vs)[k + 1]);
      LCHK(c, aw::launch_lts_cycle_rev(d, c->prm, M, w, c->stream));
    }
    w.s1 = view_at(c, (*vs)[0]);
    LCHK(c, aw::launch_lts_macro_begin_rev(d, c->prm, M, w, c->stream));
  }
  w.s1 = view_at(c, v0);
  LCHK(c, aw::launch_lts_initial_rev(d, c->prm, M, w, c->stream));
  LCHK(c, aw::launch_lts_out(d, w, Qbar0, Xbar0, c->stream));
  if (end_state && (r = state_copy(c, end_state, false))) return r;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->synced = true;
  *n_done = done;
  return 0;
}
}  // namespace

extern "C" {

int ader_adjoint_lts(ader_ctx* c, int32_t n_macro, int32_t keep_macro_steps, double t_end, const double* Qbar_dev,
                     const double* Xbar_dev, double* Qbar0_dev, double* Xbar0_dev, int32_t* n_done) {
  if (!c || !Qbar_dev || !Xbar_dev || !Qbar0_dev || !Xbar0_dev || !n_done || n_macro < 1) return ADER_E_ARG;
  if (!c->has_state) return fail(c, ADER_E_ORDER, "no state uploaded");
  if (c->cycles != 0 || c->macro_steps != 0)
    return fail(c, ADER_E_ORDER, "the LTS adjoint starts from an uploaded state with no step taken since");
  if (c->cfg.mesh_velocity != 0 && c->cfg.mesh_velocity != 1)
    return fail(c, ADER_E_ARG, "the LTS adjoint covers the mesh moving with the fluid and the fixed mesh");
  if (c->dev.K != 1) return fail(c, ADER_E_ARG, "the LTS adjoint runs one instance");
  if (c->prm.flux != ADER_FLUX_RUSANOV && c->prm.flux != ADER_FLUX_HLL)
    return fail(c, ADER_E_ARG, "the LTS adjoint covers the Rusanov and HLL fluxes");
  if (!std::isfinite(t_end)) return fail(c, ADER_E_ARG, "t_end is not finite");
  std::vector<char*> bufs;
  Pool pool;
  int done = 0;
  const int r =
      adjoint_lts_run(c, n_macro, keep_macro_steps, t_end, Qbar_dev, Xbar_dev, Qbar0_dev, Xbar0_dev, &done, pool, bufs);
  (void)hipStreamSynchronize(c->stream);
  for (char* p : bufs) (void)hipFree(p);
  pool.release();
  if (r) return r;
  *n_done = done;
  return ADER_OK;
}

int ader_probe_contraction(ader_ctx* c, int32_t use_mfma, int64_t n_elems, int32_t iters, const double* F_dev,
                           double* out_dev, float* ms) {
  if (!c || !F_dev || !out_dev || n_elems <= 0 || n_elems > INT32_MAX || iters < 1) return ADER_E_ARG;
  if (!c->bound) return fail(c, ADER_E_ORDER, "no workspace bound");
  if (c->cfg.M != 2) return fail(c, ADER_E_ARG, "the contraction probe measures M = 2");
  hipStream_t s = c->stream;
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  HIPCHK(c, hipEventRecord(e0, s));
  const int r = aw::probe_contraction(c->dev.tab, use_mfma, long(n_elems), iters, F_dev, out_dev, s, 0);
  HIPCHK(c, hipEventRecord(e1, s));
  HIPCHK(c, hipEventSynchronize(e1));
  float t = 0.f;
  HIPCHK(c, hipEventElapsedTime(&t, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (r) return hip_fail(c, r, "probe launch");
  if (ms) *ms = t;
  return ADER_OK;
}

int ader_set_schedule_replay(ader_ctx* c, const int32_t* step_ptr, const int32_t* steps, int64_t n_steps) {
  if (!c) return ADER_E_ARG;
  if (!c->bound) return fail(c, ADER_E_ORDER, "no workspace bound");
  const size_t NE = c->topo.NE;
  if (step_ptr) {
    if (n_steps < 0 || n_steps > INT32_MAX || (n_steps > 0 && !steps))
      return fail(c, ADER_E_ARG, "schedule replay: bad step count");
    if (step_ptr[0] != 0 || int64_t(step_ptr[NE]) != n_steps)
      return fail(c, ADER_E_ARG, "schedule replay: step_ptr must run from 0 to n_steps");
    for (size_t i = 0; i < NE; ++i)
      if (step_ptr[i + 1] < step_ptr[i]) return fail(c, ADER_E_ARG, "schedule replay: step_ptr decreases");
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->replay_buf) {
    HIPCHK(c, hipFree(c->replay_buf));
    c->replay_buf = nullptr;
  }
  c->dev.replay_ptr = c->dev.replay_steps = nullptr;
  c->dev.replay_pos = nullptr;
  drop_graphs(c);              // graphs hold the launch arguments they were captured with
  if (!step_ptr) return ADER_OK;
  const size_t words = (NE + 1) + size_t(n_steps) + NE;
  HIPCHK(c, hipMalloc(&c->replay_buf, words * sizeof(int)));
  std::vector<int> host(words, 0);
  std::memcpy(host.data(), step_ptr, (NE + 1) * sizeof(int));
  if (n_steps) std::memcpy(host.data() + NE + 1, steps, size_t(n_steps) * sizeof(int));
  HIPCHK(c, hipMemcpyAsync(c->replay_buf, host.data(), words * sizeof(int), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->dev.replay_ptr = c->replay_buf;
  c->dev.replay_steps = c->replay_buf + NE + 1;
  c->dev.replay_pos = c->replay_buf + NE + 1 + n_steps;
  return ADER_OK;
}

int ader_set_graphs(ader_ctx* c, int32_t on) {
  if (!c) return ADER_E_ARG;
  c->graphs = on != 0;
  return ADER_OK;
}

int ader_kernel_times(ader_ctx* c, int32_t n, double* total_ms, int64_t* launches) {
  if (!c || n < 0 || (n > 0 && (!total_ms || !launches))) return ADER_E_ARG;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  flush_events(c);
  for (int k = 0; k < n; ++k) {
    total_ms[k] = k < ADER_K_COUNT ? c->kms[k] : 0.0;
    launches[k] = k < ADER_K_COUNT ? c->klaunch[k] : 0;
  }
  return ADER_OK;
}

const char* ader_last_error(const ader_ctx* c) {
  if (!c) return "null context";
  return c->err.c_str();
}

int ader_set_delta_replay(ader_ctx* c, const double* deltas, int32_t n) {
  if (!c) return ADER_E_ARG;
  if (!c->bound) return fail(c, ADER_E_ORDER, "no workspace bound");
  if (n < 0 || (n > 0 && !deltas)) return fail(c, ADER_E_ARG, "tick-length replay: bad count");
  if (n > 0 && c->dev.K != 1) return fail(c, ADER_E_ARG, "tick-length replay runs one instance");
  for (int32_t m = 0; m < n; ++m)
    if (!(deltas[m] > 0.0) || !std::isfinite(deltas[m]))
      return fail(c, ADER_E_ARG, "tick-length replay: tick lengths must be positive and finite");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->delta_buf) {
    HIPCHK(c, hipFree(c->delta_buf));
    c->delta_buf = nullptr;
  }
  c->dev.replay_delta = nullptr;
  c->dev.replay_delta_n = 0;
  drop_graphs(c);
  if (n == 0) return ADER_OK;
  HIPCHK(c, hipMalloc(&c->delta_buf, size_t(n) * sizeof(double)));
  HIPCHK(c, hipMemcpyAsync(c->delta_buf, deltas, size_t(n) * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->dev.replay_delta = c->delta_buf;
  c->dev.replay_delta_n = n;
  return ADER_OK;
}

int ader_set_schedule_record(ader_ctx* c, int32_t steps_per_element, int32_t macro_steps) {
  if (!c) return ADER_E_ARG;
  if (!c->bound) return fail(c, ADER_E_ORDER, "no workspace bound");
  if (steps_per_element < 0 || macro_steps < 0) return fail(c, ADER_E_ARG, "schedule record: negative capacity");
  if (steps_per_element > 0 && c->dev.K != 1) return fail(c, ADER_E_ARG, "schedule record runs one instance");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->rec_buf) (void)hipFree(c->rec_buf);
  if (c->rec_delta_buf) (void)hipFree(c->rec_delta_buf);
  c->rec_buf = nullptr;
  c->rec_delta_buf = nullptr;
  aw::Dev& d = c->dev;
  d.rec_steps = d.rec_pos = nullptr;
  d.rec_cap = 0;
  d.rec_delta = nullptr;
  d.rec_delta_cap = 0;
  drop_graphs(c);
  if (steps_per_element == 0) return ADER_OK;
  const size_t NE = c->topo.NE;
  HIPCHK(c, hipMalloc(&c->rec_buf, (NE * size_t(steps_per_element) + NE) * sizeof(int)));
  HIPCHK(c, hipMemsetAsync(c->rec_buf + NE * size_t(steps_per_element), 0, NE * sizeof(int), c->stream));
  const size_t nd = size_t(macro_steps > 0 ? macro_steps : 1);
  HIPCHK(c, hipMalloc(&c->rec_delta_buf, nd * sizeof(double)));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  d.rec_steps = c->rec_buf;
  d.rec_pos = c->rec_buf + NE * size_t(steps_per_element);
  d.rec_cap = steps_per_element;
  d.rec_delta = c->rec_delta_buf;
  d.rec_delta_cap = macro_steps;
  return ADER_OK;
}

int ader_get_schedule_record(ader_ctx* c, int32_t* step_ptr, int32_t* steps, int64_t steps_cap, double* deltas,
                             int32_t deltas_cap, int64_t* n_steps, int32_t* n_deltas) {
  if (!c || !step_ptr || !n_steps || !n_deltas) return ADER_E_ARG;
  if (!c->dev.rec_steps) return fail(c, ADER_E_ORDER, "no schedule record");
  const aw::Dev& d = c->dev;
  const size_t NE = c->topo.NE;
  std::vector<int> pos(NE);
  aw::Scal sc;
  HIPCHK(c, hipMemcpyAsync(pos.data(), d.rec_pos, NE * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(&sc, d.scal, sizeof(sc), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (sc.err & aw::ERR_RECORD) return fail(c, ADER_E_ARG, "schedule record: capacity exceeded");
  step_ptr[0] = 0;
  for (size_t i = 0; i < NE; ++i) step_ptr[i + 1] = step_ptr[i] + pos[i];
  *n_steps = step_ptr[NE];
  *n_deltas = std::min(sc.macro_index, d.rec_delta_cap);
  if (steps) {
    if (steps_cap < *n_steps) return fail(c, ADER_E_ARG, "schedule record: steps buffer too small");
    std::vector<int> all(NE * size_t(d.rec_cap));
    HIPCHK(c, hipMemcpyAsync(all.data(), d.rec_steps, all.size() * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (size_t i = 0; i < NE; ++i)
      std::memcpy(steps + step_ptr[i], all.data() + i * size_t(d.rec_cap), size_t(pos[i]) * sizeof(int));
  }
  if (deltas) {
    if (deltas_cap < *n_deltas) return fail(c, ADER_E_ARG, "schedule record: tick-length buffer too small");
    HIPCHK(c, hipMemcpyAsync(deltas, d.rec_delta, size_t(*n_deltas) * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return ADER_OK;
}

void ader_destroy(ader_ctx* c) {
  if (!c) return;
  if (c->bound) (void)hipStreamSynchronize(c->stream);
  if (c->replay_buf) (void)hipFree(c->replay_buf);
  if (c->delta_buf) (void)hipFree(c->delta_buf);
  if (c->rec_buf) (void)hipFree(c->rec_buf);
  if (c->rec_delta_buf) (void)hipFree(c->rec_delta_buf);
  drop_graphs(c);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  for (int k = 0; k < ADER_K_COUNT; ++k)
    for (auto& p : c->ev[k]) {
      (void)hipEventDestroy(p.first);
      (void)hipEventDestroy(p.second);
    }
  delete c;
}

}  // extern "C"
