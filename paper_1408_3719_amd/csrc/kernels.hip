// HIP kernels (gfx950) of the ALE ADER-WENO scheme with local time stepping.
//
// One cycle of the local time stepping (paper Sec. 2.6, "computational phase"),
// read data-parallel: the active set is fixed from the cycle-start ticks, then
//   k_sched       update criterion (eq. eqn.WENOupdate) over the symmetric
//                 scheduling stencil, compacted active list
//   k_node        node solver NS_cs (eqs. eqnNScs, eqn.NScs.weights, eqn.dtau,
//                 NodesVel) and node motion (eq. eqn.newVertex)
//   k_patch       flux through every space-time patch swept by a moved edge
//                 (eqs. eqn.spacetimenodes, G_ij, eqn.STint) with the Rusanov
//                 (eqs. eqn.rusanov, A_n^V), Osher-type (eqs. eqn.osher,
//                 eqn.path) or HLL flux
//   k_update      memory variables (eq. eqn.Qm2 and the geometric memory) and
//                 the one-step update (eq. PDEfinal) with the GCL check (eqn.gcl)
//   k_reconstruct virtual projection of the stencils (eqs. eqn.virtGeom,
//                 eqn.virtCellaverage), WENO (eqs. intConsRec .. eqn.weno), local
//                 time step (eq. eqn.timestep) and dyadic level
//   k_predict     space-time Galerkin predictor of the PDE and of the mesh ODE
//                 (eqs. timeTransf .. newVertPos)
// Every write target has a single writer per kernel: no atomics on state.
// A macro step adds the per-instance tick lengths and levels (k_min_dt,
// k_macro_setup, k_levels) and its end (k_macro_end); instances of a batch
// (independent meshes) keep their own time and tick length (Inst).
//
// Lane mappings (64-wide wavefronts):
//   k_reconstruct: 8 lanes per element, lane s solves stencil s (s < 7), lane 7
//                  computes the CFL step; the WENO sum is a 3-step butterfly;
//                  the rows of a stencil are software-pipelined.
//   k_predict:     nb lanes per element, floor(64/nb) elements per wavefront,
//                  lane m owns spatial node m for all time nodes; spatial
//                  derivatives read the other nodes of the same time slice
//                  from LDS, ordered within the wavefront.
//   k_sched:       8 lanes per element over its scheduling stencil.
//   others:        one lane per node, edge or element.
// Blocks are renumbered so that each XCD works on a contiguous index range.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cfloat>

#include "aderweno.h"
#include "basis.h"
#include "common.h"

namespace aw {

namespace {

constexpr int TPB = 256;

template <int M>
struct Sz {
  static constexpr int nb = (M + 1) * (M + 2) / 2;
  static constexpr int nt = M + 1;
  static constexpr int nG = M + 1;
  static constexpr int ne = 2 * nb;
  static constexpr int nu = nb - 1;
  static constexpr int RS = rec_stride(M);
  static constexpr int TS = trace_stride(M);
  static constexpr int WS = wnod_stride(M);
  static constexpr int VV = rec_off_vv(M);
  // predictor: one lane per spatial node, as many elements per wavefront as fit
  static constexpr int EPW = 64 / nb;
};

constexpr int XE = rec_off_xe(), QO = rec_off_q(), AO = rec_off_a(), AVG = rec_off_avg();

__device__ inline void set_err(const Dev& d, int bits) { atomicOr(&d.scal->err, bits); }

// Tick length of the instance of element i / node k (one instance: no gather).
__device__ inline double elem_delta(const Dev& d, int i) {
  return d.K == 1 ? d.inst[0].delta : d.inst[d.e_inst[i]].delta;
}
__device__ inline double node_delta(const Dev& d, int k) {
  return d.K == 1 ? d.inst[0].delta : d.inst[d.v_inst[k]].delta;
}

// atomic maximum of a non-negative double through its bit pattern
__device__ inline void atomic_max_pos(unsigned long long* a, double v) {
  atomicMax(a, (unsigned long long)__double_as_longlong(v));
}

// Workgroup totals for the statistics counters: one atomic per workgroup
// instead of one per wavefront (atomics on one address serialise, ~12 ns
// each). Every thread of the workgroup calls them, once per kernel.
__device__ inline void block_add(unsigned long long* ctr, unsigned long long v) {
  __shared__ unsigned long long part_add[TPB / 64];
#pragma unroll
  for (int s = 1; s < 64; s <<= 1) v += __shfl_xor(v, s);
  if (__lane_id() == 0) part_add[threadIdx.x / 64] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < int(blockDim.x / 64); ++w) t += part_add[w];
    if (t) atomicAdd(ctr, t);
  }
}
__device__ inline void block_max_pos(unsigned long long* ctr, double v) {
  __shared__ double part_max[TPB / 64];
#pragma unroll
  for (int s = 1; s < 64; s <<= 1) v = fmax(v, __shfl_xor(v, s));
  if (__lane_id() == 0) part_max[threadIdx.x / 64] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < int(blockDim.x / 64); ++w) t = fmax(t, part_max[w]);
    if (t > 0.0) atomic_max_pos(ctr, t);
  }
}

__device__ inline double pressure(const double q[4], double g) {
  return (g - 1.0) * (q[3] - 0.5 * (q[1] * q[1] + q[2] * q[2]) / q[0]);
}

// Space-time flux F~(q) . N = f N_x + g N_y + q N_t (eq. PDEdiv3D) through an
// unnormalised space-time normal N, nxy = |N_xy|; also the ALE normal speed
// un = u . N_xy + N_t and the scaled sound speed cn = c |N_xy|, so that the
// eigenvalues of the ALE Jacobian along N (eq. A_n^V) are un - cn, un, un + cn.
__device__ inline void stflux(const double q[4], const double N[3], double nxy, double g,
                              double out[4], double& un, double& cn) {
  const double ir = 1.0 / q[0];
  const double u = q[1] * ir, v = q[2] * ir;
  const double p = (g - 1.0) * (q[3] - 0.5 * (q[1] * u + q[2] * v));
  const double uxy = u * N[0] + v * N[1];
  un = uxy + N[2];
  out[0] = q[0] * un;
  out[1] = q[1] * un + p * N[0];
  out[2] = q[2] * un + p * N[1];
  out[3] = q[3] * un + p * uxy;
  cn = sqrt(g * p * ir) * nxy;
}

// Osher-type dissipation of eq. eqn.osher: sum_s w_s |A(Psi(s))| dq along the
// straight path Psi(s) = ql + s dq of eq. eqn.path, with |A| = R |Lambda| R^-1
// applied as wave strengths alpha = R^-1 dq followed by sum_k |lambda_k| alpha_k r_k.
// r_k, R^-1 are the eigenvectors of the Euler flux Jacobian along the unit normal
// n = N_xy / |N_xy| (acoustic, entropy, shear, acoustic); the ALE eigenvalues are
// (u.n -/+ c) |N_xy| + N_t and u.n |N_xy| + N_t (entropy and shear).
__device__ inline void osher_dissipation(const Tables* tb, const double ql[4], const double qr[4],
                                         const double N[3], double nxy, double g, double D[4]) {
  double dq[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    dq[v] = qr[v] - ql[v];
    D[v] = 0.0;
  }
  if (!(nxy > 0.0)) {   // no spatial extent: A = N_t I
#pragma unroll
    for (int v = 0; v < 4; ++v) D[v] = fabs(N[2]) * dq[v];
    return;
  }
  const double inxy = 1.0 / nxy;
  const double nx = N[0] * inxy, ny = N[1] * inxy;
  const double gm = g - 1.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double s = tb->osh_s[k], w = tb->osh_w[k];
    double ps[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) ps[v] = ql[v] + s * dq[v];
    const double ir = 1.0 / ps[0];
    const double u = ps[1] * ir, v = ps[2] * ir;
    const double q2 = u * u + v * v;
    const double p = gm * (ps[3] - 0.5 * ps[0] * q2);
    const double c2 = g * p * ir, c = sqrt(c2), ic2 = 1.0 / c2;
    const double H = (ps[3] + p) * ir;
    const double un = u * nx + v * ny, ut = v * nx - u * ny;
    // wave strengths
    const double X = gm * (0.5 * q2 * dq[0] - u * dq[1] - v * dq[2] + dq[3]);
    const double Y = c * (un * dq[0] - nx * dq[1] - ny * dq[2]);
    const double a1 = 0.5 * (X + Y) * ic2, a4 = 0.5 * (X - Y) * ic2;
    const double a2 = dq[0] - X * ic2;
    const double a3 = nx * dq[2] - ny * dq[1] - ut * dq[0];
    const double l1 = fabs((un - c) * nxy + N[2]), l2 = fabs(un * nxy + N[2]);
    const double l4 = fabs((un + c) * nxy + N[2]);
    const double b1 = w * l1 * a1, b2 = w * l2 * a2, b3 = w * l2 * a3, b4 = w * l4 * a4;
    D[0] += b1 + b2 + b4;
    D[1] += b1 * (u - c * nx) + b2 * u - b3 * ny + b4 * (u + c * nx);
    D[2] += b1 * (v - c * ny) + b2 * v + b3 * nx + b4 * (v + c * ny);
    D[3] += b1 * (H - un * c) + b2 * (0.5 * q2) + b3 * ut + b4 * (H + un * c);
  }
}

// Numerical flux through the unnormalised space-time normal N of a patch
// quadrature point: Rusanov (eq. eqn.rusanov), Osher-type (eq. eqn.osher) or HLL.
__device__ inline void numerical_flux(int flux, const Tables* tb, const double ql[4],
                                      const double qr[4], const double N[3], double g,
                                      double out[4]) {
  const double nxy = sqrt(N[0] * N[0] + N[1] * N[1]);
  double fl[4], fr[4], unl, cl, unr, cr;
  stflux(ql, N, nxy, g, fl, unl, cl);
  stflux(qr, N, nxy, g, fr, unr, cr);
  if (flux == ADER_FLUX_HLL) {
    // signal speeds bounded over both states; upwind when both have one sign
    const double sl = fmin(unl - cl, unr - cr), sr = fmax(unl + cl, unr + cr);
    if (sl >= 0.0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) out[v] = fl[v];
    } else if (sr <= 0.0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) out[v] = fr[v];
    } else {
      const double id = 1.0 / (sr - sl);
#pragma unroll
      for (int v = 0; v < 4; ++v) out[v] = (sr * fl[v] - sl * fr[v] + sl * sr * (qr[v] - ql[v])) * id;
    }
  } else if (flux == ADER_FLUX_OSHER) {
    double D[4];
    osher_dissipation(tb, ql, qr, N, nxy, g, D);
#pragma unroll
    for (int v = 0; v < 4; ++v) out[v] = 0.5 * (fl[v] + fr[v]) - 0.5 * D[v];
  } else {
    // Rusanov: the largest |eigenvalue| of the ALE Jacobian over both states
    const double smax = fmax(fabs(unl) + cl, fabs(unr) + cr);
#pragma unroll
    for (int v = 0; v < 4; ++v) out[v] = 0.5 * (fl[v] + fr[v]) - 0.5 * smax * (qr[v] - ql[v]);
  }
}

// (a - b) / step: exact for the power-of-two steps of dyadic levels, a
// correctly rounded division for free steps
__device__ inline double tick_ratio(double a_minus_b, int step) {
  return (step & (step - 1)) == 0 ? ldexp(a_minus_b, -__builtin_ctz(step)) : a_minus_b / double(step);
}


template <int M>
__device__ inline const double* rec(const Dev& d, int i) {
  return d.rec + size_t(i) * Sz<M>::RS;
}

// Stored data of element j needed to place it at tick nt: its vertices and
// either its average (j at tick nt) or its predictor's nodal averages in time;
// the predictor's vertex velocities are read where they are used.
template <int M>
struct NbrRaw {
  double xe[6];
  double av[4 * (M + 1)];
  const double* vv;
};

template <int M>
__device__ inline void fetch_nbr(const Dev& d, int j, TickStep tsj, int nt, NbrRaw<M>& r) {
  constexpr int T = M + 1, VV = Sz<M>::VV;
  const double* p = rec<M>(d, j);
  r.vv = p + VV;
#pragma unroll
  for (int c = 0; c < 6; ++c) r.xe[c] = p[XE + c];
  if (tsj.tick == nt) {
#pragma unroll
    for (int v = 0; v < 4; ++v) r.av[v] = p[QO + v];
  } else {
#pragma unroll
    for (int c = 0; c < 4 * T; ++c) r.av[c] = p[AVG + c];
  }
}

// Geometry (x0 y0 x1 y1 x2 y2) and average of element j at tick nt: the real
// data when j is at that tick, else its predictor projected there.
template <int M>
__device__ inline bool place_nbr(const Tables* tb, const NbrRaw<M>& r, TickStep tsj, int nt,
                                 double delta, double X[6], double Qv[4]) {
  constexpr int T = M + 1;
  if (tsj.tick == nt) {
#pragma unroll
    for (int c = 0; c < 6; ++c) X[c] = r.xe[c];
#pragma unroll
    for (int v = 0; v < 4; ++v) Qv[v] = r.av[v];
    return true;
  }
  if (tsj.step <= 0) return false;
  const double tau = tick_ratio(double(nt - tsj.tick), tsj.step);
  const double dtj = double(tsj.step) * delta;
  double L[T], l[T];
  time_antideriv<M>(tau, L);
  time_basis<M>(tau, l);
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < T; ++q) s += L[q] * r.vv[(k * T + q) * 2 + c];
      X[2 * k + c] = r.xe[2 * k + c] + dtj * s;
    }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < T; ++q) s += l[q] * r.av[q * 4 + v];
    Qv[v] = s;
  }
  return true;
}

template <int M>
__device__ inline bool project(const Dev& d, const Tables* tb, int j, int nt, double delta,
                               double X[6], double Qv[4]) {
  const TickStep tsj = d.ts[j];
  NbrRaw<M> r;
  fetch_nbr<M>(d, j, tsj, nt, r);
  return place_nbr<M>(tb, r, tsj, nt, delta, X, Qv);
}

__device__ inline double tri_area(const double X[6]) {
  return 0.5 * ((X[2] - X[0]) * (X[5] - X[1]) - (X[4] - X[0]) * (X[3] - X[1]));
}

__device__ inline double cfl_ratio(const double X[6], const double Q[4], double g) {
  double per = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    int k1 = (k + 1) % 3;
    double dx = X[2 * k1] - X[2 * k], dy = X[2 * k1 + 1] - X[2 * k + 1];
    per += sqrt(dx * dx + dy * dy);
  }
  double dd = 4.0 * tri_area(X) / per;
  double u = Q[1] / Q[0], v = Q[2] / Q[0];
  double lam = sqrt(u * u + v * v) + sqrt(g * pressure(Q, g) / Q[0]);
  return dd / lam;
}

// Step in ticks from tick `tick` of a macro step of N ticks of length delta.
// Dyadic levels: the largest power of two p <= N with p*delta <= dt_CFL,
// limited by the alignment of the current tick (a tick is 2^-30 of the macro
// step, far below the nominal finest step). Free steps: floor(dt_CFL / delta)
// ticks, at most the ticks left. At least one tick (overshoot flagged).
__device__ inline int level_step(double dtcfl, double delta, int N, int tick, int free_steps,
                                 int* over) {
  if (free_steps) {
    const int left = N - tick;
    const double q = dtcfl / delta;
    const int p = q >= double(left) ? left : int(floor(q));
    *over = p < 1;
    return p < 1 ? 1 : p;
  }
  int p = N;
  while (p > 1 && double(p) * delta > dtcfl) p >>= 1;
  *over = double(p) * delta > dtcfl;
  if (tick > 0) {
    int low = tick & (-tick);
    if (low < p) p = low;
  }
  return p;
}

// The step an element takes: the level rule's choice `own`, or under schedule
// replay the next recorded step of the element (counted when it differs from
// `own`; a missing or out-of-range entry raises ERR_REPLAY and keeps `own`).
// *over is set for the step taken.
__device__ inline void record_step(const Dev& d, int i, int p) {
  if (!d.rec_steps) return;
  const int k = d.rec_pos[i];
  if (k < d.rec_cap)
    d.rec_steps[size_t(i) * d.rec_cap + k] = p;
  else
    set_err(d, ERR_RECORD);
  d.rec_pos[i] = k + 1;
}

__device__ inline int take_step(const Dev& d, int i, int own, int tick, int N, double dtcfl, double delta,
                                int* over) {
  if (!d.replay_steps) {
    record_step(d, i, own);
    return own;
  }
  const int pos = d.replay_ptr[i] + d.replay_pos[i];
  if (pos >= d.replay_ptr[i + 1]) {
    set_err(d, ERR_REPLAY);
    return own;
  }
  d.replay_pos[i] += 1;
  const int p = d.replay_steps[pos];
  if (p < 1 || p > N - tick) {
    set_err(d, ERR_REPLAY);
    return own;
  }
  if (p != own) {
    atomicAdd(&d.scal->replay_overrides, 1ull);
    *over = double(p) * delta > dtcfl;
  }
  record_step(d, i, p);
  return p;
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.
// This renumbering gives every XCD a contiguous range of logical blocks, so
// that with Hilbert-ordered elements, nodes and edges the neighbours that a
// block gathers were mostly fetched into the same L2 by nearby blocks.
// Only the first nwork blocks (those with work) are renumbered, among
// themselves, so that a grid sized for all elements and running a shorter
// active list still spreads its work over every XCD.
constexpr int NXCD = 8;
__device__ inline int xcd_block(int nwork) {
  const int b = blockIdx.x;
  if (nwork > (int)gridDim.x) nwork = gridDim.x;
  if (b >= nwork) return b;
  const int x = b % NXCD, r = b / NXCD;
  const int q = nwork / NXCD, rem = nwork % NXCD;
  return x * q + (x < rem ? x : rem) + r;
}
__device__ inline int xcd_block() { return xcd_block(gridDim.x); }

// Orders LDS accesses among the lanes of one wavefront. The lanes that share a
// predictor's nodal data always lie in one wavefront, and the LDS executes the
// accesses of a wavefront in issue order, so only the compiler's reordering has
// to be fenced; no workgroup barrier is needed.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A double from another lane of the same row of 16 lanes, moved by a DPP
// pattern (no LDS round trip).
template <int CTRL>
__device__ inline double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, int(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// Sum over the 8 lanes of an aligned group, the same in every lane: pairs,
// then quads, then the two quads of the group; every step adds two equal
// partial sums, so all lanes end bit-identical and both forms give the same
// bits. The DPP form (lane moves inside the VALU, no LDS round trip) needs a
// few more registers, which at M=2 would take the reconstruction past 256
// VGPRs (one wave per SIMD instead of two): it is used where that does not
// matter.
template <bool DPP>
__device__ inline double group8_sum(double v) {
  if constexpr (DPP) {
    v += dpp_move<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_move<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_move<0x141>(v);   // row_half_mirror: lane i <-> 7 - i within 8
  } else {
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
  }
  return v;
}


// ---------------------------------------------------------------------------
// Reconstruction + local time step: 8 lanes per element
// ---------------------------------------------------------------------------
template <int M>
__global__ void __launch_bounds__(TPB) k_reconstruct(Dev d, const Tables* __restrict__ tb, Params P,
                                                     int use_list, int set_level) {
  using S = Sz<M>;
  constexpr int nb = S::nb, ne = S::ne, nu = S::nu, WS = S::WS;
  const int NE = d.NE;
  const int nitems = use_list ? d.scal->n_active : NE;
  const int sl = threadIdx.x & 7;
  const int ngroups = (gridDim.x * blockDim.x) >> 3;
  const int nwork = int((8L * nitems + blockDim.x - 1) / blockDim.x);
  for (int idx = (xcd_block(nwork) * blockDim.x + threadIdx.x) >> 3; idx < nitems; idx += ngroups) {
    const int i = use_list ? d.act_list[idx] : idx;
    const double delta = elem_delta(d, i);   // stencil elements share the instance
    const int nt = d.ts[i].tick;
    const double* ri = rec<M>(d, i);
    double Xi[6], Qi[4];
#pragma unroll
    for (int c = 0; c < 6; ++c) Xi[c] = ri[XE + c];
#pragma unroll
    for (int v = 0; v < 4; ++v) Qi[v] = ri[QO + v];
    const double e1x = Xi[2] - Xi[0], e1y = Xi[3] - Xi[1];
    const double e2x = Xi[4] - Xi[0], e2y = Xi[5] - Xi[1];
    const double idet = 1.0 / (e1x * e2y - e2x * e1y);
    double W[nu][4];
#pragma unroll
    for (int l = 0; l < nu; ++l)
#pragma unroll
      for (int v = 0; v < 4; ++v) W[l][v] = 0.0;
    double om = 0.0;
    bool ok = true;
    if (sl < NSTEN && d.sten[(sl * ne) * NE + i] >= 0) {
      double R[nu][nu], z[nu][4];
#pragma unroll
      for (int a = 0; a < nu; ++a) {
#pragma unroll
        for (int b = 0; b < nu; ++b) R[a][b] = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) z[a][v] = 0.0;
      }
      // Rows are software-pipelined: while row c is folded in, the neighbour
      // data of row c+1, the tick of row c+2 and the index of row c+3 are in
      // flight, each load depending only on values that arrived one row earlier.
      const int* sidx = d.sten + size_t(sl * ne) * NE + i;   // row c at sidx[c * NE]
      int jn = sidx[2 * NE], jnn = sidx[3 * NE];              // ne >= 6
      TickStep tc = d.ts[sidx[NE]], tn = d.ts[jn];
      NbrRaw<M> rc;
      fetch_nbr<M>(d, sidx[NE], tc, nt, rc);
#pragma unroll 1
      for (int c = 1; c < ne; ++c) {
        double Xv[6], Qv[4];
        ok &= place_nbr<M>(tb, rc, tc, nt, delta, Xv, Qv);
        if (c + 1 < ne) fetch_nbr<M>(d, jn, tn, nt, rc);
        tc = tn;
        if (c + 2 < ne) tn = d.ts[jnn];
        jn = jnn;
        if (c + 3 < ne) jnn = sidx[(c + 3) * NE];
        // vertices of the virtual element in the reference frame of element i
        double rx[3], ry[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          double dx = Xv[2 * k] - Xi[0], dy = Xv[2 * k + 1] - Xi[1];
          rx[k] = (dx * e2y - dy * e2x) * idet;
          ry[k] = (e1x * dy - e1y * dx) * idet;
        }
        // means of the monomials over the virtual element (rule exact to degree
        // M); the row is taken in the monomials shifted by their means on the
        // reference triangle, which span the same space as psi_1 .. psi_nu
        double mm[nb];
        monomial_means<M>(rx, ry, mm);
        double a[nu], b[4];
#pragma unroll
        for (int l = 0; l < nu; ++l) a[l] = mm[l + 1] - RefMeans<M>::m[l + 1];
#pragma unroll
        for (int v = 0; v < 4; ++v) b[v] = Qv[v] - Qi[v];
        // Givens rotations fold the row into the triangular factor
#pragma unroll
        for (int k = 0; k < nu; ++k) {
          const double rkk = R[k][k], ak = a[k];
          const double h2 = rkk * rkk + ak * ak;
          if (h2 == 0.0) continue;
          const double rh = rsqrt(h2);
          const double cs = rkk * rh, sn = ak * rh;
          R[k][k] = h2 * rh;
#pragma unroll
          for (int c2 = k + 1; c2 < nu; ++c2) {
            const double t = cs * R[k][c2] + sn * a[c2];
            a[c2] = cs * a[c2] - sn * R[k][c2];
            R[k][c2] = t;
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const double t = cs * z[k][v] + sn * b[v];
            b[v] = cs * b[v] - sn * z[k][v];
            z[k][v] = t;
          }
        }
      }
      double u[nu][4];
#pragma unroll
      for (int k = nu - 1; k >= 0; --k) {
        const double rinv = 1.0 / R[k][k];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double t = z[k][v];
#pragma unroll
          for (int c2 = k + 1; c2 < nu; ++c2) t -= R[k][c2] * u[c2][v];
          u[k][v] = t * rinv;
        }
      }
      // oscillation indicator (eq. eqn.sigma), summed over the variables;
      // it depends only on the polynomial, so it is taken in the shifted
      // monomials with their own (constant) indicator matrix
      double sigma = 0.0;
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int l = 0; l < nu; ++l) {
          double t = 0.0;
#pragma unroll
          for (int m = 0; m < nu; ++m) t += MonoBasis<M>::c.sig[l][m] * u[m][v];
          sigma += u[l][v] * t;
        }
      const double x = sigma + P.eps;
      const double x2 = x * x, x4 = x2 * x2, x8 = x4 * x4;
      om = (sl == 0 ? P.lambda : 1.0) / x8;
#pragma unroll
      for (int l = 0; l < nu; ++l)
#pragma unroll
        for (int v = 0; v < 4; ++v) W[l][v] = om * u[l][v];
    }
    double dt = 0.0;
    if (sl == 7) {
      // local CFL time step over the element and its face neighbours (eq. eqn.timestep)
      double rmin = cfl_ratio(Xi, Qi, P.gamma);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int j = d.neigh[k * NE + i];
        if (j < 0) continue;
        double Xv[6], Qv[4];
        ok &= project<M>(d, tb, j, nt, delta, Xv, Qv);
        rmin = fmin(rmin, cfl_ratio(Xv, Qv, P.gamma));
      }
      dt = P.cfl * rmin;
    }
    if (!ok) set_err(d, ERR_PRED);
    // nonlinear combination of eq. weno: sum over the stencil lanes
#pragma unroll
    for (int l = 0; l < nu; ++l)
#pragma unroll
      for (int v = 0; v < 4; ++v) W[l][v] = group8_sum<(M == 3)>(W[l][v]);
    const double iw = 1.0 / group8_sum<(M == 3)>(om);
    double* wo = d.wnod + size_t(i) * WS;
#pragma unroll
    for (int m = 0; m < nb; ++m)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (((m * 4 + v) & 7) != sl) continue;
        double t = Qi[v];
#pragma unroll
        for (int l = 0; l < nu; ++l) t += MonoBasis<M>::c.node[m][l] * (W[l][v] * iw);
        wo[m * 4 + v] = t;
      }
    if (sl == 7) {
      d.dtcfl[i] = dt;
      if (!(dt > 0.0 && dt < DBL_MAX)) set_err(d, ERR_DT);
      if (set_level) {
        const int N = d.scal->N;
        if (nt >= N) {
          d.ts[i].step = 0;
        } else {
          int over;
          const int own = level_step(dt, delta, N, nt, d.free_steps, &over);
          d.ts[i].step = take_step(d, i, own, nt, N, dt, delta, &over);
          if (over) atomicAdd(&d.scal->overshoots, 1ull);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Space-time Galerkin predictor: nb lanes per element, lane m = spatial node m;
// floor(64/nb) elements per wavefront (an element never straddles two), the
// remaining lanes of a wavefront are spare
// ---------------------------------------------------------------------------
template <int M>
__global__ void __launch_bounds__(TPB) k_predict(Dev d, const Tables* __restrict__ tb, Params P,
                                                 int use_list) {
  using S = Sz<M>;
  constexpr int nb = S::nb, T = S::nt, nG = S::nG, RS = S::RS, TS = S::TS, WS = S::WS;
  constexpr int G = nb, EPW = S::EPW, WPB = TPB / 64;
  constexpr int SLOTS = EPW * WPB;       // elements per block
  // exchanged fields per node: q(4), f1..f3, g1..g3 (f0 = q1 and g0 = q2 are
  // not repeated), x, y; the per-element stride is padded by 16 bytes so that
  // the broadcast reads of the elements of one wavefront fall in distinct banks
  constexpr int NF = 12;
  constexpr int LSTR = NF * G + 2;
  constexpr int NPT = 1 + 3 * nG;        // element mean + edge Gauss points
  constexpr int PPL = (NPT + G - 1) / G; // points per lane
  static_assert(TPB % 64 == 0, "whole wavefronts");
  __shared__ double lds[(SLOTS + WPB) * LSTR];   // one extra slot per wavefront for its spare lanes
  __shared__ double c0[16][TPB];         // per lane: fixed parts of slice t = 0
  const int NE = d.NE;
  const int nitems = use_list ? d.scal->n_live : NE;
  const double g = P.gamma;
  unsigned long long npred = 0;    // predictors evaluated (counted on node 0)
  const int wv = threadIdx.x / 64, lw = threadIdx.x % 64;
  const bool spare = lw >= EPW * G;
  const int slot = spare ? SLOTS + wv : wv * EPW + lw / G;
  const int m = spare ? lw - EPW * G : lw % G;   // < G either way
  double* const my = lds + slot * LSTR;
  const bool node = !spare;
  const int mm = m;
  // this lane's rows of the spatial derivative matrices
  double Dx[nb], De[nb];
#pragma unroll
  for (int k = 0; k < nb; ++k) {
    Dx[k] = tb->Dxi[mm][k];
    De[k] = tb->Deta[mm][k];
  }
  // lattice coordinates of node m (ordered by j then i)
  int jj = 0, ii = mm;
  while (ii > M - jj) {
    ii -= M + 1 - jj;
    ++jj;
  }
  const double nxi = double(ii) / M, neta = double(jj) / M;
  for (int base = xcd_block((nitems + SLOTS - 1) / SLOTS) * SLOTS; base < nitems;
       base += gridDim.x * SLOTS) {
    const int idx = base + slot;
    const int i = !spare && idx < nitems ? (use_list ? d.live_list[idx] : idx) : -1;
    const int st = i >= 0 ? d.ts[i].step : 0;
    const bool live = st > 0;           // uniform across the lanes of the element
    const bool act = live && node;
    if (live && m == 0) ++npred;
    const double dt = live ? double(st) * elem_delta(d, i) : 1.0;
    const double idt = 1.0 / dt;
    double q[T][4], x[T][2];
    if (act) {
      const double* r = rec<M>(d, i);
      const double px = r[XE + 0] + (r[XE + 2] - r[XE + 0]) * nxi + (r[XE + 4] - r[XE + 0]) * neta;
      const double py = r[XE + 1] + (r[XE + 3] - r[XE + 1]) * nxi + (r[XE + 5] - r[XE + 1]) * neta;
      const double* w = d.wnod + size_t(i) * WS + m * 4;
#pragma unroll
      for (int t = 0; t < T; ++t) {
        x[t][0] = px;
        x[t][1] = py;
#pragma unroll
        for (int v = 0; v < 4; ++v) q[t][v] = w[v];
      }
    } else {
      // idle lanes carry a harmless state through the exchange
#pragma unroll
      for (int t = 0; t < T; ++t) {
        x[t][0] = x[t][1] = 0.0;
        q[t][0] = 1.0;
        q[t][1] = q[t][2] = 0.0;
        q[t][3] = 1.0;
      }
    }
    // this node's fields of slice t into the element's exchange buffer
    auto put_fields = [&](int t) {
      const double ir = 1.0 / q[t][0];
      const double u = q[t][1] * ir, v = q[t][2] * ir;
      const double p = (g - 1.0) * (q[t][3] - 0.5 * (q[t][1] * u + q[t][2] * v));
      const double h = q[t][3] + p;
      my[0 * G + m] = q[t][0];
      my[1 * G + m] = q[t][1];
      my[2 * G + m] = q[t][2];
      my[3 * G + m] = q[t][3];
      my[4 * G + m] = q[t][1] * u + p;
      my[5 * G + m] = q[t][1] * v;
      my[6 * G + m] = u * h;
      my[7 * G + m] = q[t][2] * u;
      my[8 * G + m] = q[t][2] * v + p;
      my[9 * G + m] = v * h;
      my[10 * G + m] = x[t][0];
      my[11 * G + m] = x[t][1];
    };
    // spatial metric of the isoparametric map at this node (eq. Jac) from the
    // exchanged coordinates: xi_x, xi_y, eta_x, eta_y
    auto spatial_metric = [&](double mt[4]) {
      double xx = 0.0, xe = 0.0, yx = 0.0, ye = 0.0;
#pragma unroll
      for (int k = 0; k < nb; ++k) {
        const double vx = my[10 * G + k], vy = my[11 * G + k];
        xx += Dx[k] * vx;
        xe += De[k] * vx;
        yx += Dx[k] * vy;
        ye += De[k] * vy;
      }
      const double idet = 1.0 / (xx * ye - xe * yx);
      mt[0] = ye * idet;
      mt[1] = -xe * idet;
      mt[2] = -yx * idet;
      mt[3] = xx * idet;
    };
    // xi_t, eta_t at this node and slice t from its own trajectory
    auto time_metric = [&](int t, const double mt[4], double& xi_t, double& eta_t) {
      double xtau = 0.0, ytau = 0.0;
#pragma unroll
      for (int r = 0; r < T; ++r) {
        xtau += tb->Dt[t][r] * x[r][0];
        ytau += tb->Dt[t][r] * x[r][1];
      }
      const double xt = xtau * idt, yt = ytau * idt;
      xi_t = -(mt[0] * xt + mt[1] * yt);
      eta_t = -(mt[2] * xt + mt[3] * yt);
    };
    // d/dxi (a) and d/deta (b) at this node of the exchanged fields 0..9
    auto field_derivs = [&](double da[10], double db[10]) {
#pragma unroll
      for (int f = 0; f < 10; ++f) {
        double sa = 0.0, sb = 0.0;
#pragma unroll
        for (int k = 0; k < nb; ++k) {
          const double val = my[f * G + k];
          sa += Dx[k] * val;
          sb += De[k] * val;
        }
        da[f] = sa;
        db[f] = sb;
      }
    };
    // spatial flux part of P: f_xi xi_x + f_eta eta_x + g_xi xi_y + g_eta eta_y
    // (f0 = q1 and g0 = q2 are fields 1 and 2; f1..f3 are 4..6, g1..g3 7..9)
    auto spatial_part = [&](const double da[10], const double db[10], const double mt[4],
                            double sp[4]) {
      sp[0] = da[1] * mt[0] + db[1] * mt[2] + da[2] * mt[1] + db[2] * mt[3];
#pragma unroll
      for (int v = 1; v < 4; ++v)
        sp[v] = da[3 + v] * mt[0] + db[3 + v] * mt[2] + da[6 + v] * mt[1] + db[6 + v] * mt[3];
    };
    // P = -(q_xi xi_t + q_eta eta_t + spatial part), accumulated into the sweep
    auto accumulate = [&](int t, const double da[4], const double db[4], const double sp[4],
                          double xi_t, double eta_t, double qn[M][4]) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double Pv = -(da[v] * xi_t + db[v] * eta_t + sp[v]);
#pragma unroll
        for (int r = 0; r < M; ++r) qn[r][v] += dt * tb->At[r][t] * Pv;
      }
    };
    // The slice t = 0 (q_0, x_0) is the same in every sweep, and in the first
    // sweep every slice carries q_0. So the spatial derivatives of the fields
    // at t = 0 are taken once, in the first sweep, and serve all of its slices;
    // later sweeps keep from them the derivatives of q, the spatial flux part
    // and the spatial metric at t = 0 (per lane, in LDS), and exchange only
    // their slices t >= 1.
    for (int it = 0; it < P.npic; ++it) {
      // mesh ODE at this node: x_{1:} = Bt x_0 + dt At V
      if (P.lagrangian) {
        double V[T][2];
#pragma unroll
        for (int t = 0; t < T; ++t) {
          const double ir = 1.0 / q[t][0];
          V[t][0] = q[t][1] * ir;
          V[t][1] = q[t][2] * ir;
        }
#pragma unroll
        for (int r = 0; r < M; ++r)
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            double s = 0.0;
#pragma unroll
            for (int t = 0; t < T; ++t) s += tb->At[r][t] * V[t][c];
            x[r + 1][c] = tb->Bt[r] * x[0][c] + dt * s;
          }
      }
      double qn[M][4];
#pragma unroll
      for (int r = 0; r < M; ++r)
#pragma unroll
        for (int v = 0; v < 4; ++v) qn[r][v] = tb->Bt[r] * q[0][v];
      if (it == 0) {
        put_fields(0);
        wave_sync();
        double da[10], db[10], mt0[4], sp0[4];
        field_derivs(da, db);
        spatial_metric(mt0);
        wave_sync();
        spatial_part(da, db, mt0, sp0);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          c0[v][threadIdx.x] = da[v];
          c0[4 + v][threadIdx.x] = db[v];
          c0[8 + v][threadIdx.x] = sp0[v];
          c0[12 + v][threadIdx.x] = mt0[v];
        }
#pragma unroll
        for (int t = 0; t < T; ++t) {
          double mt[4], sp[4], xi_t, eta_t;
          if (t == 0) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              mt[c] = mt0[c];
              sp[c] = sp0[c];
            }
          } else {
            my[10 * G + m] = x[t][0];
            my[11 * G + m] = x[t][1];
            wave_sync();
            spatial_metric(mt);
            wave_sync();
            spatial_part(da, db, mt, sp);
          }
          time_metric(t, mt, xi_t, eta_t);
          accumulate(t, da, db, sp, xi_t, eta_t, qn);
        }
      } else {
        {
          double da[4], db[4], sp[4], mt[4], xi_t, eta_t;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            da[v] = c0[v][threadIdx.x];
            db[v] = c0[4 + v][threadIdx.x];
            sp[v] = c0[8 + v][threadIdx.x];
            mt[v] = c0[12 + v][threadIdx.x];
          }
          time_metric(0, mt, xi_t, eta_t);
          accumulate(0, da, db, sp, xi_t, eta_t, qn);
        }
#pragma unroll
        for (int t = 1; t < T; ++t) {
          put_fields(t);
          wave_sync();
          double da[10], db[10], mt[4], sp[4], xi_t, eta_t;
          field_derivs(da, db);
          spatial_metric(mt);
          wave_sync();
          spatial_part(da, db, mt, sp);
          time_metric(t, mt, xi_t, eta_t);
          accumulate(t, da, db, sp, xi_t, eta_t, qn);
        }
      }
#pragma unroll
      for (int r = 0; r < M; ++r)
#pragma unroll
        for (int v = 0; v < 4; ++v) q[r + 1][v] = qn[r][v];
    }
    // publish: reference means and edge traces, one time slice at a time
    // through LDS; lane m evaluates points m, m + G, ... (point 0 is the
    // element mean, point 1 + e*nG + gq the Gauss point gq of edge e), all four
    // variables each
    double cw[PPL][nb];
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
      const int pt = m + G * j;
      const int eg = pt > 0 ? pt - 1 : 0;
      const double* c = pt == 0 ? tb->amean : tb->edge[eg / nG][eg % nG];
#pragma unroll
      for (int k = 0; k < nb; ++k) cw[j][k] = pt < NPT ? c[k] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < T; ++t) {
#pragma unroll
      for (int c = 0; c < 4; ++c) my[c * G + m] = q[t][c];
      wave_sync();
      if (live) {
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
          const int pt = m + G * j;
          if (pt >= NPT) continue;
          double* out = pt == 0 ? d.rec + size_t(i) * RS + AVG + t * 4
                                : d.trace + size_t(i) * TS + ((pt - 1) * T + t) * 4;
          double s4[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < nb; ++k) s += cw[j][k] * my[v * G + k];
            s4[v] = s;
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) out[v] = s4[v];
        }
      }
      wave_sync();
    }
    if (act) {
      double* rw = d.rec + size_t(i) * RS;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        if (tb->vtx[k] != m) continue;
#pragma unroll
        for (int t = 0; t < T; ++t) {
          double vx = 0.0, vy = 0.0;
          if (P.lagrangian) {
            const double ir = 1.0 / q[t][0];
            vx = q[t][1] * ir;
            vy = q[t][2] * ir;
          }
          rw[S::VV + (k * T + t) * 2 + 0] = vx;
          rw[S::VV + (k * T + t) * 2 + 1] = vy;
        }
      }
    }
  }
  block_add(&d.scal->n_pred, npred);
}

// ---------------------------------------------------------------------------
// Scheduling
// ---------------------------------------------------------------------------
__global__ void k_cycle_begin(Dev d) {
  d.scal->n_active = 0;
  d.scal->n_live = 0;
  d.scal->n_unfinished = 0;
  d.scal->cycle += 1;
}

// Each block owns a contiguous chunk of at most SCHED_CHUNK elements; 8 lanes
// per element share the scan of its scheduling stencil; the block gathers its
// active elements in LDS and reserves list space with one global atomic. A
// second list keeps the active elements that stay short of tick N: only they
// need a predictor after their update (an element reaching tick N gets its
// next one at the macro-step start, and no stage reads it before).
constexpr int SCHED_CHUNK = 1024;

constexpr int SCHED_TPB = 1024;   // 16 wavefronts: a chunk of 1024 elements in 8 passes
__global__ void __launch_bounds__(SCHED_TPB) k_sched(Dev d, int chunk) {
  const int cycle = d.scal->cycle;
  constexpr int PER_PASS = SCHED_TPB / 8;
  __shared__ int local[SCHED_CHUNK], local_live[SCHED_CHUNK];
  __shared__ int count, gbase, count_live, gbase_live;
  const int NE = d.NE;
  const int N = d.scal->N;
  const int sub = threadIdx.x & 7;
  if (threadIdx.x == 0) {
    count = 0;
    count_live = 0;
  }
  __syncthreads();
  const int begin = xcd_block() * chunk;
  const int end = min(NE, begin + chunk);
  // The element's own tick and the bounds of its stencil are loaded one pass
  // ahead, and a lane's first SCAN_U stencil entries (of ~80 at M=2) are
  // gathered together, so that a pass waits on two dependent loads (stencil
  // index, then tick) instead of one such pair per 32 entries.
  constexpr int SCAN_U = 12;
  auto head = [&](int i, TickStep& me, int& r0, int& r1) {
    me = i < end ? d.ts[i] : TickStep{N, 0};
    r0 = r1 = 0;
    if (me.tick < N) {
      r0 = d.sched_ptr[i];
      r1 = d.sched_ptr[i + 1];
    }
  };
  TickStep me_n;
  int r0_n, r1_n;
  head(begin + (threadIdx.x >> 3), me_n, r0_n, r1_n);
  for (int base = begin; base < end; base += PER_PASS) {
    const int i = base + (threadIdx.x >> 3);
    const TickStep me = me_n;
    const int r0 = r0_n, r1 = r1_n;
    if (base + PER_PASS < end) head(base + PER_PASS + (threadIdx.x >> 3), me_n, r0_n, r1_n);
    int fut = 0, mx = 0, mn = FREE_TICKS;   // no tick count exceeds FREE_TICKS
    bool unf = false;
    if (i < end && me.tick < N) {
      unf = true;
      fut = me.tick + me.step;
      int jx[SCAN_U];
#pragma unroll
      for (int u = 0; u < SCAN_U; ++u) {
        const int r = r0 + sub + 8 * u;
        jx[u] = r < r1 ? d.sched_idx[r] : -1;
      }
      TickStep o[SCAN_U];
#pragma unroll
      for (int u = 0; u < SCAN_U; ++u) o[u] = jx[u] >= 0 ? d.ts[jx[u]] : TickStep{0, FREE_TICKS};
#pragma unroll
      for (int u = 0; u < SCAN_U; ++u) {
        mx = max(mx, o[u].tick);
        mn = min(mn, o[u].tick + o[u].step);
      }
      // longer stencils: the rest four entries per lane at a time
      for (int r = r0 + 8 * SCAN_U + sub; r < r1; r += 32) {
        int jy[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) jy[u] = r + 8 * u < r1 ? d.sched_idx[r + 8 * u] : -1;
        TickStep o4[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) o4[u] = jy[u] >= 0 ? d.ts[jy[u]] : TickStep{0, FREE_TICKS};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          mx = max(mx, o4[u].tick);
          mn = min(mn, o4[u].tick + o4[u].step);
        }
      }
    }
#pragma unroll
    for (int s = 1; s < 8; s <<= 1) {
      mx = max(mx, __shfl_xor(mx, s));
      mn = min(mn, __shfl_xor(mn, s));
    }
    // append to both block lists with one LDS atomic per wavefront and list
    const bool isact = unf && sub == 0 && mx <= fut && fut <= mn;
    const bool islive = isact && fut < N;
    const unsigned long long ba = __ballot(isact), bl = __ballot(islive);
    const int lane = __lane_id();
    int pa = 0, pl = 0;
    if (lane == 0) {
      pa = ba ? atomicAdd(&count, __popcll(ba)) : 0;
      pl = bl ? atomicAdd(&count_live, __popcll(bl)) : 0;
    }
    pa = __shfl(pa, 0);
    pl = __shfl(pl, 0);
    const unsigned long long below = (1ull << lane) - 1ull;
    if (isact) {
      local[pa + __popcll(ba & below)] = i;
      d.act_stamp[i] = cycle;
    }
    if (islive) local_live[pl + __popcll(bl & below)] = i;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    gbase = gbase_live = 0;
    if (count) {
      const unsigned long long both = (unsigned long long)count | ((unsigned long long)count_live << 32);
      const unsigned long long old =
          atomicAdd(reinterpret_cast<unsigned long long*>(&d.scal->n_active), both);
      gbase = int(old & 0xffffffffull);
      gbase_live = int(old >> 32);
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < count; k += SCHED_TPB) d.act_list[gbase + k] = local[k];
  for (int k = threadIdx.x; k < count_live; k += SCHED_TPB) d.live_list[gbase_live + k] = local_live[k];
}

// ---------------------------------------------------------------------------
// Node solver and node motion
// ---------------------------------------------------------------------------
template <int M>
__global__ void __launch_bounds__(TPB) k_node(Dev d, const Tables* __restrict__ tb, Params P) {
  const int cycle = d.scal->cycle;
  constexpr int T = M + 1, VV = Sz<M>::VV;
  const int NV = d.NV;
  unsigned long long nmoved = 0;   // nodes moved by this lane
  if (blockIdx.x == 0 && threadIdx.x == 0) d.scal->updates += (unsigned long long)d.scal->n_active;
  for (int k = xcd_block() * blockDim.x + threadIdx.x; k < NV; k += gridDim.x * blockDim.x) {
    const int r0 = d.ring_ptr[k], r1 = d.ring_ptr[k + 1];
    int newt = -1;
    for (int r = r0; r < r1; ++r) {
      const int j = d.ring_ent[r] >> 2;
      if (d.act_stamp[j] == cycle) {
        const TickStep tsj = d.ts[j];
        newt = tsj.tick + tsj.step;
        break;
      }
    }
    const int nk = d.ntick[k];
    if (newt <= nk) continue;
    double mu_sum = 0.0, Vx = 0.0, Vy = 0.0;
    bool ok = true;
    for (int r = r0; r < r1; ++r) {
      const int ent = d.ring_ent[r];
      const int j = ent >> 2, lv = ent & 3;
      const TickStep tsj = d.ts[j];
      if (tsj.step <= 0) {
        ok = false;
        continue;
      }
      const double tau0 = tick_ratio(double(nk - tsj.tick), tsj.step);
      const double tau1 = tick_ratio(double(newt - tsj.tick), tsj.step);
      double L0[T], L1[T];
      time_antideriv<M>(tau0, L0);
      time_antideriv<M>(tau1, L1);
      const double* rj = rec<M>(d, j);
      double vx = 0.0, vy = 0.0;
#pragma unroll
      for (int q = 0; q < T; ++q) {
        const double I = L1[q] - L0[q];
        vx += I * rj[VV + (lv * T + q) * 2 + 0];
        vy += I * rj[VV + (lv * T + q) * 2 + 1];
      }
      const double inv = 1.0 / (tau1 - tau0);
      const double mu = rj[QO] * rj[AO];
      Vx += mu * (vx * inv);
      Vy += mu * (vy * inv);
      mu_sum += mu;
    }
    if (!ok) set_err(d, ERR_PRED);
    Vx /= mu_sum;
    Vy /= mu_sum;
    if (d.wall_pin[k]) {
      Vx = 0.0;
      Vy = 0.0;
    } else {
      const double nx = d.wall_n[k], ny = d.wall_n[NV + k];
      const double vn = Vx * nx + Vy * ny;
      Vx -= vn * nx;
      Vy -= vn * ny;
    }
    const double dtk = double(newt - nk) * node_delta(d, k);
    d.Xnew[k] = d.X[k] + dtk * Vx;
    d.Xnew[NV + k] = d.X[NV + k] + dtk * Vy;
    d.ntick_new[k] = newt;
    d.node_stamp[k] = cycle;
    ++nmoved;
  }
  block_add(&d.scal->n_node, nmoved);
}

// ---------------------------------------------------------------------------
// Space-time patch fluxes: one lane per edge; an edge with a moved node
// sweeps a patch, whose flux and normal integral go to the memory-variable
// slots of the edge in its two elements (each slot has one writer per cycle:
// its edge)
// ---------------------------------------------------------------------------
template <int M>
__global__ void __launch_bounds__(TPB) k_patch(Dev d, const Tables* __restrict__ tb, Params P) {
  const int cycle = d.scal->cycle;
  constexpr int T = M + 1, nG = M + 1, TS = Sz<M>::TS;
  const int NV = d.NV, NF = d.NF;
  const double g = P.gamma;
  unsigned long long npatch = 0;   // patches integrated by this lane
  for (int e = xcd_block() * blockDim.x + threadIdx.x; e < NF; e += gridDim.x * blockDim.x) {
    const int a = d.e_a[e], b = d.e_b[e];
    const bool ma = d.node_stamp[a] == cycle, mb = d.node_stamp[b] == cycle;
    if (!ma && !mb) continue;
    const double delta = node_delta(d, a);
    double P1[3], P2[3], P3[3], P4[3];
    const double n1 = d.ntick[a], n2 = d.ntick[b];
    const double n3 = mb ? d.ntick_new[b] : n2, n4 = ma ? d.ntick_new[a] : n1;
    P1[0] = d.X[a];
    P1[1] = d.X[NV + a];
    P1[2] = n1 * delta;
    P2[0] = d.X[b];
    P2[1] = d.X[NV + b];
    P2[2] = n2 * delta;
    P3[0] = mb ? d.Xnew[b] : P2[0];
    P3[1] = mb ? d.Xnew[NV + b] : P2[1];
    P3[2] = n3 * delta;
    P4[0] = ma ? d.Xnew[a] : P1[0];
    P4[1] = ma ? d.Xnew[NV + a] : P1[1];
    P4[2] = n4 * delta;
    const int L = d.e_L[e], el = d.e_el[e], R = d.e_R[e], er = d.e_er[e], bc = d.e_bc[e];
    const TickStep tL = d.ts[L];
    TickStep tR{0, 1};
    if (R >= 0) tR = d.ts[R];
    if (tL.step <= 0 || tR.step <= 0) {
      set_err(d, ERR_PRED);
      continue;
    }
    const double* trL = d.trace + size_t(L) * TS + el * nG * T * 4;
    const double* trR = R >= 0 ? d.trace + size_t(R) * TS + er * nG * T * 4 : trL;
    // the two memory-variable slots this edge adds to, read now so that the
    // loads overlap the flux integration
    double* sl = d.mem + (size_t(L) * 3 + el) * MEM_W;
    double* sr = d.mem + (size_t(R >= 0 ? R : L) * 3 + (R >= 0 ? er : el)) * MEM_W;
    double mL[7], mR[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) mL[c] = sl[c];
    if (R >= 0) {
#pragma unroll
      for (int c = 0; c < 7; ++c) mR[c] = sr[c];
    }
    double G[4] = {0, 0, 0, 0}, Nn[3] = {0, 0, 0};
#pragma unroll 1
    for (int gq = 0; gq < nG; ++gq) {
      double qL[T][4], qR[T][4];
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          qL[t][v] = trL[(gq * T + t) * 4 + v];
          qR[t][v] = trR[((nG - 1 - gq) * T + t) * 4 + v];
        }
      const double c = tb->gchi[gq];
#pragma unroll 1
      for (int h = 0; h < nG; ++h) {
        const double tt = tb->gchi[h];
        const double w = tb->gw[gq] * tb->gw[h];
        double dchi[3], dtau[3], N[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          dchi[k] = (1.0 - tt) * (P2[k] - P1[k]) + tt * (P3[k] - P4[k]);
          dtau[k] = (1.0 - c) * (P4[k] - P1[k]) + c * (P3[k] - P2[k]);
        }
        N[0] = dchi[1] * dtau[2] - dchi[2] * dtau[1];
        N[1] = dchi[2] * dtau[0] - dchi[0] * dtau[2];
        N[2] = dchi[0] * dtau[1] - dchi[1] * dtau[0];
        const double tk = (1.0 - c) * (1.0 - tt) * n1 + c * (1.0 - tt) * n2 + c * tt * n3 + (1.0 - c) * tt * n4;
        double lL[T];
        time_basis<M>(tick_ratio(tk - tL.tick, tL.step), lL);
        double ql[4], qr[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double s = 0.0;
#pragma unroll
          for (int t = 0; t < T; ++t) s += lL[t] * qL[t][v];
          ql[v] = s;
        }
        if (R >= 0) {
          double lR[T];
          time_basis<M>(tick_ratio(tk - tR.tick, tR.step), lR);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            double s = 0.0;
#pragma unroll
            for (int t = 0; t < T; ++t) s += lR[t] * qR[t][v];
            qr[v] = s;
          }
        } else if (bc == 2) {
          // slip wall: mirror the normal momentum
          const double inxy = rsqrt(N[0] * N[0] + N[1] * N[1]);
          const double nx = N[0] * inxy, ny = N[1] * inxy;
          const double mn = ql[1] * nx + ql[2] * ny;
          qr[0] = ql[0];
          qr[1] = ql[1] - 2.0 * mn * nx;
          qr[2] = ql[2] - 2.0 * mn * ny;
          qr[3] = ql[3];
        } else {
          // transmissive: the inner element's predicted cell mean at this
          // time (a ghost copy of the element; the inner trace as outer state
          // leaves the face without dissipation and lets boundary modes grow)
          const double* rl = rec<M>(d, L);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            double s = 0.0;
#pragma unroll
            for (int t = 0; t < T; ++t) s += lL[t] * rl[AVG + t * 4 + v];
            qr[v] = s;
          }
        }
        double fn[4];
        numerical_flux(P.flux, tb, ql, qr, N, g, fn);
#pragma unroll
        for (int v = 0; v < 4; ++v) G[v] += w * fn[v];
#pragma unroll
        for (int k = 0; k < 3; ++k) Nn[k] += w * N[k];
      }
    }
    // inflow-positive memory variables: the flux leaves L and enters R
#pragma unroll
    for (int v = 0; v < 4; ++v) sl[v] = mL[v] - G[v];
#pragma unroll
    for (int k = 0; k < 3; ++k) sl[4 + k] = mL[4 + k] - Nn[k];
    if (R >= 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) sr[v] = mR[v] + G[v];
#pragma unroll
      for (int k = 0; k < 3; ++k) sr[4 + k] = mR[4 + k] + Nn[k];
    }
    ++npatch;
  }
  block_add(&d.scal->n_patch, npatch);
}

// ---------------------------------------------------------------------------
// Memory variables and conservative update
// ---------------------------------------------------------------------------
template <int M>
__global__ void __launch_bounds__(TPB) k_update(Dev d, Params P) {
  const int cycle = d.scal->cycle;
  const int NE = d.NE, NV = d.NV;
  const int na = d.scal->n_active;
  const int nwork = (na + TPB - 1) / TPB;
  double gmax = 0.0;   // largest relative GCL residual seen by this lane
  for (int idx = xcd_block(nwork) * blockDim.x + threadIdx.x; idx < na; idx += gridDim.x * blockDim.x) {
    const int i = d.act_list[idx];
    // memory variables: the three edge slots, consumed and cleared
    double* ms = d.mem + size_t(i) * 3 * MEM_W;
    double qm[4], hm[3];
#pragma unroll
    for (int v = 0; v < 4; ++v) qm[v] = (ms[v] + ms[MEM_W + v]) + ms[2 * MEM_W + v];
#pragma unroll
    for (int c = 0; c < 3; ++c) hm[c] = (ms[4 + c] + ms[MEM_W + 4 + c]) + ms[2 * MEM_W + 4 + c];
#pragma unroll
    for (int c = 0; c < 3 * MEM_W; ++c) ms[c] = 0.0;
    double X[6];
    int nd[3];
    bool mv[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      nd[k] = d.tri[k * NE + i];
      mv[k] = d.node_stamp[nd[k]] == cycle;
      X[2 * k] = mv[k] ? d.Xnew[nd[k]] : d.X[nd[k]];
      X[2 * k + 1] = mv[k] ? d.Xnew[NV + nd[k]] : d.X[NV + nd[k]];
    }
    double* r = d.rec + size_t(i) * Sz<M>::RS;
    const double An = tri_area(X);
    const double A0 = r[AO];
    if (!(An > 0.0)) set_err(d, ERR_GEOM);
    const double res = fmax(fmax(fabs(hm[0]), fabs(hm[1])), fabs(hm[2] - (An - A0)));
    const double rel = res / (A0 + An);
    gmax = fmax(gmax, rel);
    if (!(rel <= P.gcl_tol)) set_err(d, ERR_GCL);
    double qn[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) qn[v] = (A0 * r[QO + v] + qm[v]) / An;
    const double pn = pressure(qn, P.gamma);
    if (!(qn[0] > 0.0) || !(pn > 0.0)) set_err(d, ERR_STATE);
#pragma unroll
    for (int v = 0; v < 4; ++v) r[QO + v] = qn[v];
#pragma unroll
    for (int c = 0; c < 6; ++c) r[XE + c] = X[c];
    r[AO] = An;
    TickStep me = d.ts[i];
    me.tick += me.step;
    d.ts[i] = me;
    // commit the moved nodes (every writer stores the same value)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (mv[k]) {
        d.X[nd[k]] = X[2 * k];
        d.X[NV + nd[k]] = X[2 * k + 1];
        d.ntick[nd[k]] = d.ntick_new[nd[k]];
      }
  }
  block_max_pos(&d.scal->max_gcl_bits, gmax);
}

// ---------------------------------------------------------------------------
// Macro-step boundary
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(TPB) k_reset_min(Dev d) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < d.K; k += gridDim.x * blockDim.x)
    d.inst[k].min_dt_bits = ~0ull;
}

// Smallest CFL step per instance. Instances own contiguous element ranges, so
// a wavefront's 64 consecutive elements belong to one instance except at range
// ends: their minimum then, else each lane's, goes to the instance. A
// workgroup takes MIN_U such rows per wavefront and merges its wavefronts'
// minima first, so a single instance takes one atomic per workgroup (atomics
// on one address serialise).
constexpr int MIN_U = 4;
__global__ void __launch_bounds__(TPB) k_min_dt(Dev d) {
  constexpr int WPB = TPB / 64;
  __shared__ int wk[WPB];
  __shared__ double wm[WPB];
  const int NE = d.NE, lane = __lane_id(), wv = threadIdx.x / 64;
  for (int base = blockIdx.x * blockDim.x * MIN_U; base < NE; base += gridDim.x * blockDim.x * MIN_U) {
    int ku[MIN_U];
    double mu[MIN_U];
#pragma unroll
    for (int u = 0; u < MIN_U; ++u) {
      const int i = base + (u * WPB + wv) * 64 + lane;
      ku[u] = i < NE ? d.e_inst[i] : -1;
      // a lane without a finite positive step takes no part (and raised ERR_DT)
      const double m = i < NE ? d.dtcfl[i] : DBL_MAX;
      mu[u] = m > 0.0 && m < DBL_MAX ? m : DBL_MAX;
    }
    int kw = -1;          // the wavefront's instance and minimum over its uniform rows
    double mw = DBL_MAX;
#pragma unroll
    for (int u = 0; u < MIN_U; ++u) {
      const int k0 = __shfl(ku[u], 0), klast = __shfl(ku[u], 63);
      double m = mu[u];
      if (k0 == klast) {
#pragma unroll
        for (int s = 1; s < 64; s <<= 1) m = fmin(m, __shfl_xor(m, s));
        if (k0 < 0) continue;
        if (k0 != kw) {
          if (lane == 0 && kw >= 0 && mw < DBL_MAX)
            atomicMin(&d.inst[kw].min_dt_bits, (unsigned long long)__double_as_longlong(mw));
          kw = k0;
          mw = m;
        } else {
          mw = fmin(mw, m);
        }
      } else if (ku[u] >= 0 && m < DBL_MAX) {
        atomicMin(&d.inst[ku[u]].min_dt_bits, (unsigned long long)__double_as_longlong(m));
      }
    }
    if (lane == 0) {
      wk[wv] = kw;
      wm[wv] = mw;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int kc = -1;
      double mc = DBL_MAX;
      for (int w = 0; w < WPB; ++w) {
        if (wk[w] < 0) continue;
        if (wk[w] != kc) {
          if (kc >= 0 && mc < DBL_MAX)
            atomicMin(&d.inst[kc].min_dt_bits, (unsigned long long)__double_as_longlong(mc));
          kc = wk[w];
          mc = wm[w];
        } else {
          mc = fmin(mc, wm[w]);
        }
      }
      if (kc >= 0 && mc < DBL_MAX)
        atomicMin(&d.inst[kc].min_dt_bits, (unsigned long long)__double_as_longlong(mc));
    }
    __syncthreads();
  }
}

// Tick length of the macro step per open instance: for dyadic levels the
// smallest CFL step times the step fraction, times dscale = 2^(L-1) / N (a
// power of two), clamped so that N ticks do not pass the target time; for free
// steps the interval to the target over N; 0 for closed ones. An instance that
// had no finite positive CFL step (k_min_dt left its minimum unset) raises
// ERR_DT.
__global__ void __launch_bounds__(TPB) k_macro_setup(Dev d, int N, double fraction, double dscale) {
  const double t_end = d.scal->t_end;
  if (blockIdx.x == 0 && threadIdx.x == 0) d.scal->N = N;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < d.K; k += gridDim.x * blockDim.x) {
    Inst* in = d.inst + k;
    if (!in->open) {
      in->delta = 0.0;
      continue;
    }
    const double rest = (t_end - in->T) / double(N);
    if (d.free_steps) {
      in->delta = rest;
    } else if (in->min_dt_bits == ~0ull) {
      in->delta = 0.0;
    } else {
      in->delta = fmin((__longlong_as_double((long long)in->min_dt_bits) * fraction) * dscale, rest);
    }
    const int m = d.scal->macro_index;
    if (d.replay_delta) {
      if (m < d.replay_delta_n)
        in->delta = fmin(d.replay_delta[m], rest);
      else
        set_err(d, ERR_REPLAY);
    }
    if (d.rec_delta) {
      if (m < d.rec_delta_cap)
        d.rec_delta[m] = in->delta;
      else
        set_err(d, ERR_RECORD);
    }
    if (!(in->delta > 0.0)) set_err(d, ERR_DT);
  }
}

// Levels at the macro-step start; elements of closed instances sit at tick N
// with no step, i.e. finished.
__global__ void __launch_bounds__(TPB) k_levels(Dev d) {
  const int N = d.scal->N;
  const int n = max(d.NE, d.NV);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    if (i < d.NE) {
      const double delta = d.inst[d.e_inst[i]].delta;
      TickStep me;
      if (delta > 0.0) {
        int over;
        me.tick = 0;
        const int own = level_step(d.dtcfl[i], delta, N, 0, d.free_steps, &over);
        me.step = take_step(d, i, own, 0, N, d.dtcfl[i], delta, &over);
        if (over) atomicAdd(&d.scal->overshoots, 1ull);
      } else {
        me.tick = N;
        me.step = 0;
      }
      d.ts[i] = me;
    }
    if (i < d.NV) d.ntick[i] = 0;
  }
}

// Ends the macro step: each instance's time advanced, ticks reset. With
// only_if_done, it does nothing unless every element has reached the end of
// the macro step (the host then runs further cycles and ends the step itself).
__global__ void __launch_bounds__(TPB) k_macro_end(Dev d, int only_if_done) {
  if (only_if_done && d.scal->n_unfinished != 0) return;
  const int N = d.scal->N;
  if (blockIdx.x == 0 && threadIdx.x == 0) d.scal->macro_index += 1;
  const int n = max(max(d.NE, d.NV), d.K);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    if (i < d.K) {
      Inst* in = d.inst + i;
      in->T = in->T + double(N) * in->delta;
    }
    if (i < d.NE) d.ts[i].tick = 0;
    if (i < d.NV) d.ntick[i] = 0;
  }
}

__global__ void k_set_target(Dev d, double t_end) { d.scal->t_end = t_end; }

// Which instances are short of the target time (the same test the host applies
// to a single time), and how many.
__global__ void __launch_bounds__(TPB) k_open(Dev d) {
  const double t_end = d.scal->t_end;
  const double tol = 1e-12 * fmax(1.0, fabs(t_end));
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < d.K; k += gridDim.x * blockDim.x)
    d.inst[k].open = !(t_end - d.inst[k].T <= tol);
}

__global__ void __launch_bounds__(TPB) k_count_open(Dev d) {
  __shared__ int part[TPB / 64];
  int c = 0;
  for (int k = threadIdx.x; k < d.K; k += blockDim.x) c += d.inst[k].open;
#pragma unroll
  for (int s = 1; s < 64; s <<= 1) c += __shfl_xor(c, s);
  if (__lane_id() == 0) part[threadIdx.x / 64] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < TPB / 64; ++w) t += part[w];
    d.scal->n_open = t;
  }
}

__global__ void k_count_reset(Dev d) { d.scal->n_unfinished = 0; }

__global__ void __launch_bounds__(TPB) k_count(Dev d) {
  __shared__ int part[TPB / 64];
  const int N = d.scal->N;
  int c = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < d.NE; i += gridDim.x * blockDim.x)
    c += d.ts[i].tick < N ? 1 : 0;
  // one atomic per workgroup
#pragma unroll
  for (int s = 1; s < 64; s <<= 1) c += __shfl_xor(c, s);
  if (__lane_id() == 0) part[threadIdx.x / 64] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < TPB / 64; ++w) t += part[w];
    if (t) atomicAdd(&d.scal->n_unfinished, t);
  }
}

// ---------------------------------------------------------------------------
// Set-up and I/O
// ---------------------------------------------------------------------------
template <int M>
__global__ void __launch_bounds__(TPB) k_init_geometry(Dev d) {
  const int NE = d.NE, NV = d.NV, NF = d.NF;
  const int n = max(max(NE, NV), NF);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    if (i < NE) {
      double X[6];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int nd = d.tri[k * NE + i];
        X[2 * k] = d.X[nd];
        X[2 * k + 1] = d.X[NV + nd];
      }
      double* r = d.rec + size_t(i) * Sz<M>::RS;
#pragma unroll
      for (int c = 0; c < 6; ++c) r[XE + c] = X[c];
      r[AO] = tri_area(X);
      if (!(r[AO] > 0.0)) set_err(d, ERR_GEOM);
      d.ts[i] = TickStep{0, 0};
      d.act_stamp[i] = -1;
#pragma unroll
      for (int c = 0; c < 3 * MEM_W; ++c) d.mem[size_t(i) * 3 * MEM_W + c] = 0.0;
      if (d.replay_pos) d.replay_pos[i] = 0;
    }
    if (i < NV) {
      d.ntick[i] = 0;
      d.node_stamp[i] = -1;
    }
  }
}

template <int M>
__global__ void __launch_bounds__(TPB) k_check_state(Dev d, double g) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < d.NE; i += gridDim.x * blockDim.x) {
    const double* r = d.rec + size_t(i) * Sz<M>::RS;
    double q[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) q[v] = r[QO + v];
    if (!(q[0] > 0.0) || !(pressure(q, g) > 0.0)) set_err(d, ERR_STATE);
  }
}

template <int M>
__global__ void __launch_bounds__(TPB) k_download_q(Dev d, double* out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < d.NE; i += gridDim.x * blockDim.x) {
    const double* r = d.rec + size_t(i) * Sz<M>::RS;
#pragma unroll
    for (int v = 0; v < 4; ++v) out[size_t(v) * d.NE + i] = r[QO + v];
  }
}

template <int M>
__global__ void __launch_bounds__(TPB) k_upload_q(Dev d, const double* in) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < d.NE; i += gridDim.x * blockDim.x) {
    double* r = d.rec + size_t(i) * Sz<M>::RS;
#pragma unroll
    for (int v = 0; v < 4; ++v) r[QO + v] = in[size_t(v) * d.NE + i];
  }
}

__global__ void __launch_bounds__(TPB) k_download_xy(Dev d, double* out) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < d.NV; k += gridDim.x * blockDim.x) {
    out[2 * k] = d.X[k];
    out[2 * k + 1] = d.X[d.NV + k];
  }
}

__global__ void __launch_bounds__(TPB) k_upload_xy(Dev d, const double* in) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < d.NV; k += gridDim.x * blockDim.x) {
    d.X[k] = in[2 * k];
    d.X[d.NV + k] = in[2 * k + 1];
  }
}

__global__ void __launch_bounds__(TPB) k_elem_times(Dev d, double* out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < d.NE; i += gridDim.x * blockDim.x) {
    const Inst in = d.inst[d.e_inst[i]];
    out[i] = in.T + double(d.ts[i].tick) * in.delta;
  }
}

int grid_for(long n) {
  long b = (n + TPB - 1) / TPB;
  if (b < 1) b = 1;
  if (b > 16384) b = 16384;
  return int(b);
}

// Start and stop events for the next grid launch (per-kernel timing): that
// launch then takes its two timestamps from the kernel's own execution rather
// than from markers queued before and after it.
thread_local hipEvent_t t_ev_start = nullptr, t_ev_stop = nullptr;

#define AW_LAUNCH_GB(kern, grid, block, stream, ...)                                                \
  do {                                                                                              \
    if (t_ev_start) {                                                                               \
      hipEvent_t _a = t_ev_start, _b = t_ev_stop;                                                   \
      t_ev_start = t_ev_stop = nullptr;                                                             \
      hipExtLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, (hipStream_t)(stream), _a, _b, 0,     \
                            __VA_ARGS__);                                                           \
    } else {                                                                                        \
      hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, (hipStream_t)(stream), __VA_ARGS__);     \
    }                                                                                               \
    hipError_t _e = hipGetLastError();                                                              \
    if (_e != hipSuccess) return int(_e);                                                           \
  } while (0)
#define AW_LAUNCH_G(kern, grid, stream, ...) AW_LAUNCH_GB(kern, grid, TPB, stream, __VA_ARGS__)

#define AW_LAUNCH(kern, n, stream, ...) AW_LAUNCH_G(kern, grid_for(n), stream, __VA_ARGS__)

#define AW_LAUNCH1(kern, stream, ...)                                                     \
  do {                                                                                    \
    hipLaunchKernelGGL(kern, dim3(1), dim3(1), 0, (hipStream_t)(stream), __VA_ARGS__);    \
    hipError_t _e = hipGetLastError();                                                    \
    if (_e != hipSuccess) return int(_e);                                                 \
  } while (0)

#define AW_DISPATCH(M, ...)                                    \
  switch (M) {                                                 \
    case 1: { constexpr int MM = 1; __VA_ARGS__; } break;      \
    case 2: { constexpr int MM = 2; __VA_ARGS__; } break;      \
    case 3: { constexpr int MM = 3; __VA_ARGS__; } break;      \
    default: return int(hipErrorInvalidValue);                 \
  }

}  // namespace

void set_next_launch_events(void* start, void* stop) {
  t_ev_start = static_cast<hipEvent_t>(start);
  t_ev_stop = static_cast<hipEvent_t>(stop);
}
bool next_launch_events_pending() { return t_ev_start != nullptr; }

int launch_init_geometry(const Dev& d, void* s) {
  int n = d.NE > d.NV ? d.NE : d.NV;
  if (d.NF > n) n = d.NF;
  AW_DISPATCH(d.M, AW_LAUNCH(k_init_geometry<MM>, n, s, d));
  return 0;
}

// Workgroups of a list-driven launch: enough for every element, or (when
// tuned) a persistent grid of list_wg_per_cu workgroups per CU striding over
// the active list.
static int list_grid(const Dev& d, long blocks_for_all, int use_list) {
  long b = blocks_for_all;
  if (use_list && d.list_wg_per_cu > 0) {
    const long cap = long(d.list_wg_per_cu) * (d.n_cu > 0 ? d.n_cu : 256);
    if (b > cap) b = cap;
  }
  if (b < 1) b = 1;
  if (b > 16384) b = 16384;
  return int(b);
}

int launch_reconstruct(const Dev& d, const Params& p, int M, int use_list, int set_level, void* s) {
  // 8 lanes per element
  const int g = list_grid(d, (8L * d.NE + TPB - 1) / TPB, use_list);
  AW_DISPATCH(M, AW_LAUNCH_G(k_reconstruct<MM>, g, s, d, d.tab, p, use_list, set_level));
  return 0;
}

int launch_predict(const Dev& d, const Params& p, int M, int use_list, void* s) {
  AW_DISPATCH(M, {
    constexpr int per_block = Sz<MM>::EPW * (TPB / 64);
    const int g = list_grid(d, (long(d.NE) + per_block - 1) / per_block, use_list);
    AW_LAUNCH_G(k_predict<MM>, g, s, d, d.tab, p, use_list);
  });
  return 0;
}

int launch_set_target(const Dev& d, double t_end, void* s) {
  AW_LAUNCH1(k_set_target, s, d, t_end);
  return 0;
}

int launch_macro_begin(const Dev& d, int N, int nominal, double fraction, void* s) {
  AW_LAUNCH(k_reset_min, d.K, s, d);
  AW_LAUNCH(k_min_dt, (long(d.NE) + MIN_U - 1) / MIN_U, s, d);
  AW_LAUNCH(k_macro_setup, d.K, s, d, N, fraction, double(nominal) / double(N));
  AW_LAUNCH(k_levels, d.NE > d.NV ? d.NE : d.NV, s, d);
  return 0;
}

int launch_cycle_begin(const Dev& d, void* s) {
  AW_LAUNCH1(k_cycle_begin, s, d);
  return 0;
}

int launch_sched(const Dev& d, void* s) {
  // chunks of at most SCHED_CHUNK elements, at least ~1024 blocks when possible,
  // unless a chunk size was chosen; at least one pass of SCHED_TPB / 8 elements.
  // Each block reserves its list space with one atomic, and atomics on one
  // address serialise, so larger chunks mean fewer of them.
  int chunk = d.sched_chunk > 0 ? d.sched_chunk : (d.NE + 1023) / 1024;
  chunk = chunk < SCHED_TPB / 8 ? SCHED_TPB / 8 : (chunk > SCHED_CHUNK ? SCHED_CHUNK : chunk);
  const int blocks = (d.NE + chunk - 1) / chunk;
  AW_LAUNCH_GB(k_sched, blocks, SCHED_TPB, s, d, chunk);
  return 0;
}

// Grid of a launch that sweeps every node or edge: one lane per item, or the
// persistent grid of the launch settings (workgroups per CU), whose
// workgroups stride the items.
static int sweep_grid(const Dev& d, long n) {
  long b = (n + TPB - 1) / TPB;
  if (d.sweep_wg_per_cu > 0) {
    const long cap = long(d.sweep_wg_per_cu) * (d.n_cu > 0 ? d.n_cu : 256);
    if (b > cap) b = cap;
  }
  if (b < 1) b = 1;
  if (b > 16384) b = 16384;
  return int(b);
}

int launch_node(const Dev& d, const Params& p, int M, void* s) {
  AW_DISPATCH(M, AW_LAUNCH_G(k_node<MM>, sweep_grid(d, d.NV), s, d, d.tab, p));
  return 0;
}

int launch_patch(const Dev& d, const Params& p, int M, void* s) {
  AW_DISPATCH(M, AW_LAUNCH_G(k_patch<MM>, sweep_grid(d, d.NF), s, d, d.tab, p));
  return 0;
}

// The update kernel runs over the cycle's active list, whose length only the
// device knows: a grid sized for every element (or the persistent grid of the
// launch settings), blocks beyond the list exit at once.
int launch_update(const Dev& d, const Params& p, void* s) {
  const int g = list_grid(d, (long(d.NE) + TPB - 1) / TPB, 1);
  AW_DISPATCH(d.M, AW_LAUNCH_G(k_update<MM>, g, s, d, p));
  return 0;
}

int launch_status(const Dev& d, void* s) {
  AW_LAUNCH1(k_count_reset, s, d);
  {
    const int g = grid_for(d.NE), cap = 2 * (d.n_cu > 0 ? d.n_cu : 256);
    AW_LAUNCH_G(k_count, g < cap ? g : cap, s, d);
  }
  return 0;
}

int launch_macro_end(const Dev& d, int only_if_done, void* s) {
  long n = d.NE > d.NV ? d.NE : d.NV;
  if (d.K > n) n = d.K;
  AW_LAUNCH(k_macro_end, n, s, d, only_if_done);
  return 0;
}

int launch_open(const Dev& d, void* s) {
  AW_LAUNCH(k_open, d.K, s, d);
  AW_LAUNCH_G(k_count_open, 1, s, d);
  return 0;
}

int launch_download_xy(const Dev& d, double* out, void* s) {
  AW_LAUNCH(k_download_xy, d.NV, s, d, out);
  return 0;
}

int launch_upload_xy(const Dev& d, const double* in, void* s) {
  AW_LAUNCH(k_upload_xy, d.NV, s, d, in);
  return 0;
}

int launch_download_q(const Dev& d, double* out, void* s) {
  AW_DISPATCH(d.M, AW_LAUNCH(k_download_q<MM>, d.NE, s, d, out));
  return 0;
}

int launch_upload_q(const Dev& d, const double* in, void* s) {
  AW_DISPATCH(d.M, AW_LAUNCH(k_upload_q<MM>, d.NE, s, d, in));
  return 0;
}

int launch_elem_times(const Dev& d, double* out, void* s) {
  AW_LAUNCH(k_elem_times, d.NE, s, d, out);
  return 0;
}

int launch_check_state(const Dev& d, double gamma, void* s) {
  AW_DISPATCH(d.M, AW_LAUNCH(k_check_state<MM>, d.NE, s, d, gamma));
  return 0;
}

}  // namespace aw
