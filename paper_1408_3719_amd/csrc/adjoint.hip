// Reverse mode (adjoint) of one global time step on a fixed mesh (gfx950).
//
// The step map Q^n -> Q^{n+1} of global time stepping with the mesh held fixed
// (mesh velocity V = 0, eq. ODEmesh) and a given time step dt:
//   WENO reconstruction with real neighbour data (eqs. intConsRec .. eqn.weno)
//   -> space-time predictor (eq. CGfinal; the metric of the fixed affine map,
//   no time derivative of the mesh) -> edge traces -> Rusanov (eq.
//   eqn.rusanov) or HLL fluxes over the space-time faces of the fixed edges
//   ((M+1)^2 Gauss points, eq. eqn.STint) -> one-step update (eq. PDEfinal,
//   |T'| = |T|).
// Given qbar_next = dL/dQ^{n+1} the kernels return qbar = dL/dQ^n, with dt
// held fixed (the CFL step of eq. eqn.timestep is not differentiated):
//   k_adj_recon<fwd>  reconstruction from the current averages (8 lanes per
//                     element, lane s solves stencil s by Givens rotations)
//   k_adj_pred_fwd    predictor sweeps, each iterate kept, edge traces and
//                     cell means at the time nodes
//   k_adj_patch       adjoint of the fluxes: per edge, the flux adjoint
//                     -qbar_L/|T_L| + qbar_R/|T_R| pulled back through the
//                     Rusanov flux at every Gauss point onto the two elements'
//                     trace adjoints (each (element, edge) slot has one
//                     writer), and on a transmissive edge onto the inner
//                     element's mean adjoint in the edge's own slot
//   k_adj_pred_rev    the sweeps in reverse: trace adjoint -> adjoint of the
//                     reconstruction's nodal values
//   k_adj_recon<rev>  WENO weights and least squares in reverse from the data
//                     the forward pass kept; each stencil row's adjoint goes to
//                     a slot of its own
//   k_adj_gather      qbar_j = qbar_next_j (the identity part of the update) +
//                     the slots of every stencil row that names element j, in a
//                     fixed order (no atomics: each average is named by ~80 rows)
// Subgradients: the larger Rusanov signal speed and the bounding HLL speeds are
// taken from the left state on ties, and |x| has derivative sign(x), 0 at 0.
// The least-squares adjoint uses A R^-1 = Q of the QR factorisation: the
// adjoint of the right-hand side is A R^-1 R^-T wbar, so the rotations need
// not be kept.
#include <hip/hip_runtime.h>

#include <type_traits>

#include <mutex>
#include <vector>

#include "aderweno.h"
#include "basis.h"
#include "common.h"
#include "lagadj.h"

namespace aw {

// Scratch of ader_adjoint_gts_step_static (callers that cannot allocate): a
// file-scope device array, one copy on every GPU the library runs on, held
// until the process ends. Host code never passes `scratch` itself to a kernel
// (on the host it is only a stand-in for the symbol): its device address on
// the current GPU comes from static_scratch() below.
static __device__ __align__(256) char scratch[ADER_STATIC_SCRATCH_BYTES];

int static_scratch(void** ptr, size_t* bytes) {
  static std::mutex mu;
  static std::vector<void*> addr;   // per device, looked up once
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return int(e);
  std::lock_guard<std::mutex> lock(mu);
  if (dev >= int(addr.size())) addr.resize(dev + 1, nullptr);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return int(e);
    addr[dev] = p;
  }
  *ptr = addr[dev];
  *bytes = ADER_STATIC_SCRATCH_BYTES;
  return 0;
}

namespace {

constexpr int TPB = 256;
constexpr int XE = rec_off_xe(), QO = rec_off_q(), AO = rec_off_a();

template <int M>
struct AZ {
  static constexpr int nb = (M + 1) * (M + 2) / 2;
  static constexpr int T = M + 1;
  static constexpr int nG = M + 1;
  static constexpr int ne = 2 * nb;
  static constexpr int nu = nb - 1;
  static constexpr int RS = rec_stride(M);
  static constexpr int TS = trace_stride(M);
  static constexpr int WS = wnod_stride(M);
  static constexpr int QS = nb * T * 4;   // nodal space-time values of one element
  // kept per stencil lane by the forward reconstruction: R (upper triangle),
  // solution, weight and indicator (the rows are rebuilt in reverse)
  static constexpr int L_R = 0, L_W = nu * (nu + 1) / 2, L_OM = L_W + 4 * nu, L_SIG = L_OM + 1,
                       LB = L_SIG + 1;
};

// Euler fluxes f, g (eq. eulerTerms) with p from eq. eqn.eos.
__device__ inline void euler_fg(const double q[4], double gam, double f[4], double g[4]) {
  const double r = q[0], u = q[1] / r, v = q[2] / r, E = q[3];
  const double p = (gam - 1.0) * (E - 0.5 * r * (u * u + v * v));
  f[0] = r * u;
  f[1] = r * u * u + p;
  f[2] = r * u * v;
  f[3] = u * (E + p);
  g[0] = r * v;
  g[1] = r * u * v;
  g[2] = r * v * v + p;
  g[3] = v * (E + p);
}

// Adjoint of the primitive variables (rho, u, v, p, E written as rb, ub, vb,
// pb, Eb) pulled back to the conserved ones: qb += d(rho, u, v, p, E)/dq ^T (.).
__device__ inline void prim_pullback(const double q[4], double gam, double rb, double ub, double vb,
                                     double pb, double Eb, double qb[4]) {
  const double r = q[0], u = q[1] / r, v = q[2] / r;
  const double gm = gam - 1.0;
  Eb += gm * pb;
  rb += -gm * 0.5 * (u * u + v * v) * pb;
  ub += -gm * r * u * pb;
  vb += -gm * r * v * pb;
  qb[0] += rb - (ub * u + vb * v) / r;
  qb[1] += ub / r;
  qb[2] += vb / r;
  qb[3] += Eb;
}

// qb += J_f(q)^T fb + J_g(q)^T gb
__device__ inline void euler_fg_vjp(const double q[4], double gam, const double fb[4],
                                    const double gb[4], double qb[4]) {
  const double r = q[0], u = q[1] / r, v = q[2] / r, E = q[3];
  const double p = (gam - 1.0) * (E - 0.5 * r * (u * u + v * v));
  const double H = E + p;
  double rb = 0.0, ub = 0.0, vb = 0.0, pb = 0.0, Eb = 0.0;
  rb += fb[0] * u;            ub += fb[0] * r;
  rb += fb[1] * u * u;        ub += fb[1] * 2.0 * r * u;   pb += fb[1];
  rb += fb[2] * u * v;        ub += fb[2] * r * v;         vb += fb[2] * r * u;
  ub += fb[3] * H;            Eb += fb[3] * u;             pb += fb[3] * u;
  rb += gb[0] * v;            vb += gb[0] * r;
  rb += gb[1] * u * v;        ub += gb[1] * r * v;         vb += gb[1] * r * u;
  rb += gb[2] * v * v;        vb += gb[2] * 2.0 * r * v;   pb += gb[2];
  vb += gb[3] * H;            Eb += gb[3] * v;             pb += gb[3] * v;
  prim_pullback(q, gam, rb, ub, vb, pb, Eb, qb);
}

// ALE signal speed |u.N_xy + N_t| + c |N_xy| (eq. eqn.rusanov)
__device__ inline double signal_speed(const double q[4], const double N[3], double nxy, double gam) {
  const double r = q[0], u = q[1] / r, v = q[2] / r;
  const double p = (gam - 1.0) * (q[3] - 0.5 * r * (u * u + v * v));
  return fabs(u * N[0] + v * N[1] + N[2]) + sqrt(gam * p / r) * nxy;
}

// qb += sb * d(signal speed)/dq
__device__ inline void signal_speed_vjp(const double q[4], const double N[3], double nxy, double gam,
                                        double sb, double qb[4]) {
  const double r = q[0], u = q[1] / r, v = q[2] / r;
  const double p = (gam - 1.0) * (q[3] - 0.5 * r * (u * u + v * v));
  const double un = u * N[0] + v * N[1] + N[2];
  const double sg = (un > 0.0) ? 1.0 : (un < 0.0 ? -1.0 : 0.0);
  const double c = sqrt(gam * p / r);
  const double cb = sb * nxy;
  prim_pullback(q, gam, -cb * c / (2.0 * r), sb * sg * N[0], sb * sg * N[1], cb * gam / (2.0 * c * r),
                0.0, qb);
}

// Adjoint of the Rusanov flux 0.5 (F(ql) + F(qr)) . N - 0.5 smax (qr - ql).
__device__ inline void rusanov_vjp(const double ql[4], const double qr[4], const double N[3],
                                   double gam, const double Gb[4], double qlb[4], double qrb[4]) {
  const double nxy = sqrt(N[0] * N[0] + N[1] * N[1]);
  const double sl = signal_speed(ql, N, nxy, gam), sr = signal_speed(qr, N, nxy, gam);
  const bool left = sl >= sr;
  const double smax = left ? sl : sr;
  double fb[4], gb[4], sbar = 0.0;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    fb[v] = 0.5 * N[0] * Gb[v];
    gb[v] = 0.5 * N[1] * Gb[v];
    qlb[v] += 0.5 * N[2] * Gb[v] + 0.5 * smax * Gb[v];
    qrb[v] += 0.5 * N[2] * Gb[v] - 0.5 * smax * Gb[v];
    sbar -= 0.5 * Gb[v] * (qr[v] - ql[v]);
  }
  euler_fg_vjp(ql, gam, fb, gb, qlb);
  euler_fg_vjp(qr, gam, fb, gb, qrb);
  if (left)
    signal_speed_vjp(ql, N, nxy, gam, sbar, qlb);
  else
    signal_speed_vjp(qr, N, nxy, gam, sbar, qrb);
}

// ALE signal speeds u.N_xy + N_t -/+ c|N_xy|
__device__ inline void hll_speeds(const double q[4], const double N[3], double nxy, double gam,
                                  double& lo, double& hi) {
  const double r = q[0], u = q[1] / r, v = q[2] / r;
  const double p = (gam - 1.0) * (q[3] - 0.5 * r * (u * u + v * v));
  const double un = u * N[0] + v * N[1] + N[2];
  const double c = sqrt(gam * p / r) * nxy;
  lo = un - c;
  hi = un + c;
}

// qb += sb * d(u.N_xy + N_t + sgn * c|N_xy|)/dq
__device__ inline void hll_speed_vjp(const double q[4], const double N[3], double nxy, double gam,
                                     double sgn, double sb, double qb[4]) {
  const double r = q[0], u = q[1] / r, v = q[2] / r;
  const double p = (gam - 1.0) * (q[3] - 0.5 * r * (u * u + v * v));
  const double c = sqrt(gam * p / r);
  const double cb = sgn * sb * nxy;
  prim_pullback(q, gam, -cb * c / (2.0 * r), sb * N[0], sb * N[1], cb * gam / (2.0 * c * r), 0.0, qb);
}

// qb += J_ft(q)^T gb with ft = f N_x + g N_y + q N_t
__device__ inline void ft_vjp(const double q[4], const double N[3], double gam, const double gb[4],
                              double qb[4]) {
  double fb[4], gg[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    fb[v] = N[0] * gb[v];
    gg[v] = N[1] * gb[v];
    qb[v] += N[2] * gb[v];
  }
  euler_fg_vjp(q, gam, fb, gg, qb);
}

// Adjoint of the HLL flux: speeds bounded over both states (the left state's
// speed on ties), upwind when both have one sign, else
// (sr F(ql) - sl F(qr) + sl sr (qr - ql)) / (sr - sl).
__device__ inline void hll_vjp(const double ql[4], const double qr[4], const double N[3], double gam,
                               const double Gb[4], double qlb[4], double qrb[4]) {
  const double nxy = sqrt(N[0] * N[0] + N[1] * N[1]);
  double l1, r1, l2, r2;
  hll_speeds(ql, N, nxy, gam, l1, r1);
  hll_speeds(qr, N, nxy, gam, l2, r2);
  const bool left_lo = l1 <= l2, left_hi = r1 >= r2;
  const double sl = left_lo ? l1 : l2, sr = left_hi ? r1 : r2;
  if (sl >= 0.0) {
    ft_vjp(ql, N, gam, Gb, qlb);
    return;
  }
  if (sr <= 0.0) {
    ft_vjp(qr, N, gam, Gb, qrb);
    return;
  }
  double fl[4], fr[4], f[4], g[4];
  euler_fg(ql, gam, f, g);
#pragma unroll
  for (int v = 0; v < 4; ++v) fl[v] = f[v] * N[0] + g[v] * N[1] + ql[v] * N[2];
  euler_fg(qr, gam, f, g);
#pragma unroll
  for (int v = 0; v < 4; ++v) fr[v] = f[v] * N[0] + g[v] * N[1] + qr[v] * N[2];
  const double id = 1.0 / (sr - sl);
  double flb[4], frb[4], slb = 0.0, srb = 0.0;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double d = qr[v] - ql[v];
    const double F = (sr * fl[v] - sl * fr[v] + sl * sr * d) * id;
    flb[v] = sr * id * Gb[v];
    frb[v] = -sl * id * Gb[v];
    qrb[v] += sl * sr * id * Gb[v];
    qlb[v] -= sl * sr * id * Gb[v];
    srb += Gb[v] * (fl[v] + sl * d - F) * id;
    slb += Gb[v] * (-fr[v] + sr * d + F) * id;
  }
  ft_vjp(ql, N, gam, flb, qlb);
  ft_vjp(qr, N, gam, frb, qrb);
  if (left_lo)
    hll_speed_vjp(ql, N, nxy, gam, -1.0, slb, qlb);
  else
    hll_speed_vjp(qr, N, nxy, gam, -1.0, slb, qrb);
  if (left_hi)
    hll_speed_vjp(ql, N, nxy, gam, 1.0, srb, qlb);
  else
    hll_speed_vjp(qr, N, nxy, gam, 1.0, srb, qrb);
}

__device__ inline double group8_sum(double v) {
  v += __shfl_xor(v, 1);
  v += __shfl_xor(v, 2);
  v += __shfl_xor(v, 4);
  return v;
}

// The same sum with the lane moves done by DPP inside the VALU (no LDS round
// trip); each step adds two equal partial sums, so the bits are those of
// group8_sum. Every lane of the 8-lane group must be active.
template <int CTRL>
__device__ inline double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, int(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
__device__ inline double group8_sum_dpp(double v) {
  v += dpp_move<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_move<0x141>(v);   // row_half_mirror: lane i <-> 7 - i within 8
  return v;
}

// Row of the least-squares system for stencil element j seen from element i:
// the means over T_j, mapped into the reference frame of T_i (vertices Xi,
// inverse edge matrix through e1, e2, idet), of the monomials shifted by their
// reference means, the basis the forward reconstruction solves in.
template <int M>
__device__ inline void ls_row(const double* Xj, const double Xi[6], double e1x, double e1y,
                              double e2x, double e2y, double idet, double a[AZ<M>::nu]) {
  constexpr int nb = AZ<M>::nb, nu = AZ<M>::nu;
  double rx[3], ry[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double dx = Xj[2 * k] - Xi[0], dy = Xj[2 * k + 1] - Xi[1];
    rx[k] = (dx * e2y - dy * e2x) * idet;
    ry[k] = (e1x * dy - e1y * dx) * idet;
  }
  double mm[nb];
  monomial_means<M>(rx, ry, mm);
#pragma unroll
  for (int l = 0; l < nu; ++l) a[l] = mm[l + 1] - RefMeans<M>::m[l + 1];
}

// The context's averages as [4][NE].
template <int M>
__global__ void __launch_bounds__(TPB) k_adj_state(Dev d, AdjWork w) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < d.NE; i += gridDim.x * blockDim.x) {
    const double* r = d.rec + size_t(i) * AZ<M>::RS;
#pragma unroll
    for (int v = 0; v < 4; ++v) w.qcopy[size_t(v) * d.NE + i] = r[QO + v];
  }
}

// qbar_j = qbar_next_j + own terms of j (row 0, 8 lanes) + rows naming j.
// 8 lanes per element: lane s takes own slot s and every 8th naming row, two
// rows in flight; a butterfly sums the lanes (a fixed order: deterministic).
// GEO: the same for the vertex adjoints of the rows, added to xeb_j.
template <int M, bool GEO = false>
__global__ void __launch_bounds__(TPB) k_adj_gather(Dev d, AdjWork w) {
  constexpr int NA = GEO ? 10 : 4;
  const int NE = d.NE;
  const int sl = threadIdx.x & 7;
  const int ngroups = (gridDim.x * blockDim.x) >> 3;
  for (int j = (blockIdx.x * blockDim.x + threadIdx.x) >> 3; j < NE; j += ngroups) {
    double acc[NA];
    // a row slot holds NA doubles: the right-hand side's adjoint (4), then
    // with GEO the stencil element's vertex adjoints (6)
    auto add = [&](size_t slot) {
      const double* r = w.rowbar + slot * NA;
#pragma unroll
      for (int v = 0; v < NA; ++v) acc[v] += r[v];
    };
#pragma unroll
    for (int v = 0; v < NA; ++v) acc[v] = 0.0;
    add(size_t(j) * AZ<M>::ne * 8 + sl);
    const int k1 = d.tsten_ptr[j + 1];
    int k = d.tsten_ptr[j] + sl;
    for (; k + 8 < k1; k += 16) {
      const size_t s0 = size_t(d.tsten_idx[k]), s1 = size_t(d.tsten_idx[k + 8]);
      double a0[NA], a1[NA];
#pragma unroll
      for (int v = 0; v < NA; ++v) {
        a0[v] = w.rowbar[s0 * NA + v];
        a1[v] = w.rowbar[s1 * NA + v];
      }
#pragma unroll
      for (int v = 0; v < NA; ++v) acc[v] += a0[v] + a1[v];
    }
    if (k < k1) add(size_t(d.tsten_idx[k]));
#pragma unroll
    for (int v = 0; v < NA; ++v) acc[v] = group8_sum(acc[v]);
    double mine = acc[0];
#pragma unroll
    for (int v = 1; v < NA; ++v)
      if (sl == v) mine = acc[v];
    if (sl < 4) w.qbar[size_t(sl) * NE + j] = w.qbar_next[size_t(sl) * NE + j] + mine;
    if (GEO) {
      // lanes 0..5 hold the vertex sums in acc[4 + lane]
      double xm = acc[4];
#pragma unroll
      for (int v = 1; v < 6; ++v)
        if (sl == v) xm = acc[4 + v];
      if (sl < 6) w.xeb[size_t(j) * 6 + sl] += xm;
    }
  }
}

// Element j of the saved state s placed at tick nt (eqs. eqn.virtGeom and
// eqn.virtCellaverage): its stored vertices and average when it is at that
// tick, else its predictor's vertex trajectories and cell means at the
// rescaled time (nt - tick) / step.
template <int M>
__device__ inline void lts_place(const Tables* __restrict__ tb, const LtsView& s, int j, int nt, double delta,
                                 double X[6], double Q[4]) {
  constexpr int T = M + 1, RS = AZ<M>::RS, AVG = rec_off_avg(), VV = rec_off_vv(M);
  const TickStep tj = s.ts[j];
  const double* rj = s.rec + size_t(j) * RS;
  if (tj.tick == nt) {
#pragma unroll
    for (int k = 0; k < 6; ++k) X[k] = rj[XE + k];
#pragma unroll
    for (int v = 0; v < 4; ++v) Q[v] = rj[QO + v];
    return;
  }
  const double tau = double(nt - tj.tick) / double(tj.step);
  const double dtj = double(tj.step) * delta;
  double L[T], l[T];
  lag::tanti<M>(*tb, tau, L);
  lag::tbasis<M>(*tb, tau, l);
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    double sum = 0.0;
#pragma unroll
    for (int q = 0; q < T; ++q) sum += L[q] * rj[VV + ((k / 2) * T + q) * 2 + (k % 2)];
    X[k] = rj[XE + k] + dtj * sum;
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    double sum = 0.0;
#pragma unroll
    for (int q = 0; q < T; ++q) sum += l[q] * rj[AVG + q * 4 + v];
    Q[v] = sum;
  }
}

// Reconstruction (REV = false: write the nodal values) or its adjoint (REV =
// true: read their adjoint, add to qbar). 8 lanes per element. GEO: the rows
// depend on vertices that are differentiated too (a moving mesh): with w = the
// least-squares solution, z = (A^T A)^-1 wbar and the residual r_c = b_c - a_c w,
// the adjoint of row a_c is sum over the variables of r_c z - (a_c . z) w, pulled
// back to the vertices of the stencil element (its slot) and of element i
// (row 0 of the lane).
// VIRT (local time stepping): the elements of lw.act_list, their own data
// from the state lw.s1, the stencil elements placed at the element's tick
// (real or projected, lts_place).
template <int M, bool REV, bool GEO = false, bool VIRT = false>
__global__ void __launch_bounds__(TPB) k_adj_recon(Dev d, const Tables* __restrict__ tb, Params P,
                                                   AdjWork w, LtsWork lw) {
  using S = AZ<M>;
  constexpr int nb = S::nb, ne = S::ne, nu = S::nu, WS = S::WS;
  const int NE = d.NE;
  const int sl = threadIdx.x & 7;
  const int ngroups = (gridDim.x * blockDim.x) >> 3;
  const double* gbase = VIRT ? lw.s1.rec + XE : (w.geo ? w.geo : d.rec + XE);
  const size_t gs = VIRT ? size_t(S::RS) : (w.geo ? size_t(w.geo_stride) : size_t(S::RS));
  const int n_el = VIRT ? lw.counts[0] : NE;
  for (int idx = (blockIdx.x * blockDim.x + threadIdx.x) >> 3; idx < n_el; idx += ngroups) {
    const int i = VIRT ? lw.act_list[idx] : idx;
    const double* ri = gbase + size_t(i) * gs;
    double Xi[6], Qi[4];
#pragma unroll
    for (int c = 0; c < 6; ++c) Xi[c] = ri[c];
#pragma unroll
    for (int v = 0; v < 4; ++v) Qi[v] = VIRT ? lw.s1.rec[size_t(i) * S::RS + QO + v] : w.q[size_t(v) * NE + i];
    const int nt = VIRT ? lw.s1.ts[i].tick : 0;
    // stencil row c of this lane: the element's vertices (xv when placed) and average
    auto row = [&](int c, double xv[6], double qv[4]) -> const double* {
      const int j = d.sten[size_t(sl * ne + c) * NE + i];
      if (VIRT) {
        lts_place<M>(tb, lw.s1, j, nt, lw.delta, xv, qv);
        return xv;
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) qv[v] = w.q[size_t(v) * NE + j];
      return gbase + size_t(j) * gs;
    };
    const double e1x = Xi[2] - Xi[0], e1y = Xi[3] - Xi[1];
    const double e2x = Xi[4] - Xi[0], e2y = Xi[5] - Xi[1];
    const double idet = 1.0 / (e1x * e2y - e2x * e1y);
    const int* sidx = d.sten + size_t(sl * ne) * NE + i;    // row c at sidx[c * NE]
    const bool valid = sl < NSTEN && sidx[0] >= 0;
    // kept data of this lane: slot k at lq[k * 8 * NE]
    double* lq = w.lsq + size_t(i) * 8 + sl;
    const size_t LS = size_t(8) * NE;
    double R[nu][nu], ws[nu][4];
    double om = 0.0, sig = 0.0;
#pragma unroll
    for (int a = 0; a < nu; ++a) {
#pragma unroll
      for (int b = 0; b < nu; ++b) R[a][b] = 0.0;
#pragma unroll
      for (int v = 0; v < 4; ++v) ws[a][v] = 0.0;
    }
    if (REV && valid) {
      int k = S::L_R;
#pragma unroll
      for (int a = 0; a < nu; ++a)
#pragma unroll
        for (int b = a; b < nu; ++b) R[a][b] = lq[(k++) * LS];
#pragma unroll
      for (int a = 0; a < nu; ++a)
#pragma unroll
        for (int v = 0; v < 4; ++v) ws[a][v] = lq[(S::L_W + a * 4 + v) * LS];
      om = lq[S::L_OM * LS];
      sig = lq[S::L_SIG * LS];
    } else if (valid) {
      double z[nu][4];
#pragma unroll
      for (int a = 0; a < nu; ++a)
#pragma unroll
        for (int v = 0; v < 4; ++v) z[a][v] = 0.0;
#pragma unroll 1
      for (int c = 1; c < ne; ++c) {
        double xv[6], qv[4];
        const double* rj = row(c, xv, qv);
        double a[nu], b[4];
        ls_row<M>(rj, Xi, e1x, e1y, e2x, e2y, idet, a);
#pragma unroll
        for (int v = 0; v < 4; ++v) b[v] = qv[v] - Qi[v];
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
#pragma unroll
      for (int k = nu - 1; k >= 0; --k) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double t = z[k][v];
#pragma unroll
          for (int c2 = k + 1; c2 < nu; ++c2) t -= R[k][c2] * ws[c2][v];
          ws[k][v] = t / R[k][k];
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int l = 0; l < nu; ++l) {
          double t = 0.0;
#pragma unroll
          for (int m = 0; m < nu; ++m) t += MonoBasis<M>::c.sig[l][m] * ws[m][v];
          sig += ws[l][v] * t;
        }
      const double x = sig + P.eps;
      const double x2 = x * x, x4 = x2 * x2;
      om = (sl == 0 ? P.lambda : 1.0) / (x4 * x4);
      int k = S::L_R;
#pragma unroll
      for (int a = 0; a < nu; ++a)
#pragma unroll
        for (int b = a; b < nu; ++b) lq[(k++) * LS] = R[a][b];
#pragma unroll
      for (int a = 0; a < nu; ++a)
#pragma unroll
        for (int v = 0; v < 4; ++v) lq[(S::L_W + a * 4 + v) * LS] = ws[a][v];
      lq[S::L_OM * LS] = om;
      lq[S::L_SIG * LS] = sig;
    }
    // combined reconstruction W = sum_s om_s w_s / sum_s om_s
    const double Ssum = group8_sum(om);
    double W[nu][4];
#pragma unroll
    for (int l = 0; l < nu; ++l)
#pragma unroll
      for (int v = 0; v < 4; ++v) W[l][v] = group8_sum(om * ws[l][v]) / Ssum;
    if (!REV) {
      double* wo = w.wnod + size_t(i) * WS;
#pragma unroll
      for (int m = 0; m < nb; ++m)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if (((m * 4 + v) & 7) != sl) continue;
          double t = Qi[v];
#pragma unroll
          for (int l = 0; l < nu; ++l) t += MonoBasis<M>::c.node[m][l] * W[l][v];
          wo[m * 4 + v] = t;
        }
      continue;
    }
    // adjoint of the nodal values -> adjoint of (Q_i, W)
    const double* wbi = w.wbar + size_t(i) * WS;
    double Wb[nu][4], q0b[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      q0b[v] = 0.0;
#pragma unroll
      for (int l = 0; l < nu; ++l) Wb[l][v] = 0.0;
    }
#pragma unroll
    for (int m = 0; m < nb; ++m)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double b = wbi[m * 4 + v];
        q0b[v] += b;
#pragma unroll
        for (int l = 0; l < nu; ++l) Wb[l][v] += MonoBasis<M>::c.node[m][l] * b;
      }
    // row c of this lane's stencil: slot ((i * ne + c) * 8 + sl); row 0 holds
    // the element's own terms
    constexpr int SW = GEO ? 10 : 4;   // doubles per row slot
    double* rb = w.rowbar + (size_t(i) * ne * 8 + sl) * SW;
    constexpr int RB = 8 * SW;
    if (!valid) {
#pragma unroll
      for (int v = 0; v < 4; ++v) rb[v] = sl == 7 ? q0b[v] : 0.0;
      if (GEO) {
#pragma unroll
        for (int c = 0; c < 6; ++c) rb[4 + c] = 0.0;
      }
      continue;
    }
    // weights: om_s = lambda_s / (sigma_s + eps)^8, W = sum om_s w_s / sum om_s
    double omb = 0.0;
#pragma unroll
    for (int l = 0; l < nu; ++l)
#pragma unroll
      for (int v = 0; v < 4; ++v) omb += Wb[l][v] * (ws[l][v] - W[l][v]);
    omb /= Ssum;
    const double sigb = omb * (-8.0) * om / (sig + P.eps);
    double u[nu][4];   // wbar_s, then R^-T wbar_s, then R^-1 R^-T wbar_s
#pragma unroll
    for (int l = 0; l < nu; ++l)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double t = 0.0;
#pragma unroll
        for (int m = 0; m < nu; ++m) t += (MonoBasis<M>::c.sig[l][m] + MonoBasis<M>::c.sig[m][l]) * ws[m][v];
        u[l][v] = (om / Ssum) * Wb[l][v] + sigb * t;
      }
#pragma unroll
    for (int k = 0; k < nu; ++k)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double t = u[k][v];
#pragma unroll
        for (int c2 = 0; c2 < k; ++c2) t -= R[c2][k] * u[c2][v];
        u[k][v] = t / R[k][k];
      }
#pragma unroll
    for (int k = nu - 1; k >= 0; --k)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double t = u[k][v];
#pragma unroll
        for (int c2 = k + 1; c2 < nu; ++c2) t -= R[k][c2] * u[c2][v];
        u[k][v] = t / R[k][k];
      }
    // right-hand sides b_c = Q_j - Q_i: their adjoints are a_c . u
    double sumb[4] = {0.0, 0.0, 0.0, 0.0};
    double Xib[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
    for (int c = 1; c < ne; ++c) {
      double xv[6], qv[4];
      const double* Xj = row(c, xv, qv);
      double a[nu], bb[4];
      ls_row<M>(Xj, Xi, e1x, e1y, e2x, e2y, idet, a);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double t = 0.0;
#pragma unroll
        for (int l = 0; l < nu; ++l) t += a[l] * u[l][v];
        rb[c * RB + v] = t;
        sumb[v] += t;
        bb[v] = t;
      }
      if (GEO) {
        double ab[nu], xj[6], Xjb[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int l = 0; l < nu; ++l) ab[l] = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double r = qv[v] - Qi[v];
#pragma unroll
          for (int l = 0; l < nu; ++l) r -= a[l] * ws[l][v];
#pragma unroll
          for (int l = 0; l < nu; ++l) ab[l] += r * u[l][v] - bb[v] * ws[l][v];
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) xj[k] = Xj[k];
        lag::ls_row_geom_vjp<M>(xj, Xi, ab, Xjb, Xib);
        double* xo = rb + c * RB + 4;
#pragma unroll
        for (int k = 0; k < 6; ++k) xo[k] = Xjb[k];
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) rb[v] = -sumb[v];
    if (GEO) {
      double* xo = rb + 4;
#pragma unroll
      for (int k = 0; k < 6; ++k) xo[k] = Xib[k];
    }
  }
}

// Metric of the fixed affine map of element i: xi_x, xi_y, eta_x, eta_y.
__device__ inline void affine_metric(const double X[6], double m[4]) {
  const double e1x = X[2] - X[0], e1y = X[3] - X[1], e2x = X[4] - X[0], e2y = X[5] - X[1];
  const double det = e1x * e2y - e2x * e1y;
  m[0] = e2y / det;
  m[1] = -e2x / det;
  m[2] = -e1y / det;
  m[3] = e1x / det;
}

// Predictor sweeps from the reconstruction, each iterate kept; edge traces.
// One lane per element; nodal data element-minor in the sweep store.
template <int M>
__global__ void __launch_bounds__(TPB) k_adj_pred_fwd(Dev d, const Tables* __restrict__ tb, Params P,
                                                      AdjWork w, double dt) {
  using S = AZ<M>;
  constexpr int nb = S::nb, T = S::T, nG = S::nG, QS = S::QS;
  const int NE = d.NE;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < NE; i += gridDim.x * blockDim.x) {
    const double* ri = d.rec + size_t(i) * S::RS;
    double X[6], mt[4];
#pragma unroll
    for (int c = 0; c < 6; ++c) X[c] = ri[XE + c];
    affine_metric(X, mt);
    double q[nb][T][4];
    const double* wn = w.wnod + size_t(i) * S::WS;
#pragma unroll
    for (int m = 0; m < nb; ++m)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double x = wn[m * 4 + v];
#pragma unroll
        for (int t = 0; t < T; ++t) q[m][t][v] = x;
      }
#pragma unroll 1
    for (int k = 0; k < P.npic; ++k) {
      double* st = w.sweeps + size_t(k) * QS * NE + i;
#pragma unroll
      for (int m = 0; m < nb; ++m)
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
          for (int v = 0; v < 4; ++v) st[size_t((m * T + t) * 4 + v) * NE] = q[m][t][v];
      double qn[nb][M][4];
#pragma unroll
      for (int m = 0; m < nb; ++m)
#pragma unroll
        for (int r = 0; r < M; ++r)
#pragma unroll
          for (int v = 0; v < 4; ++v) qn[m][r][v] = tb->Bt[r] * q[m][0][v];
#pragma unroll
      for (int t = 0; t < T; ++t) {
        double f[nb][4], g[nb][4];
#pragma unroll
        for (int m = 0; m < nb; ++m) euler_fg(q[m][t], P.gamma, f[m], g[m]);
#pragma unroll
        for (int kk = 0; kk < nb; ++kk)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            double fx = 0.0, fe = 0.0, gx = 0.0, ge = 0.0;
#pragma unroll
            for (int m = 0; m < nb; ++m) {
              fx += tb->Dxi[kk][m] * f[m][v];
              fe += tb->Deta[kk][m] * f[m][v];
              gx += tb->Dxi[kk][m] * g[m][v];
              ge += tb->Deta[kk][m] * g[m][v];
            }
            const double s = mt[0] * fx + mt[2] * fe + mt[1] * gx + mt[3] * ge;
#pragma unroll
            for (int r = 0; r < M; ++r) qn[kk][r][v] += dt * tb->At[r][t] * (-s);
          }
      }
#pragma unroll
      for (int m = 0; m < nb; ++m)
#pragma unroll
        for (int r = 0; r < M; ++r)
#pragma unroll
          for (int v = 0; v < 4; ++v) q[m][r + 1][v] = qn[m][r][v];
    }
    double* av = w.avg + size_t(i) * T * 4;
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double s = 0.0;
#pragma unroll
        for (int m = 0; m < nb; ++m) s += tb->amean[m] * q[m][t][v];
        av[t * 4 + v] = s;
      }
    double* tr = w.trace + size_t(i) * S::TS;
#pragma unroll
    for (int e = 0; e < 3; ++e)
#pragma unroll
      for (int g = 0; g < nG; ++g)
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            double s = 0.0;
#pragma unroll
            for (int m = 0; m < nb; ++m) s += tb->edge[e][g][m] * q[m][t][v];
            tr[((e * nG + g) * T + t) * 4 + v] = s;
          }
  }
}

// Adjoint of the fluxes through the space-time faces of the fixed edges.
template <int M>
__global__ void __launch_bounds__(TPB) k_adj_patch(Dev d, const Tables* __restrict__ tb, Params P,
                                                   AdjWork w, double dt) {
  using S = AZ<M>;
  constexpr int T = S::T, nG = S::nG, TS = S::TS;
  const int NE = d.NE, NV = d.NV, NF = d.NF;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < NF; e += gridDim.x * blockDim.x) {
    const int a = d.e_a[e], b = d.e_b[e];
    const int L = d.e_L[e], el = d.e_el[e], R = d.e_R[e], er = d.e_er[e], bc = d.e_bc[e];
    const double P1[3] = {d.X[a], d.X[NV + a], 0.0};
    const double P2[3] = {d.X[b], d.X[NV + b], 0.0};
    const double P3[3] = {d.X[b], d.X[NV + b], dt};
    const double P4[3] = {d.X[a], d.X[NV + a], dt};
    // flux adjoint: Q_L' = Q_L - G / |T_L|, Q_R' = Q_R + G / |T_R|
    double Gb[4];
    const double AL = d.rec[size_t(L) * S::RS + AO];
    const double AR = R >= 0 ? d.rec[size_t(R) * S::RS + AO] : 1.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Gb[v] = -w.qbar_next[size_t(v) * NE + L] / AL;
      if (R >= 0) Gb[v] += w.qbar_next[size_t(v) * NE + R] / AR;
    }
    const double* trL = w.trace + size_t(L) * TS + el * nG * T * 4;
    const double* trR = R >= 0 ? w.trace + size_t(R) * TS + er * nG * T * 4 : trL;
    const bool open_edge = R < 0 && bc != 2;
    const double* avL = w.avg + size_t(L) * T * 4;
    double bL[nG][T][4], bR[nG][T][4], bA[T][4];
#pragma unroll
    for (int t = 0; t < T; ++t) {
#pragma unroll
      for (int g = 0; g < nG; ++g)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          bL[g][t][v] = 0.0;
          bR[g][t][v] = 0.0;
        }
#pragma unroll
      for (int v = 0; v < 4; ++v) bA[t][v] = 0.0;
    }
#pragma unroll
    for (int gq = 0; gq < nG; ++gq) {
      const double c = tb->gchi[gq];
#pragma unroll
      for (int h = 0; h < nG; ++h) {
        const double tt = tb->gchi[h];
        const double wgt = tb->gw[gq] * tb->gw[h];
        double dchi[3], dtau[3], N[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          dchi[k] = (1.0 - tt) * (P2[k] - P1[k]) + tt * (P3[k] - P4[k]);
          dtau[k] = (1.0 - c) * (P4[k] - P1[k]) + c * (P3[k] - P2[k]);
        }
        N[0] = dchi[1] * dtau[2] - dchi[2] * dtau[1];
        N[1] = dchi[2] * dtau[0] - dchi[0] * dtau[2];
        N[2] = dchi[0] * dtau[1] - dchi[1] * dtau[0];
        // corner ticks 0, 0, 1, 1 of a one-tick step: tau at the point
        const double tk = c * tt + (1.0 - c) * tt;
        double l[T];
        time_basis<M>(tk, l);
        double ql[4], qr[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double s = 0.0, s2 = 0.0;
#pragma unroll
          for (int t = 0; t < T; ++t) {
            s += l[t] * trL[(gq * T + t) * 4 + v];
            s2 += l[t] * trR[((nG - 1 - gq) * T + t) * 4 + v];
          }
          ql[v] = s;
          qr[v] = s2;
        }
        double nx = 0.0, ny = 0.0;
        if (R < 0 && bc == 2) {
          const double inxy = 1.0 / sqrt(N[0] * N[0] + N[1] * N[1]);
          nx = N[0] * inxy;
          ny = N[1] * inxy;
          const double mn = ql[1] * nx + ql[2] * ny;
          qr[0] = ql[0];
          qr[1] = ql[1] - 2.0 * mn * nx;
          qr[2] = ql[2] - 2.0 * mn * ny;
          qr[3] = ql[3];
        } else if (open_edge) {
          // transmissive: the inner element's predicted mean at this time
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            double s = 0.0;
#pragma unroll
            for (int t = 0; t < T; ++t) s += l[t] * avL[t * 4 + v];
            qr[v] = s;
          }
        }
        double Gw[4], qlb[4] = {0, 0, 0, 0}, qrb[4] = {0, 0, 0, 0};
#pragma unroll
        for (int v = 0; v < 4; ++v) Gw[v] = wgt * Gb[v];
        if (P.flux == ADER_FLUX_HLL)
          hll_vjp(ql, qr, N, P.gamma, Gw, qlb, qrb);
        else
          rusanov_vjp(ql, qr, N, P.gamma, Gw, qlb, qrb);
        if (R >= 0) {
#pragma unroll
          for (int t = 0; t < T; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) bR[nG - 1 - gq][t][v] += l[t] * qrb[v];
        } else if (bc == 2) {
          // the mirror map is a symmetric reflection of the momentum
          const double mb = qrb[1] * nx + qrb[2] * ny;
          qlb[0] += qrb[0];
          qlb[1] += qrb[1] - 2.0 * mb * nx;
          qlb[2] += qrb[2] - 2.0 * mb * ny;
          qlb[3] += qrb[3];
        } else {
#pragma unroll
          for (int t = 0; t < T; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) bA[t][v] += l[t] * qrb[v];
        }
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
          for (int v = 0; v < 4; ++v) bL[gq][t][v] += l[t] * qlb[v];
      }
    }
    double* oL = w.tbar + size_t(L) * TS + el * nG * T * 4;
#pragma unroll
    for (int g = 0; g < nG; ++g)
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) oL[(g * T + t) * 4 + v] = bL[g][t][v];
    if (open_edge) {
      // adjoint of the inner element's means, in this edge's own slot
      double* aL = w.abar + size_t(e) * T * 4;
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) aL[t * 4 + v] = bA[t][v];
    }
    if (R >= 0) {
      double* oR = w.tbar + size_t(R) * TS + er * nG * T * 4;
#pragma unroll
      for (int g = 0; g < nG; ++g)
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
          for (int v = 0; v < 4; ++v) oR[(g * T + t) * 4 + v] = bR[g][t][v];
    }
  }
}

// Predictor sweeps in reverse: trace adjoint -> adjoint of the reconstruction.
template <int M>
__global__ void __launch_bounds__(TPB) k_adj_pred_rev(Dev d, const Tables* __restrict__ tb, Params P,
                                                      AdjWork w, double dt) {
  using S = AZ<M>;
  constexpr int nb = S::nb, T = S::T, nG = S::nG, QS = S::QS;
  const int NE = d.NE;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < NE; i += gridDim.x * blockDim.x) {
    const double* ri = d.rec + size_t(i) * S::RS;
    double X[6], mt[4];
#pragma unroll
    for (int c = 0; c < 6; ++c) X[c] = ri[XE + c];
    affine_metric(X, mt);
    // adjoint of the means, from the element's transmissive edges (if any)
    double ab[T][4];
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) ab[t][v] = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int e = d.elem_edges[k * NE + i];
      if (d.e_R[e] < 0 && d.e_bc[e] != 2) {
        const double* a = w.abar + size_t(e) * T * 4;
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
          for (int v = 0; v < 4; ++v) ab[t][v] += a[t * 4 + v];
      }
    }
    double qb[nb][T][4];
    const double* tb_i = w.tbar + size_t(i) * S::TS;
#pragma unroll
    for (int m = 0; m < nb; ++m)
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double s = 0.0;
#pragma unroll
          for (int e = 0; e < 3; ++e)
#pragma unroll
            for (int g = 0; g < nG; ++g) s += tb->edge[e][g][m] * tb_i[((e * nG + g) * T + t) * 4 + v];
          qb[m][t][v] = s + tb->amean[m] * ab[t][v];
        }
#pragma unroll 1
    for (int k = P.npic - 1; k >= 0; --k) {
      const double* st = w.sweeps + size_t(k) * QS * NE + i;
      // q_new[m][r+1] = Bt[r] q[m][0] + dt sum_t At[r][t] P[m][t];  q_new[m][0] = q[m][0]
      double nb0[nb][4];
#pragma unroll
      for (int m = 0; m < nb; ++m)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double s = qb[m][0][v];
#pragma unroll
          for (int r = 0; r < M; ++r) s += tb->Bt[r] * qb[m][r + 1][v];
          nb0[m][v] = s;
        }
      double nq[nb][T][4];
#pragma unroll
      for (int t = 0; t < T; ++t) {
        // Pbar at time node t for every spatial node
        double Pb[nb][4];
#pragma unroll
        for (int m = 0; m < nb; ++m)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            double s = 0.0;
#pragma unroll
            for (int r = 0; r < M; ++r) s += tb->At[r][t] * qb[m][r + 1][v];
            Pb[m][v] = dt * s;
          }
        // P[kk] = -sum_m (xi_x Dxi + eta_x Deta)[kk][m] f[m] + (xi_y Dxi + eta_y Deta)[kk][m] g[m]
#pragma unroll
        for (int m = 0; m < nb; ++m) {
          double fb[4], gb[4], q[4], acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            double ax = 0.0, ae = 0.0;
#pragma unroll
            for (int kk = 0; kk < nb; ++kk) {
              ax += tb->Dxi[kk][m] * Pb[kk][v];
              ae += tb->Deta[kk][m] * Pb[kk][v];
            }
            fb[v] = -(mt[0] * ax + mt[2] * ae);
            gb[v] = -(mt[1] * ax + mt[3] * ae);
            q[v] = st[size_t((m * T + t) * 4 + v) * NE];
          }
          euler_fg_vjp(q, P.gamma, fb, gb, acc);
#pragma unroll
          for (int v = 0; v < 4; ++v) nq[m][t][v] = acc[v] + (t == 0 ? nb0[m][v] : 0.0);
        }
      }
#pragma unroll
      for (int m = 0; m < nb; ++m)
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
          for (int v = 0; v < 4; ++v) qb[m][t][v] = nq[m][t][v];
    }
    // the first iterate repeats the reconstruction at every time node
    double* wb = w.wbar + size_t(i) * S::WS;
#pragma unroll
    for (int m = 0; m < nb; ++m)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < T; ++t) s += qb[m][t][v];
        wb[m * 4 + v] = s;
      }
  }
}

// ---------------------------------------------------------------------------
// Adjoint of one global step with the mesh moving with the fluid (V = v in eq.
// ODEmesh): (Q^n, X^n) -> (Q^{n+1}, X^{n+1}) for a fixed dt. Forward:
// reconstruction on the current geometry, the predictor of the PDE and the
// mesh ODE (eqs. CGfinal, VCG, newVertPos), the node solver (eqs. eqnNScs,
// eqn.NScs.weights, NodesVel, eqn.newVertex over the whole step), the fluxes
// over the bilinear space-time patches of the moving edges (eqs.
// eqn.spacetimenodes, G_ij, eqn.STint) and the update with the new areas (eq.
// PDEfinal). Reverse, each sum in a fixed order (no atomics): patch adjoints
// per edge; update adjoints per element; node solver adjoints per node, into
// (element, vertex) slots; predictor in reverse per element; reconstruction
// in reverse with row slots; gathers per element and per node.
// ---------------------------------------------------------------------------

// The edges of node k, each once: those of the ring elements j at local edges
// lv (node = a) and lv + 2 (node = b) of which j is the left element.
template <class F>
__device__ inline void node_edges(const Dev& d, int k, F f) {
  const int NE = d.NE;
  for (int r = d.ring_ptr[k]; r < d.ring_ptr[k + 1]; ++r) {
    const int j = d.ring_ent[r] >> 2, lv = d.ring_ent[r] & 3;
    const int ea = d.elem_edges[lv * NE + j], eb = d.elem_edges[((lv + 2) % 3) * NE + j];
    if (d.e_L[ea] == j) f(ea, 0);
    if (d.e_L[eb] == j) f(eb, 1);
  }
}

// Positions (from the caller or the context) and averages, vertices, areas.
template <int M>
__global__ void __launch_bounds__(TPB) k_lag_geom(Dev d, LagWork w, int x_from_ctx, int q_from_ctx) {
  const int NE = d.NE, NV = d.NV;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < NV && x_from_ctx; k += gridDim.x * blockDim.x) {
    w.xcopy[2 * k] = d.X[k];
    w.xcopy[2 * k + 1] = d.X[NV + k];
  }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < NE; i += gridDim.x * blockDim.x) {
    if (q_from_ctx) {
      const double* r = d.rec + size_t(i) * AZ<M>::RS;
#pragma unroll
      for (int v = 0; v < 4; ++v) w.a.qcopy[size_t(v) * NE + i] = r[QO + v];
    }
    const double* X = x_from_ctx ? nullptr : w.x;
    double xe[6];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int n = d.tri[c * NE + i];
      xe[2 * c] = X ? X[2 * n] : d.X[n];
      xe[2 * c + 1] = X ? X[2 * n + 1] : d.X[NV + n];
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) w.xe[size_t(i) * 6 + c] = xe[c];
    w.area[i] = lag::area3(xe);
  }
}

// Orders LDS accesses among the lanes of one wavefront (the lanes of an
// element's predictor always share one, and the LDS serves a wavefront's
// accesses in issue order, so only the compiler's reordering is fenced).
__device__ inline void lag_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lane layout of the moving-mesh predictor kernels: one lane per spatial node
// of the nodal basis, floor(64 / nb) elements per wavefront (the spare lanes
// of a wavefront exchange into a slot of their own); LDS holds NX values per
// node of each element.
template <int M>
struct LP {
  static constexpr int nb = (M + 1) * (M + 2) / 2, T = M + 1, nG = M + 1, G = nb;
  static constexpr int EPW = 64 / nb, WPB = TPB / 64, SLOTS = EPW * WPB;
  static constexpr int NX = 28;
  static constexpr int LSTR = NX * G + 2;
  static constexpr int QS = nb * T * 4;
};

// Predictor iterate k of element i, time node t, variable v, spatial node m:
// the nb nodes of an element adjacent, then the elements, so that the lanes of
// a wavefront (ten elements x six nodes at M = 2) touch one contiguous run.
template <int M>
__device__ inline size_t keep_at(int k, int t, int v, int i, int m, int NE) {
  return ((size_t(k * (M + 1) + t) * 4 + v) * NE + i) * LP<M>::nb + m;
}

// Predictor with the mesh ODE (eqs. CGfinal, VCG, newVertPos), one lane per
// spatial node: each node's space-time values and trajectory stay in its
// lane, the spatial derivatives at a node take the element's other nodes
// through LDS. Every iterate is kept (element-minor) for the reverse sweeps;
// traces, means and vertex velocities as in the forward step.
// LTS: the elements of lw.going_list, each with its own step (ticks x
// tick length) from the state lw.s1; only the iterates are kept.
template <int M, bool LTS = false>
__global__ void __launch_bounds__(TPB) k_lag_pred_fwd(Dev d, const Tables* __restrict__ tb, Params P,
                                                      LagWork w, double dt_all, LtsWork lz) {
  using S = AZ<M>;
  using L = LP<M>;
  constexpr int nb = L::nb, T = L::T, nG = L::nG, G = L::G, EPW = L::EPW, SLOTS = L::SLOTS;
  constexpr int NPT = 1 + 3 * nG;
  __shared__ double lds[(SLOTS + L::WPB) * L::LSTR];
  const int NE = d.NE;
  const double gam = P.gamma;
  const double vs = P.lagrangian ? 1.0 : 0.0;   // mesh velocity V = v, or V = 0 (fixed mesh)
  const int wv = threadIdx.x / 64, lw = threadIdx.x % 64;
  const bool spare = lw >= EPW * G;
  const int slot = spare ? SLOTS + wv : wv * EPW + lw / G;
  const int m = spare ? lw - EPW * G : lw % G;
  double* const my = lds + slot * L::LSTR;
  double Dx[nb], De[nb];
#pragma unroll
  for (int k = 0; k < nb; ++k) {
    Dx[k] = tb->Dxi[m][k];
    De[k] = tb->Deta[m][k];
  }
  double nxi, neta;
  lag::lattice<M>(m, nxi, neta);
  const int n_el = LTS ? lz.counts[1] : NE;
  for (int base = blockIdx.x * SLOTS; base < n_el; base += gridDim.x * SLOTS) {
    const int idx = spare ? -1 : base + slot;
    const bool live = idx >= 0 && idx < n_el;
    const int i = !live ? -1 : (LTS ? lz.going_list[idx] : idx);
    const double dt = LTS ? (live ? double(lz.s1.ts[i].step) * lz.delta : 1.0) : dt_all;
    double q[T][4], x[T][2], x0[2];
    if (live) {
      const double* X = LTS ? lz.s1.rec + size_t(i) * S::RS + XE : w.xe + size_t(i) * 6;
      x0[0] = X[0] + (X[2] - X[0]) * nxi + (X[4] - X[0]) * neta;
      x0[1] = X[1] + (X[3] - X[1]) * nxi + (X[5] - X[1]) * neta;
      const double* wn = (LTS ? lz.s1.wnod : w.a.wnod) + size_t(i) * S::WS + m * 4;
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) q[t][v] = wn[v];
    } else {
      // idle lanes: the reference triangle at rest
      x0[0] = nxi;
      x0[1] = neta;
#pragma unroll
      for (int t = 0; t < T; ++t) {
        q[t][0] = 1.0;
        q[t][1] = q[t][2] = 0.0;
        q[t][3] = 2.5;
      }
    }
#pragma unroll 1
    for (int k = 0; k < P.npic; ++k) {
      if (live) {
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
          for (int v = 0; v < 4; ++v) w.keep[keep_at<M>(k, t, v, i, m, NE)] = q[t][v];
      }
      // mesh ODE of this node
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        x[0][c] = x0[c];
#pragma unroll
        for (int r = 0; r < M; ++r) {
          double s = 0.0;
#pragma unroll
          for (int t = 0; t < T; ++t) s += tb->At[r][t] * q[t][1 + c] / q[t][0];
          x[r + 1][c] = tb->Bt[r] * x0[c] + dt * (vs * s);
        }
      }
      double qn[M][4];
#pragma unroll
      for (int r = 0; r < M; ++r)
#pragma unroll
        for (int v = 0; v < 4; ++v) qn[r][v] = tb->Bt[r] * q[0][v];
#pragma unroll
      for (int t = 0; t < T; ++t) {
        double f[4], g[4];
        lag::euler_f_g(q[t], gam, f, g);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          my[v * G + m] = q[t][v];
          my[(4 + v) * G + m] = f[v];
          my[(8 + v) * G + m] = g[v];
        }
        my[12 * G + m] = x[t][0];
        my[13 * G + m] = x[t][1];
        lag_wave_sync();
        double xx = 0, xe = 0, yx = 0, ye = 0;
#pragma unroll
        for (int kk = 0; kk < nb; ++kk) {
          xx += Dx[kk] * my[12 * G + kk];
          xe += De[kk] * my[12 * G + kk];
          yx += Dx[kk] * my[13 * G + kk];
          ye += De[kk] * my[13 * G + kk];
        }
        double xtau = 0, ytau = 0;
#pragma unroll
        for (int r = 0; r < T; ++r) {
          xtau += tb->Dt[t][r] * x[r][0];
          ytau += tb->Dt[t][r] * x[r][1];
        }
        const double det = xx * ye - xe * yx;
        const double xi_x = ye / det, xi_y = -xe / det, eta_x = -yx / det, eta_y = xx / det;
        const double xt = xtau / dt, yt = ytau / dt;
        const double xi_t = -(xi_x * xt + xi_y * yt), eta_t = -(eta_x * xt + eta_y * yt);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double dqx = 0, dqe = 0, dfx = 0, dfe = 0, dgx = 0, dge = 0;
#pragma unroll
          for (int kk = 0; kk < nb; ++kk) {
            dqx += Dx[kk] * my[v * G + kk];
            dqe += De[kk] * my[v * G + kk];
            dfx += Dx[kk] * my[(4 + v) * G + kk];
            dfe += De[kk] * my[(4 + v) * G + kk];
            dgx += Dx[kk] * my[(8 + v) * G + kk];
            dge += De[kk] * my[(8 + v) * G + kk];
          }
          const double Pv = -(dqx * xi_t + dqe * eta_t + dfx * xi_x + dfe * eta_x + dgx * xi_y + dge * eta_y);
#pragma unroll
          for (int r = 0; r < M; ++r) qn[r][v] += dt * tb->At[r][t] * Pv;
        }
        lag_wave_sync();
      }
#pragma unroll
      for (int r = 0; r < M; ++r)
#pragma unroll
        for (int v = 0; v < 4; ++v) q[r + 1][v] = qn[r][v];
    }
    if (live) {
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) w.keep[keep_at<M>(P.npic, t, v, i, m, NE)] = q[t][v];
    }
    if (LTS) continue;   // traces, means and velocities are in the saved state
    if (live) {
#pragma unroll
      for (int kv = 0; kv < 3; ++kv) {
        if (tb->vtx[kv] != m) continue;
        double* vv = w.vvel + (size_t(i) * 3 + kv) * T * 2;
#pragma unroll
        for (int t = 0; t < T; ++t) {
          vv[2 * t] = q[t][1] / q[t][0];
          vv[2 * t + 1] = q[t][2] / q[t][0];
        }
      }
    }
    // cell means and edge traces, one time slice at a time through LDS; lane m
    // evaluates points m, m + G, ... (point 0 the mean, 1 + e nG + gq the Gauss
    // point gq of edge e)
#pragma unroll
    for (int t = 0; t < T; ++t) {
#pragma unroll
      for (int v = 0; v < 4; ++v) my[v * G + m] = q[t][v];
      lag_wave_sync();
      if (live) {
        for (int pt = m; pt < NPT; pt += G) {
          const double* c = pt == 0 ? tb->amean : tb->edge[(pt - 1) / nG][(pt - 1) % nG];
          double* out = pt == 0 ? w.a.avg + size_t(i) * T * 4 + t * 4
                                : w.a.trace + size_t(i) * S::TS + ((pt - 1) * T + t) * 4;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            double s = 0.0;
#pragma unroll
            for (int kk = 0; kk < nb; ++kk) s += c[kk] * my[v * G + kk];
            out[v] = s;
          }
        }
      }
      lag_wave_sync();
    }
  }
}

// Node solver: mass-weighted ring mean of the time-averaged vertex velocities,
// slip walls slide and pinned nodes stay; new positions.
template <int M>
__global__ void __launch_bounds__(TPB) k_lag_node_fwd(Dev d, const Tables* __restrict__ tb, LagWork w,
                                                      double dt) {
  constexpr int T = M + 1;
  const int NE = d.NE, NV = d.NV;
  double I[T];
  lag::tint01<M>(*tb, I);
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < NV; k += gridDim.x * blockDim.x) {
    double num[2] = {0.0, 0.0}, den = 0.0;
    for (int r = d.ring_ptr[k]; r < d.ring_ptr[k + 1]; ++r) {
      const int j = d.ring_ent[r] >> 2, lv = d.ring_ent[r] & 3;
      const double* vv = w.vvel + (size_t(j) * 3 + lv) * T * 2;
      double vb[2] = {0.0, 0.0};
#pragma unroll
      for (int q = 0; q < T; ++q) {
        vb[0] += I[q] * vv[2 * q];
        vb[1] += I[q] * vv[2 * q + 1];
      }
      const double mu = w.a.q[j] * w.area[j];
      num[0] += mu * vb[0];
      num[1] += mu * vb[1];
      den += mu;
    }
    const double Vx = num[0] / den, Vy = num[1] / den;
    w.vraw[2 * k] = Vx;
    w.vraw[2 * k + 1] = Vy;
    w.den[k] = den;
    double Wx = Vx, Wy = Vy;
    if (d.wall_pin[k]) {
      Wx = Wy = 0.0;
    } else {
      const double nx = d.wall_n[k], ny = d.wall_n[NV + k];
      const double vn = Vx * nx + Vy * ny;
      Wx -= vn * nx;
      Wy -= vn * ny;
    }
    const double* x = w.x + 2 * size_t(k);
    w.xn[2 * k] = x[0] + dt * Wx;
    w.xn[2 * k + 1] = x[1] + dt * Wy;
  }
  (void)NE;
}

template <int M>
__global__ void __launch_bounds__(TPB) k_lag_area_new(Dev d, LagWork w) {
  const int NE = d.NE;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < NE; i += gridDim.x * blockDim.x) {
    double xe[6];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int n = d.tri[c * NE + i];
      xe[2 * c] = w.xn[2 * n];
      xe[2 * c + 1] = w.xn[2 * n + 1];
    }
    w.an[i] = lag::area3(xe);
  }
}

// Per edge: the patch flux (into the two (element, edge) slots, inflow
// positive) and, in the same pass, its adjoint for Gbar = -Qbar'_L / |T_L'| + Qbar'_R / |T_R'|
// onto the traces, the inner element's means (transmissive edge) and the
// four corners.
template <int M>
__global__ void __launch_bounds__(TPB) k_lag_patch(Dev d, const Tables* __restrict__ tb, Params P, LagWork w,
                                                   double dt) {
  using S = AZ<M>;
  constexpr int T = S::T, nG = S::nG, TS = S::TS, NT = nG * T * 4;
  const int NE = d.NE, NF = d.NF;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < NF; e += gridDim.x * blockDim.x) {
    const int a = d.e_a[e], b = d.e_b[e];
    const int L = d.e_L[e], el = d.e_el[e], R = d.e_R[e], er = d.e_er[e];
    const bool hasR = R >= 0;
    const int kind = hasR ? lag::INTERIOR : (d.e_bc[e] == 2 ? lag::SLIP : lag::TRANSMISSIVE);
    const double xa[2] = {w.x[2 * a], w.x[2 * a + 1]}, xb[2] = {w.x[2 * b], w.x[2 * b + 1]};
    const double xan[2] = {w.xn[2 * a], w.xn[2 * a + 1]}, xbn[2] = {w.xn[2 * b], w.xn[2 * b + 1]};
    const double* trL = w.a.trace + size_t(L) * TS + el * NT;
    const double* trR = hasR ? w.a.trace + size_t(R) * TS + er * NT : trL;
    const double* avL = w.a.avg + size_t(L) * T * 4;
    double Gb[4];
    const double anL = w.an[L], anR = hasR ? w.an[R] : 1.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Gb[v] = -w.a.qbar_next[size_t(v) * NE + L] / anL;
      if (hasR) Gb[v] += w.a.qbar_next[size_t(v) * NE + R] / anR;
    }
    double G[4] = {0.0, 0.0, 0.0, 0.0}, bA[T * 4];
#pragma unroll
    for (int k = 0; k < T * 4; ++k) bA[k] = 0.0;
    double c[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double* oL = w.a.tbar + size_t(L) * TS + el * NT;
    double* oR = hasR ? w.a.tbar + size_t(R) * TS + er * NT : oL;
    lag::patch_flux_vjp<M>(*tb, P.gamma, xa, xb, xan, xbn, dt, trL, trR, avL, kind, Gb, G, oL, oR, bA, c, c + 2,
                           c + 4, c + 6, P.flux == ADER_FLUX_HLL);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      w.gslot[(size_t(L) * 3 + el) * 4 + v] = -G[v];
      if (hasR) w.gslot[(size_t(R) * 3 + er) * 4 + v] = G[v];
    }
    if (kind == lag::TRANSMISSIVE) {
      double* aL = w.a.abar + size_t(e) * T * 4;
#pragma unroll
      for (int k = 0; k < T * 4; ++k) aL[k] = bA[k];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) w.xs[size_t(e) * 8 + k] = c[k];
  }
}

// Per element: the update Q' = (|T| Q + sum of inflows) / |T'| and the
// adjoints of its direct inputs: Q (qdir), |T| and |T'| pulled back to the
// old (xeb) and new (xnbe) vertices.
template <int M>
__global__ void __launch_bounds__(TPB) k_lag_update_rev(Dev d, LagWork w) {
  const int NE = d.NE;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < NE; i += gridDim.x * blockDim.x) {
    const double A = w.area[i], An = w.an[i];
    double qn[4], q[4], qb[4], Ab = 0.0, Anb = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double* g = w.gslot + size_t(i) * 12 + v;
      q[v] = w.a.q[size_t(v) * NE + i];
      qn[v] = (A * q[v] + ((g[0] + g[4]) + g[8])) / An;
      qb[v] = w.a.qbar_next[size_t(v) * NE + i];
      Ab += qb[v] * q[v] / An;
      Anb -= qb[v] * qn[v] / An;
      w.qdir[size_t(v) * NE + i] = (A / An) * qb[v];
      if (w.qnext) w.qnext[size_t(v) * NE + i] = qn[v];
    }
    double xe[6], xne[6], g0[6] = {0, 0, 0, 0, 0, 0}, g1[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int n = d.tri[c * NE + i];
      xe[2 * c] = w.xe[size_t(i) * 6 + 2 * c];
      xe[2 * c + 1] = w.xe[size_t(i) * 6 + 2 * c + 1];
      xne[2 * c] = w.xn[2 * n];
      xne[2 * c + 1] = w.xn[2 * n + 1];
    }
    lag::area3_grad(xe, Ab, g0);
    lag::area3_grad(xne, Anb, g1);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      w.a.xeb[size_t(i) * 6 + c] = g0[c];
      w.xnbe[size_t(i) * 6 + c] = g1[c];
    }
  }
}

// Per node: adjoint of the new position (the caller's, the new areas, the
// patch corners at the step end) -> that of the old position (direct part) and
// of the ring's vertex velocities and masses, into (element, vertex) slots.
template <int M>
__global__ void __launch_bounds__(TPB) k_lag_node_rev(Dev d, const Tables* __restrict__ tb, LagWork w,
                                                      double dt) {
  constexpr int T = M + 1;
  const int NV = d.NV;
  double I[T];
  lag::tint01<M>(*tb, I);
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < NV; k += gridDim.x * blockDim.x) {
    double xb[2] = {w.xbar_next[2 * k], w.xbar_next[2 * k + 1]};
    for (int r = d.ring_ptr[k]; r < d.ring_ptr[k + 1]; ++r) {
      const int j = d.ring_ent[r] >> 2, lv = d.ring_ent[r] & 3;
      xb[0] += w.xnbe[size_t(j) * 6 + 2 * lv];
      xb[1] += w.xnbe[size_t(j) * 6 + 2 * lv + 1];
    }
    node_edges(d, k, [&](int e, int isb) {
      xb[0] += w.xs[size_t(e) * 8 + 4 + 2 * isb];
      xb[1] += w.xs[size_t(e) * 8 + 5 + 2 * isb];
    });
    w.xbar[2 * k] = xb[0];
    w.xbar[2 * k + 1] = xb[1];
    if (w.xnext) {
      w.xnext[2 * k] = w.xn[2 * k];
      w.xnext[2 * k + 1] = w.xn[2 * k + 1];
    }
    // x' = x + dt P V, P the (symmetric) wall constraint
    double Vb[2] = {dt * xb[0], dt * xb[1]};
    if (d.wall_pin[k]) {
      Vb[0] = Vb[1] = 0.0;
    } else {
      const double nx = d.wall_n[k], ny = d.wall_n[NV + k];
      const double vn = Vb[0] * nx + Vb[1] * ny;
      Vb[0] -= vn * nx;
      Vb[1] -= vn * ny;
    }
    // V = num / den
    const double den = w.den[k];
    const double numb[2] = {Vb[0] / den, Vb[1] / den};
    const double denb = -(numb[0] * w.vraw[2 * k] + numb[1] * w.vraw[2 * k + 1]);
    for (int r = d.ring_ptr[k]; r < d.ring_ptr[k + 1]; ++r) {
      const int j = d.ring_ent[r] >> 2, lv = d.ring_ent[r] & 3;
      const double* vv = w.vvel + (size_t(j) * 3 + lv) * T * 2;
      double vb[2] = {0.0, 0.0};
#pragma unroll
      for (int q = 0; q < T; ++q) {
        vb[0] += I[q] * vv[2 * q];
        vb[1] += I[q] * vv[2 * q + 1];
      }
      const double mu = w.a.q[j] * w.area[j];
      double* o = w.nslot + (size_t(j) * 3 + lv) * 3;
      o[0] = mu * numb[0];
      o[1] = mu * numb[1];
      o[2] = numb[0] * vb[0] + numb[1] * vb[1] + denb;
    }
  }
}

// Predictor in reverse, one lane per spatial node as in k_lag_pred_fwd: the
// adjoints of the traces, of the means (transmissive edges) and of the vertex
// velocities -> those of the reconstruction's nodal values and of the
// element's vertices; the ring masses rho |T| (qdir, vertices through the
// area). Per sweep and time node the lanes exchange their forward fields,
// then the products their node's equation sends to the other nodes (the
// transposed spatial derivatives).
// LTS: the elements of lw.going_list with their own steps (state lw.s1); the
// adjoints of the traces (g.a.tbar), means (avb) and vertex velocities (vvb)
// are the element's own, added to the reconstruction's and the vertices'
// adjoints and then cleared (the predictor's outputs are overwritten here).
template <int M, bool LTS = false>
__global__ void __launch_bounds__(TPB) k_lag_pred_rev(Dev d, const Tables* __restrict__ tb, Params P,
                                                      LagWork w, double dt_all, LtsWork lz) {
  using S = AZ<M>;
  using L = LP<M>;
  constexpr int nb = L::nb, T = L::T, nG = L::nG, G = L::G, EPW = L::EPW, SLOTS = L::SLOTS;
  __shared__ double lds[(SLOTS + L::WPB) * L::LSTR];
  const int NE = d.NE;
  const double gam = P.gamma;
  const double vs = P.lagrangian ? 1.0 : 0.0;   // mesh velocity V = v, or V = 0 (fixed mesh)
  const int wv = threadIdx.x / 64, lw = threadIdx.x % 64;
  const bool spare = lw >= EPW * G;
  const int slot = spare ? SLOTS + wv : wv * EPW + lw / G;
  const int m = spare ? lw - EPW * G : lw % G;
  double* const my = lds + slot * L::LSTR;
  // this node's rows (its derivatives) and columns (its share of the others')
  double Dx[nb], De[nb], DxT[nb], DeT[nb];
#pragma unroll
  for (int k = 0; k < nb; ++k) {
    Dx[k] = tb->Dxi[m][k];
    De[k] = tb->Deta[m][k];
    DxT[k] = tb->Dxi[k][m];
    DeT[k] = tb->Deta[k][m];
  }
  double I[T];
  lag::tint01<M>(*tb, I);
  double nxi, neta;
  lag::lattice<M>(m, nxi, neta);
  const int n_el = LTS ? lz.counts[1] : NE;
  for (int base = blockIdx.x * SLOTS; base < n_el; base += gridDim.x * SLOTS) {
    const int idx = spare ? -1 : base + slot;
    const bool live = idx >= 0 && idx < n_el;
    const int i = !live ? -1 : (LTS ? lz.going_list[idx] : idx);
    const double dt = LTS ? (live ? double(lz.s1.ts[i].step) * lz.delta : 1.0) : dt_all;
    // the element's trace adjoints into LDS, a share per lane, then every lane
    // reads the ones its node contributes to
    constexpr int NTB = 3 * nG * T * 4;
    if (live) {
      const double* tbi = w.a.tbar + size_t(i) * S::TS;
      for (int c = m; c < NTB; c += G) my[c] = tbi[c];
    }
    lag_wave_sync();
    double x0[2], qb[T][4];
    if (live) {
      const double* X = LTS ? lz.s1.rec + size_t(i) * S::RS + XE : w.xe + size_t(i) * 6;
      x0[0] = X[0] + (X[2] - X[0]) * nxi + (X[4] - X[0]) * neta;
      x0[1] = X[1] + (X[3] - X[1]) * nxi + (X[5] - X[1]) * neta;
      // adjoint of the final iterate at this node: traces, means, vertex velocity
      double ab[T][4];
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) ab[t][v] = LTS ? lz.avb[(size_t(i) * T + t) * 4 + v] : 0.0;
#pragma unroll
      for (int le = 0; le < 3 && !LTS; ++le) {
        const int e = d.elem_edges[le * NE + i];
        if (d.e_R[e] < 0 && d.e_bc[e] != 2) {
          const double* a = w.a.abar + size_t(e) * T * 4;
#pragma unroll
          for (int t = 0; t < T; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) ab[t][v] += a[t * 4 + v];
        }
      }
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double s = tb->amean[m] * ab[t][v];
#pragma unroll
          for (int e = 0; e < 3; ++e)
#pragma unroll
            for (int gq = 0; gq < nG; ++gq) s += tb->edge[e][gq][m] * my[((e * nG + gq) * T + t) * 4 + v];
          qb[t][v] = s;
        }
#pragma unroll
      for (int kv = 0; kv < 3; ++kv) {
        if (tb->vtx[kv] != m) continue;
        const double* o = w.nslot + (size_t(i) * 3 + kv) * 3;
        const double* ov = lz.vvb + (size_t(i) * 3 + kv) * T * 2;
#pragma unroll
        for (int t = 0; t < T; ++t) {
          const double q0 = w.keep[keep_at<M>(P.npic, t, 0, i, m, NE)];
          const double q1 = w.keep[keep_at<M>(P.npic, t, 1, i, m, NE)];
          const double q2 = w.keep[keep_at<M>(P.npic, t, 2, i, m, NE)];
          const double vxb = vs * (LTS ? ov[2 * t] : I[t] * o[0]), vyb = vs * (LTS ? ov[2 * t + 1] : I[t] * o[1]);
          qb[t][0] -= (vxb * q1 + vyb * q2) / (q0 * q0);
          qb[t][1] += vxb / q0;
          qb[t][2] += vyb / q0;
        }
      }
    } else {
      x0[0] = nxi;
      x0[1] = neta;
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) qb[t][v] = 0.0;
    }
    lag_wave_sync();   // the staged trace adjoints are read before the sweeps reuse the buffer
    double x0b[2] = {0.0, 0.0};
#pragma unroll 1
    for (int k = P.npic - 1; k >= 0; --k) {
      double q[T][4];
      if (live) {
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
          for (int v = 0; v < 4; ++v) q[t][v] = w.keep[keep_at<M>(k, t, v, i, m, NE)];
      } else {
#pragma unroll
        for (int t = 0; t < T; ++t) {
          q[t][0] = 1.0;
          q[t][1] = q[t][2] = 0.0;
          q[t][3] = 2.5;
        }
      }
      // this node's trajectory in the sweep
      double x[T][2];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        x[0][c] = x0[c];
#pragma unroll
        for (int r = 0; r < M; ++r) {
          double s = 0.0;
#pragma unroll
          for (int t = 0; t < T; ++t) s += tb->At[r][t] * q[t][1 + c] / q[t][0];
          x[r + 1][c] = tb->Bt[r] * x0[c] + dt * (vs * s);
        }
      }
      // q_out[0] = q[0]; q_out[r+1] = Bt[r] q[0] + dt sum_t At[r][t] P[t]
      double qi[T][4], Pb[T][4], xb[T][2];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double s = qb[0][v];
#pragma unroll
        for (int r = 0; r < M; ++r) s += tb->Bt[r] * qb[r + 1][v];
        qi[0][v] = s;
#pragma unroll
        for (int t = 1; t < T; ++t) qi[t][v] = 0.0;
#pragma unroll
        for (int t = 0; t < T; ++t) {
          double p = 0.0;
#pragma unroll
          for (int r = 0; r < M; ++r) p += tb->At[r][t] * qb[r + 1][v];
          Pb[t][v] = dt * p;
        }
      }
#pragma unroll
      for (int t = 0; t < T; ++t) xb[t][0] = xb[t][1] = 0.0;
#pragma unroll
      for (int t = 0; t < T; ++t) {
        double f[4], g[4];
        lag::euler_f_g(q[t], gam, f, g);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          my[v * G + m] = q[t][v];
          my[(4 + v) * G + m] = f[v];
          my[(8 + v) * G + m] = g[v];
        }
        my[12 * G + m] = x[t][0];
        my[13 * G + m] = x[t][1];
        lag_wave_sync();
        double xx = 0, xe = 0, yx = 0, ye = 0;
#pragma unroll
        for (int kk = 0; kk < nb; ++kk) {
          xx += Dx[kk] * my[12 * G + kk];
          xe += De[kk] * my[12 * G + kk];
          yx += Dx[kk] * my[13 * G + kk];
          ye += De[kk] * my[13 * G + kk];
        }
        double xtau = 0, ytau = 0;
#pragma unroll
        for (int r = 0; r < T; ++r) {
          xtau += tb->Dt[t][r] * x[r][0];
          ytau += tb->Dt[t][r] * x[r][1];
        }
        const double det = xx * ye - xe * yx;
        const double xi_x = ye / det, xi_y = -xe / det, eta_x = -yx / det, eta_y = xx / det;
        const double xt = xtau / dt, yt = ytau / dt;
        const double xi_t = -(xi_x * xt + xi_y * yt), eta_t = -(eta_x * xt + eta_y * yt);
        double xitb = 0, etatb = 0, xixb = 0, xiyb = 0, etaxb = 0, etayb = 0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double dqx = 0, dqe = 0, dfx = 0, dfe = 0, dgx = 0, dge = 0;
#pragma unroll
          for (int kk = 0; kk < nb; ++kk) {
            dqx += Dx[kk] * my[v * G + kk];
            dqe += De[kk] * my[v * G + kk];
            dfx += Dx[kk] * my[(4 + v) * G + kk];
            dfe += De[kk] * my[(4 + v) * G + kk];
            dgx += Dx[kk] * my[(8 + v) * G + kk];
            dge += De[kk] * my[(8 + v) * G + kk];
          }
          const double pb = Pb[t][v];
          xitb -= pb * dqx;
          etatb -= pb * dqe;
          xixb -= pb * dfx;
          etaxb -= pb * dfe;
          xiyb -= pb * dgx;
          etayb -= pb * dge;
        }
        // xi_t = -(xi_x xt + xi_y yt), eta_t = -(eta_x xt + eta_y yt)
        xixb -= xitb * xt;
        xiyb -= xitb * yt;
        etaxb -= etatb * xt;
        etayb -= etatb * yt;
        const double xtb = -(xitb * xi_x + etatb * eta_x), ytb = -(xitb * xi_y + etatb * eta_y);
        const double detb = -(xixb * xi_x + xiyb * xi_y + etaxb * eta_x + etayb * eta_y) / det;
        const double xxb = etayb / det + detb * ye;
        const double yeb = xixb / det + detb * xx;
        const double xeb = -xiyb / det - detb * yx;
        const double yxb = -etaxb / det - detb * xe;
#pragma unroll
        for (int r = 0; r < T; ++r) {
          xb[r][0] += tb->Dt[t][r] * xtb / dt;
          xb[r][1] += tb->Dt[t][r] * ytb / dt;
        }
        lag_wave_sync();
        // what this node's equation sends to every node: the transposed sums
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double pb = Pb[t][v];
          my[v * G + m] = pb * xi_t;
          my[(4 + v) * G + m] = pb * eta_t;
          my[(8 + v) * G + m] = pb * xi_x;
          my[(12 + v) * G + m] = pb * eta_x;
          my[(16 + v) * G + m] = pb * xi_y;
          my[(20 + v) * G + m] = pb * eta_y;
        }
        my[24 * G + m] = xxb;
        my[25 * G + m] = xeb;
        my[26 * G + m] = yxb;
        my[27 * G + m] = yeb;
        lag_wave_sync();
        double fb[4], gb[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double sq = 0.0, sf = 0.0, sg = 0.0;
#pragma unroll
          for (int kk = 0; kk < nb; ++kk) {
            sq += DxT[kk] * my[v * G + kk] + DeT[kk] * my[(4 + v) * G + kk];
            sf += DxT[kk] * my[(8 + v) * G + kk] + DeT[kk] * my[(12 + v) * G + kk];
            sg += DxT[kk] * my[(16 + v) * G + kk] + DeT[kk] * my[(20 + v) * G + kk];
          }
          qi[t][v] -= sq;
          fb[v] = -sf;
          gb[v] = -sg;
        }
        {
          double sx = 0.0, sy = 0.0;
#pragma unroll
          for (int kk = 0; kk < nb; ++kk) {
            sx += DxT[kk] * my[24 * G + kk] + DeT[kk] * my[25 * G + kk];
            sy += DxT[kk] * my[26 * G + kk] + DeT[kk] * my[27 * G + kk];
          }
          xb[t][0] += sx;
          xb[t][1] += sy;
        }
        lag::euler_f_g_vjp(q[t], gam, fb, gb, qi[t]);
        lag_wave_sync();
      }
      // mesh ODE of this node in reverse: x[0] = x0, x[r+1] = Bt[r] x0 + dt sum_t At[r][t] V[t]
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        double s = xb[0][c];
#pragma unroll
        for (int r = 0; r < M; ++r) s += tb->Bt[r] * xb[r + 1][c];
        x0b[c] += s;
      }
#pragma unroll
      for (int t = 0; t < T; ++t) {
        double vb[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          double s = 0.0;
#pragma unroll
          for (int r = 0; r < M; ++r) s += tb->At[r][t] * xb[r + 1][c];
          vb[c] = vs * (dt * s);
        }
        qi[t][0] -= (vb[0] * q[t][1] + vb[1] * q[t][2]) / (q[t][0] * q[t][0]);
        qi[t][1] += vb[0] / q[t][0];
        qi[t][2] += vb[1] / q[t][0];
      }
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) qb[t][v] = qi[t][v];
    }
    // the first iterate repeats the reconstruction at every time node
    if (live) {
      double* wb = w.a.wbar + size_t(i) * S::WS + m * 4;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < T; ++t) s += qb[t][v];
        wb[v] = LTS ? wb[v] + s : s;
      }
    }
    // x0 = (1 - xi - eta) X0 + xi X1 + eta X2: the element's vertex adjoints,
    // summed over its nodes by lane 0
    const double bw[3] = {1.0 - nxi - neta, nxi, neta};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      my[(2 * c) * G + m] = bw[c] * x0b[0];
      my[(2 * c + 1) * G + m] = bw[c] * x0b[1];
    }
    lag_wave_sync();
    if (LTS && live && m == 0) {
      double* xo = w.a.xeb + size_t(i) * 6;
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        double s = 0.0;
#pragma unroll
        for (int kk = 0; kk < nb; ++kk) s += my[c * G + kk];
        xo[c] += s;
      }
      double* av = lz.avb + size_t(i) * T * 4;
#pragma unroll
      for (int k = 0; k < T * 4; ++k) av[k] = 0.0;
      double* vv = lz.vvb + size_t(i) * 3 * T * 2;
#pragma unroll
      for (int k = 0; k < 3 * T * 2; ++k) vv[k] = 0.0;
    }
    if (LTS && live) {
      double* tbi = w.a.tbar + size_t(i) * S::TS;
      for (int c = m; c < NTB; c += G) tbi[c] = 0.0;
    }
    if (!LTS && live && m == 0) {
      double xb6[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        double s = 0.0;
#pragma unroll
        for (int kk = 0; kk < nb; ++kk) s += my[c * G + kk];
        xb6[c] = s;
      }
      // mu = rho |T| of the ring means
      double mub = 0.0;
#pragma unroll
      for (int kv = 0; kv < 3; ++kv) mub += w.nslot[(size_t(i) * 3 + kv) * 3 + 2];
      double xe[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) xe[c] = w.xe[size_t(i) * 6 + c];
      w.qdir[i] += mub * w.area[i];
      lag::area3_grad(xe, mub * w.a.q[i], xb6);
#pragma unroll
      for (int c = 0; c < 6; ++c) w.a.xeb[size_t(i) * 6 + c] += xb6[c];
    }
    lag_wave_sync();
  }
}

// Per node: the old position's adjoint = direct part + ring elements' vertex
// adjoints + the patch corners at the step start.
template <int M>
__global__ void __launch_bounds__(TPB) k_lag_node_gather(Dev d, LagWork w) {
  const int NV = d.NV;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < NV; k += gridDim.x * blockDim.x) {
    double xb[2] = {w.xbar[2 * k], w.xbar[2 * k + 1]};
    for (int r = d.ring_ptr[k]; r < d.ring_ptr[k + 1]; ++r) {
      const int j = d.ring_ent[r] >> 2, lv = d.ring_ent[r] & 3;
      xb[0] += w.a.xeb[size_t(j) * 6 + 2 * lv];
      xb[1] += w.a.xeb[size_t(j) * 6 + 2 * lv + 1];
    }
    node_edges(d, k, [&](int e, int isb) {
      xb[0] += w.xs[size_t(e) * 8 + 2 * isb];
      xb[1] += w.xs[size_t(e) * 8 + 1 + 2 * isb];
    });
    w.xbar[2 * k] = xb[0];
    w.xbar[2 * k + 1] = xb[1];
  }
}

int grid_for(long n) {
  long b = (n + TPB - 1) / TPB;
  if (b < 1) b = 1;
  if (b > 16384) b = 16384;
  return int(b);
}

#define AD_LAUNCH(kern, n, stream, ...)                                                      \
  do {                                                                                       \
    hipLaunchKernelGGL(kern, dim3(grid_for(n)), dim3(TPB), 0, (hipStream_t)(stream),         \
                       __VA_ARGS__);                                                         \
    hipError_t _e = hipGetLastError();                                                       \
    if (_e != hipSuccess) return int(_e);                                                    \
  } while (0)

template <int M>
int adjoint_gts(const Dev& d, const Params& p, const AdjWork& w, double dt, bool from_ctx, void* s) {
  if (from_ctx) AD_LAUNCH(k_adj_state<M>, d.NE, s, d, w);
  AD_LAUNCH((k_adj_recon<M, false>), 8L * d.NE, s, d, d.tab, p, w, LtsWork{});
  AD_LAUNCH(k_adj_pred_fwd<M>, d.NE, s, d, d.tab, p, w, dt);
  AD_LAUNCH(k_adj_patch<M>, d.NF, s, d, d.tab, p, w, dt);
  AD_LAUNCH(k_adj_pred_rev<M>, d.NE, s, d, d.tab, p, w, dt);
  AD_LAUNCH((k_adj_recon<M, true>), 8L * d.NE, s, d, d.tab, p, w, LtsWork{});
  AD_LAUNCH(k_adj_gather<M>, 8L * d.NE, s, d, w);
  return 0;
}

#define AD_LAUNCH_BLOCKS(kern, blocks, stream, ...)                                          \
  do {                                                                                       \
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(TPB), 0, (hipStream_t)(stream), __VA_ARGS__); \
    hipError_t _e = hipGetLastError();                                                       \
    if (_e != hipSuccess) return int(_e);                                                    \
  } while (0)

template <int M>
int adjoint_lagrangian(const Dev& d, const Params& p, LagWork w, double dt, bool qctx, bool xctx, void* s) {
  long pb = (long(d.NE) + LP<M>::SLOTS - 1) / LP<M>::SLOTS;   // predictor blocks: SLOTS elements each
  if (pb > 16384) pb = 16384;
  if (qctx) w.a.q = w.a.qcopy;
  if (xctx) w.x = w.xcopy;
  AD_LAUNCH(k_lag_geom<M>, d.NE > d.NV ? d.NE : d.NV, s, d, w, int(xctx), int(qctx));
  AD_LAUNCH((k_adj_recon<M, false, true>), 8L * d.NE, s, d, d.tab, p, w.a, LtsWork{});
  AD_LAUNCH_BLOCKS(k_lag_pred_fwd<M>, pb, s, d, d.tab, p, w, dt, LtsWork{});
  AD_LAUNCH(k_lag_node_fwd<M>, d.NV, s, d, d.tab, w, dt);
  AD_LAUNCH(k_lag_area_new<M>, d.NE, s, d, w);
  AD_LAUNCH(k_lag_patch<M>, d.NF, s, d, d.tab, p, w, dt);
  AD_LAUNCH(k_lag_update_rev<M>, d.NE, s, d, w);
  AD_LAUNCH(k_lag_node_rev<M>, d.NV, s, d, d.tab, w, dt);
  AD_LAUNCH_BLOCKS(k_lag_pred_rev<M>, pb, s, d, d.tab, p, w, dt, LtsWork{});
  AD_LAUNCH((k_adj_recon<M, true, true>), 8L * d.NE, s, d, d.tab, p, w.a, LtsWork{});
  AdjWork g = w.a;
  g.qbar_next = w.qdir;
  AD_LAUNCH((k_adj_gather<M, true>), 8L * d.NE, s, d, g);
  AD_LAUNCH(k_lag_node_gather<M>, d.NV, s, d, w);
  return 0;
}

// ---------------------------------------------------------------------------
// Local time stepping in reverse, schedule frozen: one cycle (update criterion
// already decided) is the node motion, the swept patches, the update of the
// active elements, their reconstruction from the stencil placed at their new
// tick, and the predictors of those that stay short of the macro-step end.
// Its reverse reads the saved states before (s0) and after (s1) the cycle.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(TPB) k_lts_clear_counts(LtsWork lw) {
  if (blockIdx.x == 0 && threadIdx.x < 3) lw.counts[threadIdx.x] = 0;
}

// Appends the flagged items of one workgroup pass to a global list with one
// atomic per workgroup (atomics on one address serialise); every thread of the
// workgroup calls it. The order of a list is free: each item is processed on
// its own. sh: TPB + 2 ints of LDS.
__device__ inline void block_append(int* list, int* counter, bool flag, int item, int* sh) {
  if (threadIdx.x == 0) sh[TPB] = 0;
  __syncthreads();
  if (flag) sh[atomicAdd(&sh[TPB], 1)] = item;
  __syncthreads();
  const int cnt = sh[TPB];
  if (threadIdx.x == 0) sh[TPB + 1] = cnt ? atomicAdd(counter, cnt) : 0;
  __syncthreads();
  const int base = sh[TPB + 1];
  for (int k = threadIdx.x; k < cnt; k += blockDim.x) list[base + k] = sh[k];
  __syncthreads();
}

// Flags and lists of the cycle from the ticks on both sides of it; all = 1:
// every element updated and predicted, no node moved.
__global__ void __launch_bounds__(TPB) k_lts_marks(Dev d, LtsWork lw, int all) {
  __shared__ int sh[TPB + 2];
  const int NE = d.NE, NV = d.NV;
  for (int base = blockIdx.x * blockDim.x; base < NE; base += gridDim.x * blockDim.x) {
    const int i = base + threadIdx.x;
    int f = 0;
    if (i < NE) {
      f = 3;
      if (!all) {
        const int t0 = lw.s0.ts[i].tick, t1 = lw.s1.ts[i].tick;
        f = t1 != t0 ? (1 | (t1 < MACRO_TICKS ? 2 : 0)) : 0;
      }
      lw.eflag[i] = f;
    }
    block_append(lw.act_list, &lw.counts[0], (f & 1) != 0, i, sh);
    block_append(lw.going_list, &lw.counts[1], (f & 2) != 0, i, sh);
  }
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < NV; k += gridDim.x * blockDim.x)
    lw.nflag[k] = all ? 0 : int(lw.s1.ntick[k] != lw.s0.ntick[k]);
}

// The swept edges (a moved end) listed.
__global__ void __launch_bounds__(TPB) k_lts_edges(Dev d, LtsWork lw) {
  __shared__ int sh[TPB + 2];
  const int NF = d.NF;
  for (int base = blockIdx.x * blockDim.x; base < NF; base += gridDim.x * blockDim.x) {
    const int e = base + threadIdx.x;
    const bool swept = e < NF && (lw.nflag[d.e_a[e]] || lw.nflag[d.e_b[e]]);
    block_append(lw.edge_list, &lw.counts[2], swept, e, sh);
  }
}

// Per element j, 8 lanes: the own terms of its reconstruction (updated j) and
// the rows of updated elements' stencils that name j, through the placement
// in reverse: into j's average and vertices (same tick) or into its
// predictor's means and vertex velocities and its vertices (projected). The
// updated elements' reconstruction adjoints are consumed.
template <int M>
__global__ void __launch_bounds__(TPB) k_lts_gather(Dev d, const Tables* __restrict__ tb, LtsWork lw) {
  using S = AZ<M>;
  constexpr int ne = S::ne, T = M + 1, WS = S::WS;
  constexpr int OA = 10, OV = 10 + 4 * T, NACC = 10 + 10 * T;
  const int NE = d.NE;
  const int sl = threadIdx.x & 7;
  const int ngroups = (gridDim.x * blockDim.x) >> 3;
  const double* rowbar = lw.g.a.rowbar;
  for (int j = (blockIdx.x * blockDim.x + threadIdx.x) >> 3; j < NE; j += ngroups) {
    double acc[NACC];
#pragma unroll
    for (int k = 0; k < NACC; ++k) acc[k] = 0.0;
    const int fj = lw.eflag[j];
    if (fj & 1) {
      const double* r = rowbar + (size_t(j) * ne * 8 + sl) * 10;
#pragma unroll
      for (int k = 0; k < 10; ++k) acc[k] += r[k];
    }
    bool touched = (fj & 1) != 0;
    const TickStep tj = lw.s1.ts[j];
    const int k0 = d.tsten_ptr[j], k1 = d.tsten_ptr[j + 1];
    // a lane's first GU entries (of ~80 per element at M=2) and their
    // elements' flags are loaded together; the rows of the updated ones follow
    constexpr int GU = 12;
    int gslot[GU], gflag[GU];
#pragma unroll
    for (int u = 0; u < GU; ++u) {
      const int k = k0 + sl + 8 * u;
      gslot[u] = k < k1 ? d.tsten_idx[k] : -1;
    }
#pragma unroll
    for (int u = 0; u < GU; ++u) gflag[u] = gslot[u] >= 0 ? lw.eflag[gslot[u] / (ne * 8)] : 0;
    for (int k = k0 + sl, u = 0; k < k1; k += 8, ++u) {
      int slot, fi;
      if (u < GU) {
        // constant-index selects keep the batch in registers
        slot = gslot[0];
        fi = gflag[0];
#pragma unroll
        for (int q = 1; q < GU; ++q)
          if (u == q) {
            slot = gslot[q];
            fi = gflag[q];
          }
      } else {
        slot = d.tsten_idx[k];
        fi = lw.eflag[slot / (ne * 8)];
      }
      if (!(fi & 1)) continue;
      touched = true;
      const int i = slot / (ne * 8);
      const double* r = rowbar + size_t(slot) * 10;
      double rv[10];
#pragma unroll
      for (int c = 0; c < 10; ++c) rv[c] = r[c];
      const int ti = lw.s1.ts[i].tick;
#pragma unroll
      for (int c = 4; c < 10; ++c) acc[c] += rv[c];
      if (ti == tj.tick) {
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] += rv[v];
      } else {
        const double tau = double(ti - tj.tick) / double(tj.step);
        const double dtj = double(tj.step) * lw.delta;
        double L[T], l[T];
        lag::tanti<M>(*tb, tau, L);
        lag::tbasis<M>(*tb, tau, l);
#pragma unroll
        for (int q = 0; q < T; ++q) {
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[OA + q * 4 + v] += l[q] * rv[v];
#pragma unroll
          for (int kc = 0; kc < 6; ++kc) acc[OV + ((kc / 2) * T + q) * 2 + (kc % 2)] += dtj * L[q] * rv[4 + kc];
        }
      }
    }
    // an element that no updated element's stencil names (and not updated
    // itself) receives nothing: its 8 lanes skip the sums and the writes
    const unsigned long long tmask = __ballot(touched);
    if (((tmask >> (__lane_id() & 56)) & 0xffull) == 0ull) continue;
#pragma unroll
    for (int k = 0; k < NACC; ++k) acc[k] = group8_sum_dpp(acc[k]);
#pragma unroll
    for (int k = 0; k < NACC; ++k) {
      if ((k & 7) != sl) continue;
      if (k < 4)
        lw.qb[size_t(j) * 4 + k] += acc[k];
      else if (k < 10)
        lw.g.a.xeb[size_t(j) * 6 + k - 4] += acc[k];
      else if (k < OV)
        lw.avb[size_t(j) * T * 4 + k - OA] += acc[k];
      else
        lw.vvb[size_t(j) * 3 * T * 2 + k - OV] += acc[k];
    }
    if (fj & 1)
      for (int c = sl; c < WS; c += 8) lw.g.a.wbar[size_t(j) * WS + c] = 0.0;
  }
}

// Update of each updated element in reverse: Q' = (|T| Q + sum of its memory
// variables) / |T'|, |T'| the area of its new vertices, which it stores with
// |T'|. Its new vertices' adjoints go to (element, vertex) slots for the nodes.
template <int M>
__global__ void __launch_bounds__(TPB) k_lts_update_rev(Dev d, LtsWork lw) {
  using S = AZ<M>;
  const int NE = d.NE;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < NE; i += gridDim.x * blockDim.x) {
    if (!(lw.eflag[i] & 1)) continue;
    const double* r0 = lw.s0.rec + size_t(i) * S::RS;
    const double* r1 = lw.s1.rec + size_t(i) * S::RS;
    const double A0 = r0[AO], An = r1[AO];
    double Anb = lw.ab[i], A0b = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double qb = lw.qb[size_t(i) * 4 + v];
      Anb -= qb * r1[QO + v] / An;
      A0b += qb * r0[QO + v] / An;
      lw.qb[size_t(i) * 4 + v] = (A0 / An) * qb;
      lw.mb[size_t(i) * 4 + v] = qb / An;
    }
    lw.ab[i] = A0b;
    double xn[6], g[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      xn[c] = r1[XE + c];
      g[c] = lw.g.a.xeb[size_t(i) * 6 + c];
      lw.g.a.xeb[size_t(i) * 6 + c] = 0.0;
    }
    lag::area3_grad(xn, Anb, g);
#pragma unroll
    for (int c = 0; c < 6; ++c) lw.g.xnbe[size_t(i) * 6 + c] = g[c];
  }
}

// Swept patches in reverse, one lane per edge with a moved node: the flux's
// adjoint is that of the memory variables it was added to (inflow positive
// into R, outflow from L); onto both sides' traces (added), the inner mean
// (transmissive, per edge) and the four corners (per edge).
template <int M>
__global__ void __launch_bounds__(TPB) k_lts_patch(Dev d, const Tables* __restrict__ tb, Params P, LtsWork lw) {
  using S = AZ<M>;
  constexpr int T = S::T, nG = S::nG, TS = S::TS, NT = nG * T * 4;
  const int NV = d.NV, n_e = lw.counts[2];
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n_e; idx += gridDim.x * blockDim.x) {
    const int e = lw.edge_list[idx];
    const int a = d.e_a[e], b = d.e_b[e];
    const bool ma = lw.nflag[a] != 0, mvb = lw.nflag[b] != 0;
    const double* X0 = lw.s0.X;
    const double* X1 = lw.s1.X;
    const double xa[2] = {X0[a], X0[NV + a]}, xb[2] = {X0[b], X0[NV + b]};
    const double xan[2] = {ma ? X1[a] : xa[0], ma ? X1[NV + a] : xa[1]};
    const double xbn[2] = {mvb ? X1[b] : xb[0], mvb ? X1[NV + b] : xb[1]};
    const int L = d.e_L[e], el = d.e_el[e], R = d.e_R[e], er = d.e_er[e];
    const bool hasR = R >= 0;
    const int kind = hasR ? lag::INTERIOR : (d.e_bc[e] == 2 ? lag::SLIP : lag::TRANSMISSIVE);
    lag::PatchTimes pt;
    pt.tk[0] = double(lw.s0.ntick[a]);
    pt.tk[1] = double(lw.s0.ntick[b]);
    pt.tk[2] = double(lw.s1.ntick[b]);
    pt.tk[3] = double(lw.s1.ntick[a]);
    const TickStep tL = lw.s0.ts[L];
    const TickStep tR = hasR ? lw.s0.ts[R] : tL;
    pt.nL = double(tL.tick);
    pt.sL = double(tL.step);
    pt.nR = double(tR.tick);
    pt.sR = double(tR.step);
    pt.delta = lw.delta;
    const double* trL = lw.s0.trace + size_t(L) * TS + el * NT;
    const double* trR = hasR ? lw.s0.trace + size_t(R) * TS + er * NT : trL;
    const double* avL = lw.s0.rec + size_t(L) * S::RS + rec_off_avg();
    double Gb[4], G[4] = {0.0, 0.0, 0.0, 0.0}, bA[T * 4];
#pragma unroll
    for (int v = 0; v < 4; ++v) Gb[v] = -lw.mb[size_t(L) * 4 + v] + (hasR ? lw.mb[size_t(R) * 4 + v] : 0.0);
#pragma unroll
    for (int k = 0; k < T * 4; ++k) bA[k] = 0.0;
    double c[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double* oL = lw.g.a.tbar + size_t(L) * TS + el * NT;
    double* oR = hasR ? lw.g.a.tbar + size_t(R) * TS + er * NT : oL;
    lag::patch_flux_vjp_lts<M>(*tb, P.gamma, xa, xb, xan, xbn, pt, trL, trR, avL, kind, Gb, G, oL, oR, bA, c,
                               c + 2, c + 4, c + 6, P.flux == ADER_FLUX_HLL);
    if (kind == lag::TRANSMISSIVE) {
      double* aL = lw.abar_e + size_t(e) * T * 4;
#pragma unroll
      for (int k = 0; k < T * 4; ++k) aL[k] = bA[k];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) lw.g.xs[size_t(e) * 8 + k] = c[k];
  }
}

// Per node: the adjoint of its position after the cycle (carried, the updated
// ring elements' new vertices, the swept patches' end corners) and, for a
// moved node, the node solver over its own interval in reverse (eqs.
// eqn.dtau, NodesVel, eqnNScs, eqn.NScs.weights, eqn.newVertex): into the
// ring's vertex velocities (each (element, vertex) written by its node only)
// and masses ((element, vertex) slots); the patches' start corners.
template <int M>
__global__ void __launch_bounds__(TPB) k_lts_node_rev(Dev d, const Tables* __restrict__ tb, LtsWork lw) {
  using S = AZ<M>;
  constexpr int T = M + 1, VV = rec_off_vv(M);
  const int NV = d.NV, NE = d.NE;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < NV; k += gridDim.x * blockDim.x) {
    double xn[2] = {lw.xb[2 * k], lw.xb[2 * k + 1]};
    double xo[2] = {0.0, 0.0};
    const int r0 = d.ring_ptr[k], r1 = d.ring_ptr[k + 1];
    const int fk = lw.nflag[k];
    // the ring element's corner slots (new vertex), then the edges leaving
    // this node in that element (local edges lv and lv + 2, whose L side
    // holds the edge's corner adjoints; an edge is swept when one of its two
    // nodes moved), in ring order; the first RING_U entries' indices and flags
    // are loaded together
    auto corner = [&](int j, int lv) {
      xn[0] += lw.g.xnbe[size_t(j) * 6 + 2 * lv];
      xn[1] += lw.g.xnbe[size_t(j) * 6 + 2 * lv + 1];
    };
    auto edge_end = [&](int e, int isb) {
      xn[0] += lw.g.xs[size_t(e) * 8 + 4 + 2 * isb];
      xn[1] += lw.g.xs[size_t(e) * 8 + 5 + 2 * isb];
      xo[0] += lw.g.xs[size_t(e) * 8 + 2 * isb];
      xo[1] += lw.g.xs[size_t(e) * 8 + 1 + 2 * isb];
    };
    constexpr int RING_U = 8;
    int ent[RING_U], ef[RING_U], ea[RING_U], eb[RING_U], oa[RING_U], ob[RING_U];
#pragma unroll
    for (int u = 0; u < RING_U; ++u) ent[u] = r0 + u < r1 ? d.ring_ent[r0 + u] : -1;
#pragma unroll
    for (int u = 0; u < RING_U; ++u) {
      ef[u] = ea[u] = eb[u] = oa[u] = ob[u] = 0;
      if (ent[u] >= 0) {
        const int j = ent[u] >> 2, lv = ent[u] & 3, l1 = lv == 2 ? 0 : lv + 1, l2 = lv == 0 ? 2 : lv - 1;
        ef[u] = lw.eflag[j];
        ea[u] = d.elem_edges[lv * NE + j];
        eb[u] = d.elem_edges[l2 * NE + j];
        oa[u] = d.tri[l1 * NE + j];
        ob[u] = d.tri[l2 * NE + j];
      }
    }
#pragma unroll
    for (int u = 0; u < RING_U; ++u)
      if (ent[u] >= 0 && (ef[u] & 1)) corner(ent[u] >> 2, ent[u] & 3);
    for (int r = r0 + RING_U; r < r1; ++r) {
      const int j = d.ring_ent[r] >> 2, lv = d.ring_ent[r] & 3;
      if (lw.eflag[j] & 1) corner(j, lv);
    }
    int la[RING_U], lb[RING_U], fa[RING_U], fb[RING_U];
#pragma unroll
    for (int u = 0; u < RING_U; ++u) {
      la[u] = lb[u] = -1;
      fa[u] = fb[u] = 0;
      if (ent[u] >= 0) {
        la[u] = d.e_L[ea[u]];
        lb[u] = d.e_L[eb[u]];
        fa[u] = fk | lw.nflag[oa[u]];
        fb[u] = fk | lw.nflag[ob[u]];
      }
    }
#pragma unroll
    for (int u = 0; u < RING_U; ++u) {
      if (ent[u] < 0) continue;
      const int j = ent[u] >> 2;
      if (la[u] == j && fa[u]) edge_end(ea[u], 0);
      if (lb[u] == j && fb[u]) edge_end(eb[u], 1);
    }
    for (int r = r0 + RING_U; r < r1; ++r) {
      const int j = d.ring_ent[r] >> 2, lv = d.ring_ent[r] & 3;
      const int e1 = d.elem_edges[lv * NE + j], e2 = d.elem_edges[((lv + 2) % 3) * NE + j];
      if (d.e_L[e1] == j && (lw.nflag[d.e_a[e1]] || lw.nflag[d.e_b[e1]])) edge_end(e1, 0);
      if (d.e_L[e2] == j && (lw.nflag[d.e_a[e2]] || lw.nflag[d.e_b[e2]])) edge_end(e2, 1);
    }
    lw.xb[2 * k] = xn[0] + xo[0];
    lw.xb[2 * k + 1] = xn[1] + xo[1];
    if (!lw.nflag[k]) continue;
    const int nk = lw.s0.ntick[k], newt = lw.s1.ntick[k];
    // the ring mean, recomputed from the state before the cycle
    double num[2] = {0.0, 0.0}, den = 0.0;
    for (int r = d.ring_ptr[k]; r < d.ring_ptr[k + 1]; ++r) {
      const int j = d.ring_ent[r] >> 2, lv = d.ring_ent[r] & 3;
      const TickStep tj = lw.s0.ts[j];
      const double tau0 = double(nk - tj.tick) / double(tj.step), tau1 = double(newt - tj.tick) / double(tj.step);
      double L0[T], L1[T];
      lag::tanti<M>(*tb, tau0, L0);
      lag::tanti<M>(*tb, tau1, L1);
      const double* rj = lw.s0.rec + size_t(j) * S::RS;
      const double inv = 1.0 / (tau1 - tau0);
      double vx = 0.0, vy = 0.0;
#pragma unroll
      for (int q = 0; q < T; ++q) {
        vx += (L1[q] - L0[q]) * rj[VV + (lv * T + q) * 2];
        vy += (L1[q] - L0[q]) * rj[VV + (lv * T + q) * 2 + 1];
      }
      const double mu = rj[QO] * rj[AO];
      num[0] += mu * (vx * inv);
      num[1] += mu * (vy * inv);
      den += mu;
    }
    const double V[2] = {num[0] / den, num[1] / den};
    const double dtk = double(newt - nk) * lw.delta;
    double Vb[2] = {dtk * xn[0], dtk * xn[1]};
    if (d.wall_pin[k]) {
      Vb[0] = Vb[1] = 0.0;
    } else {
      const double nx = d.wall_n[k], ny = d.wall_n[NV + k];
      const double vn = Vb[0] * nx + Vb[1] * ny;
      Vb[0] -= vn * nx;
      Vb[1] -= vn * ny;
    }
    const double numb[2] = {Vb[0] / den, Vb[1] / den};
    const double denb = -(numb[0] * V[0] + numb[1] * V[1]);
    for (int r = d.ring_ptr[k]; r < d.ring_ptr[k + 1]; ++r) {
      const int j = d.ring_ent[r] >> 2, lv = d.ring_ent[r] & 3;
      const TickStep tj = lw.s0.ts[j];
      const double tau0 = double(nk - tj.tick) / double(tj.step), tau1 = double(newt - tj.tick) / double(tj.step);
      double L0[T], L1[T];
      lag::tanti<M>(*tb, tau0, L0);
      lag::tanti<M>(*tb, tau1, L1);
      const double* rj = lw.s0.rec + size_t(j) * S::RS;
      const double inv = 1.0 / (tau1 - tau0);
      double vx = 0.0, vy = 0.0;
      double* vo = lw.vvb + (size_t(j) * 3 + lv) * T * 2;
      const double mu = rj[QO] * rj[AO];
#pragma unroll
      for (int q = 0; q < T; ++q) {
        const double I = L1[q] - L0[q];
        vx += I * rj[VV + (lv * T + q) * 2];
        vy += I * rj[VV + (lv * T + q) * 2 + 1];
        vo[2 * q] += mu * numb[0] * I * inv;
        vo[2 * q + 1] += mu * numb[1] * I * inv;
      }
      lw.g.nslot[(size_t(j) * 3 + lv) * 3] = numb[0] * (vx * inv) + numb[1] * (vy * inv) + denb;
    }
  }
}

// Per element: the ring masses rho |T| of its moved vertices (state before
// the cycle) and the means' adjoints of its transmissive swept edges.
template <int M>
__global__ void __launch_bounds__(TPB) k_lts_elem(Dev d, LtsWork lw) {
  using S = AZ<M>;
  constexpr int T = M + 1;
  const int NE = d.NE;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < NE; j += gridDim.x * blockDim.x) {
    const double* r0 = lw.s0.rec + size_t(j) * S::RS;
#pragma unroll
    for (int lv = 0; lv < 3; ++lv) {
      if (!lw.nflag[d.tri[lv * NE + j]]) continue;
      const double mub = lw.g.nslot[(size_t(j) * 3 + lv) * 3];
      lw.qb[size_t(j) * 4] += mub * r0[AO];
      lw.ab[j] += mub * r0[QO];
    }
#pragma unroll
    for (int le = 0; le < 3; ++le) {
      const int e = d.elem_edges[le * NE + j];
      if (d.e_L[e] != j || d.e_R[e] >= 0 || d.e_bc[e] == 2) continue;
      if (!lw.nflag[d.e_a[e]] && !lw.nflag[d.e_b[e]]) continue;
#pragma unroll
      for (int k = 0; k < T * 4; ++k) lw.avb[size_t(j) * T * 4 + k] += lw.abar_e[size_t(e) * T * 4 + k];
    }
  }
}

// Where the stored vertices and areas are those of the node positions (a
// macro-step boundary, the uploaded state): their adjoints added to the
// nodes' (view s1), then cleared by k_lts_clear_geo.
template <int M>
__global__ void __launch_bounds__(TPB) k_lts_fold(Dev d, LtsWork lw) {
  using S = AZ<M>;
  const int NV = d.NV;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < NV; k += gridDim.x * blockDim.x) {
    double x[2] = {0.0, 0.0};
    for (int r = d.ring_ptr[k]; r < d.ring_ptr[k + 1]; ++r) {
      const int j = d.ring_ent[r] >> 2, lv = d.ring_ent[r] & 3;
      double xe[6], g[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        xe[c] = lw.s1.rec[size_t(j) * S::RS + XE + c];
        g[c] = lw.g.a.xeb[size_t(j) * 6 + c];
      }
      lag::area3_grad(xe, lw.ab[j], g);
      x[0] += g[2 * lv];
      x[1] += g[2 * lv + 1];
    }
    lw.xb[2 * k] += x[0];
    lw.xb[2 * k + 1] += x[1];
  }
}

__global__ void __launch_bounds__(TPB) k_lts_clear_geo(Dev d, LtsWork lw) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < d.NE; i += gridDim.x * blockDim.x) {
    lw.ab[i] = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) lw.g.a.xeb[size_t(i) * 6 + c] = 0.0;
  }
}

template <int M>
__global__ void __launch_bounds__(TPB) k_lts_init(Dev d, LtsWork lw, const double* Qbar, const double* Xbar) {
  using S = AZ<M>;
  constexpr int T = M + 1;
  const int NE = d.NE, NV = d.NV;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < NE; i += gridDim.x * blockDim.x) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      lw.qb[size_t(i) * 4 + v] = Qbar[size_t(v) * NE + i];
      lw.mb[size_t(i) * 4 + v] = 0.0;
    }
    lw.ab[i] = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) lw.g.a.xeb[size_t(i) * 6 + c] = 0.0;
#pragma unroll
    for (int c = 0; c < S::WS; ++c) lw.g.a.wbar[size_t(i) * S::WS + c] = 0.0;
    for (int c = 0; c < S::TS; ++c) lw.g.a.tbar[size_t(i) * S::TS + c] = 0.0;
#pragma unroll
    for (int c = 0; c < T * 4; ++c) lw.avb[size_t(i) * T * 4 + c] = 0.0;
#pragma unroll
    for (int c = 0; c < 6 * T; ++c) lw.vvb[size_t(i) * 6 * T + c] = 0.0;
  }
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < NV; k += gridDim.x * blockDim.x) {
    lw.xb[2 * k] = Xbar[2 * k];
    lw.xb[2 * k + 1] = Xbar[2 * k + 1];
  }
}

__global__ void __launch_bounds__(TPB) k_lts_out(Dev d, LtsWork lw, double* Qbar, double* Xbar) {
  const int NE = d.NE, NV = d.NV;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < NE; i += gridDim.x * blockDim.x)
#pragma unroll
    for (int v = 0; v < 4; ++v) Qbar[size_t(v) * NE + i] = lw.qb[size_t(i) * 4 + v];
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < 2 * NV; k += gridDim.x * blockDim.x) Xbar[k] = lw.xb[k];
}

template <int M>
int lts_pred_rev(const Dev& d, const Params& p, const LtsWork& w, void* s) {
  long pb = (long(d.NE) + LP<M>::SLOTS - 1) / LP<M>::SLOTS;
  if (pb > 16384) pb = 16384;
  AD_LAUNCH_BLOCKS((k_lag_pred_fwd<M, true>), pb, s, d, d.tab, p, w.g, 0.0, w);
  AD_LAUNCH_BLOCKS((k_lag_pred_rev<M, true>), pb, s, d, d.tab, p, w.g, 0.0, w);
  return 0;
}

template <int M>
int lts_recon_rev(const Dev& d, const Params& p, const LtsWork& w, void* s) {
  AD_LAUNCH((k_adj_recon<M, false, true, true>), 8L * d.NE, s, d, d.tab, p, w.g.a, w);
  AD_LAUNCH((k_adj_recon<M, true, true, true>), 8L * d.NE, s, d, d.tab, p, w.g.a, w);
  AD_LAUNCH(k_lts_gather<M>, 8L * d.NE, s, d, d.tab, w);
  return 0;
}

template <int M>
int lts_cycle_rev(const Dev& d, const Params& p, const LtsWork& w, void* s) {
  AD_LAUNCH(k_lts_clear_counts, 1, s, w);
  AD_LAUNCH(k_lts_marks, d.NE > d.NV ? d.NE : d.NV, s, d, w, 0);
  AD_LAUNCH(k_lts_edges, d.NF, s, d, w);
  int r;
  if ((r = lts_pred_rev<M>(d, p, w, s))) return r;
  if ((r = lts_recon_rev<M>(d, p, w, s))) return r;
  AD_LAUNCH(k_lts_update_rev<M>, d.NE, s, d, w);
  AD_LAUNCH(k_lts_patch<M>, d.NF, s, d, d.tab, p, w);
  AD_LAUNCH(k_lts_node_rev<M>, d.NV, s, d, d.tab, w);
  AD_LAUNCH(k_lts_elem<M>, d.NE, s, d, w);
  return 0;
}

template <int M>
int lts_macro_begin_rev(const Dev& d, const Params& p, const LtsWork& w, void* s) {
  AD_LAUNCH(k_lts_clear_counts, 1, s, w);
  AD_LAUNCH(k_lts_marks, d.NE > d.NV ? d.NE : d.NV, s, d, w, 1);
  int r;
  if ((r = lts_pred_rev<M>(d, p, w, s))) return r;
  AD_LAUNCH(k_lts_fold<M>, d.NV, s, d, w);
  AD_LAUNCH(k_lts_clear_geo, d.NE, s, d, w);
  return 0;
}

template <int M>
int lts_initial_rev(const Dev& d, const Params& p, const LtsWork& w, void* s) {
  AD_LAUNCH(k_lts_clear_counts, 1, s, w);
  AD_LAUNCH(k_lts_marks, d.NE > d.NV ? d.NE : d.NV, s, d, w, 1);
  int r;
  if ((r = lts_recon_rev<M>(d, p, w, s))) return r;
  AD_LAUNCH(k_lts_fold<M>, d.NV, s, d, w);
  AD_LAUNCH(k_lts_clear_geo, d.NE, s, d, w);
  return 0;
}

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

int lsq_slots(int M) {
  switch (M) {
    case 1: return AZ<1>::LB;
    case 2: return AZ<2>::LB;
    default: return AZ<3>::LB;
  }
}

// Buffer sizes in bytes: nodal values, traces, sweeps, kept least-squares data.
void adjoint_sizes(int M, int NE, int NF, int npic, size_t& ws, size_t& ts, size_t& sw, size_t& lq,
                   size_t& rb, size_t& qc, size_t& mb) {
  const size_t nb = size_t(M + 1) * (M + 2) / 2, T = M + 1, D = sizeof(double);
  ws = align256(NE * size_t(wnod_stride(M)) * D);
  ts = align256(NE * size_t(trace_stride(M)) * D);
  sw = align256(size_t(npic) * nb * T * 4 * NE * D);
  lq = align256(size_t(lsq_slots(M)) * 8 * NE * D);
  rb = align256(size_t(2 * nb) * NE * 32 * D);
  qc = align256(size_t(4) * NE * D);
  mb = align256(size_t(T) * 4 * (NE + NF) * D);   // means, and their adjoints per edge
}

}  // namespace

size_t adjoint_work_bytes(int M, int NE, int NF, int npic) {
  size_t ws, ts, sw, lq, rb, qc, mb;
  adjoint_sizes(M, NE, NF, npic, ws, ts, sw, lq, rb, qc, mb);
  return 2 * ws + 2 * ts + sw + lq + rb + qc + mb;
}

void adjoint_carve(int M, int NE, int NF, int npic, char* base, AdjWork& w) {
  size_t ws, ts, sw, lq, rb, qc, mb;
  adjoint_sizes(M, NE, NF, npic, ws, ts, sw, lq, rb, qc, mb);
  w.wnod = (double*)base;
  w.wbar = (double*)(base + ws);
  w.trace = (double*)(base + 2 * ws);
  w.tbar = (double*)(base + 2 * ws + ts);
  w.sweeps = (double*)(base + 2 * ws + 2 * ts);
  w.lsq = (double*)(base + 2 * ws + 2 * ts + sw);
  w.rowbar = (double*)(base + 2 * ws + 2 * ts + sw + lq);
  w.qcopy = (double*)(base + 2 * ws + 2 * ts + sw + lq + rb);
  w.avg = (double*)(base + 2 * ws + 2 * ts + sw + lq + rb + qc);
  w.abar = w.avg + size_t(NE) * (M + 1) * 4;   // [NF][M+1][4]
}

namespace {
// Buffers of the moving-mesh adjoint, in carve order (bytes, 256-aligned each).
struct LagPlan {
  size_t off[32];
  size_t total = 0;
  int n = 0;
  void add(size_t bytes) {
    off[n++] = total;
    total += align256(bytes);
  }
};

LagPlan lag_plan(int M, int NE, int NV, int NF, int npic) {
  const size_t D = sizeof(double), nb = size_t(M + 1) * (M + 2) / 2, T = M + 1, ne = 2 * nb;
  LagPlan p;
  p.add(4 * size_t(NE) * D);                       // 0 qcopy
  p.add(2 * size_t(NV) * D);                       // 1 xcopy
  p.add(6 * size_t(NE) * D);                       // 2 xe
  p.add(size_t(NE) * D);                           // 3 area
  p.add(size_t(NE) * D);                           // 4 an
  p.add(2 * size_t(NV) * D);                       // 5 xn
  p.add(2 * size_t(NV) * D);                       // 6 vraw
  p.add(size_t(NV) * D);                           // 7 den
  p.add(size_t(NE) * wnod_stride(M) * D);          // 8 wnod
  p.add(size_t(NE) * wnod_stride(M) * D);          // 9 wbar
  p.add(size_t(npic + 1) * nb * T * 4 * NE * D);   // 10 keep
  p.add(size_t(NE) * trace_stride(M) * D);         // 11 trace
  p.add(size_t(NE) * trace_stride(M) * D);         // 12 tbar
  p.add(size_t(NE) * T * 4 * D);                   // 13 avg
  p.add(size_t(NF) * T * 4 * D);                   // 14 abar
  p.add(size_t(NE) * 3 * T * 2 * D);               // 15 vvel
  p.add(size_t(NE) * 12 * D);                      // 16 gslot
  p.add(size_t(NF) * 8 * D);                       // 17 xs
  p.add(size_t(NE) * 6 * D);                       // 18 xeb
  p.add(size_t(NE) * 6 * D);                       // 19 xnbe
  p.add(size_t(NE) * 9 * D);                       // 20 nslot
  p.add(4 * size_t(NE) * D);                       // 21 qdir
  p.add(size_t(lsq_slots(M)) * 8 * NE * D);        // 22 lsq
  p.add(ne * NE * 80 * D);                         // 23 row slots (10 doubles)
  return p;
}

// Buffers of the local-time-stepping adjoint, in carve order.
LagPlan lts_plan(int M, int NE, int NV, int NF, int npic) {
  const size_t D = sizeof(double), I = sizeof(int), nb = size_t(M + 1) * (M + 2) / 2, T = M + 1, ne = 2 * nb;
  LagPlan p;
  p.add(size_t(NE) * wnod_stride(M) * D);          // 0 recomputed reconstruction
  p.add(size_t(NE) * wnod_stride(M) * D);          // 1 wbar
  p.add(size_t(NE) * trace_stride(M) * D);         // 2 tbar
  p.add(size_t(npic + 1) * nb * T * 4 * NE * D);   // 3 keep
  p.add(size_t(lsq_slots(M)) * 8 * NE * D);        // 4 lsq
  p.add(ne * NE * 80 * D);                         // 5 row slots
  p.add(size_t(NF) * 8 * D);                       // 6 xs
  p.add(size_t(NE) * 6 * D);                       // 7 xnbe
  p.add(size_t(NE) * 9 * D);                       // 8 nslot
  p.add(size_t(NE) * 6 * D);                       // 9 xeb
  p.add(size_t(NE) * 4 * D);                       // 10 qb
  p.add(size_t(NE) * D);                           // 11 ab
  p.add(size_t(NE) * 4 * D);                       // 12 mb
  p.add(size_t(NE) * T * 4 * D);                   // 13 avb
  p.add(size_t(NE) * 6 * T * D);                   // 14 vvb
  p.add(size_t(NV) * 2 * D);                       // 15 xb
  p.add(size_t(NF) * T * 4 * D);                   // 16 abar_e
  p.add(8);                                        // 17 (unused)
  p.add(size_t(NE) * I);                           // 18 eflag
  p.add(size_t(NV) * I);                           // 19 nflag
  p.add(size_t(NE) * I);                           // 20 act_list
  p.add(size_t(NE) * I);                           // 21 going_list
  p.add(3 * I);                                    // 22 counts
  p.add(size_t(NF) * I);                           // 23 edge_list
  return p;
}
}  // namespace

size_t lts_work_bytes(int M, int NE, int NV, int NF, int npic) { return lts_plan(M, NE, NV, NF, npic).total; }

void lts_carve(int M, int NE, int NV, int NF, int npic, char* base, LtsWork& w) {
  const LagPlan p = lts_plan(M, NE, NV, NF, npic);
  auto at = [&](int k) { return reinterpret_cast<double*>(base + p.off[k]); };
  auto ai = [&](int k) { return reinterpret_cast<int*>(base + p.off[k]); };
  w = LtsWork{};
  w.g.a.wnod = at(0);
  w.g.a.wbar = at(1);
  w.g.a.tbar = at(2);
  w.g.keep = at(3);
  w.g.a.lsq = at(4);
  w.g.a.rowbar = at(5);
  w.g.xs = at(6);
  w.g.xnbe = at(7);
  w.g.nslot = at(8);
  w.g.a.xeb = at(9);
  w.qb = at(10);
  w.ab = at(11);
  w.mb = at(12);
  w.avb = at(13);
  w.vvb = at(14);
  w.xb = at(15);
  w.abar_e = at(16);
  w.eflag = ai(18);
  w.nflag = ai(19);
  w.act_list = ai(20);
  w.going_list = ai(21);
  w.counts = ai(22);
  w.edge_list = ai(23);
}

#define LTS_DISPATCH(fn, ...)                          \
  switch (M) {                                         \
    case 1: return fn<1>(__VA_ARGS__);                 \
    case 2: return fn<2>(__VA_ARGS__);                 \
    case 3: return fn<3>(__VA_ARGS__);                 \
    default: return int(hipErrorInvalidValue);         \
  }

int launch_lts_init(const Dev& d, const LtsWork& w, const double* Qbar, const double* Xbar, void* s) {
  const int M = d.M;
  auto go = [&](auto tag) -> int {
    constexpr int MM = decltype(tag)::value;
    AD_LAUNCH(k_lts_init<MM>, d.NE > d.NV ? d.NE : d.NV, s, d, w, Qbar, Xbar);
    return 0;
  };
  switch (M) {
    case 1: return go(std::integral_constant<int, 1>{});
    case 2: return go(std::integral_constant<int, 2>{});
    case 3: return go(std::integral_constant<int, 3>{});
    default: return int(hipErrorInvalidValue);
  }
}

int launch_lts_cycle_rev(const Dev& d, const Params& p, int M, const LtsWork& w, void* s) {
  LTS_DISPATCH(lts_cycle_rev, d, p, w, s)
}

int launch_lts_macro_begin_rev(const Dev& d, const Params& p, int M, const LtsWork& w, void* s) {
  LTS_DISPATCH(lts_macro_begin_rev, d, p, w, s)
}

int launch_lts_initial_rev(const Dev& d, const Params& p, int M, const LtsWork& w, void* s) {
  LTS_DISPATCH(lts_initial_rev, d, p, w, s)
}

int launch_lts_out(const Dev& d, const LtsWork& w, double* Qbar, double* Xbar, void* s) {
  AD_LAUNCH(k_lts_out, d.NE > 2 * d.NV ? d.NE : 2 * d.NV, s, d, w, Qbar, Xbar);
  return 0;
}

size_t lagadj_work_bytes(int M, int NE, int NV, int NF, int npic) {
  return lag_plan(M, NE, NV, NF, npic).total;
}

void lagadj_carve(int M, int NE, int NV, int NF, int npic, char* base, LagWork& w) {
  const LagPlan p = lag_plan(M, NE, NV, NF, npic);
  auto at = [&](int k) { return reinterpret_cast<double*>(base + p.off[k]); };
  w.a.qcopy = at(0);
  w.xcopy = at(1);
  w.xe = at(2);
  w.area = at(3);
  w.an = at(4);
  w.xn = at(5);
  w.vraw = at(6);
  w.den = at(7);
  w.a.wnod = at(8);
  w.a.wbar = at(9);
  w.keep = at(10);
  w.a.sweeps = nullptr;
  w.a.trace = at(11);
  w.a.tbar = at(12);
  w.a.avg = at(13);
  w.a.abar = at(14);
  w.vvel = at(15);
  w.gslot = at(16);
  w.xs = at(17);
  w.a.xeb = at(18);
  w.xnbe = at(19);
  w.nslot = at(20);
  w.qdir = at(21);
  w.a.lsq = at(22);
  w.a.rowbar = at(23);
  w.a.geo = w.xe;
  w.a.geo_stride = 6;
}

int launch_adjoint_lagrangian(const Dev& d, const Params& p, int M, const LagWork& w, double dt,
                              bool q_from_context, bool x_from_context, void* s) {
  switch (M) {
    case 1: return adjoint_lagrangian<1>(d, p, w, dt, q_from_context, x_from_context, s);
    case 2: return adjoint_lagrangian<2>(d, p, w, dt, q_from_context, x_from_context, s);
    case 3: return adjoint_lagrangian<3>(d, p, w, dt, q_from_context, x_from_context, s);
    default: return int(hipErrorInvalidValue);
  }
}

int launch_adjoint_gts(const Dev& d, const Params& p, int M, const AdjWork& w, double dt,
                       bool state_from_context, void* s) {
  switch (M) {
    case 1: return adjoint_gts<1>(d, p, w, dt, state_from_context, s);
    case 2: return adjoint_gts<2>(d, p, w, dt, state_from_context, s);
    case 3: return adjoint_gts<3>(d, p, w, dt, state_from_context, s);
    default: return int(hipErrorInvalidValue);
  }
}

}  // namespace aw
