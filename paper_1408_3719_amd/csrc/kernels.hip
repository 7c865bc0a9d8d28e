// HIP kernels (gfx950) of the ALE ADER-WENO scheme with local time stepping.
//
// One cycle of the local time stepping (paper Sec. 2.6, "computational phase"),
// read data-parallel: the active set is fixed from the cycle-start ticks, then
//   k_sched      update criterion (eq. eqn.WENOupdate) over the symmetric
//                scheduling stencil, compacted active list
//   k_node       node solver NS_cs (eqs. eqnNScs, eqn.NScs.weights, eqn.dtau,
//                NodesVel) and node motion (eq. eqn.newVertex)
//   k_patch      flux through every space-time patch swept by a moved edge
//                (eqs. eqn.spacetimenodes, G_ij, eqn.rusanov, A_n^V, eqn.STint)
//   k_update     memory variables (eq. eqn.Qm2 and the geometric memory) and
//                the one-step update (eq. PDEfinal) with the GCL check (eqn.gcl)
//   k_reconstruct virtual projection of the stencil (eqs. eqn.virtGeom,
//                eqn.virtCellaverage), WENO (eqs. intConsRec .. eqn.weno), local
//                time step (eq. eqn.timestep) and dyadic level
//   k_predict    space-time Galerkin predictor of the PDE and of the mesh ODE
//                (eqs. timeTransf .. newVertPos)
// Every write target has a single writer per kernel: no atomics on state.
#include <hip/hip_runtime.h>

#include <cfloat>

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
};

__device__ inline void set_err(const Dev& d, int bits) { atomicOr(&d.scal->err, bits); }

// count the calling lanes of the wavefront with one atomic
__device__ inline void wave_count(unsigned long long* ctr) {
  unsigned long long m = __ballot(1);
  if ((int)__lane_id() == __ffsll((long long)m) - 1) atomicAdd(ctr, (unsigned long long)__popcll(m));
}

__device__ inline void atomic_max_pos(unsigned long long* a, double v) {
  atomicMax(a, (unsigned long long)__double_as_longlong(v));
}

__device__ inline double pressure(const double q[4], double g) {
  return (g - 1.0) * (q[3] - 0.5 * (q[1] * q[1] + q[2] * q[2]) / q[0]);
}

// F~(q) . N = f N_x + g N_y + q N_t (eq. PDEdiv3D)
__device__ inline void stflux(const double q[4], const double N[3], double g, double out[4]) {
  double u = q[1] / q[0], v = q[2] / q[0];
  double p = pressure(q, g);
  double un = u * N[0] + v * N[1] + N[2];
  out[0] = q[0] * un;
  out[1] = q[1] * un + p * N[0];
  out[2] = q[2] * un + p * N[1];
  out[3] = q[3] * un + p * (u * N[0] + v * N[1]);
}

__device__ inline double stspeed(const double q[4], const double N[3], double g) {
  double u = q[1] / q[0], v = q[2] / q[0];
  double c = sqrt(g * pressure(q, g) / q[0]);
  return fabs(u * N[0] + v * N[1] + N[2]) + c * sqrt(N[0] * N[0] + N[1] * N[1]);
}

template <int M>
__device__ inline void time_basis(const Tables* tb, double tau, double l[M + 1]) {
#pragma unroll
  for (int q = 0; q <= M; ++q) {
    double s = tb->lag[q][M];
#pragma unroll
    for (int k = M - 1; k >= 0; --k) s = s * tau + tb->lag[q][k];
    l[q] = s;
  }
}

template <int M>
__device__ inline void time_antideriv(const Tables* tb, double tau, double L[M + 1]) {
#pragma unroll
  for (int q = 0; q <= M; ++q) {
    double s = tb->Lint[q][M + 1];
#pragma unroll
    for (int k = M; k >= 0; --k) s = s * tau + tb->Lint[q][k];
    L[q] = s;
  }
}

// Geometry (x0 y0 x1 y1 x2 y2) and average of element j projected to tick nt.
template <int M>
__device__ inline bool project(const Dev& d, const Tables* tb, int j, int nt, double delta,
                               double X[6], double Qv[4]) {
  const int NE = d.NE;
  int nj = d.tick[j];
  if (nj == nt) {
#pragma unroll
    for (int c = 0; c < 6; ++c) X[c] = d.Xe[c * NE + j];
#pragma unroll
    for (int v = 0; v < 4; ++v) Qv[v] = d.Q[v * NE + j];
    return true;
  }
  int sj = d.step[j];
  if (sj <= 0) return false;
  double tau = double(nt - nj) / double(sj);
  double dtj = double(sj) * delta;
  double L[M + 1], l[M + 1];
  time_antideriv<M>(tb, tau, L);
  time_basis<M>(tb, tau, l);
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q <= M; ++q) s += L[q] * d.vvel[((k * (M + 1) + q) * 2 + c) * NE + j];
      X[2 * k + c] = d.Xe[(2 * k + c) * NE + j] + dtj * s;
    }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q <= M; ++q) s += l[q] * d.avg[(q * 4 + v) * NE + j];
    Qv[v] = s;
  }
  return true;
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

__device__ inline int level_step(double dtcfl, double delta, int N, int tick, int* over) {
  int p = N;
  while (p > 1 && double(p) * delta > dtcfl) p >>= 1;
  *over = double(p) * delta > dtcfl;
  if (tick > 0) {
    int low = tick & (-tick);
    if (low < p) p = low;
  }
  return p;
}

// ---------------------------------------------------------------------------
// Reconstruction + local time step
// ---------------------------------------------------------------------------
template <int M>
__global__ void __launch_bounds__(TPB) k_reconstruct(Dev d, const Tables* __restrict__ tb, Params P,
                                                     int use_list, int set_level) {
  using S = Sz<M>;
  constexpr int nb = S::nb, ne = S::ne, nu = S::nu;
  const int NE = d.NE;
  const int nitems = use_list ? d.scal->n_active : NE;
  const double delta = d.scal->delta;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < nitems; idx += gridDim.x * blockDim.x) {
    const int i = use_list ? d.act_list[idx] : idx;
    const int nt = d.tick[i];
    double Xi[6], Qi[4];
#pragma unroll
    for (int c = 0; c < 6; ++c) Xi[c] = d.Xe[c * NE + i];
#pragma unroll
    for (int v = 0; v < 4; ++v) Qi[v] = d.Q[v * NE + i];
    const double e1x = Xi[2] - Xi[0], e1y = Xi[3] - Xi[1];
    const double e2x = Xi[4] - Xi[0], e2y = Xi[5] - Xi[1];
    const double idet = 1.0 / (e1x * e2y - e2x * e1y);
    double W[nu][4];
#pragma unroll
    for (int l = 0; l < nu; ++l)
#pragma unroll
      for (int v = 0; v < 4; ++v) W[l][v] = 0.0;
    double Wsum = 0.0;
    bool ok = true;
    for (int s = 0; s < NSTEN; ++s) {
      if (d.sten[(s * ne) * NE + i] < 0) continue;
      double R[nu][nu], z[nu][4];
#pragma unroll
      for (int a = 0; a < nu; ++a) {
#pragma unroll
        for (int b = 0; b < nu; ++b) R[a][b] = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) z[a][v] = 0.0;
      }
      for (int c = 1; c < ne; ++c) {
        const int j = d.sten[(s * ne + c) * NE + i];
        double Xv[6], Qv[4];
        ok &= project<M>(d, tb, j, nt, delta, Xv, Qv);
        // vertices of the virtual element in the reference frame of element i
        double rx[3], ry[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          double dx = Xv[2 * k] - Xi[0], dy = Xv[2 * k + 1] - Xi[1];
          rx[k] = (dx * e2y - dy * e2x) * idet;
          ry[k] = (e1x * dy - e1y * dx) * idet;
        }
        // means of the monomials over the virtual element (rule exact to degree M)
        double mm[nb];
#pragma unroll
        for (int k = 0; k < nb; ++k) mm[k] = 0.0;
        for (int r = 0; r < tb->nrq; ++r) {
          double px = tb->rqb[r][0] * rx[0] + tb->rqb[r][1] * rx[1] + tb->rqb[r][2] * rx[2];
          double py = tb->rqb[r][0] * ry[0] + tb->rqb[r][1] * ry[1] + tb->rqb[r][2] * ry[2];
          double w = tb->rqw[r];
          double xp[M + 1], yp[M + 1];
          xp[0] = 1.0;
          yp[0] = 1.0;
#pragma unroll
          for (int a = 1; a <= M; ++a) {
            xp[a] = xp[a - 1] * px;
            yp[a] = yp[a - 1] * py;
          }
          int k = 0;
#pragma unroll
          for (int dg = 0; dg <= M; ++dg)
#pragma unroll
            for (int b = 0; b <= dg; ++b) {
              mm[k] += w * xp[dg - b] * yp[b];
              ++k;
            }
        }
        double a[nu], b[4];
#pragma unroll
        for (int l = 0; l < nu; ++l) {
          double s2 = 0.0;
#pragma unroll
          for (int k = 0; k < nb; ++k) s2 += tb->psiC[l + 1][k] * mm[k];
          a[l] = s2;
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) b[v] = Qv[v] - Qi[v];
        // Givens rotations fold the row into the triangular factor
#pragma unroll
        for (int k = 0; k < nu; ++k) {
          double rkk = R[k][k], ak = a[k];
          double h = sqrt(rkk * rkk + ak * ak);
          if (h == 0.0) continue;
          double cs = rkk / h, sn = ak / h;
          R[k][k] = h;
#pragma unroll
          for (int c2 = k + 1; c2 < nu; ++c2) {
            double t = cs * R[k][c2] + sn * a[c2];
            a[c2] = cs * a[c2] - sn * R[k][c2];
            R[k][c2] = t;
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            double t = cs * z[k][v] + sn * b[v];
            b[v] = cs * b[v] - sn * z[k][v];
            z[k][v] = t;
          }
        }
      }
      double w[nu][4];
#pragma unroll
      for (int k = nu - 1; k >= 0; --k)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double t = z[k][v];
#pragma unroll
          for (int c2 = k + 1; c2 < nu; ++c2) t -= R[k][c2] * w[c2][v];
          w[k][v] = t / R[k][k];
        }
      double sigma = 0.0;
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int l = 0; l < nu; ++l) {
          double t = 0.0;
#pragma unroll
          for (int m = 0; m < nu; ++m) t += tb->Sigma[l + 1][m + 1] * w[m][v];
          sigma += w[l][v] * t;
        }
      double x = sigma + P.eps;
      double x2 = x * x, x4 = x2 * x2, x8 = x4 * x4;
      double om = (s == 0 ? P.lambda : 1.0) / x8;
      Wsum += om;
#pragma unroll
      for (int l = 0; l < nu; ++l)
#pragma unroll
        for (int v = 0; v < 4; ++v) W[l][v] += om * w[l][v];
    }
    if (!ok) set_err(d, ERR_PRED);
    const double iw = 1.0 / Wsum;
#pragma unroll
    for (int m = 0; m < nb; ++m)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double t = tb->psiNodes[m][0] * Qi[v];
#pragma unroll
        for (int l = 0; l < nu; ++l) t += tb->psiNodes[m][l + 1] * (W[l][v] * iw);
        d.wnod[(m * 4 + v) * NE + i] = t;
      }
    // local CFL time step over the element and its face neighbours (eq. eqn.timestep)
    double rmin = cfl_ratio(Xi, Qi, P.gamma);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      int j = d.neigh[k * NE + i];
      if (j < 0) continue;
      double Xv[6], Qv[4];
      if (!project<M>(d, tb, j, nt, delta, Xv, Qv)) set_err(d, ERR_PRED);
      rmin = fmin(rmin, cfl_ratio(Xv, Qv, P.gamma));
    }
    const double dt = P.cfl * rmin;
    d.dtcfl[i] = dt;
    if (set_level) {
      const int N = d.scal->N;
      if (nt >= N) {
        d.step[i] = 0;
      } else {
        int over;
        d.step[i] = level_step(dt, delta, N, nt, &over);
        if (over) atomicAdd(&d.scal->overshoots, 1ull);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Space-time Galerkin predictor
// ---------------------------------------------------------------------------
template <int M>
__global__ void __launch_bounds__(TPB) k_predict(Dev d, const Tables* __restrict__ tb, Params P,
                                                 int use_list) {
  using S = Sz<M>;
  constexpr int nb = S::nb, nt = S::nt, nG = S::nG;
  const int NE = d.NE;
  const int nitems = use_list ? d.scal->n_active : NE;
  const double delta = d.scal->delta;
  const double g = P.gamma;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < nitems; idx += gridDim.x * blockDim.x) {
    const int i = use_list ? d.act_list[idx] : idx;
    const int st = d.step[i];
    if (st <= 0) continue;
    wave_count(&d.scal->n_pred);
    const double dt = double(st) * delta;
    double q[nb][nt][4], x[nb][nt][2];
    {
      double X[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) X[c] = d.Xe[c * NE + i];
      int m = 0;
#pragma unroll
      for (int jj = 0; jj <= M; ++jj)
#pragma unroll
        for (int ii = 0; ii + jj <= M; ++ii) {
          double xi = double(ii) / M, eta = double(jj) / M;
          double px = X[0] + (X[2] - X[0]) * xi + (X[4] - X[0]) * eta;
          double py = X[1] + (X[3] - X[1]) * xi + (X[5] - X[1]) * eta;
#pragma unroll
          for (int t = 0; t < nt; ++t) {
            x[m][t][0] = px;
            x[m][t][1] = py;
#pragma unroll
            for (int v = 0; v < 4; ++v) q[m][t][v] = d.wnod[(m * 4 + v) * NE + i];
          }
          ++m;
        }
    }
    for (int it = 0; it < P.npic; ++it) {
      // mesh ODE: x_{m,1:} = Bt x_{m,0} + dt At V_m
      if (P.lagrangian) {
#pragma unroll
        for (int m = 0; m < nb; ++m) {
          double V[nt][2];
#pragma unroll
          for (int t = 0; t < nt; ++t) {
            V[t][0] = q[m][t][1] / q[m][t][0];
            V[t][1] = q[m][t][2] / q[m][t][0];
          }
#pragma unroll
          for (int r = 0; r < M; ++r)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
              double s = 0.0;
#pragma unroll
              for (int t = 0; t < nt; ++t) s += tb->At[r][t] * V[t][c];
              x[m][r + 1][c] = tb->Bt[r] * x[m][0][c] + dt * s;
            }
        }
      }
      double qn[nb][M][4];
#pragma unroll
      for (int m = 0; m < nb; ++m)
#pragma unroll
        for (int r = 0; r < M; ++r)
#pragma unroll
          for (int v = 0; v < 4; ++v) qn[m][r][v] = tb->Bt[r] * q[m][0][v];
#pragma unroll
      for (int t = 0; t < nt; ++t) {
        double f[nb][4], gg[nb][4];
#pragma unroll
        for (int m = 0; m < nb; ++m) {
          double u = q[m][t][1] / q[m][t][0], v = q[m][t][2] / q[m][t][0];
          double p = pressure(q[m][t], g);
          f[m][0] = q[m][t][1];
          f[m][1] = q[m][t][1] * u + p;
          f[m][2] = q[m][t][1] * v;
          f[m][3] = u * (q[m][t][3] + p);
          gg[m][0] = q[m][t][2];
          gg[m][1] = q[m][t][2] * u;
          gg[m][2] = q[m][t][2] * v + p;
          gg[m][3] = v * (q[m][t][3] + p);
        }
#pragma unroll
        for (int m = 0; m < nb; ++m) {
          double xx = 0, xe = 0, yx = 0, ye = 0, xtau = 0, ytau = 0;
#pragma unroll
          for (int k = 0; k < nb; ++k) {
            xx += tb->Dxi[m][k] * x[k][t][0];
            yx += tb->Dxi[m][k] * x[k][t][1];
            xe += tb->Deta[m][k] * x[k][t][0];
            ye += tb->Deta[m][k] * x[k][t][1];
          }
#pragma unroll
          for (int r = 0; r < nt; ++r) {
            xtau += tb->Dt[t][r] * x[m][r][0];
            ytau += tb->Dt[t][r] * x[m][r][1];
          }
          double det = xx * ye - xe * yx;
          double xi_x = ye / det, xi_y = -xe / det, eta_x = -yx / det, eta_y = xx / det;
          double xt = xtau / dt, yt = ytau / dt;
          double xi_t = -(xi_x * xt + xi_y * yt), eta_t = -(eta_x * xt + eta_y * yt);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            double qxi = 0, qeta = 0, fxi = 0, feta = 0, gxi = 0, geta = 0;
#pragma unroll
            for (int k = 0; k < nb; ++k) {
              qxi += tb->Dxi[m][k] * q[k][t][v];
              qeta += tb->Deta[m][k] * q[k][t][v];
              fxi += tb->Dxi[m][k] * f[k][v];
              feta += tb->Deta[m][k] * f[k][v];
              gxi += tb->Dxi[m][k] * gg[k][v];
              geta += tb->Deta[m][k] * gg[k][v];
            }
            double Pv = -(qxi * xi_t + qeta * eta_t + fxi * xi_x + feta * eta_x + gxi * xi_y + geta * eta_y);
#pragma unroll
            for (int r = 0; r < M; ++r) qn[m][r][v] += dt * tb->At[r][t] * Pv;
          }
        }
      }
#pragma unroll
      for (int m = 0; m < nb; ++m)
#pragma unroll
        for (int r = 0; r < M; ++r)
#pragma unroll
          for (int v = 0; v < 4; ++v) q[m][r + 1][v] = qn[m][r][v];
    }
    // publish: reference means, edge traces, vertex velocities of the final iterate
#pragma unroll
    for (int t = 0; t < nt; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double s = 0.0;
#pragma unroll
        for (int m = 0; m < nb; ++m) s += tb->amean[m] * q[m][t][v];
        d.avg[(t * 4 + v) * NE + i] = s;
      }
#pragma unroll
    for (int e = 0; e < 3; ++e)
#pragma unroll
      for (int gq = 0; gq < nG; ++gq)
#pragma unroll
        for (int t = 0; t < nt; ++t)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            double s = 0.0;
#pragma unroll
            for (int m = 0; m < nb; ++m) s += tb->edge[e][gq][m] * q[m][t][v];
            d.trace[(((e * nG + gq) * nt + t) * 4 + v) * NE + i] = s;
          }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int m = tb->vtx[k];
#pragma unroll
      for (int t = 0; t < nt; ++t) {
        double vx = 0.0, vy = 0.0;
        if (P.lagrangian) {
          vx = q[m][t][1] / q[m][t][0];
          vy = q[m][t][2] / q[m][t][0];
        }
        d.vvel[((k * nt + t) * 2 + 0) * NE + i] = vx;
        d.vvel[((k * nt + t) * 2 + 1) * NE + i] = vy;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Scheduling
// ---------------------------------------------------------------------------
__global__ void k_cycle_begin(Dev d) {
  d.scal->n_active = 0;
  d.scal->n_unfinished = 0;
}

__global__ void __launch_bounds__(TPB) k_sched(Dev d, int cycle) {
  const int NE = d.NE;
  const int N = d.scal->N;
  const int lane = threadIdx.x & 63;
  for (int base = blockIdx.x * blockDim.x; base < NE; base += gridDim.x * blockDim.x) {
    const int i = base + threadIdx.x;
    bool act = false, unf = false;
    if (i < NE) {
      const int n = d.tick[i];
      if (n < N) {
        unf = true;
        const int fut = n + d.step[i];
        int mx = 0, mn = 1 << 30;
        for (int r = d.sched_ptr[i]; r < d.sched_ptr[i + 1]; ++r) {
          int j = d.sched_idx[r];
          int nj = d.tick[j];
          mx = max(mx, nj);
          mn = min(mn, nj + d.step[j]);
        }
        act = (mx <= fut) && (fut <= mn);
      }
    }
    unsigned long long ma = __ballot(act);
    unsigned long long mu = __ballot(unf);
    int base_slot = 0;
    if (lane == 0) {
      if (ma) base_slot = atomicAdd(&d.scal->n_active, __popcll(ma));
      if (mu) atomicAdd(&d.scal->n_unfinished, __popcll(mu));
      if (ma) atomicAdd(&d.scal->updates, (unsigned long long)__popcll(ma));
    }
    base_slot = __shfl(base_slot, 0);
    if (act) {
      int pos = base_slot + __popcll(ma & ((1ull << lane) - 1ull));
      d.act_list[pos] = i;
      d.act_stamp[i] = cycle;
    }
  }
}

// ---------------------------------------------------------------------------
// Node solver and node motion
// ---------------------------------------------------------------------------
template <int M>
__global__ void __launch_bounds__(TPB) k_node(Dev d, const Tables* __restrict__ tb, Params P, int cycle) {
  constexpr int nt = M + 1;
  const int NE = d.NE, NV = d.NV;
  const double delta = d.scal->delta;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < NV; k += gridDim.x * blockDim.x) {
    const int r0 = d.ring_ptr[k], r1 = d.ring_ptr[k + 1];
    int newt = -1;
    for (int r = r0; r < r1; ++r) {
      int j = d.ring_ent[r] >> 2;
      if (d.act_stamp[j] == cycle) {
        newt = d.tick[j] + d.step[j];
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
      const int nj = d.tick[j], sj = d.step[j];
      if (sj <= 0) {
        ok = false;
        continue;
      }
      const double tau0 = double(nk - nj) / double(sj), tau1 = double(newt - nj) / double(sj);
      double L0[nt], L1[nt];
      time_antideriv<M>(tb, tau0, L0);
      time_antideriv<M>(tb, tau1, L1);
      double vx = 0.0, vy = 0.0;
#pragma unroll
      for (int q = 0; q < nt; ++q) {
        double I = L1[q] - L0[q];
        vx += I * d.vvel[((lv * nt + q) * 2 + 0) * NE + j];
        vy += I * d.vvel[((lv * nt + q) * 2 + 1) * NE + j];
      }
      const double inv = 1.0 / (tau1 - tau0);
      const double mu = d.Q[j] * d.A[j];
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
    const double dtk = double(newt - nk) * delta;
    d.Xnew[k] = d.X[k] + dtk * Vx;
    d.Xnew[NV + k] = d.X[NV + k] + dtk * Vy;
    d.ntick_new[k] = newt;
    d.node_stamp[k] = cycle;
    wave_count(&d.scal->n_node);
  }
}

// ---------------------------------------------------------------------------
// Space-time patch fluxes
// ---------------------------------------------------------------------------
template <int M>
__global__ void __launch_bounds__(TPB) k_patch(Dev d, const Tables* __restrict__ tb, Params P, int cycle) {
  constexpr int nt = M + 1, nG = M + 1;
  const int NE = d.NE, NV = d.NV, NF = d.NF;
  const double delta = d.scal->delta;
  const double g = P.gamma;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < NF; e += gridDim.x * blockDim.x) {
    const int a = d.e_a[e], b = d.e_b[e];
    const bool ma = d.node_stamp[a] == cycle, mb = d.node_stamp[b] == cycle;
    if (!ma && !mb) continue;
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
    const int sL = d.step[L];
    const double nL = d.tick[L];
    int sR = 1;
    double nR = 0.0;
    if (R >= 0) {
      sR = d.step[R];
      nR = d.tick[R];
    }
    if (sL <= 0 || sR <= 0) {
      set_err(d, ERR_PRED);
      continue;
    }
    double G[4] = {0, 0, 0, 0}, Nn[3] = {0, 0, 0};
#pragma unroll
    for (int gq = 0; gq < nG; ++gq) {
      double trL[nt][4], trR[nt][4];
#pragma unroll
      for (int t = 0; t < nt; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          trL[t][v] = d.trace[(((el * nG + gq) * nt + t) * 4 + v) * NE + L];
          trR[t][v] = R >= 0 ? d.trace[(((er * nG + (nG - 1 - gq)) * nt + t) * 4 + v) * NE + R] : 0.0;
        }
      const double c = tb->gchi[gq];
#pragma unroll
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
        double lL[nt];
        time_basis<M>(tb, (tk - nL) / double(sL), lL);
        double ql[4], qr[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double s = 0.0;
#pragma unroll
          for (int t = 0; t < nt; ++t) s += lL[t] * trL[t][v];
          ql[v] = s;
        }
        if (R >= 0) {
          double lR[nt];
          time_basis<M>(tb, (tk - nR) / double(sR), lR);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            double s = 0.0;
#pragma unroll
            for (int t = 0; t < nt; ++t) s += lR[t] * trR[t][v];
            qr[v] = s;
          }
        } else if (bc == 2) {
          const double nxy = sqrt(N[0] * N[0] + N[1] * N[1]);
          const double nx = N[0] / nxy, ny = N[1] / nxy;
          const double mn = ql[1] * nx + ql[2] * ny;
          qr[0] = ql[0];
          qr[1] = ql[1] - 2.0 * mn * nx;
          qr[2] = ql[2] - 2.0 * mn * ny;
          qr[3] = ql[3];
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v) qr[v] = ql[v];
        }
        double fl[4], fr[4];
        stflux(ql, N, g, fl);
        stflux(qr, N, g, fr);
        const double smax = fmax(stspeed(ql, N, g), stspeed(qr, N, g));
#pragma unroll
        for (int v = 0; v < 4; ++v) G[v] += w * (0.5 * (fl[v] + fr[v]) - 0.5 * smax * (qr[v] - ql[v]));
#pragma unroll
        for (int k = 0; k < 3; ++k) Nn[k] += w * N[k];
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) d.G[v * NF + e] = G[v];
#pragma unroll
    for (int k = 0; k < 3; ++k) d.Nint[k * NF + e] = Nn[k];
    d.edge_stamp[e] = cycle;
    wave_count(&d.scal->n_patch);
  }
}

// ---------------------------------------------------------------------------
// Memory variables and conservative update
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(TPB) k_update(Dev d, Params P, int cycle) {
  const int NE = d.NE, NV = d.NV, NF = d.NF;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < NE; i += gridDim.x * blockDim.x) {
    const bool act = d.act_stamp[i] == cycle;
    int es[3];
    bool any = false;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      es[k] = d.elem_edges[k * NE + i];
      if (d.edge_stamp[es[k]] != cycle) es[k] = -1;
      any |= es[k] >= 0;
    }
    if (!any && !act) continue;
    double qm[4], hm[3];
#pragma unroll
    for (int v = 0; v < 4; ++v) qm[v] = d.QM[v * NE + i];
#pragma unroll
    for (int c = 0; c < 3; ++c) hm[c] = d.HM[c * NE + i];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int e = es[k];
      if (e < 0) continue;
      const double sg = d.e_L[e] == i ? -1.0 : 1.0;
#pragma unroll
      for (int v = 0; v < 4; ++v) qm[v] += sg * d.G[v * NF + e];
#pragma unroll
      for (int c = 0; c < 3; ++c) hm[c] += sg * d.Nint[c * NF + e];
    }
    if (!act) {
#pragma unroll
      for (int v = 0; v < 4; ++v) d.QM[v * NE + i] = qm[v];
#pragma unroll
      for (int c = 0; c < 3; ++c) d.HM[c * NE + i] = hm[c];
      continue;
    }
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
    const double An = tri_area(X);
    const double A0 = d.A[i];
    if (!(An > 0.0)) set_err(d, ERR_GEOM);
    const double r = fmax(fmax(fabs(hm[0]), fabs(hm[1])), fabs(hm[2] - (An - A0)));
    const double rel = r / (A0 + An);
    atomic_max_pos(&d.scal->max_gcl_bits, rel);
    if (!(rel <= P.gcl_tol)) set_err(d, ERR_GCL);
    double qn[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) qn[v] = (A0 * d.Q[v * NE + i] + qm[v]) / An;
    const double pn = pressure(qn, P.gamma);
    if (!(qn[0] > 0.0) || !(pn > 0.0)) set_err(d, ERR_STATE);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      d.Q[v * NE + i] = qn[v];
      d.QM[v * NE + i] = 0.0;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) d.HM[c * NE + i] = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) d.Xe[c * NE + i] = X[c];
    d.A[i] = An;
    d.tick[i] = d.tick[i] + d.step[i];
    // commit the moved nodes (every writer stores the same value)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (mv[k]) {
        d.X[nd[k]] = X[2 * k];
        d.X[NV + nd[k]] = X[2 * k + 1];
        d.ntick[nd[k]] = d.ntick_new[nd[k]];
      }
  }
}

// ---------------------------------------------------------------------------
// Macro-step boundary
// ---------------------------------------------------------------------------
__global__ void k_reset_min(Dev d) { d.scal->min_dt_bits = ~0ull; }

__global__ void __launch_bounds__(TPB) k_min_dt(Dev d) {
  __shared__ double red[TPB];
  double m = DBL_MAX;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < d.NE; i += gridDim.x * blockDim.x)
    m = fmin(m, d.dtcfl[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = TPB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0 && red[0] > 0.0 && red[0] < DBL_MAX)
    atomicMin(&d.scal->min_dt_bits, (unsigned long long)__double_as_longlong(red[0]));
}

__global__ void k_macro_setup(Dev d, double t_end, int N) {
  Scal* s = d.scal;
  double dmin = __longlong_as_double((long long)s->min_dt_bits);
  double rest = (t_end - s->T) / double(N);
  s->delta = fmin(dmin, rest);
  s->N = N;
  s->t_end = t_end;
}

__global__ void __launch_bounds__(TPB) k_levels(Dev d) {
  const int N = d.scal->N;
  const double delta = d.scal->delta;
  const int n = max(d.NE, d.NV);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    if (i < d.NE) {
      int over;
      d.tick[i] = 0;
      d.step[i] = level_step(d.dtcfl[i], delta, N, 0, &over);
      if (over) atomicAdd(&d.scal->overshoots, 1ull);
    }
    if (i < d.NV) d.ntick[i] = 0;
  }
}

// All elements met at tick N: advance the common time and restart the ticks.
__global__ void __launch_bounds__(TPB) k_macro_end(Dev d) {
  const int n = max(d.NE, d.NV);
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid == 0) {
    Scal* s = d.scal;
    s->T = s->T + double(s->N) * s->delta;
  }
  for (int i = gid; i < n; i += gridDim.x * blockDim.x) {
    if (i < d.NE) d.tick[i] = 0;
    if (i < d.NV) d.ntick[i] = 0;
  }
}

__global__ void k_count_reset(Dev d) { d.scal->n_unfinished = 0; }

__global__ void __launch_bounds__(TPB) k_count(Dev d) {
  const int N = d.scal->N;
  for (int base = blockIdx.x * blockDim.x; base < d.NE; base += gridDim.x * blockDim.x) {
    const int i = base + threadIdx.x;
    bool unf = i < d.NE && d.tick[i] < N;
    unsigned long long m = __ballot(unf);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(&d.scal->n_unfinished, __popcll(m));
  }
}

// ---------------------------------------------------------------------------
// Set-up and I/O
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(TPB) k_init_geometry(Dev d) {
  const int NE = d.NE, NV = d.NV, NF = d.NF;
  const int n = max(max(NE, NV), NF);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    if (i < NE) {
      double X[6];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        int nd = d.tri[k * NE + i];
        X[2 * k] = d.X[nd];
        X[2 * k + 1] = d.X[NV + nd];
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) d.Xe[c * NE + i] = X[c];
      d.A[i] = tri_area(X);
      d.tick[i] = 0;
      d.step[i] = 0;
      d.act_stamp[i] = -1;
#pragma unroll
      for (int v = 0; v < 4; ++v) d.QM[v * NE + i] = 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c) d.HM[c * NE + i] = 0.0;
    }
    if (i < NV) {
      d.ntick[i] = 0;
      d.node_stamp[i] = -1;
    }
    if (i < NF) d.edge_stamp[i] = -1;
  }
}

__global__ void __launch_bounds__(TPB) k_check_state(Dev d, double g) {
  const int NE = d.NE;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < NE; i += gridDim.x * blockDim.x) {
    double q[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) q[v] = d.Q[v * NE + i];
    if (!(q[0] > 0.0) || !(pressure(q, g) > 0.0)) set_err(d, ERR_STATE);
  }
}

__global__ void __launch_bounds__(TPB) k_download_xy(Dev d, double* out) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < d.NV; k += gridDim.x * blockDim.x) {
    out[2 * k] = d.X[k];
    out[2 * k + 1] = d.X[d.NV + k];
  }
}

__global__ void __launch_bounds__(TPB) k_elem_times(Dev d, double* out) {
  const double T = d.scal->T, delta = d.scal->delta;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < d.NE; i += gridDim.x * blockDim.x)
    out[i] = T + double(d.tick[i]) * delta;
}

int grid_for(int n) {
  int b = (n + TPB - 1) / TPB;
  if (b < 1) b = 1;
  if (b > 8192) b = 8192;
  return b;
}

#define AW_LAUNCH(kern, n, stream, ...)                                                   \
  do {                                                                                    \
    hipLaunchKernelGGL(kern, dim3(grid_for(n)), dim3(TPB), 0, (hipStream_t)(stream),      \
                       __VA_ARGS__);                                                      \
    hipError_t _e = hipGetLastError();                                                    \
    if (_e != hipSuccess) return int(_e);                                                 \
  } while (0)

#define AW_LAUNCH1(kern, stream, ...)                                                     \
  do {                                                                                    \
    hipLaunchKernelGGL(kern, dim3(1), dim3(1), 0, (hipStream_t)(stream), __VA_ARGS__);    \
    hipError_t _e = hipGetLastError();                                                    \
    if (_e != hipSuccess) return int(_e);                                                 \
  } while (0)

template <int M>
int reconstruct_m(const Dev& d, const Params& p, int use_list, int set_level, void* s) {
  AW_LAUNCH(k_reconstruct<M>, d.NE, s, d, d.tab, p, use_list, set_level);
  return 0;
}

template <int M>
int predict_m(const Dev& d, const Params& p, int use_list, void* s) {
  AW_LAUNCH(k_predict<M>, d.NE, s, d, d.tab, p, use_list);
  return 0;
}

template <int M>
int node_m(const Dev& d, const Params& p, int cycle, void* s) {
  AW_LAUNCH(k_node<M>, d.NV, s, d, d.tab, p, cycle);
  return 0;
}

template <int M>
int patch_m(const Dev& d, const Params& p, int cycle, void* s) {
  AW_LAUNCH(k_patch<M>, d.NF, s, d, d.tab, p, cycle);
  return 0;
}

}  // namespace

int launch_init_geometry(const Dev& d, void* s) {
  int n = d.NE > d.NV ? d.NE : d.NV;
  if (d.NF > n) n = d.NF;
  AW_LAUNCH(k_init_geometry, n, s, d);
  return 0;
}

int launch_reconstruct(const Dev& d, const Params& p, int M, int use_list, int set_level, void* s) {
  switch (M) {
    case 1: return reconstruct_m<1>(d, p, use_list, set_level, s);
    case 2: return reconstruct_m<2>(d, p, use_list, set_level, s);
    case 3: return reconstruct_m<3>(d, p, use_list, set_level, s);
  }
  return int(hipErrorInvalidValue);
}

int launch_predict(const Dev& d, const Params& p, int M, int use_list, void* s) {
  switch (M) {
    case 1: return predict_m<1>(d, p, use_list, s);
    case 2: return predict_m<2>(d, p, use_list, s);
    case 3: return predict_m<3>(d, p, use_list, s);
  }
  return int(hipErrorInvalidValue);
}

int launch_macro_begin(const Dev& d, double t_end, int N, void* s) {
  AW_LAUNCH1(k_reset_min, s, d);
  AW_LAUNCH(k_min_dt, d.NE, s, d);
  AW_LAUNCH1(k_macro_setup, s, d, t_end, N);
  AW_LAUNCH(k_levels, d.NE > d.NV ? d.NE : d.NV, s, d);
  return 0;
}

int launch_cycle_begin(const Dev& d, void* s) {
  AW_LAUNCH1(k_cycle_begin, s, d);
  return 0;
}

int launch_sched(const Dev& d, int cycle, void* s) {
  AW_LAUNCH(k_sched, d.NE, s, d, cycle);
  return 0;
}

int launch_node(const Dev& d, const Params& p, int M, int cycle, void* s) {
  switch (M) {
    case 1: return node_m<1>(d, p, cycle, s);
    case 2: return node_m<2>(d, p, cycle, s);
    case 3: return node_m<3>(d, p, cycle, s);
  }
  return int(hipErrorInvalidValue);
}

int launch_patch(const Dev& d, const Params& p, int M, int cycle, void* s) {
  switch (M) {
    case 1: return patch_m<1>(d, p, cycle, s);
    case 2: return patch_m<2>(d, p, cycle, s);
    case 3: return patch_m<3>(d, p, cycle, s);
  }
  return int(hipErrorInvalidValue);
}

int launch_update(const Dev& d, const Params& p, int cycle, void* s) {
  AW_LAUNCH(k_update, d.NE, s, d, p, cycle);
  return 0;
}

int launch_status(const Dev& d, void* s) {
  AW_LAUNCH1(k_count_reset, s, d);
  AW_LAUNCH(k_count, d.NE, s, d);
  return 0;
}

int launch_macro_end(const Dev& d, void* s) {
  AW_LAUNCH(k_macro_end, d.NE > d.NV ? d.NE : d.NV, s, d);
  return 0;
}

int launch_download_xy(const Dev& d, double* out, void* s) {
  AW_LAUNCH(k_download_xy, d.NV, s, d, out);
  return 0;
}

int launch_elem_times(const Dev& d, double* out, void* s) {
  AW_LAUNCH(k_elem_times, d.NE, s, d, out);
  return 0;
}

int launch_check_state(const Dev& d, double gamma, void* s) {
  AW_LAUNCH(k_check_state, d.NE, s, d, gamma);
  return 0;
}

}  // namespace aw
