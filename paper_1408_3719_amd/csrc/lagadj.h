// Per-edge and per-row pieces of the adjoint of one global time step with the
// mesh moving with the fluid (Lagrangian mode): the Rusanov and HLL fluxes
// through an unnormalised space-time normal, the flux over a bilinear space-time patch
// (interior, transmissive and slip-wall edges) and the geometry part of a
// least-squares row of the reconstruction, each with its vector-Jacobian
// product; triangle areas. Written for host and device so that the products
// can be checked against central differences on the CPU.
#pragma once

#include <cmath>

#include "common.h"

#if defined(__HIPCC__)
#define AWHD __host__ __device__
#else
#define AWHD
#endif

namespace aw {
namespace lag {

template <int M>
struct Dim {
  static constexpr int nb = (M + 1) * (M + 2) / 2, T = M + 1, nG = M + 1, nu = nb - 1;
};

// Lattice point m of the nodal set (i/M, j/M), ordered by j then i.
template <int M>
AWHD inline void lattice(int m, double& xi, double& eta) {
  int jj = 0, ii = m;
  while (ii > M - jj) {
    ii -= M + 1 - jj;
    ++jj;
  }
  xi = double(ii) / M;
  eta = double(jj) / M;
}

// Lagrange time basis l_q(tau) from the host tables' monomial coefficients.
template <int M>
AWHD inline void tbasis(const Tables& tb, double tau, double l[M + 1]) {
  for (int q = 0; q <= M; ++q) {
    double s = tb.lag[q][M];
    for (int k = M - 1; k >= 0; --k) s = s * tau + tb.lag[q][k];
    l[q] = s;
  }
}

// int_0^tau l_q
template <int M>
AWHD inline void tanti(const Tables& tb, double tau, double L[M + 1]) {
  for (int q = 0; q <= M; ++q) {
    double s = tb.Lint[q][M + 1];
    for (int k = M; k >= 0; --k) s = s * tau + tb.Lint[q][k];
    L[q] = s;
  }
}

// int_0^1 l_q
template <int M>
AWHD inline void tint01(const Tables& tb, double I[M + 1]) {
  for (int q = 0; q <= M; ++q) {
    double s = 0.0;
    for (int k = 0; k <= M + 1; ++k) s += tb.Lint[q][k];
    I[q] = s;
  }
}

AWHD inline void euler_f_g(const double q[4], double gam, double f[4], double g[4]) {
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

// qb += J_f(q)^T fb + J_g(q)^T gb
AWHD inline void euler_f_g_vjp(const double q[4], double gam, const double fb[4], const double gb[4],
                               double qb[4]) {
  const double r = q[0], u = q[1] / r, v = q[2] / r, E = q[3];
  const double gm = gam - 1.0;
  const double p = gm * (E - 0.5 * r * (u * u + v * v));
  const double H = E + p;
  double rb = 0.0, ub = 0.0, vb = 0.0, pb = 0.0, Eb = 0.0;
  rb += fb[0] * u;       ub += fb[0] * r;
  rb += fb[1] * u * u;   ub += fb[1] * 2.0 * r * u;   pb += fb[1];
  rb += fb[2] * u * v;   ub += fb[2] * r * v;         vb += fb[2] * r * u;
  ub += fb[3] * H;       Eb += fb[3] * u;             pb += fb[3] * u;
  rb += gb[0] * v;       vb += gb[0] * r;
  rb += gb[1] * u * v;   ub += gb[1] * r * v;         vb += gb[1] * r * u;
  rb += gb[2] * v * v;   vb += gb[2] * 2.0 * r * v;   pb += gb[2];
  vb += gb[3] * H;       Eb += gb[3] * v;             pb += gb[3] * v;
  // p = gm (E - (q1^2 + q2^2) / (2 q0)), u = q1 / q0, v = q2 / q0, r = q0
  Eb += gm * pb;
  rb += -gm * 0.5 * (u * u + v * v) * pb;
  ub += -gm * r * u * pb;
  vb += -gm * r * v * pb;
  qb[0] += rb - (ub * u + vb * v) / r;
  qb[1] += ub / r;
  qb[2] += vb / r;
  qb[3] += Eb;
}

// ------------------------------------------------------------------------
// Rusanov flux through an unnormalised space-time normal and its product
// ------------------------------------------------------------------------
AWHD inline double rus_speed(const double q[4], const double N[3], double gam, double* un_out, double* c_out) {
  const double r = q[0], u = q[1] / r, v = q[2] / r;
  const double p = (gam - 1.0) * (q[3] - 0.5 * r * (u * u + v * v));
  const double nxy = sqrt(N[0] * N[0] + N[1] * N[1]);
  const double un = u * N[0] + v * N[1] + N[2];
  const double c = sqrt(gam * p / r);
  *un_out = un;
  *c_out = c;
  return fabs(un) + c * nxy;
}

// qlb, qrb, Nb += the product of Fb with the Rusanov flux's Jacobian (the
// larger signal speed taken from the left state on ties, d|x|/dx = 0 at 0);
// the flux itself into F when F is not null.
AWHD inline void rusanov_flux_vjp(const double ql[4], const double qr[4], const double N[3], double gam,
                                  const double Fb[4], double qlb[4], double qrb[4], double Nb[3],
                                  double* F = nullptr) {
  double fl[4], gl[4], fr[4], gr[4], unl, cl, unr, cr;
  euler_f_g(ql, gam, fl, gl);
  euler_f_g(qr, gam, fr, gr);
  const double sl = rus_speed(ql, N, gam, &unl, &cl), sr = rus_speed(qr, N, gam, &unr, &cr);
  const bool left = sl >= sr;
  const double s = left ? sl : sr;
  if (F)
    for (int v = 0; v < 4; ++v)
      F[v] = 0.5 * ((fl[v] + fr[v]) * N[0] + (gl[v] + gr[v]) * N[1] + (ql[v] + qr[v]) * N[2]) -
             0.5 * s * (qr[v] - ql[v]);
  double fb[4], gb[4], sb = 0.0;
  for (int v = 0; v < 4; ++v) {
    fb[v] = 0.5 * N[0] * Fb[v];
    gb[v] = 0.5 * N[1] * Fb[v];
    qlb[v] += 0.5 * N[2] * Fb[v] + 0.5 * s * Fb[v];
    qrb[v] += 0.5 * N[2] * Fb[v] - 0.5 * s * Fb[v];
    sb -= 0.5 * Fb[v] * (qr[v] - ql[v]);
    Nb[0] += 0.5 * Fb[v] * (fl[v] + fr[v]);
    Nb[1] += 0.5 * Fb[v] * (gl[v] + gr[v]);
    Nb[2] += 0.5 * Fb[v] * (ql[v] + qr[v]);
  }
  euler_f_g_vjp(ql, gam, fb, gb, qlb);
  euler_f_g_vjp(qr, gam, fb, gb, qrb);
  // s = |u N0 + v N1 + N2| + c |N_xy| of the state that gives the maximum
  const double* q = left ? ql : qr;
  double* qsb = left ? qlb : qrb;
  const double un = left ? unl : unr, c = left ? cl : cr;
  const double nxy = sqrt(N[0] * N[0] + N[1] * N[1]);
  const double sg = un > 0.0 ? 1.0 : (un < 0.0 ? -1.0 : 0.0);
  const double r = q[0], u = q[1] / r, v = q[2] / r;
  Nb[0] += sb * (sg * u + c * N[0] / nxy);
  Nb[1] += sb * (sg * v + c * N[1] / nxy);
  Nb[2] += sb * sg;
  // through u, v and c = sqrt(gam p / r)
  const double gm = gam - 1.0;
  const double ub = sb * sg * N[0], vb = sb * sg * N[1];
  const double cb = sb * nxy;
  const double p = gm * (q[3] - 0.5 * r * (u * u + v * v));
  double rb = -cb * c / (2.0 * r), pb = cb * gam / (2.0 * c * r);
  double ubb = ub - gm * r * u * pb, vbb = vb - gm * r * v * pb;
  rb += -gm * 0.5 * (u * u + v * v) * pb;
  (void)p;
  qsb[0] += rb - (ubb * u + vbb * v) / r;
  qsb[1] += ubb / r;
  qsb[2] += vbb / r;
  qsb[3] += gm * pb;
}

// ------------------------------------------------------------------------
// HLL flux through an unnormalised space-time normal and its product
// ------------------------------------------------------------------------
// F~(q) . N = f N_x + g N_y + q N_t; its product: qb += J^T fb, Nb += (f . fb, g . fb, q . fb)
AWHD inline void ft_dot(const double q[4], const double N[3], double gam, double out[4]) {
  double f[4], g[4];
  euler_f_g(q, gam, f, g);
  for (int v = 0; v < 4; ++v) out[v] = f[v] * N[0] + g[v] * N[1] + q[v] * N[2];
}

AWHD inline void ft_dot_vjp(const double q[4], const double N[3], double gam, const double ob[4], double qb[4],
                            double Nb[3]) {
  double f[4], g[4], fb[4], gb[4];
  euler_f_g(q, gam, f, g);
  for (int v = 0; v < 4; ++v) {
    fb[v] = N[0] * ob[v];
    gb[v] = N[1] * ob[v];
    qb[v] += N[2] * ob[v];
    Nb[0] += f[v] * ob[v];
    Nb[1] += g[v] * ob[v];
    Nb[2] += q[v] * ob[v];
  }
  euler_f_g_vjp(q, gam, fb, gb, qb);
}

// u . N_xy + N_t + sgn c |N_xy| and its product with sb onto q and N
AWHD inline double hll_speed(const double q[4], const double N[3], double gam, double sgn) {
  const double r = q[0], u = q[1] / r, v = q[2] / r;
  const double p = (gam - 1.0) * (q[3] - 0.5 * r * (u * u + v * v));
  return u * N[0] + v * N[1] + N[2] + sgn * sqrt(gam * p / r) * sqrt(N[0] * N[0] + N[1] * N[1]);
}

AWHD inline void hll_speed_vjp(const double q[4], const double N[3], double gam, double sgn, double sb, double qb[4],
                               double Nb[3]) {
  const double r = q[0], u = q[1] / r, v = q[2] / r;
  const double gm = gam - 1.0;
  const double p = gm * (q[3] - 0.5 * r * (u * u + v * v));
  const double c = sqrt(gam * p / r);
  const double nxy = sqrt(N[0] * N[0] + N[1] * N[1]);
  Nb[0] += sb * (u + sgn * c * N[0] / nxy);
  Nb[1] += sb * (v + sgn * c * N[1] / nxy);
  Nb[2] += sb;
  // through u, v and c = sqrt(gam p / r)
  const double cb = sgn * sb * nxy;
  double rb = -cb * c / (2.0 * r), pb = cb * gam / (2.0 * c * r);
  const double ub = sb * N[0] - gm * r * u * pb, vb = sb * N[1] - gm * r * v * pb;
  rb += -gm * 0.5 * (u * u + v * v) * pb;
  qb[0] += rb - (ub * u + vb * v) / r;
  qb[1] += ub / r;
  qb[2] += vb / r;
  qb[3] += gm * pb;
}

// qlb, qrb, Nb += the product of Fb with the HLL flux's Jacobian: signal
// speeds bounded over both states (the left state's speed on ties), upwind
// when both have one sign, else (sr F(ql) - sl F(qr) + sl sr (qr - ql)) /
// (sr - sl); the flux itself into F when F is not null.
AWHD inline void hll_flux_vjp(const double ql[4], const double qr[4], const double N[3], double gam,
                              const double Fb[4], double qlb[4], double qrb[4], double Nb[3], double* F = nullptr) {
  const double l1 = hll_speed(ql, N, gam, -1.0), r1 = hll_speed(ql, N, gam, 1.0);
  const double l2 = hll_speed(qr, N, gam, -1.0), r2 = hll_speed(qr, N, gam, 1.0);
  const bool left_lo = l1 <= l2, left_hi = r1 >= r2;
  const double sl = left_lo ? l1 : l2, sr = left_hi ? r1 : r2;
  double fl[4], fr[4];
  ft_dot(ql, N, gam, fl);
  ft_dot(qr, N, gam, fr);
  if (sl >= 0.0) {
    if (F)
      for (int v = 0; v < 4; ++v) F[v] = fl[v];
    ft_dot_vjp(ql, N, gam, Fb, qlb, Nb);
    return;
  }
  if (sr <= 0.0) {
    if (F)
      for (int v = 0; v < 4; ++v) F[v] = fr[v];
    ft_dot_vjp(qr, N, gam, Fb, qrb, Nb);
    return;
  }
  const double id = 1.0 / (sr - sl);
  double flb[4], frb[4], slb = 0.0, srb = 0.0;
  for (int v = 0; v < 4; ++v) {
    const double d = qr[v] - ql[v];
    const double Fv = (sr * fl[v] - sl * fr[v] + sl * sr * d) * id;
    if (F) F[v] = Fv;
    flb[v] = sr * id * Fb[v];
    frb[v] = -sl * id * Fb[v];
    qrb[v] += sl * sr * id * Fb[v];
    qlb[v] -= sl * sr * id * Fb[v];
    srb += Fb[v] * (fl[v] + sl * d - Fv) * id;
    slb += Fb[v] * (-fr[v] + sr * d + Fv) * id;
  }
  ft_dot_vjp(ql, N, gam, flb, qlb, Nb);
  ft_dot_vjp(qr, N, gam, frb, qrb, Nb);
  hll_speed_vjp(left_lo ? ql : qr, N, gam, -1.0, slb, left_lo ? qlb : qrb, Nb);
  hll_speed_vjp(left_hi ? ql : qr, N, gam, 1.0, srb, left_hi ? qlb : qrb, Nb);
}

// ------------------------------------------------------------------------
// One edge's bilinear space-time patch over a global step (eqs.
// eqn.spacetimenodes, G_ij, eqn.STint): old nodes a, b at time 0, new nodes at
// dt; trL (nG, T, 4) the left element's trace along the edge. Outer state by
// edge kind: INTERIOR the right element's trace trR (read in reverse),
// TRANSMISSIVE the left element's predicted cell means avL (T, 4), SLIP the
// inner state with its normal momentum mirrored about the patch normal.
// ------------------------------------------------------------------------
enum { INTERIOR = 0, TRANSMISSIVE = 1, SLIP = 2 };

// q with the momentum reflected about the unit normal of N's space part
AWHD inline void mirror(const double q[4], const double N[3], double out[4]) {
  const double inxy = 1.0 / sqrt(N[0] * N[0] + N[1] * N[1]);
  const double nx = N[0] * inxy, ny = N[1] * inxy;
  const double mn = q[1] * nx + q[2] * ny;
  out[0] = q[0];
  out[1] = q[1] - 2.0 * mn * nx;
  out[2] = q[2] - 2.0 * mn * ny;
  out[3] = q[3];
}

// qb, Nb += the product of ob with mirror's Jacobian
AWHD inline void mirror_vjp(const double q[4], const double N[3], const double ob[4], double qb[4], double Nb[3]) {
  const double nxy = sqrt(N[0] * N[0] + N[1] * N[1]);
  const double nx = N[0] / nxy, ny = N[1] / nxy;
  const double mn = q[1] * nx + q[2] * ny, mb = ob[1] * nx + ob[2] * ny;
  qb[0] += ob[0];
  qb[1] += ob[1] - 2.0 * mb * nx;
  qb[2] += ob[2] - 2.0 * mb * ny;
  qb[3] += ob[3];
  // n = N_xy / |N_xy|: nbar = -2 (mb q_m + mn ob_m), projected off n
  const double bx = -2.0 * (mb * q[1] + mn * ob[1]), by = -2.0 * (mb * q[2] + mn * ob[2]);
  const double bn = bx * nx + by * ny;
  Nb[0] += (bx - bn * nx) / nxy;
  Nb[1] += (by - bn * ny) / nxy;
}
template <int M>
AWHD inline void patch_corners(const double xa[2], const double xb[2], const double xan[2], const double xbn[2],
                               double dt, double P[4][3]) {
  P[0][0] = xa[0];  P[0][1] = xa[1];  P[0][2] = 0.0;
  P[1][0] = xb[0];  P[1][1] = xb[1];  P[1][2] = 0.0;
  P[2][0] = xbn[0]; P[2][1] = xbn[1]; P[2][2] = dt;
  P[3][0] = xan[0]; P[3][1] = xan[1]; P[3][2] = dt;
}

template <int M>
AWHD inline void patch_point(const Tables& tb, int gq, int h, const double P[4][3], double N[3], double lt[M + 1],
                             double dchi[3], double dtau[3]) {
  const double c = tb.gchi[gq], t = tb.gchi[h];
  for (int k = 0; k < 3; ++k) {
    dchi[k] = (1.0 - t) * (P[1][k] - P[0][k]) + t * (P[2][k] - P[3][k]);
    dtau[k] = (1.0 - c) * (P[3][k] - P[0][k]) + c * (P[2][k] - P[1][k]);
  }
  N[0] = dchi[1] * dtau[2] - dchi[2] * dtau[1];
  N[1] = dchi[2] * dtau[0] - dchi[0] * dtau[2];
  N[2] = dchi[0] * dtau[1] - dchi[1] * dtau[0];
  tbasis<M>(tb, t, lt);
}

template <int M>
AWHD inline void patch_states(const double* trL, const double* trR, const double* avL, int kind, int gq,
                              const double lt[M + 1], const double N[3], double ql[4], double qr[4]) {
  constexpr int T = M + 1, nG = M + 1;
  for (int v = 0; v < 4; ++v) {
    double a = 0.0, b = 0.0;
    for (int s = 0; s < T; ++s) {
      a += lt[s] * trL[(gq * T + s) * 4 + v];
      if (kind == INTERIOR) b += lt[s] * trR[((nG - 1 - gq) * T + s) * 4 + v];
      if (kind == TRANSMISSIVE) b += lt[s] * avL[s * 4 + v];
    }
    ql[v] = a;
    qr[v] = b;
  }
  if (kind == SLIP) mirror(ql, N, qr);
}

// The flux through the patch, G (added to; Rusanov, or HLL when hll), and the
// products of Gb with its Jacobian: the rows of the trace adjoints trLb and (interior) trRb are
// written, the means' adjoint avLb (transmissive) and the four corner nodes'
// adjoints (xab, xbb, xanb, xbnb: x, y) are added to.
template <int M>
AWHD inline void patch_flux_vjp(const Tables& tb, double gam, const double xa[2], const double xb[2],
                                const double xan[2], const double xbn[2], double dt, const double* trL,
                                const double* trR, const double* avL, int kind, const double Gb[4], double G[4],
                                double* trLb, double* trRb, double* avLb, double xab[2], double xbb[2],
                                double xanb[2], double xbnb[2], bool hll = false) {
  constexpr int T = M + 1, nG = M + 1;
  double P[4][3], Pb[4][3] = {};
  patch_corners<M>(xa, xb, xan, xbn, dt, P);
  for (int gq = 0; gq < nG; ++gq) {
    double rl[T][4] = {}, rr[T][4] = {};
    for (int h = 0; h < nG; ++h) {
      double N[3], lt[M + 1], dc[3], dtau[3], ql[4], qr[4];
      patch_point<M>(tb, gq, h, P, N, lt, dc, dtau);
      patch_states<M>(trL, trR, avL, kind, gq, lt, N, ql, qr);
      const double w = tb.gw[gq] * tb.gw[h];
      double Fb[4], F[4], qlb[4] = {}, qrb[4] = {}, Nb[3] = {};
      for (int v = 0; v < 4; ++v) Fb[v] = w * Gb[v];
      if (hll)
        hll_flux_vjp(ql, qr, N, gam, Fb, qlb, qrb, Nb, F);
      else
        rusanov_flux_vjp(ql, qr, N, gam, Fb, qlb, qrb, Nb, F);
      for (int v = 0; v < 4; ++v) G[v] += w * F[v];
      if (kind == SLIP) mirror_vjp(ql, N, qrb, qlb, Nb);
      for (int s = 0; s < T; ++s)
        for (int v = 0; v < 4; ++v) {
          rl[s][v] += lt[s] * qlb[v];
          if (kind == INTERIOR) rr[s][v] += lt[s] * qrb[v];
          if (kind == TRANSMISSIVE) avLb[s * 4 + v] += lt[s] * qrb[v];
        }
      // N = dchi x dtau
      double dcb[3], dtb[3];
      dcb[0] = dtau[1] * Nb[2] - dtau[2] * Nb[1];
      dcb[1] = dtau[2] * Nb[0] - dtau[0] * Nb[2];
      dcb[2] = dtau[0] * Nb[1] - dtau[1] * Nb[0];
      dtb[0] = Nb[1] * dc[2] - Nb[2] * dc[1];
      dtb[1] = Nb[2] * dc[0] - Nb[0] * dc[2];
      dtb[2] = Nb[0] * dc[1] - Nb[1] * dc[0];
      const double c = tb.gchi[gq], t = tb.gchi[h];
      for (int k = 0; k < 3; ++k) {
        Pb[1][k] += (1.0 - t) * dcb[k] - c * dtb[k];
        Pb[0][k] -= (1.0 - t) * dcb[k] + (1.0 - c) * dtb[k];
        Pb[2][k] += t * dcb[k] + c * dtb[k];
        Pb[3][k] += -t * dcb[k] + (1.0 - c) * dtb[k];
      }
    }
    for (int s = 0; s < T; ++s)
      for (int v = 0; v < 4; ++v) {
        trLb[(gq * T + s) * 4 + v] = rl[s][v];
        if (kind == INTERIOR) trRb[((nG - 1 - gq) * T + s) * 4 + v] = rr[s][v];
      }
  }
  for (int c = 0; c < 2; ++c) {
    xab[c] += Pb[0][c];
    xbb[c] += Pb[1][c];
    xbnb[c] += Pb[2][c];
    xanb[c] += Pb[3][c];
  }
}

// Times of a patch swept in a cycle of the local time stepping: its corners
// (old a, old b, new b, new a) at ticks tk, and each side's predictor slab
// [n, n + s) in ticks (the right side unused on boundary edges); delta the
// tick length.
struct PatchTimes {
  double tk[4];
  double nL, sL, nR, sR;
  double delta;
};

// patch_flux_vjp for a patch with corners at different times: each side's
// traces are read at the rescaled time (tick - n) / s of the point.
template <int M>
AWHD inline void patch_flux_vjp_lts(const Tables& tb, double gam, const double xa[2], const double xb[2],
                                    const double xan[2], const double xbn[2], const PatchTimes& pt,
                                    const double* trL, const double* trR, const double* avL, int kind,
                                    const double Gb[4], double G[4], double* trLb, double* trRb, double* avLb,
                                    double xab[2], double xbb[2], double xanb[2], double xbnb[2], bool hll) {
  constexpr int T = M + 1, nG = M + 1;
  double P[4][3], Pb[4][3] = {};
  P[0][0] = xa[0];  P[0][1] = xa[1];  P[0][2] = pt.tk[0] * pt.delta;
  P[1][0] = xb[0];  P[1][1] = xb[1];  P[1][2] = pt.tk[1] * pt.delta;
  P[2][0] = xbn[0]; P[2][1] = xbn[1]; P[2][2] = pt.tk[2] * pt.delta;
  P[3][0] = xan[0]; P[3][1] = xan[1]; P[3][2] = pt.tk[3] * pt.delta;
  for (int gq = 0; gq < nG; ++gq) {
    double rl[T][4] = {}, rr[T][4] = {};
    for (int h = 0; h < nG; ++h) {
      double N[3], lt[M + 1], dc[3], dtau[3], ql[4], qr[4];
      patch_point<M>(tb, gq, h, P, N, lt, dc, dtau);
      const double c = tb.gchi[gq], t = tb.gchi[h];
      const double tkp = (1.0 - c) * (1.0 - t) * pt.tk[0] + c * (1.0 - t) * pt.tk[1] + c * t * pt.tk[2] +
                         (1.0 - c) * t * pt.tk[3];
      double lL[T], lR[T];
      tbasis<M>(tb, (tkp - pt.nL) / pt.sL, lL);
      tbasis<M>(tb, kind == INTERIOR ? (tkp - pt.nR) / pt.sR : 0.0, lR);
      for (int v = 0; v < 4; ++v) {
        double a = 0.0, b = 0.0;
        for (int s = 0; s < T; ++s) {
          a += lL[s] * trL[(gq * T + s) * 4 + v];
          if (kind == INTERIOR) b += lR[s] * trR[((nG - 1 - gq) * T + s) * 4 + v];
          if (kind == TRANSMISSIVE) b += lL[s] * avL[s * 4 + v];
        }
        ql[v] = a;
        qr[v] = b;
      }
      if (kind == SLIP) mirror(ql, N, qr);
      const double w = tb.gw[gq] * tb.gw[h];
      double Fb[4], F[4], qlb[4] = {}, qrb[4] = {}, Nb[3] = {};
      for (int v = 0; v < 4; ++v) Fb[v] = w * Gb[v];
      if (hll)
        hll_flux_vjp(ql, qr, N, gam, Fb, qlb, qrb, Nb, F);
      else
        rusanov_flux_vjp(ql, qr, N, gam, Fb, qlb, qrb, Nb, F);
      for (int v = 0; v < 4; ++v) G[v] += w * F[v];
      if (kind == SLIP) mirror_vjp(ql, N, qrb, qlb, Nb);
      for (int s = 0; s < T; ++s)
        for (int v = 0; v < 4; ++v) {
          rl[s][v] += lL[s] * qlb[v];
          if (kind == INTERIOR) rr[s][v] += lR[s] * qrb[v];
          if (kind == TRANSMISSIVE) avLb[s * 4 + v] += lL[s] * qrb[v];
        }
      double dcb[3], dtb[3];
      dcb[0] = dtau[1] * Nb[2] - dtau[2] * Nb[1];
      dcb[1] = dtau[2] * Nb[0] - dtau[0] * Nb[2];
      dcb[2] = dtau[0] * Nb[1] - dtau[1] * Nb[0];
      dtb[0] = Nb[1] * dc[2] - Nb[2] * dc[1];
      dtb[1] = Nb[2] * dc[0] - Nb[0] * dc[2];
      dtb[2] = Nb[0] * dc[1] - Nb[1] * dc[0];
      for (int k = 0; k < 3; ++k) {
        Pb[1][k] += (1.0 - t) * dcb[k] - c * dtb[k];
        Pb[0][k] -= (1.0 - t) * dcb[k] + (1.0 - c) * dtb[k];
        Pb[2][k] += t * dcb[k] + c * dtb[k];
        Pb[3][k] += -t * dcb[k] + (1.0 - c) * dtb[k];
      }
    }
    for (int s = 0; s < T; ++s)
      for (int v = 0; v < 4; ++v) {
        trLb[(gq * T + s) * 4 + v] += rl[s][v];
        if (kind == INTERIOR) trRb[((nG - 1 - gq) * T + s) * 4 + v] += rr[s][v];
      }
  }
  for (int c = 0; c < 2; ++c) {
    xab[c] += Pb[0][c];
    xbb[c] += Pb[1][c];
    xbnb[c] += Pb[2][c];
    xanb[c] += Pb[3][c];
  }
}

// Signed area of a triangle and its gradient with respect to the vertices.
AWHD inline double area3(const double X[6]) {
  return 0.5 * ((X[2] - X[0]) * (X[5] - X[1]) - (X[4] - X[0]) * (X[3] - X[1]));
}
AWHD inline void area3_grad(const double X[6], double s, double Xb[6]) {
  Xb[0] += s * 0.5 * (X[3] - X[5]);
  Xb[1] += s * 0.5 * (X[4] - X[2]);
  Xb[2] += s * 0.5 * (X[5] - X[1]);
  Xb[3] += s * 0.5 * (X[0] - X[4]);
  Xb[4] += s * 0.5 * (X[1] - X[3]);
  Xb[5] += s * 0.5 * (X[2] - X[0]);
}

// ------------------------------------------------------------------------
// Geometry of a least-squares row: the means over the triangle Xj of the
// monomials shifted by their reference means, in the reference frame of the
// triangle Xi (the rule exact to degree M of the reconstruction: centroid;
// edge midpoints; vertices, edge midpoints and centroid with 3/60, 8/60, 27/60)
// ------------------------------------------------------------------------
template <int M>
AWHD inline void mono_point(double w, double px, double py, double* mm) {
  double xp[M + 1], yp[M + 1];
  xp[0] = yp[0] = 1.0;
  for (int a = 1; a <= M; ++a) {
    xp[a] = xp[a - 1] * px;
    yp[a] = yp[a - 1] * py;
  }
  int k = 0;
  for (int dg = 0; dg <= M; ++dg)
    for (int b = 0; b <= dg; ++b) mm[k++] += w * xp[dg - b] * yp[b];
}

template <int M>
AWHD inline void mono_point_vjp(double w, double px, double py, const double* mmb, double& pxb, double& pyb) {
  double xp[M + 1], yp[M + 1];
  xp[0] = yp[0] = 1.0;
  for (int a = 1; a <= M; ++a) {
    xp[a] = xp[a - 1] * px;
    yp[a] = yp[a - 1] * py;
  }
  pxb = pyb = 0.0;
  int k = 0;
  for (int dg = 0; dg <= M; ++dg)
    for (int b = 0; b <= dg; ++b) {
      const int a = dg - b;
      if (a > 0) pxb += mmb[k] * w * a * xp[a - 1] * yp[b];
      if (b > 0) pyb += mmb[k] * w * b * xp[a] * yp[b - 1];
      ++k;
    }
}

// The rule's points as barycentric combinations of the three vertices.
template <int M>
struct RowRule {
  static constexpr int NP = M == 1 ? 1 : (M == 2 ? 3 : 7);
};

template <int M>
AWHD inline void row_rule_point(int p, double& w, double bc[3]) {
  const double third = 1.0 / 3.0;
  bc[0] = bc[1] = bc[2] = 0.0;
  if (M == 1) {
    w = 1.0;
    bc[0] = bc[1] = bc[2] = third;
  } else if (M == 2) {
    w = third;
    bc[p] = 0.5;
    bc[p == 2 ? 0 : p + 1] = 0.5;
  } else {
    if (p < 3) {
      w = 3.0 / 60.0;
      bc[p] = 1.0;
    } else if (p < 6) {
      w = 8.0 / 60.0;
      bc[p - 3] = 0.5;
      bc[p - 3 == 2 ? 0 : p - 2] = 0.5;
    } else {
      w = 27.0 / 60.0;
      bc[0] = bc[1] = bc[2] = third;
    }
  }
}

// Row a (nu values) of neighbour triangle Xj in the frame of Xi, given the
// shifted monomials' reference means refm (nb values).
template <int M>
AWHD inline void ls_row_geom(const double Xj[6], const double Xi[6], const double* refm, double* a) {
  constexpr int nb = Dim<M>::nb;
  const double e1x = Xi[2] - Xi[0], e1y = Xi[3] - Xi[1], e2x = Xi[4] - Xi[0], e2y = Xi[5] - Xi[1];
  const double idet = 1.0 / (e1x * e2y - e2x * e1y);
  double rx[3], ry[3];
  for (int k = 0; k < 3; ++k) {
    const double dx = Xj[2 * k] - Xi[0], dy = Xj[2 * k + 1] - Xi[1];
    rx[k] = (dx * e2y - dy * e2x) * idet;
    ry[k] = (e1x * dy - e1y * dx) * idet;
  }
  double mm[nb] = {};
  for (int p = 0; p < RowRule<M>::NP; ++p) {
    double w, bc[3];
    row_rule_point<M>(p, w, bc);
    mono_point<M>(w, bc[0] * rx[0] + bc[1] * rx[1] + bc[2] * rx[2], bc[0] * ry[0] + bc[1] * ry[1] + bc[2] * ry[2],
                  mm);
  }
  for (int l = 0; l + 1 < nb; ++l) a[l] = mm[l + 1] - refm[l + 1];
}

// Xjb, Xib += the product of ab (nu values) with ls_row_geom's Jacobian.
template <int M>
AWHD inline void ls_row_geom_vjp(const double Xj[6], const double Xi[6], const double* ab, double Xjb[6],
                                 double Xib[6]) {
  constexpr int nb = Dim<M>::nb;
  const double e1x = Xi[2] - Xi[0], e1y = Xi[3] - Xi[1], e2x = Xi[4] - Xi[0], e2y = Xi[5] - Xi[1];
  const double det = e1x * e2y - e2x * e1y;
  const double idet = 1.0 / det;
  double rx[3], ry[3], dx[3], dy[3];
  for (int k = 0; k < 3; ++k) {
    dx[k] = Xj[2 * k] - Xi[0];
    dy[k] = Xj[2 * k + 1] - Xi[1];
    rx[k] = (dx[k] * e2y - dy[k] * e2x) * idet;
    ry[k] = (e1x * dy[k] - e1y * dx[k]) * idet;
  }
  double mmb[nb];
  mmb[0] = 0.0;
  for (int l = 0; l + 1 < nb; ++l) mmb[l + 1] = ab[l];
  double rxb[3] = {}, ryb[3] = {};
  for (int p = 0; p < RowRule<M>::NP; ++p) {
    double w, bc[3], pxb, pyb;
    row_rule_point<M>(p, w, bc);
    mono_point_vjp<M>(w, bc[0] * rx[0] + bc[1] * rx[1] + bc[2] * rx[2],
                      bc[0] * ry[0] + bc[1] * ry[1] + bc[2] * ry[2], mmb, pxb, pyb);
    for (int k = 0; k < 3; ++k) {
      rxb[k] += bc[k] * pxb;
      ryb[k] += bc[k] * pyb;
    }
  }
  double e1xb = 0, e1yb = 0, e2xb = 0, e2yb = 0, idetb = 0;
  for (int k = 0; k < 3; ++k) {
    const double dxb = (rxb[k] * e2y - ryb[k] * e1y) * idet;
    const double dyb = (-rxb[k] * e2x + ryb[k] * e1x) * idet;
    Xjb[2 * k] += dxb;
    Xjb[2 * k + 1] += dyb;
    Xib[0] -= dxb;
    Xib[1] -= dyb;
    e2yb += rxb[k] * dx[k] * idet;
    e2xb -= rxb[k] * dy[k] * idet;
    e1xb += ryb[k] * dy[k] * idet;
    e1yb -= ryb[k] * dx[k] * idet;
    idetb += rxb[k] * rx[k] * det + ryb[k] * ry[k] * det;   // d rx / d idet = rx / idet
  }
  const double detb = -idetb * idet * idet;
  e1xb += detb * e2y;
  e2yb += detb * e1x;
  e2xb -= detb * e1y;
  e1yb -= detb * e2x;
  Xib[2] += e1xb;
  Xib[3] += e1yb;
  Xib[0] -= e1xb + e2xb;
  Xib[1] -= e1yb + e2yb;
  Xib[4] += e2xb;
  Xib[5] += e2yb;
}

}  // namespace lag
}  // namespace aw
