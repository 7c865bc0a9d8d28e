// Central-difference check of the vector-Jacobian products in
// paper_1408_3719_amd/csrc/lagadj.h (host build, no GPU): for each piece, a
// seeded random point and random output adjoint ybar, the product xbar =
// J^T ybar against (L(x + h e_k) - L(x - h e_k)) / 2h with L = ybar . f(x),
// for every input component k. Prints one line per piece and order:
// "<piece> M=<M> <max relative deviation>".
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "host.h"
#include "lagadj.h"

using namespace aw;
using namespace aw::lag;

static std::mt19937_64 rng(20140815);
static double uni(double a, double b) { return std::uniform_real_distribution<double>(a, b)(rng); }

// a state near rho = 1, p = 1 with a moderate velocity
static void state(double q[4]) {
  const double r = uni(0.8, 1.2), u = uni(-0.3, 0.3), v = uni(-0.3, 0.3), p = uni(0.8, 1.2);
  q[0] = r;
  q[1] = r * u;
  q[2] = r * v;
  q[3] = p / 0.4 + 0.5 * r * (u * u + v * v);
}

static void triangle(double X[6], double cx, double cy, double h) {
  X[0] = cx + uni(-0.1, 0.1) * h;
  X[1] = cy + uni(-0.1, 0.1) * h;
  X[2] = cx + h + uni(-0.1, 0.1) * h;
  X[3] = cy + uni(-0.1, 0.1) * h;
  X[4] = cx + 0.3 * h + uni(-0.1, 0.1) * h;
  X[5] = cy + 0.9 * h + uni(-0.1, 0.1) * h;
}

// max over k of |fd_k - an_k| / (max_k |fd_k| + 1e-300)
template <class F>
static double check(std::vector<double>& x, const std::vector<double>& an, F L, double h) {
  double dmax = 0.0, scale = 0.0;
  for (size_t k = 0; k < x.size(); ++k) {
    const double x0 = x[k];
    const double hk = h * fmax(1.0, fabs(x0));
    x[k] = x0 + hk;
    const double lp = L(x);
    x[k] = x0 - hk;
    const double lm = L(x);
    x[k] = x0;
    const double fd = (lp - lm) / (2.0 * hk);
    dmax = fmax(dmax, fabs(fd - an[k]));
    scale = fmax(scale, fabs(fd));
  }
  return dmax / (scale + 1e-300);
}

template <int M>
static void run(const Tables& tb) {
  using D = Dim<M>;
  constexpr int nb = D::nb, T = D::T, nG = D::nG, nu = D::nu;
  const double gam = 1.4, dt = 0.02;
  // ---- space-time patch flux ------------------------------------------------
  for (int kh = 0; kh < 6; ++kh) {
    const int kind = kh % 3;
    const bool hll = kh >= 3;
    const int NT = nG * T * 4;
    std::vector<double> x(2 * NT + T * 4 + 8);
    for (int k = 0; k < 2 * nG * T; ++k) state(&x[k * 4]);
    for (int t = 0; t < T; ++t) state(&x[2 * NT + t * 4]);
    double* c = &x[2 * NT + T * 4];
    c[0] = 0.0 + uni(-0.01, 0.01);
    c[1] = 0.0 + uni(-0.01, 0.01);
    c[2] = 0.1 + uni(-0.01, 0.01);
    c[3] = 0.05 + uni(-0.01, 0.01);
    c[4] = c[0] + uni(-0.004, 0.004);
    c[5] = c[1] + uni(-0.004, 0.004);
    c[6] = c[2] + uni(-0.004, 0.004);
    c[7] = c[3] + uni(-0.004, 0.004);
    double Gb[4];
    for (auto& v : Gb) v = uni(-1, 1);
    auto L = [&](const std::vector<double>& y) {
      const double* cc = &y[2 * NT + T * 4];
      double G[4] = {0, 0, 0, 0}, c8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      std::vector<double> t1(NT), t2(NT), t3(T * 4);
      patch_flux_vjp<M>(tb, gam, cc, cc + 2, cc + 4, cc + 6, dt, y.data(), y.data() + NT, y.data() + 2 * NT, kind,
                        Gb, G, t1.data(), t2.data(), t3.data(), c8, c8 + 2, c8 + 4, c8 + 6, hll);
      return Gb[0] * G[0] + Gb[1] * G[1] + Gb[2] * G[2] + Gb[3] * G[3];
    };
    std::vector<double> an(x.size(), 0.0);
    double* ac = &an[2 * NT + T * 4];
    double G[4] = {0, 0, 0, 0};
    patch_flux_vjp<M>(tb, gam, c, c + 2, c + 4, c + 6, dt, x.data(), x.data() + NT, x.data() + 2 * NT, kind, Gb, G,
                      an.data(), an.data() + NT, an.data() + 2 * NT, ac, ac + 2, ac + 4, ac + 6, hll);
    const char* name[3] = {"interior", "transmissive", "slip"};
    std::printf("patch_%s%s M=%d %.3e\n", hll ? "hll_" : "", name[kind], M, check(x, an, L, 1e-6));
    // the same patch swept in a cycle of the local time stepping: corners at
    // different ticks, each side read over its own slab
    PatchTimes pt;
    pt.tk[0] = 0.0;
    pt.tk[1] = 2.0;
    pt.tk[2] = 4.0;
    pt.tk[3] = 3.0;
    pt.nL = 0.0;
    pt.sL = 4.0;
    pt.nR = 2.0;
    pt.sR = 2.0;
    pt.delta = dt / 4.0;
    auto Lt = [&](const std::vector<double>& y) {
      const double* cc = &y[2 * NT + T * 4];
      double G[4] = {0, 0, 0, 0}, c8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      std::vector<double> t1(NT), t2(NT), t3(T * 4);
      patch_flux_vjp_lts<M>(tb, gam, cc, cc + 2, cc + 4, cc + 6, pt, y.data(), y.data() + NT, y.data() + 2 * NT,
                            kind, Gb, G, t1.data(), t2.data(), t3.data(), c8, c8 + 2, c8 + 4, c8 + 6, hll);
      return Gb[0] * G[0] + Gb[1] * G[1] + Gb[2] * G[2] + Gb[3] * G[3];
    };
    std::vector<double> at(x.size(), 0.0);
    double* act = &at[2 * NT + T * 4];
    double Gt[4] = {0, 0, 0, 0};
    patch_flux_vjp_lts<M>(tb, gam, c, c + 2, c + 4, c + 6, pt, x.data(), x.data() + NT, x.data() + 2 * NT, kind, Gb,
                          Gt, at.data(), at.data() + NT, at.data() + 2 * NT, act, act + 2, act + 4, act + 6, hll);
    std::printf("patch_lts_%s%s M=%d %.3e\n", hll ? "hll_" : "", name[kind], M, check(x, at, Lt, 1e-6));
  }
  // ---- least-squares row geometry ------------------------------------------
  {
    std::vector<double> x(12);
    triangle(&x[0], 0.15, 0.1, 0.2);
    triangle(&x[6], 0.0, 0.0, 0.2);
    double refm[nb], ab[nu];
    for (auto& v : refm) v = uni(0, 1);
    for (auto& v : ab) v = uni(-1, 1);
    auto L = [&](const std::vector<double>& y) {
      double a[nu];
      ls_row_geom<M>(&y[0], &y[6], refm, a);
      double s = 0.0;
      for (int l = 0; l < nu; ++l) s += ab[l] * a[l];
      return s;
    };
    std::vector<double> an(12, 0.0);
    ls_row_geom_vjp<M>(&x[0], &x[6], ab, &an[0], &an[6]);
    std::printf("ls_row M=%d %.3e\n", M, check(x, an, L, 1e-6));
    // the row itself: means of the monomials over Xj in the frame of Xi by a
    // collapsed 12 x 12 Gauss rule (exact far beyond degree M)
    double zero[nb] = {}, a[nu];
    ls_row_geom<M>(&x[0], &x[6], zero, a);
    const double* Xi = &x[6];
    const double e1x = Xi[2] - Xi[0], e1y = Xi[3] - Xi[1], e2x = Xi[4] - Xi[0], e2y = Xi[5] - Xi[1];
    const double det = e1x * e2y - e2x * e1y;
    double gx[12], gw[12], mm[nb] = {}, wsum = 0.0;
    gauss_legendre01(12, gx, gw);
    for (int p = 0; p < 12; ++p)
      for (int q = 0; q < 12; ++q) {
        const double l1 = gx[p], l2 = gx[q] * (1.0 - gx[p]), w = gw[p] * gw[q] * (1.0 - gx[p]);
        const double px = (1.0 - l1 - l2) * x[0] + l1 * x[2] + l2 * x[4];
        const double py = (1.0 - l1 - l2) * x[1] + l1 * x[3] + l2 * x[5];
        const double dx = px - Xi[0], dy = py - Xi[1];
        const double xi = (dx * e2y - dy * e2x) / det, eta = (e1x * dy - e1y * dx) / det;
        int k = 0;
        for (int dg = 0; dg <= M; ++dg)
          for (int b = 0; b <= dg; ++b) mm[k++] += w * std::pow(xi, dg - b) * std::pow(eta, b);
        wsum += w;
      }
    double dev = 0.0;
    for (int l = 0; l < nu; ++l) dev = fmax(dev, fabs(a[l] - mm[l + 1] / wsum) / fmax(1.0, fabs(a[l])));
    std::printf("ls_row_means M=%d %.3e\n", M, dev);
  }
}

int main() {
  for (int M = 1; M <= 3; ++M) {
    Tables tb;
    build_tables(M, tb);
    if (M == 1) run<1>(tb);
    if (M == 2) run<2>(tb);
    if (M == 3) run<3>(tb);
  }
  // ---- area and Rusanov flux (order independent) ---------------------------
  {
    std::vector<double> x(6);
    triangle(x.data(), 0.0, 0.0, 1.0);
    const double sb = uni(-1, 1);
    std::vector<double> an(6, 0.0);
    area3_grad(x.data(), sb, an.data());
    std::printf("area M=0 %.3e\n", check(x, an, [&](const std::vector<double>& y) { return sb * area3(y.data()); }, 1e-6));
  }
  for (int rep = 0; rep < 6; ++rep) {
    // N_t chosen so that the two signal speeds straddle 0, or both are
    // positive (upwind left), or both negative (upwind right)
    std::vector<double> x(11);
    state(&x[0]);
    state(&x[4]);
    x[8] = uni(-0.1, 0.1);
    x[9] = uni(-0.1, 0.1);
    const double shift = rep < 2 ? 0.0 : (rep < 4 ? 1.0 : -1.0);
    x[10] = uni(-0.02, 0.02) + shift;
    double Fb[4];
    for (auto& v : Fb) v = uni(-1, 1);
    auto L = [&](const std::vector<double>& y) {
      double F[4], d1[4], d2[4], d3[3];
      hll_flux_vjp(&y[0], &y[4], &y[8], 1.4, Fb, d1, d2, d3, F);
      return Fb[0] * F[0] + Fb[1] * F[1] + Fb[2] * F[2] + Fb[3] * F[3];
    };
    std::vector<double> an(11, 0.0);
    hll_flux_vjp(&x[0], &x[4], &x[8], 1.4, Fb, &an[0], &an[4], &an[8]);
    const char* nm[3] = {"hll_middle", "hll_upwind_left", "hll_upwind_right"};
    std::printf("%s M=0 %.3e\n", nm[rep / 2], check(x, an, L, 1e-7));
  }
  for (int rep = 0; rep < 4; ++rep) {
    std::vector<double> x(11);
    state(&x[0]);
    state(&x[4]);
    x[8] = uni(-0.1, 0.1);
    x[9] = uni(-0.1, 0.1);
    x[10] = uni(-0.05, 0.05);
    double Fb[4];
    for (auto& v : Fb) v = uni(-1, 1);
    auto L = [&](const std::vector<double>& y) {
      double F[4], d1[4], d2[4], d3[3];
      rusanov_flux_vjp(&y[0], &y[4], &y[8], 1.4, Fb, d1, d2, d3, F);
      return Fb[0] * F[0] + Fb[1] * F[1] + Fb[2] * F[2] + Fb[3] * F[3];
    };
    std::vector<double> an(11, 0.0);
    rusanov_flux_vjp(&x[0], &x[4], &x[8], 1.4, Fb, &an[0], &an[4], &an[8]);
    std::printf("rusanov M=0 %.3e\n", check(x, an, L, 1e-7));
  }
  return 0;
}
