// Compile-time constants of the reference element shared by the step and
// adjoint kernels (gfx950): the time basis and the reconstruction's basis of
// shifted monomials, with the quadrature of monomial means on a triangle.
#pragma once

#include <hip/hip_runtime.h>

namespace aw {
// internal linkage: each kernel file folds these constants into its own code
namespace {

// Monomial coefficients of the Lagrange polynomials l_q on the time nodes
// q/M (q = 0..M) and of their integrals from 0, evaluated at compile time so
// that they enter the kernels as constants (the same polynomials as the host
// tables, built as products of the linear factors (tau - j/M) / ((q - j)/M)).
template <int M>
struct TimePoly {
  static constexpr int T = M + 1;
  struct Coef {
    double lag[T][T];
    double lint[T][T + 1];
  };
  static constexpr Coef make() {
    Coef c{};
    for (int q = 0; q < T; ++q) {
      double p[T] = {};
      p[0] = 1.0;
      int deg = 0;
      for (int j = 0; j < T; ++j) {
        if (j == q) continue;
        const double tj = double(j) / M, den = double(q - j) / M;
        double np[T] = {};
        for (int k = 0; k <= deg; ++k) {
          np[k + 1] += p[k] / den;
          np[k] -= p[k] * tj / den;
        }
        ++deg;
        for (int k = 0; k < T; ++k) p[k] = np[k];
      }
      c.lint[q][0] = 0.0;
      for (int k = 0; k < T; ++k) {
        c.lag[q][k] = p[k];
        c.lint[q][k + 1] = p[k] / (k + 1);
      }
    }
    return c;
  }
  static constexpr Coef c = make();
};

template <int M>
__device__ inline void time_basis(double tau, double l[M + 1]) {
  constexpr auto& C = TimePoly<M>::c;
#pragma unroll
  for (int q = 0; q <= M; ++q) {
    double s = C.lag[q][M];
#pragma unroll
    for (int k = M - 1; k >= 0; --k) s = s * tau + C.lag[q][k];
    l[q] = s;
  }
}

template <int M>
__device__ inline void time_antideriv(double tau, double L[M + 1]) {
  constexpr auto& C = TimePoly<M>::c;
#pragma unroll
  for (int q = 0; q <= M; ++q) {
    double s = C.lint[q][M + 1];
#pragma unroll
    for (int k = M; k >= 0; --k) s = s * tau + C.lint[q][k];
    L[q] = s;
  }
}

// Means of the monomials x^a y^b over the reference triangle (0,0), (1,0),
// (0,1): 2 a! b! / (a + b + 2)!, in the order of increasing degree, then b.
template <int M>
struct RefMeans {
  static constexpr double fact(int n) { return n <= 1 ? 1.0 : n * fact(n - 1); }
  struct Arr {
    double v[(M + 1) * (M + 2) / 2];
    constexpr double operator[](int k) const { return v[k]; }
  };
  static constexpr Arr make() {
    Arr r{};
    int k = 0;
    for (int d = 0; d <= M; ++d)
      for (int b = 0; b <= d; ++b) r.v[k++] = 2.0 * fact(d - b) * fact(b) / fact(d + 2);
    return r;
  }
  static constexpr Arr m = make();
};

// The reconstruction's basis: the monomials x^a y^b (1 <= a + b <= M, by
// degree, then b) minus their means on the reference triangle. For it, at
// compile time: the oscillation-indicator matrix (sum over all derivatives of
// orders 1..M of the integral of their products over the reference triangle,
// eq. eqn.sigma) and the values at the nodal lattice (i/M, j/M), i + j <= M,
// ordered by j then i. Integrals of x^p y^q over the triangle: p! q! / (p+q+2)!.
template <int M>
struct MonoBasis {
  static constexpr int nb = (M + 1) * (M + 2) / 2, nu = nb - 1;
  struct Coef {
    double sig[nu][nu];
    double node[nb][nu];
  };
  static constexpr double fact(int n) { return n <= 1 ? 1.0 : n * fact(n - 1); }
  static constexpr double falling(int n, int k) { return k == 0 ? 1.0 : n * falling(n - 1, k - 1); }
  static constexpr double ipow(double x, int n) { return n == 0 ? 1.0 : x * ipow(x, n - 1); }
  static constexpr Coef make() {
    Coef c{};
    int ea[nb] = {}, eb[nb] = {};
    int k = 0;
    for (int d = 0; d <= M; ++d)
      for (int b = 0; b <= d; ++b) {
        ea[k] = d - b;
        eb[k] = b;
        ++k;
      }
    for (int l = 1; l < nb; ++l)
      for (int m = 1; m < nb; ++m) {
        double s = 0.0;
        for (int ord = 1; ord <= M; ++ord)
          for (int be = 0; be <= ord; ++be) {
            const int al = ord - be;
            if (ea[l] < al || eb[l] < be || ea[m] < al || eb[m] < be) continue;
            const int p = ea[l] + ea[m] - 2 * al, q = eb[l] + eb[m] - 2 * be;
            s += falling(ea[l], al) * falling(eb[l], be) * falling(ea[m], al) * falling(eb[m], be) *
                 fact(p) * fact(q) / fact(p + q + 2);
          }
        c.sig[l - 1][m - 1] = s;
      }
    int n = 0;
    for (int j = 0; j <= M; ++j)
      for (int i = 0; i + j <= M; ++i) {
        const double x = double(i) / M, y = double(j) / M;
        for (int l = 1; l < nb; ++l)
          c.node[n][l - 1] = ipow(x, ea[l]) * ipow(y, eb[l]) -
                             2.0 * fact(ea[l]) * fact(eb[l]) / fact(ea[l] + eb[l] + 2);
        ++n;
      }
    return c;
  }
  static constexpr Coef c = make();
};

// Means of the monomials x^a y^b (a + b <= M) over a triangle with vertices
// (x[k], y[k]), by a rule exact to degree M with its points written out: the
// centroid (M=1), the edge midpoints (M=2), and the vertices, edge midpoints
// and centroid with weights 3/60, 8/60, 27/60 (M=3).
template <int M>
__device__ inline void monomial_means(const double x[3], const double y[3], double mm[]) {
  constexpr int nb = (M + 1) * (M + 2) / 2;
#pragma unroll
  for (int k = 0; k < nb; ++k) mm[k] = 0.0;
  auto point = [&](double w, double px, double py) {
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
  };
  constexpr double third = 1.0 / 3.0;
  if constexpr (M == 1) {
    point(1.0, (x[0] + x[1] + x[2]) * third, (y[0] + y[1] + y[2]) * third);
  } else if constexpr (M == 2) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int k1 = k == 2 ? 0 : k + 1;
      point(third, 0.5 * (x[k] + x[k1]), 0.5 * (y[k] + y[k1]));
    }
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) point(3.0 / 60.0, x[k], y[k]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int k1 = k == 2 ? 0 : k + 1;
      point(8.0 / 60.0, 0.5 * (x[k] + x[k1]), 0.5 * (y[k] + y[k1]));
    }
    point(27.0 / 60.0, (x[0] + x[1] + x[2]) * third, (y[0] + y[1] + y[2]) * third);
  }
}

}  // namespace
}  // namespace aw
