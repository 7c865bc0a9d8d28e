// Reference-element tables of the scheme, built on the host in FP64.
//
// Reconstruction basis: the orthogonal Dubiner polynomials on the reference
// triangle (the paper's Sec. 2.2 asks for an orthogonal basis), written as
//   psi_pq = [sum_s C(p,s)^2 (xi+eta-1)^s xi^(p-s)]
//          * [sum_t C(q+2p+1, q-t) C(q,t) (eta-1)^t eta^(q-t)],
// i.e. P_p(2xi/(1-eta)-1)(1-eta)^p P_q^(2p+1,0)(2eta-1) expanded in monomials,
// scaled to unit mean square.  psi_00 = 1.
// Predictor basis: Lagrange polynomials on the equispaced lattice (i/M, j/M)
// times Lagrange polynomials on the time nodes q/M (eq. thetaSol); the time
// factors of K_tau and M (eq. Ktau) and the reduced system that keeps only
// test functions with tau > 0 (eq. CGfinal with the tau = 0 values fixed).
#include <cmath>
#include <cstring>
#include <stdexcept>
#include <vector>

#include "common.h"
#include "host.h"

namespace aw {
namespace {

constexpr int PD = 8;  // polynomial coefficient array dimension (degree <= 7)

struct Poly {
  double c[PD][PD];
  Poly() { std::memset(c, 0, sizeof(c)); }
};

Poly pmul(const Poly& x, const Poly& y) {
  Poly r;
  for (int a = 0; a < PD; ++a)
    for (int b = 0; b < PD; ++b)
      if (x.c[a][b] != 0.0)
        for (int e = 0; a + e < PD; ++e)
          for (int f = 0; b + f < PD; ++f) r.c[a + e][b + f] += x.c[a][b] * y.c[e][f];
  return r;
}

Poly pdiff(const Poly& x, int da, int db) {
  Poly r;
  for (int a = da; a < PD; ++a)
    for (int b = db; b < PD; ++b) {
      double f = 1.0;
      for (int t = 0; t < da; ++t) f *= (a - t);
      for (int t = 0; t < db; ++t) f *= (b - t);
      r.c[a - da][b - db] += f * x.c[a][b];
    }
  return r;
}

double fact(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}

double binom(int n, int k) {
  if (k < 0 || k > n) return 0.0;
  return fact(n) / (fact(k) * fact(n - k));
}

// exact integral of xi^a eta^b over the reference triangle
double mono_int(int a, int b) { return fact(a) * fact(b) / fact(a + b + 2); }

double pint(const Poly& x) {
  double s = 0.0;
  for (int a = 0; a < PD; ++a)
    for (int b = 0; a + b < PD; ++b) s += x.c[a][b] * mono_int(a, b);
  return s;
}

// (u*xi + v*eta + w)^n as a polynomial
Poly lin_pow(double u, double v, double w, int n) {
  Poly r;
  r.c[0][0] = 1.0;
  Poly lin;
  lin.c[1][0] = u;
  lin.c[0][1] = v;
  lin.c[0][0] = w;
  for (int i = 0; i < n; ++i) r = pmul(r, lin);
  return r;
}

Poly dubiner(int p, int q) {
  Poly A, B;
  for (int s = 0; s <= p; ++s) {
    Poly t = pmul(lin_pow(1, 1, -1, s), lin_pow(1, 0, 0, p - s));
    double c = binom(p, s) * binom(p, s);
    for (int a = 0; a < PD; ++a)
      for (int b = 0; b < PD; ++b) A.c[a][b] += c * t.c[a][b];
  }
  for (int t = 0; t <= q; ++t) {
    Poly u = pmul(lin_pow(0, 1, -1, t), lin_pow(0, 1, 0, q - t));
    double c = binom(q + 2 * p + 1, q - t) * binom(q, t);
    for (int a = 0; a < PD; ++a)
      for (int b = 0; b < PD; ++b) B.c[a][b] += c * u.c[a][b];
  }
  return pmul(A, B);
}

double peval(const Poly& x, double xi, double eta) {
  double s = 0.0;
  for (int a = 0; a < PD; ++a)
    for (int b = 0; a + b < PD; ++b)
      if (x.c[a][b] != 0.0) s += x.c[a][b] * std::pow(xi, a) * std::pow(eta, b);
  return s;
}

// Gauss-Jordan inverse with partial pivoting (small dense matrices)
std::vector<double> invert(std::vector<double> A, int n) {
  std::vector<double> I(n * n, 0.0);
  for (int i = 0; i < n; ++i) I[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (A[piv * n + c] == 0.0) throw std::runtime_error("singular table matrix");
    for (int k = 0; k < n; ++k) {
      std::swap(A[c * n + k], A[piv * n + k]);
      std::swap(I[c * n + k], I[piv * n + k]);
    }
    double d = A[c * n + c];
    for (int k = 0; k < n; ++k) {
      A[c * n + k] /= d;
      I[c * n + k] /= d;
    }
    for (int r = 0; r < n; ++r)
      if (r != c) {
        double f = A[r * n + c];
        if (f == 0.0) continue;
        for (int k = 0; k < n; ++k) {
          A[r * n + k] -= f * A[c * n + k];
          I[r * n + k] -= f * I[c * n + k];
        }
      }
  }
  return I;
}

}  // namespace

void gauss_legendre01(int n, double* x, double* w) {
  // roots of P_n by Newton iteration, mapped to [0,1]
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    // z descends with i; store ascending on [0,1]
    x[n - 1 - i] = 0.5 * (1.0 + z);
    w[n - 1 - i] = 1.0 / ((1.0 - z * z) * dp * dp);
  }
}

void build_tables(int M, Tables& T) {
  std::memset(&T, 0, sizeof(T));
  if (M < 1 || M > MAXM) throw std::runtime_error("M out of range");
  const int nb = (M + 1) * (M + 2) / 2;
  T.M = M;
  T.nb = nb;
  T.nt = M + 1;
  T.nG = M + 1;
  T.ne = 2 * nb;
  {
    int k = 0;
    for (int d = 0; d <= M; ++d)
      for (int b = 0; b <= d; ++b) {
        T.monoA[k] = d - b;
        T.monoB[k] = b;
        ++k;
      }
  }
  // --- modal basis and Sigma -------------------------------------------------
  std::vector<Poly> psi;
  for (int d = 0; d <= M; ++d)
    for (int q = 0; q <= d; ++q) {
      int p = d - q;
      Poly P = dubiner(p, q);
      double ms = 2.0 * pint(pmul(P, P));
      double sc = 1.0 / std::sqrt(ms);
      if (p == 0 && q == 0) sc = 1.0 / P.c[0][0];
      for (int a = 0; a < PD; ++a)
        for (int b = 0; b < PD; ++b) P.c[a][b] *= sc;
      psi.push_back(P);
    }
  for (int l = 0; l < nb; ++l)
    for (int k = 0; k < nb; ++k) T.psiC[l][k] = psi[l].c[T.monoA[k]][T.monoB[k]];
  for (int l = 0; l < nb; ++l)
    for (int m = 0; m < nb; ++m) {
      double s = 0.0;
      for (int ord = 1; ord <= M; ++ord)
        for (int be = 0; be <= ord; ++be) {
          int al = ord - be;
          s += pint(pmul(pdiff(psi[l], al, be), pdiff(psi[m], al, be)));
        }
      T.Sigma[l][m] = s;
    }
  // --- nodal lattice ---------------------------------------------------------
  std::vector<double> nx, ny;
  for (int j = 0; j <= M; ++j)
    for (int i = 0; i + j <= M; ++i) {
      nx.push_back(double(i) / M);
      ny.push_back(double(j) / M);
    }
  for (int m = 0; m < nb; ++m) {
    if (nx[m] == 0.0 && ny[m] == 0.0) T.vtx[0] = m;
    if (nx[m] == 1.0 && ny[m] == 0.0) T.vtx[1] = m;
    if (nx[m] == 0.0 && ny[m] == 1.0) T.vtx[2] = m;
  }
  std::vector<double> V(nb * nb);
  for (int m = 0; m < nb; ++m)
    for (int k = 0; k < nb; ++k) V[m * nb + k] = std::pow(nx[m], T.monoA[k]) * std::pow(ny[m], T.monoB[k]);
  std::vector<double> Vi = invert(V, nb);   // Vi[k][m]: coefficient of mono k in phi_m
  std::vector<Poly> phi(nb);
  for (int m = 0; m < nb; ++m)
    for (int k = 0; k < nb; ++k) phi[m].c[T.monoA[k]][T.monoB[k]] = Vi[k * nb + m];
  for (int m = 0; m < nb; ++m) {
    Poly dx = pdiff(phi[m], 1, 0), dy = pdiff(phi[m], 0, 1);
    for (int mp = 0; mp < nb; ++mp) {
      T.Dxi[mp][m] = peval(dx, nx[mp], ny[mp]);
      T.Deta[mp][m] = peval(dy, nx[mp], ny[mp]);
    }
    T.amean[m] = 2.0 * pint(phi[m]);
    for (int l = 0; l < nb; ++l) T.psiNodes[m][l] = peval(psi[l], nx[m], ny[m]);
  }
  gauss_legendre01(M + 1, T.gchi, T.gw);
  gauss_legendre01(3, T.osh_s, T.osh_w);
  const double vx[3] = {0.0, 1.0, 0.0}, vy[3] = {0.0, 0.0, 1.0};
  for (int e = 0; e < 3; ++e)
    for (int g = 0; g <= M; ++g) {
      double c = T.gchi[g];
      double px = vx[e] + (vx[(e + 1) % 3] - vx[e]) * c;
      double py = vy[e] + (vy[(e + 1) % 3] - vy[e]) * c;
      for (int m = 0; m < nb; ++m) T.edge[e][g][m] = peval(phi[m], px, py);
    }
  // --- time basis --------------------------------------------------------------
  const int nt = M + 1;
  std::vector<double> Vt(nt * nt);
  for (int q = 0; q < nt; ++q)
    for (int k = 0; k < nt; ++k) Vt[q * nt + k] = std::pow(double(q) / M, k);
  std::vector<double> Vti = invert(Vt, nt);   // Vti[k][q]
  for (int q = 0; q < nt; ++q)
    for (int k = 0; k < nt; ++k) {
      T.lag[q][k] = Vti[k * nt + q];
      T.Lint[q][k + 1] = Vti[k * nt + q] / (k + 1);
    }
  // Kt[k][l] = int l_k l_l',  Mt[k][l] = int l_k l_l
  std::vector<double> Kt(nt * nt, 0.0), Mt(nt * nt, 0.0);
  for (int k = 0; k < nt; ++k)
    for (int l = 0; l < nt; ++l)
      for (int a = 0; a < nt; ++a)
        for (int b = 0; b < nt; ++b) {
          Mt[k * nt + l] += T.lag[k][a] * T.lag[l][b] / (a + b + 1);
          if (b > 0) Kt[k * nt + l] += T.lag[k][a] * T.lag[l][b] * b / (a + b);
        }
  std::vector<double> K11(M * M);
  for (int r = 0; r < M; ++r)
    for (int c = 0; c < M; ++c) K11[r * M + c] = Kt[(r + 1) * nt + (c + 1)];
  std::vector<double> K11i = invert(K11, M);
  for (int r = 0; r < M; ++r) {
    double b = 0.0;
    for (int c = 0; c < M; ++c) b -= K11i[r * M + c] * Kt[(c + 1) * nt + 0];
    T.Bt[r] = b;
    for (int q = 0; q < nt; ++q) {
      double a = 0.0;
      for (int c = 0; c < M; ++c) a += K11i[r * M + c] * Mt[(c + 1) * nt + q];
      T.At[r][q] = a;
    }
  }
  for (int qp = 0; qp < nt; ++qp)
    for (int q = 0; q < nt; ++q) {
      double tau = double(qp) / M, s = 0.0;
      for (int k = 1; k < nt; ++k) s += k * T.lag[q][k] * std::pow(tau, k - 1);
      T.Dt[qp][q] = s;
    }
  // --- triangle rule exact to degree M (barycentric) -----------------------------
  auto add = [&](double w, double a, double b, double c) {
    T.rqw[T.nrq] = w;
    T.rqb[T.nrq][0] = a;
    T.rqb[T.nrq][1] = b;
    T.rqb[T.nrq][2] = c;
    T.nrq++;
  };
  if (M == 1) {
    add(1.0, 1.0 / 3, 1.0 / 3, 1.0 / 3);
  } else if (M == 2) {
    add(1.0 / 3, 0.5, 0.5, 0.0);
    add(1.0 / 3, 0.0, 0.5, 0.5);
    add(1.0 / 3, 0.5, 0.0, 0.5);
  } else {
    add(3.0 / 60, 1, 0, 0);
    add(3.0 / 60, 0, 1, 0);
    add(3.0 / 60, 0, 0, 1);
    add(8.0 / 60, 0.5, 0.5, 0.0);
    add(8.0 / 60, 0.0, 0.5, 0.5);
    add(8.0 / 60, 0.5, 0.0, 0.5);
    add(27.0 / 60, 1.0 / 3, 1.0 / 3, 1.0 / 3);
  }
}

}  // namespace aw
