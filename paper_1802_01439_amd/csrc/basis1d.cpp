// 1D nodal basis, quadrature and the 1D SIPG matrices (host side).
#include "basis1d.h"

#include <cmath>

namespace dgmf {

namespace {

// Legendre P_n(t) and P_n'(t) on [-1,1] by the three-term recurrence.
void legendre(int n, double t, double& p, double& dp) {
  double p0 = 1.0, p1 = t;
  if (n == 0) { p = 1.0; dp = 0.0; return; }
  for (int j = 1; j < n; ++j) {
    double p2 = ((2.0 * j + 1.0) * t * p1 - j * p0) / (j + 1.0);
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  // derivative from (t^2-1) P_n' = n (t P_n - P_{n-1}); end points separately
  if (std::fabs(std::fabs(t) - 1.0) < 1e-300)
    dp = (t > 0 ? 1.0 : ((n % 2) ? 1.0 : -1.0)) * 0.5 * n * (n + 1.0);
  else
    dp = n * (t * p1 - p0) / (t * t - 1.0);
}

}  // namespace

void lgl_nodes(int k, double* x) {
  const int n = k + 1;
  x[0] = 0.0;
  x[n - 1] = 1.0;
  // interior: roots of P_k' on [-1,1]; Newton from Chebyshev-Lobatto guesses,
  // P_k'' from Legendre's equation (1-t^2) P'' = 2t P' - k(k+1) P.  Newton
  // converges quadratically: after a step below 1e-12 the error is at the
  // rounding level (a tighter test is never met and ran all 100 steps).
  for (int j = 1; j < k; ++j) {
    double t = -std::cos(M_PI * j / k);
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(k, t, p, dp);
      double d2 = (2.0 * t * dp - k * (k + 1.0) * p) / (1.0 - t * t);
      double dt = dp / d2;
      t -= dt;
      if (std::fabs(dt) < 1e-12) break;
    }
    x[j] = t;
  }
  // symmetrise about 0, then map to [0,1]
  for (int j = 1; j < k; ++j) {
    double s = 0.5 * (x[j] - x[n - 1 - j]);
    if (j <= n - 1 - j) {
      x[j] = s;
      x[n - 1 - j] = -s;
    }
  }
  for (int j = 1; j < k; ++j) x[j] = 0.5 * (x[j] + 1.0);
}

void gauss_rule(int m, double* x, double* w) {
  for (int j = 0; j < m; ++j) {
    double t = -std::cos(M_PI * (j + 0.75) / (m + 0.5));
    double p = 0, dp = 1;
    for (int it = 0; it < 100; ++it) {
      legendre(m, t, p, dp);
      double dt = p / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-12) break;
    }
    legendre(m, t, p, dp);
    x[j] = t;
    w[j] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
  for (int j = 0; j < m / 2; ++j) {  // exact symmetry
    double s = 0.5 * (x[m - 1 - j] - x[j]);
    double ww = 0.5 * (w[j] + w[m - 1 - j]);
    x[j] = -s;
    x[m - 1 - j] = s;
    w[j] = w[m - 1 - j] = ww;
  }
  if (m % 2) x[m / 2] = 0.0;
  for (int j = 0; j < m; ++j) {
    x[j] = 0.5 * (x[j] + 1.0);
    w[j] *= 0.5;
  }
}

namespace {

double lag(const std::vector<double>& xi, int a, double t) {
  double v = 1.0;
  for (size_t j = 0; j < xi.size(); ++j)
    if ((int)j != a) v *= (t - xi[j]) / (xi[a] - xi[j]);
  return v;
}

double lag_d(const std::vector<double>& xi, int a, double t) {
  double s = 0.0;
  const int n = (int)xi.size();
  for (int j = 0; j < n; ++j) {
    if (j == a) continue;
    double v = 1.0 / (xi[a] - xi[j]);
    for (int l = 0; l < n; ++l)
      if (l != a && l != j) v *= (t - xi[l]) / (xi[a] - xi[l]);
    s += v;
  }
  return s;
}

// derivative matrix of the Lagrange basis on points z at the points z
std::vector<double> colloc_deriv(const std::vector<double>& z) {
  const int m = (int)z.size();
  std::vector<double> D(m * m);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) D[i * m + j] = lag_d(z, j, z[i]);
  return D;
}

}  // namespace

std::vector<double> child_interp(int k, int c) {
  const int n = k + 1;
  std::vector<double> xi(n);
  lgl_nodes(k, xi.data());
  std::vector<double> P(n * n);
  for (int i = 0; i < n; ++i)
    for (int a = 0; a < n; ++a) P[i * n + a] = lag(xi, a, 0.5 * (xi[i] + c));
  return P;
}

Basis1D make_basis(int k, int m) {
  Basis1D B;
  B.k = k;
  B.n = k + 1;
  B.m = m;
  const int n = B.n;
  B.xi.resize(n);
  lgl_nodes(k, B.xi.data());
  B.zq.resize(m);
  B.wq.resize(m);
  gauss_rule(m, B.zq.data(), B.wq.data());
  B.S.resize(m * n);
  B.G.resize(m * n);
  for (int q = 0; q < m; ++q)
    for (int a = 0; a < n; ++a) {
      B.S[q * n + a] = lag(B.xi, a, B.zq[q]);
      B.G[q * n + a] = lag_d(B.xi, a, B.zq[q]);
    }
  B.D.resize(n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) B.D[i * n + j] = lag_d(B.xi, j, B.xi[i]);
  B.Mref.assign(n * n, 0.0);
  B.Kcell.assign(n * n, 0.0);
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      double sm = 0, sk = 0;
      for (int q = 0; q < m; ++q) {
        sm += B.wq[q] * B.S[q * n + a] * B.S[q * n + b];
        sk += B.wq[q] * B.G[q * n + a] * B.G[q * n + b];
      }
      B.Mref[a * n + b] = sm;
      B.Kcell[a * n + b] = sk;
    }
  B.Dg = colloc_deriv(B.zq);
  return B;
}

Sipg1D make_sipg_1d(const Basis1D& B, double sigma) {
  // On [0,1] with the own element's outward normal n = -1 at 0 and +1 at 1:
  //  right end, jump J = u(1) - uR(0), mean slope G = (u'(1) + uR'(0))/2:
  //    y_i += -1/2 l_i'(1) J - l_i(1) G + sigma l_i(1) J
  //  left end, J = u(0) - uL(1), G = (u'(0) + uL'(1))/2, n = -1:
  //    y_i += +1/2 l_i'(0) J + l_i(0) G + sigma l_i(0) J
  // With LGL nodes l_i(0) = delta_{i,0}, l_i(1) = delta_{i,n-1}.
  const int n = B.n;
  const double* D = B.D.data();
  const double* d0 = D;                  // row of l_b'(0)
  const double* d1 = D + (n - 1) * n;    // row of l_b'(1)
  Sipg1D S;
  S.Kown = B.Kcell;
  S.Kl.assign(n * n, 0.0);
  S.Kr.assign(n * n, 0.0);
  const int L = 0, R = n - 1;
  for (int i = 0; i < n; ++i)
    for (int b = 0; b < n; ++b) {
      double own = 0, kl = 0, kr = 0;
      const double iR = (i == R), iL = (i == L), bR = (b == R), bL = (b == L);
      // right end
      own += -0.5 * d1[i] * bR - iR * 0.5 * d1[b] + sigma * iR * bR;
      kr += +0.5 * d1[i] * (b == L) - iR * 0.5 * d0[b] - sigma * iR * (b == L);
      // left end
      own += +0.5 * d0[i] * bL + iL * 0.5 * d0[b] + sigma * iL * bL;
      kl += -0.5 * d0[i] * (b == R) + iL * 0.5 * d1[b] - sigma * iL * (b == R);
      S.Kown[i * n + b] += own;
      S.Kl[i * n + b] = kl;
      S.Kr[i * n + b] = kr;
    }
  return S;
}

}  // namespace dgmf
