// Compile-time 1D tables for kernels whose tables depend on the degree alone:
// LGL nodes (Sec. 3.2: end points and the roots of P_k'), the m-point Gauss
// rule and the LGL Lagrange basis and its derivative at the Gauss points.
// Evaluated by the compiler in double precision, so that kernels see every
// entry as an immediate constant (no table loads at run time).
//
// Roots are bracketed by interlacing: the roots of P_{j+1} are separated by
// those of P_j (and -1, 1), and the roots of P_k' by those of P_k; each
// bracket is bisected to a width below the spacing of doubles near 1.  Node
// sets are then symmetrised.
#pragma once

namespace dgmf {
namespace ct {

constexpr int kMaxPts = 32;

struct LegPair {
  double p, pm1;   // P_n(t), P_{n-1}(t)
};

constexpr LegPair legendre2(int n, double t) {
  if (n == 0) return {1.0, 0.0};
  double p0 = 1.0, p1 = t;
  for (int j = 1; j < n; ++j) {
    const double p2 = ((2.0 * j + 1.0) * t * p1 - j * p0) / (j + 1.0);
    p0 = p1;
    p1 = p2;
  }
  return {p1, p0};
}

// f(t) = P_n(t) (kind 0) or t P_n(t) - P_{n-1}(t) = (t^2-1) P_n'(t) / n
// (kind 1, same roots as P_n' inside (-1, 1)).
constexpr double leg_f(int kind, int n, double t) {
  const LegPair r = legendre2(n, t);
  return kind == 0 ? r.p : t * r.p - r.pm1;
}

constexpr double bisect(int kind, int n, double lo, double hi) {
  const bool neg_lo = leg_f(kind, n, lo) < 0;
  for (int it = 0; it < 64; ++it) {   // bracket width <= 2^-63 after 64 halvings
    const double mid = 0.5 * (lo + hi);
    if (!(mid > lo && mid < hi)) break;
    if ((leg_f(kind, n, mid) < 0) == neg_lo) lo = mid;
    else hi = mid;
  }
  return 0.5 * (lo + hi);
}

// roots of P_m on (-1, 1), ascending, into r[0..m)
constexpr void legendre_roots(int m, double (&r)[kMaxPts]) {
  double prev[kMaxPts] = {};
  int np = 0;
  for (int j = 1; j <= m; ++j) {
    double cur[kMaxPts] = {};
    for (int i = 0; i < j; ++i) {
      const double lo = i == 0 ? -1.0 : prev[i - 1];
      const double hi = i == j - 1 ? 1.0 : prev[i];
      cur[i] = bisect(0, j, lo, hi);
    }
    for (int i = 0; i < j; ++i) prev[i] = cur[i];
    np = j;
  }
  for (int i = 0; i < np; ++i) r[i] = prev[i];
}

template <int N, int Q>
struct Tables {
  double xi[N];     // LGL nodes on [0, 1]
  double z[Q];      // Gauss points on [0, 1]
  double w[Q];      // Gauss weights on [0, 1]
  double S[Q][N];   // l_a(z_q)
  double G[Q][N];   // l_a'(z_q)

  constexpr Tables() : xi{}, z{}, w{}, S{}, G{} {
    // LGL nodes: -1, roots of P_k' between consecutive roots of P_k, 1
    const int k = N - 1;
    double t[kMaxPts] = {};
    t[0] = -1.0;
    t[N - 1] = 1.0;
    if (k >= 2) {
      double rk[kMaxPts] = {};
      legendre_roots(k, rk);
      for (int i = 1; i < k; ++i) t[i] = bisect(1, k, rk[i - 1], rk[i]);
    }
    for (int i = 0; i < N / 2; ++i) {
      const double s = 0.5 * (t[N - 1 - i] - t[i]);
      t[i] = -s;
      t[N - 1 - i] = s;
    }
    if (N % 2) t[N / 2] = 0.0;
    for (int i = 0; i < N; ++i) xi[i] = 0.5 * (t[i] + 1.0);

    // Gauss rule: roots of P_Q, w = 2 / ((1 - t^2) P_Q'(t)^2), mapped to [0, 1]
    double g[kMaxPts] = {};
    legendre_roots(Q, g);
    double wr[kMaxPts] = {};
    for (int i = 0; i < Q; ++i) {
      const LegPair r = legendre2(Q, g[i]);
      const double dp = Q * (g[i] * r.p - r.pm1) / (g[i] * g[i] - 1.0);
      wr[i] = 2.0 / ((1.0 - g[i] * g[i]) * dp * dp);
    }
    for (int i = 0; i < Q / 2; ++i) {
      const double s = 0.5 * (g[Q - 1 - i] - g[i]);
      const double ww = 0.5 * (wr[i] + wr[Q - 1 - i]);
      g[i] = -s;
      g[Q - 1 - i] = s;
      wr[i] = wr[Q - 1 - i] = ww;
    }
    if (Q % 2) g[Q / 2] = 0.0;
    for (int i = 0; i < Q; ++i) {
      z[i] = 0.5 * (g[i] + 1.0);
      w[i] = 0.5 * wr[i];
    }

    // Lagrange basis of the LGL nodes and its derivative at the Gauss points
    for (int q = 0; q < Q; ++q)
      for (int a = 0; a < N; ++a) {
        double v = 1.0, d = 0.0;
        for (int b = 0; b < N; ++b) {
          if (b == a) continue;
          const double f = (z[q] - xi[b]) / (xi[a] - xi[b]);
          d = d * f + v / (xi[a] - xi[b]);
          v *= f;
        }
        S[q][a] = v;
        G[q][a] = d;
      }
  }
};

}  // namespace ct
}  // namespace dgmf
