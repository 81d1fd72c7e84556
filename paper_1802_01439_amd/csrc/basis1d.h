// 1D nodal basis and quadrature for the HIP operators (host side).
//
// Sec. 3.2: tensor-product Lagrange polynomials on the Legendre-Gauss-Lobatto
// (LGL) nodes of degree k, Gauss quadrature.  Everything lives on the
// reference interval [0, 1].  These are small dense tables (n, m <= 24)
// computed once per (k, n_q) and handed to the kernels.
#pragma once

#include <vector>

namespace dgmf {

// LGL nodes of degree k on [0,1] (end points + roots of P_k'), ascending.
void lgl_nodes(int k, double* x);
// m-point Gauss-Legendre rule on [0,1].
void gauss_rule(int m, double* x, double* w);
// Embedding of the degree-k LGL basis of [0,1] in its half c (0: [0,1/2],
// 1: [1/2,1]) mapped to [0,1]: P[i*n+a] = l_a((xi_i + c)/2), n = k+1.
std::vector<double> child_interp(int k, int c);

struct Basis1D {
  int k = 0, n = 0, m = 0;
  std::vector<double> xi;     // n LGL nodes
  std::vector<double> zq, wq; // m Gauss points and weights
  std::vector<double> S;      // m x n: S[q*n+a] = l_a(z_q)
  std::vector<double> G;      // m x n: G[q*n+a] = l_a'(z_q)
  std::vector<double> D;      // n x n: D[i*n+j] = l_j'(xi_i)
  std::vector<double> Mref;   // n x n mass on [0,1]: sum_q w_q l_a l_b
  std::vector<double> Kcell;  // n x n stiffness on [0,1]: sum_q w_q l_a' l_b'
  std::vector<double> Dg;     // m x m collocation derivative on the Gauss points
};

Basis1D make_basis(int k, int m);

// 1D SIPG operator on [0,1] with penalty sigma (= tau*h) split into the part
// acting on the own element (cell stiffness plus the own-side face terms of
// both ends) and the rank-two couplings to the left and right neighbours:
//   y_i = sum_b Kown[i][b] u[b] + sum_b Kl[i][b] uL[b] + sum_b Kr[i][b] uR[b].
struct Sipg1D {
  std::vector<double> Kown, Kl, Kr;  // n x n each
};
Sipg1D make_sipg_1d(const Basis1D& B, double sigma);

}  // namespace dgmf
