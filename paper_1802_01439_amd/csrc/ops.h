// Internal launch interface between the C ABI layer and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "common.h"

namespace dgmf {

// Everything a Laplace launch needs, in double; kernels cast to their type.
struct LaplacePlan {
  int k = 0;
  int n_comp = 1;
  MeshArgs mesh{};
  std::vector<double> Mref;  // n x n 1D mass on [0,1]
  std::vector<double> Kown;  // n x n 1D SIPG own-element part on [0,1]
  std::vector<double> D;     // n x n l_j'(xi_i) at the LGL nodes
  std::vector<double> Lown;  // n x n  M^-1 Kown
  std::vector<double> cR, cL, gR, gL;  // M^-1 times the neighbour coupling columns
  double c[3] = {0, 0, 0};   // scale * vol / h_d^2
  double sigma = 0;          // penalty_factor * (k+1)^2
  double shift = 0;          // y = (Mx(x)My(x)Mz)(shift I + sum_d c_d L_d) u: mass_factor * vol
};

// tab: the kernel's device table of plan P (bytes written by lap_table_fill),
// or nullptr to take it from the library's table cache (uploaded on first use).
hipError_t launch_laplace(const LaplacePlan& P, bool f32, const void* src, void* dst,
                          hipStream_t stream, const void* tab = nullptr);
// Size of the device table of plan P's Laplace kernels (FP32 or FP64); with
// host_out, also writes the table there (for an upload by the caller).
size_t lap_table_fill(const LaplacePlan& P, bool f32, void* host_out);

// Multigrid smoother steps fused into the Laplace apply (T = double, float):
// d <- c1 d + c2 D^-1 (b - A x), xout = x + d (xout must not be x: x is read
// for neighbour DoFs); res = b - A x.  dinv: one element's n^3 values.
template <typename T>
hipError_t mg_apply_cheb(const LaplacePlan& P, const T* x, const T* b, const T* dinv, T c1, T c2, T* d, T* xout,
                         hipStream_t s);
template <typename T>
hipError_t mg_apply_residual(const LaplacePlan& P, const T* x, const T* b, T* res, hipStream_t s);
// the Chebyshev step of mg_apply_cheb with its new iterate added to y
// (y += x + d') instead of stored
template <typename T>
hipError_t mg_apply_cheb_add(const LaplacePlan& P, const T* x, const T* b, const T* dinv, T c1, T c2, const T* d, T* y,
                             hipStream_t s);
// res = b - A x and the first step of a zero-start Chebyshev smoother on it,
// d = e = scale * dinv[node] * res
template <typename T>
hipError_t mg_apply_residual_cheb_first(const LaplacePlan& P, const T* x, const T* b, const T* dinv, T scale, T* res,
                                        T* d, T* e, hipStream_t s);

// Convective form and its VJP: 1D tables on [0,1] and the cell/face scalings.
struct ConvPlan {
  int k = 0;
  int m = 0;                 // Gauss points per direction (floor(3k/2)+1)
  MeshArgs mesh{};
  std::vector<double> S;     // m x n: l_a(z_q)
  std::vector<double> G;     // m x n: l_a'(z_q)
  std::vector<double> w;     // m Gauss weights
  double cell[3] = {0, 0, 0};   // -vol/h_j
  double area[3] = {0, 0, 0};   // vol/h_d
  double lf = 1.0;
};

hipError_t launch_convective(const ConvPlan& P, bool f32, const void* u, void* r, hipStream_t s);
hipError_t launch_convective_vjp(const ConvPlan& P, bool f32, const void* u, const void* w,
                                 void* g, hipStream_t s);

// Central-flux divergence: 1D mass and the 1D divergence operator on [0,1].
struct DivPlan {
  int k = 0;
  MeshArgs mesh{};
  std::vector<double> Mref;  // n x n
  std::vector<double> Bown;  // n x n: -sum_q w l_i' l_j + own central-flux end terms
  double c[3] = {0, 0, 0};   // vol/h_d
};

hipError_t launch_divergence(const DivPlan& P, bool f32, const void* u, void* b, hipStream_t s);
// inverse-mass-preconditioned CG step on element blocks (FP64): x += alpha p,
// r -= alpha q, z = M^-1 r, block sums of r.r and r.z (2 * grid doubles)
long long pcg_precond_grid(int k, long long nblocks);
hipError_t launch_pcg_precond(int k, const std::vector<double>& Minv, double scale, long long nblocks, double* x,
                              double* r, const double* p, const double* q, double* z, const double* st,
                              double* partial, hipStream_t s);
// h-multigrid level transfers between a mesh (coarse) and the mesh with every
// element split in two per direction: P[c] = child_interp(k, c)
struct TransferPlan {
  int k = 0, nxc = 0, nyc = 0, nzc = 0, n_comp = 1;
  std::vector<double> P[2];
};
hipError_t launch_transfer(const TransferPlan& P, bool prolong, bool f32, const void* src, void* dst,
                           hipStream_t s);
// dst += the prolongation of src (a V-cycle's coarse-grid correction)
hipError_t launch_prolongate_add(const TransferPlan& P, bool f32, const void* src, void* dst, hipStream_t s);
// rc = the restriction of rf (one component) and the first step of a
// zero-start Chebyshev smoother on it: d = x = scale * dinv[node] * rc, with
// scale rounded to the transfer's precision
hipError_t launch_restrict_cheb_first(const TransferPlan& P, bool f32, const void* rf, void* rc, const void* dinv,
                                      double scale, void* d, void* x, hipStream_t s);

// pressure gradient: the divergence's 1D tables, G = -B^T
hipError_t launch_gradient(const DivPlan& P, bool f32, const void* p, void* y, hipStream_t s);

// Projection-step operator (mass + divergence and continuity penalties):
// 1D tables on [0,1] with k+1 Gauss points and the cell scalings.
struct ProjPlan {
  int k = 0;
  MeshArgs mesh{};
  std::vector<double> S, Dg, M1, w;   // n x n, n x n, n x n, n
  double vol = 0, ih[3] = {0, 0, 0}, area[3] = {0, 0, 0};
};
// dot_partial (optional): one partial sum of u.y per workgroup,
// projection_grid(P) of them
hipError_t launch_projection(const ProjPlan& P, bool f32, const void* u, void* y, const void* tau_d,
                             const void* tau_c, hipStream_t s, void* dot_partial = nullptr);
long long projection_grid(const ProjPlan& P);

// x = M^-1 b on nblocks consecutive element blocks: Minv = inverse of the 1D
// mass on [0,1] (n x n row major), scale = 1/(h_x h_y h_z).
hipError_t launch_inverse_mass(int k, const std::vector<double>& Minv, double scale, long long nblocks, bool f32,
                               const void* src, void* dst, hipStream_t s);
// FP64, nblocks element blocks: uhat = a0 un + a1 unm1 + a2 M^-1 (b0 cn + b1 cm),
// cm and unm1 optional (then their terms are absent); the operations of
// launch_lincomb, launch_inverse_mass, launch_lincomb in one pass
hipError_t launch_convective_substep(int k, const std::vector<double>& Minv, double scale, long long nblocks,
                                    const double* cn, const double* cm, double b0, double b1, const double* un,
                                    const double* unm1, double a0, double a1, double a2, double* uhat,
                                    hipStream_t s);

int vjp_max_degree(bool f32);

// Dual-splitting step kernels (mixed.hip).  Mixed-order divergence
// (grad = false: u [3][N_el][(k+1)^3] -> [N_el][k^3]) and gradient (grad =
// true: p [N_el][k^3] -> [3][N_el][(k+1)^3]) of plan P (velocity degree
// P.k >= 2), times scale.
hipError_t launch_mixed(const DivPlan& P, bool grad, bool f32, const void* src, void* dst, double scale,
                        hipStream_t s);
// tau_d[e] = fd |u|_e, tau_c[e] = fc |u|_e, |u|_e the element average of the
// velocity magnitude (FP64, degree k, k+1 Gauss points)
hipError_t launch_penalty(int k, const MeshArgs& mesh, const double* u, double* tau_d, double* tau_c, double fd,
                          double fc, hipStream_t s);
// out2 = (sum_e int |u|^2, sum_e int grad u : grad u); partial: 2 N_el doubles
hipError_t launch_diagnostics(int k, const MeshArgs& mesh, const double* u, double* partial, double* out2,
                              double vol, const double ih[3], hipStream_t s);
// y = a0 x0 + a1 x1 + a2 x2 (x1, x2 may be null); y may be one of the x
hipError_t launch_lincomb(double* y, const double* x0, const double* x1, const double* x2, double a0, double a1,
                          double a2, long long n, hipStream_t s);

}  // namespace dgmf
