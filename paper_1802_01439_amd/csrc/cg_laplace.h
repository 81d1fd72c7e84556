// Operator applications of the CG solver with the vector work of the
// iteration fused into the Laplace kernels (Sec. 3.3: CG preconditioned by
// a Chebyshev smoother, or by the diagonal).  Each call is one launch of the
// Laplace kernel for the plan's degree and dtype; reductions write one
// partial sum per workgroup, cg_apply_grid() of them per quantity, laid out
// [quantity][workgroup].  Scalars (means, beta) are read from the device
// state array of the CG loop (indices in cg_kernels.h).
#pragma once

#include <hip/hip_runtime.h>

#include "ops.h"

namespace dgmf {

// Workgroups of one apply of plan P in FP32 or FP64 (partials per quantity).
long cg_apply_grid(const LaplacePlan& P, bool f32);

// FP64 q = A p; partial[wg] = sum of p.q over the workgroup.
hipError_t cg_apply_dot(const LaplacePlan& P, const double* p, double* q, double* partial, hipStream_t s);

// One FP32 Chebyshev step with its operator apply t = A x:
//   d <- c1 d + c2 D^-1 (r' - t),   x_out = x + d
// first: x = D^-1 r' / theta (= d) is formed from r (FP64) on the fly and
//        r' = (float)(r - mu_r) is stored in r32 for the later steps;
// last:  d is not stored; x_out is the smoother output z, and the partials
//        sum z, r'.z, r'.(zprev - mu_z_prev) are written (3 quantities).
struct ChebStepArgs {
  const double* r;      // FP64 residual (first, last)
  const float* xin;     // current iterate (not first)
  float* xout;          // next iterate; differs from xin
  float* d;             // step vector, updated in place
  float* r32;           // r' in FP32 (written by first, read by the middle steps)
  const float* dinv;    // D^-1 of one element (n^3 values)
  const float* zprev;   // previous smoother output (last)
  const double* st;     // CG state (mu_r, previous mu_z)
  double* partial;      // 3 x cg_apply_grid() partials (last)
  float c1, c2, inv_theta;
};
hipError_t cg_apply_cheb(const LaplacePlan& P, bool first, bool last, const ChebStepArgs& a, hipStream_t s);

}  // namespace dgmf
