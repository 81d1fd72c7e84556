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

// FP64 q = A p; partial[wg] = sum of p.q over the workgroup.  tab: device
// table as in launch_laplace (nullptr: from the table cache).
hipError_t cg_apply_dot(const LaplacePlan& P, const double* p, double* q, double* partial, hipStream_t s,
                        const void* tab = nullptr);

// One FP32 Chebyshev step with its operator apply t = A x_k, in three-term
// form (d_k = x_{k+1} - x_k of the two-term recurrence is not stored):
//   x_{k+1} = x_k + c1 (x_k - x_{k-1}) + c2 D^-1 (r' - t)
// step 1: x_0 = 0 and the operand x_1 = D^-1 r' / theta is formed from r
//         (FP64) on the fly; r' = (float)(r - mu_r) is stored in r32;
// step 2: x_1 is recomputed from r32;
// later:  x_{k-1} is read from xprev, and xout may be xprev (in place);
// last:   x_{k+1} is the smoother output z, and the partials sum z, r'.z,
//         r'.(zprev - mu_z_prev) are written (3 quantities).
struct ChebStepArgs {
  const double* r;      // FP64 residual (step 1, last)
  const float* xin;     // x_k (steps >= 2)
  const float* xprev;   // x_{k-1} (steps >= 3)
  float* xout;          // x_{k+1}; differs from xin
  float* r32;           // r' in FP32 (written by step 1, read by the later steps)
  const float* dinv;    // D^-1 of one element (n^3 values)
  const float* zprev;   // previous smoother output (last)
  const double* st;     // CG state (mu_r, previous mu_z)
  double* partial;      // 3 x cg_apply_grid() partials (last)
  float c1, c2, inv_theta;
};
hipError_t cg_apply_cheb(const LaplacePlan& P, int step, bool last, const ChebStepArgs& a, hipStream_t s,
                         const void* tab = nullptr);

}  // namespace dgmf
