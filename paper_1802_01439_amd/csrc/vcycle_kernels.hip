// Elementwise steps of the Chebyshev smoother of the multigrid V-cycle
// (FP64): D^-1 is one element's diagonal inverse (n3 values), the same on
// every element of a uniform periodic mesh.
#include <hip/hip_runtime.h>

#include "cg_kernels.h"

namespace dgmf {

namespace {

constexpr int kThreads = kCgThreads;

// d = s D^-1 b; x = d
__global__ void __launch_bounds__(kThreads) k_cheb_first(const double* __restrict__ b, const double* __restrict__ dinv,
                                                         int n3, double s, double* __restrict__ d,
                                                         double* __restrict__ x, long long n) {
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
    const double v = s * dinv[i % n3] * b[i];
    d[i] = v;
    x[i] = v;
  }
}

// d = c1 d + c2 D^-1 (b - t); x += d
__global__ void __launch_bounds__(kThreads) k_cheb_next(const double* __restrict__ b, const double* __restrict__ t,
                                                        const double* __restrict__ dinv, int n3, double c1, double c2,
                                                        double* __restrict__ d, double* __restrict__ x, long long n) {
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
    const double v = c1 * d[i] + c2 * dinv[i % n3] * (b[i] - t[i]);
    d[i] = v;
    x[i] += v;
  }
}

// y = b - t
__global__ void __launch_bounds__(kThreads) k_sub(const double* __restrict__ b, const double* __restrict__ t,
                                                  double* __restrict__ y, long long n) {
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads)
    y[i] = b[i] - t[i];
}

// x += t
__global__ void __launch_bounds__(kThreads) k_add(double* __restrict__ x, const double* __restrict__ t, long long n) {
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads)
    x[i] += t[i];
}

}  // namespace

hipError_t mg_cheb_first(const double* b, const double* dinv, int n3, double s, double* d, double* x, long long n,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_cheb_first, dim3(kCgBlocks), dim3(kThreads), 0, st, b, dinv, n3, s, d, x, n);
  return hipGetLastError();
}

hipError_t mg_cheb_next(const double* b, const double* t, const double* dinv, int n3, double c1, double c2, double* d,
                        double* x, long long n, hipStream_t st) {
  hipLaunchKernelGGL(k_cheb_next, dim3(kCgBlocks), dim3(kThreads), 0, st, b, t, dinv, n3, c1, c2, d, x, n);
  return hipGetLastError();
}

hipError_t mg_sub(const double* b, const double* t, double* y, long long n, hipStream_t st) {
  hipLaunchKernelGGL(k_sub, dim3(kCgBlocks), dim3(kThreads), 0, st, b, t, y, n);
  return hipGetLastError();
}

hipError_t mg_add(double* x, const double* t, long long n, hipStream_t st) {
  hipLaunchKernelGGL(k_add, dim3(kCgBlocks), dim3(kThreads), 0, st, x, t, n);
  return hipGetLastError();
}

}  // namespace dgmf
