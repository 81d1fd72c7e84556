// Elementwise steps of the Chebyshev smoother of the multigrid V-cycle
// (FP64 and FP32): D^-1 is one element's diagonal inverse (n3 values), the
// same on every element of a uniform periodic mesh; conversions between the
// FP64 outer CG and an FP32 cycle.
#include <hip/hip_runtime.h>

#include "cg_kernels.h"

namespace dgmf {

namespace {

constexpr int kThreads = kCgThreads;

// d = s D^-1 b; x = d
template <typename T>
__global__ void __launch_bounds__(kThreads) k_cheb_first(const T* __restrict__ b, const T* __restrict__ dinv, int n3,
                                                         T s, T* __restrict__ d, T* __restrict__ x, long long n) {
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
    const T v = s * dinv[i % n3] * b[i];
    d[i] = v;
    x[i] = v;
  }
}

// d = c1 d + c2 D^-1 (b - t); x += d
template <typename T>
__global__ void __launch_bounds__(kThreads) k_cheb_next(const T* __restrict__ b, const T* __restrict__ t,
                                                        const T* __restrict__ dinv, int n3, T c1, T c2,
                                                        T* __restrict__ d, T* __restrict__ x, long long n) {
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
    const T v = c1 * d[i] + c2 * dinv[i % n3] * (b[i] - t[i]);
    d[i] = v;
    x[i] += v;
  }
}

// x += t
template <typename T>
__global__ void __launch_bounds__(kThreads) k_add(T* __restrict__ x, const T* __restrict__ t, long long n) {
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads)
    x[i] += t[i];
}

template <typename A, typename B>
__global__ void __launch_bounds__(kThreads) k_convert(const A* __restrict__ a, B* __restrict__ b, long long n) {
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads)
    b[i] = (B)a[i];
}

}  // namespace

hipError_t mg_cheb_first(const double* b, const double* dinv, int n3, double s, double* d, double* x, long long n,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_cheb_first<double>, dim3(kCgBlocks), dim3(kThreads), 0, st, b, dinv, n3, s, d, x, n);
  return hipGetLastError();
}
hipError_t mg_cheb_next(const double* b, const double* t, const double* dinv, int n3, double c1, double c2, double* d, double* x,
                        long long n, hipStream_t st) {
  hipLaunchKernelGGL(k_cheb_next<double>, dim3(kCgBlocks), dim3(kThreads), 0, st, b, t, dinv, n3, c1, c2, d, x, n);
  return hipGetLastError();
}
hipError_t mg_add(double* x, const double* t, long long n, hipStream_t st) {
  hipLaunchKernelGGL(k_add<double>, dim3(kCgBlocks), dim3(kThreads), 0, st, x, t, n);
  return hipGetLastError();
}

hipError_t mg_cheb_first(const float* b, const float* dinv, int n3, float s, float* d, float* x, long long n,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_cheb_first<float>, dim3(kCgBlocks), dim3(kThreads), 0, st, b, dinv, n3, s, d, x, n);
  return hipGetLastError();
}
hipError_t mg_cheb_next(const float* b, const float* t, const float* dinv, int n3, float c1, float c2, float* d, float* x,
                        long long n, hipStream_t st) {
  hipLaunchKernelGGL(k_cheb_next<float>, dim3(kCgBlocks), dim3(kThreads), 0, st, b, t, dinv, n3, c1, c2, d, x, n);
  return hipGetLastError();
}
hipError_t mg_add(float* x, const float* t, long long n, hipStream_t st) {
  hipLaunchKernelGGL(k_add<float>, dim3(kCgBlocks), dim3(kThreads), 0, st, x, t, n);
  return hipGetLastError();
}

hipError_t mg_convert(const double* a, float* b, long long n, hipStream_t st) {
  hipLaunchKernelGGL((k_convert<double, float>), dim3(kCgBlocks), dim3(kThreads), 0, st, a, b, n);
  return hipGetLastError();
}
hipError_t mg_convert(const float* a, double* b, long long n, hipStream_t st) {
  hipLaunchKernelGGL((k_convert<float, double>), dim3(kCgBlocks), dim3(kThreads), 0, st, a, b, n);
  return hipGetLastError();
}

}  // namespace dgmf
