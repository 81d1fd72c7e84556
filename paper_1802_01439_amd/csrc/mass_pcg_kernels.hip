// Scalar steps of the inverse-mass-preconditioned CG with its scalars kept on
// the device (the state array of the CG solver: kRZ, kBeta, kRN2, kDone,
// kStatus, kIter, kTol2, kMaxIt), so that iterations run in batches between
// host reads.  p.Ap and alpha come from the CG kernels, the x/r update with
// z = M^-1 r and the sums r.r, r.z from the fused inverse mass kernel.
#include "cg_kernels.h"

namespace dgmf {

namespace {

constexpr int kThreads = kCgThreads;

// sum of partial[0 .. nblocks) in a fixed order (thread 0 holds it)
__device__ double fixed_sum(const double* __restrict__ partial, int nblocks) {
  __shared__ double sh[kThreads];
  double s = 0;
  for (int i = threadIdx.x; i < nblocks; i += kThreads) s += partial[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int st = kThreads / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// r.z of the initial residual
__global__ void __launch_bounds__(kThreads) k_mp_start(const double* __restrict__ partial, int nblocks,
                                                       double* __restrict__ st) {
  const double rz = fixed_sum(partial, nblocks);
  if (threadIdx.x != 0) return;
  st[kRZ] = rz;
  if (!(rz > 0.0) || !isfinite(rz)) {
    st[kDone] = 1.0;
    st[kStatus] = 2.0;
  }
}

// after x/r update and z = M^-1 r: r.r (second quantity of the update's
// partials) and r.z; convergence test, iteration count, beta
__global__ void __launch_bounds__(kThreads) k_mp_beta(const double* __restrict__ rr_partial,
                                                      const double* __restrict__ rz_partial, int nblocks,
                                                      double* __restrict__ st) {
  const double rr = fixed_sum(rr_partial, nblocks);
  const double rz = fixed_sum(rz_partial, nblocks);
  if (threadIdx.x != 0) return;
  if (st[kDone] != 0.0) {
    st[kBeta] = 0.0;
    return;
  }
  const double it = st[kIter] + 1.0;
  st[kIter] = it;
  st[kRN2] = rr;
  st[kBeta] = 0.0;
  if (rr <= st[kTol2]) {
    st[kDone] = 1.0;
    return;
  }
  if (it >= st[kMaxIt]) {
    st[kDone] = 1.0;
    st[kStatus] = 1.0;
    return;
  }
  if (!(rz > 0.0) || !isfinite(rz)) {
    st[kDone] = 1.0;
    st[kStatus] = 2.0;
    return;
  }
  st[kBeta] = rz / st[kRZ];
  st[kRZ] = rz;
}

// p = z + beta p (beta from the state)
__global__ void __launch_bounds__(kThreads) k_mp_xpby(double* __restrict__ p, const double* __restrict__ z,
                                                      const double* __restrict__ st, long long n) {
  const double beta = st[kBeta];
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads)
    p[i] = beta != 0.0 ? z[i] + beta * p[i] : z[i];
}

}  // namespace

hipError_t mpcg_start(const double* partial, double* st, hipStream_t s) {
  hipLaunchKernelGGL(k_mp_start, dim3(1), dim3(kThreads), 0, s, partial, kCgBlocks, st);
  return hipGetLastError();
}

hipError_t mpcg_beta(const double* rr_partial, const double* rz_partial, int nblocks, double* st, hipStream_t s) {
  hipLaunchKernelGGL(k_mp_beta, dim3(1), dim3(kThreads), 0, s, rr_partial, rz_partial, nblocks, st);
  return hipGetLastError();
}

hipError_t mpcg_xpby(double* p, const double* z, const double* st, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_mp_xpby, dim3(kCgBlocks), dim3(kThreads), 0, s, p, z, st, n);
  return hipGetLastError();
}

}  // namespace dgmf
