// Vector kernels of the preconditioned CG solver (Sec. 3.3): fused updates
// with per-block partial sums and a fixed-order final reduction, so every dot
// product is bitwise reproducible run to run.  All CG vectors are FP64; the
// Chebyshev preconditioner's vectors are FP32.
#include "cg_kernels.h"

namespace dgmf {

namespace {

constexpr int kThreads = kCgThreads;

// Block sum of NQ doubles; thread 0 writes partial[q * gridDim.x + blockIdx.x].
template <int NQ>
__device__ __forceinline__ void block_partials(double (&v)[NQ], double* partial) {
  __shared__ double sh[NQ][kThreads];
#pragma unroll
  for (int q = 0; q < NQ; ++q) sh[q][threadIdx.x] = v[q];
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) partial[q * gridDim.x + blockIdx.x] = sh[q][0];
  }
}

__global__ void __launch_bounds__(kThreads) k_finalize(const double* __restrict__ partial, int nblocks, int nq,
                                                       double* __restrict__ out) {
  __shared__ double sh[kThreads];
  for (int q = 0; q < nq; ++q) {
    double s = 0;
    for (int i = threadIdx.x; i < nblocks; i += kThreads) s += partial[q * nblocks + i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int st = kThreads / 2; st > 0; st >>= 1) {
      if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[q] = sh[0];
    __syncthreads();
  }
}

// r = b - q; partials: sum r, sum r^2, sum b, sum b^2
__global__ void __launch_bounds__(kThreads) k_residual(const double* __restrict__ b, const double* __restrict__ q,
                                                       double* __restrict__ r, long long n, double* partial) {
  double v[4] = {0, 0, 0, 0};
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
    const double bi = b[i];
    const double ri = bi - q[i];
    r[i] = ri;
    v[0] += ri;
    v[1] += ri * ri;
    v[2] += bi;
    v[3] += bi * bi;
  }
  block_partials<4>(v, partial);
}

// partial x.y
__global__ void __launch_bounds__(kThreads) k_dot(const double* __restrict__ x, const double* __restrict__ y,
                                                  long long n, double* partial) {
  double v[1] = {0};
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads)
    v[0] += x[i] * y[i];
  block_partials<1>(v, partial);
}

// x += alpha p; r -= alpha q; partial sum r
__global__ void __launch_bounds__(kThreads) k_update_xr(double* __restrict__ x, double* __restrict__ r,
                                                        const double* __restrict__ p, const double* __restrict__ q,
                                                        double alpha, long long n, double* partial) {
  double v[1] = {0};
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    v[0] += ri;
  }
  block_partials<1>(v, partial);
}

// r <- r - mu_r; z = dinv * r; partials: sum z, r.z, r.zold, r.r
__global__ void __launch_bounds__(kThreads) k_jacobi(double* __restrict__ r, double* __restrict__ z,
                                                     const double* __restrict__ zold, const double* __restrict__ dinv,
                                                     int n3, double mu_r, long long n, double* partial) {
  double v[4] = {0, 0, 0, 0};
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
    const double ri = r[i] - mu_r;
    r[i] = ri;
    const double zi = dinv[i % n3] * ri;
    z[i] = zi;
    v[0] += zi;
    v[1] += ri * zi;
    v[2] += ri * zold[i];
    v[3] += ri * ri;
  }
  block_partials<4>(v, partial);
}

// z <- z - mu_z; p = z + beta p; zold = z
__global__ void __launch_bounds__(kThreads) k_update_p(double* __restrict__ z, double* __restrict__ p,
                                                       double* __restrict__ zold, double mu_z, double beta,
                                                       long long n) {
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
    const double zi = z[i] - mu_z;
    zold[i] = zi;
    p[i] = zi + beta * p[i];
  }
}

// Chebyshev start (FP32): r <- r - mu_r (FP64, written back); r32 = r;
// x32 = d32 = dinv32 * r32 / theta
__global__ void __launch_bounds__(kThreads) k_cheb_init(double* __restrict__ r, float* __restrict__ r32,
                                                        float* __restrict__ x32, float* __restrict__ d32,
                                                        const float* __restrict__ dinv32, int n3, double mu_r,
                                                        float inv_theta, long long n) {
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
    const double ri = r[i] - mu_r;
    r[i] = ri;
    const float rf = (float)ri;
    r32[i] = rf;
    const float di = dinv32[i % n3] * rf * inv_theta;
    x32[i] = di;
    d32[i] = di;
  }
}

// d32 = c1 d32 + c2 dinv32 (r32 - t32); x32 += d32
__global__ void __launch_bounds__(kThreads) k_cheb_step(float* __restrict__ x32, float* __restrict__ d32,
                                                        const float* __restrict__ r32, const float* __restrict__ t32,
                                                        const float* __restrict__ dinv32, int n3, float c1, float c2,
                                                        long long n) {
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
    const float d = c1 * d32[i] + c2 * dinv32[i % n3] * (r32[i] - t32[i]);
    d32[i] = d;
    x32[i] += d;
  }
}

// z = (double) x32; partials: sum z, r.z, r.zold, r.r   (r already projected)
__global__ void __launch_bounds__(kThreads) k_cheb_final(const double* __restrict__ r, double* __restrict__ z,
                                                         const double* __restrict__ zold, const float* __restrict__ x32,
                                                         long long n, double* partial) {
  double v[4] = {0, 0, 0, 0};
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
    const double ri = r[i];
    const double zi = (double)x32[i];
    z[i] = zi;
    v[0] += zi;
    v[1] += ri * zi;
    v[2] += ri * zold[i];
    v[3] += ri * ri;
  }
  block_partials<4>(v, partial);
}

// v[i] = uniform[-1,1) from a splitmix64 hash of (i, seed); partial sum v
__global__ void __launch_bounds__(kThreads) k_hash_fill(double* __restrict__ v, unsigned long long seed, long long n,
                                                        double* partial) {
  double s[1] = {0};
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
    unsigned long long z = (unsigned long long)i + seed * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    const double x = (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
    v[i] = x;
    s[0] += x;
  }
  block_partials<1>(s, partial);
}

__global__ void __launch_bounds__(kThreads) k_axpb(double* __restrict__ y, const double* __restrict__ x, double a,
                                                   double c, long long n) {
  // y = a * x + c
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads)
    y[i] = a * x[i] + c;
}

__global__ void __launch_bounds__(kThreads) k_fill(double* __restrict__ y, double c, long long n) {
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads)
    y[i] = c;
}

}  // namespace

#define DG_LAUNCH(kern, ...)                                                                  \
  do {                                                                                        \
    hipLaunchKernelGGL(kern, dim3(kCgBlocks), dim3(kThreads), 0, s, __VA_ARGS__);             \
    return hipGetLastError();                                                                 \
  } while (0)

hipError_t cg_finalize(const double* partial, int nq, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, s, partial, kCgBlocks, nq, out);
  return hipGetLastError();
}
hipError_t cg_residual(const double* b, const double* q, double* r, long long n, double* partial, hipStream_t s) {
  DG_LAUNCH(k_residual, b, q, r, n, partial);
}
hipError_t cg_dot(const double* x, const double* y, long long n, double* partial, hipStream_t s) {
  DG_LAUNCH(k_dot, x, y, n, partial);
}
hipError_t cg_update_xr(double* x, double* r, const double* p, const double* q, double alpha, long long n,
                        double* partial, hipStream_t s) {
  DG_LAUNCH(k_update_xr, x, r, p, q, alpha, n, partial);
}
hipError_t cg_jacobi(double* r, double* z, const double* zold, const double* dinv, int n3, double mu_r, long long n,
                     double* partial, hipStream_t s) {
  DG_LAUNCH(k_jacobi, r, z, zold, dinv, n3, mu_r, n, partial);
}
hipError_t cg_update_p(double* z, double* p, double* zold, double mu_z, double beta, long long n, hipStream_t s) {
  DG_LAUNCH(k_update_p, z, p, zold, mu_z, beta, n);
}
hipError_t cg_cheb_init(double* r, float* r32, float* x32, float* d32, const float* dinv32, int n3, double mu_r,
                        float inv_theta, long long n, hipStream_t s) {
  DG_LAUNCH(k_cheb_init, r, r32, x32, d32, dinv32, n3, mu_r, inv_theta, n);
}
hipError_t cg_cheb_step(float* x32, float* d32, const float* r32, const float* t32, const float* dinv32, int n3,
                        float c1, float c2, long long n, hipStream_t s) {
  DG_LAUNCH(k_cheb_step, x32, d32, r32, t32, dinv32, n3, c1, c2, n);
}
hipError_t cg_cheb_final(const double* r, double* z, const double* zold, const float* x32, long long n,
                         double* partial, hipStream_t s) {
  DG_LAUNCH(k_cheb_final, r, z, zold, x32, n, partial);
}
hipError_t cg_hash_fill(double* v, unsigned long long seed, long long n, double* partial, hipStream_t s) {
  DG_LAUNCH(k_hash_fill, v, seed, n, partial);
}
hipError_t cg_axpb(double* y, const double* x, double a, double c, long long n, hipStream_t s) {
  DG_LAUNCH(k_axpb, y, x, a, c, n);
}
hipError_t cg_fill(double* y, double c, long long n, hipStream_t s) { DG_LAUNCH(k_fill, y, c, n); }

}  // namespace dgmf
