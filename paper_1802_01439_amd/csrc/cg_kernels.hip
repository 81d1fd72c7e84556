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
    p[i] = beta != 0.0 ? zi + beta * p[i] : zi;   // a zero beta never reads the old direction
  }
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

// y = x + b y
__global__ void __launch_bounds__(kThreads) k_xpby(double* __restrict__ y, const double* __restrict__ x, double b,
                                                   long long n) {
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads)
    y[i] = b != 0.0 ? x[i] + b * y[i] : x[i];
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

// ---------------------------------------------------------------------------
// Main-loop kernels with the iteration scalars kept on the device (state
// array st, indices in cg_kernels.h): the host enqueues several iterations at
// a time and reads the state once per batch.  Once st[kDone] is set every
// update below becomes a no-op, so iterations queued past convergence change
// nothing.
//
// Mean projection on periodic meshes, folded into the sums: with r' = r - mu
// (mu = mean r), z' = D^-1 r' - mu_z (mu_z = mean of D^-1 r') and d = D^-1 1,
//   |r'|^2    = S_rr - 2 mu S_r + n mu^2
//   r'.D^-1r' = S_rdr - 2 mu S_dr + mu^2 S_d
//   mu_z      = (S_dr - mu S_d) / n
//   r'.z'     = r'.D^-1r' - mu_z (S_r - n mu)
// from one pass computing S_r = sum r, S_rr = sum r^2, S_dr = sum d r,
// S_rdr = sum d r^2 (S_d = sum d is a setup constant).  r itself is stored
// unprojected; every use subtracts mu.

// Sums of partial[q * nblocks + i] over i for q < NQ, in a fixed order
// (thread-strided, then across the wavefront, then across the 4 wavefronts);
// valid in thread 0.
template <int NQ>
__device__ __forceinline__ void block_sums(const double* __restrict__ partial, int nblocks, double (&out)[NQ]) {
  static_assert(kThreads == 256, "four full wavefronts");
  __shared__ double sh[NQ][kThreads / 64];
  double s[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) s[q] = 0.0;
  for (int i = threadIdx.x; i < nblocks; i += kThreads) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) s[q] += partial[(size_t)q * nblocks + i];
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s[q] += __shfl_xor(s[q], o, 64);
  }
  const int w = threadIdx.x / 64;
  if (threadIdx.x % 64 == 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) sh[q][w] = s[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NQ; ++q) out[q] = ((sh[q][0] + sh[q][1]) + sh[q][2]) + sh[q][3];
}

// alpha = rz / p.q  (p.q from one partial), breakdown if p.q <= 0 or not finite
__global__ void __launch_bounds__(kThreads) k_fin_alpha(const double* __restrict__ partial, int nblocks,
                                                        double* __restrict__ st) {
  double v[1];
  block_sums<1>(partial, nblocks, v);
  const double pq = v[0];
  if (threadIdx.x != 0) return;
  if (st[kDone] != 0.0) {
    st[kAlpha] = 0.0;
    return;
  }
  st[kPQ] = pq;
  if (!(pq > 0.0) || !isfinite(pq)) {
    st[kAlpha] = 0.0;
    st[kDone] = 1.0;
    st[kStatus] = 2.0;
    return;
  }
  st[kAlpha] = st[kRZ] / pq;
}

// x += alpha p; r -= alpha q; partials S_r, S_rr and (JAC) S_dr, S_rdr
template <bool JAC>
__global__ void __launch_bounds__(kThreads) k_update_xr_st(double* __restrict__ x, double* __restrict__ r,
                                                           const double* __restrict__ p, const double* __restrict__ q,
                                                           const double* __restrict__ dinv, int n3,
                                                           const double* __restrict__ st, long long n,
                                                           double* partial) {
  const double alpha = st[kAlpha];
  double v[JAC ? 4 : 2] = {};
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
    double ri = r[i];
    if (alpha != 0.0) {
      x[i] += alpha * p[i];
      ri -= alpha * q[i];
      r[i] = ri;
    }
    v[0] += ri;
    v[1] += ri * ri;
    if constexpr (JAC) {
      const double d = dinv[i % n3];
      v[2] += d * ri;
      v[3] += d * ri * ri;
    }
  }
  block_partials<JAC ? 4 : 2>(v, partial);
}

// count the iteration (not for the start) and test convergence / limits
__device__ void account(double* st, double rn2, double rz, bool start) {
  if (!start) st[kIter] += 1.0;
  if (!isfinite(rn2) || !isfinite(rz)) {
    st[kDone] = 1.0;
    st[kStatus] = 2.0;
  } else if (rn2 <= st[kTol2]) {
    st[kDone] = 1.0;
  } else if (st[kIter] >= st[kMaxIt]) {
    st[kDone] = 1.0;
    st[kStatus] = 1.0;
  }
}

// Jacobi: scalars of the new residual (sums from k_update_xr_st<true>);
// beta = rz_new / rz (a fixed symmetric preconditioner: standard PCG)
__global__ void __launch_bounds__(kThreads) k_fin_jacobi(const double* __restrict__ partial, int nblocks,
                                                         double* __restrict__ st, int start) {
  double v[4];
  block_sums<4>(partial, nblocks, v);
  const double Sr = v[0], Srr = v[1], Sdr = v[2], Srdr = v[3];
  if (threadIdx.x != 0) return;
  if (!start && st[kDone] != 0.0) return;
  const double n = st[kN], Sd = st[kSumD];
  const bool proj = st[kProj] != 0.0;
  const double mu = proj ? Sr / n : 0.0;
  const double rn2 = Srr - 2.0 * mu * Sr + n * mu * mu;
  const double muz = proj ? (Sdr - mu * Sd) / n : 0.0;
  const double rz = (Srdr - 2.0 * mu * Sdr + mu * mu * Sd) - muz * (Sr - n * mu);
  st[kBeta] = start ? 0.0 : rz / st[kRZ];
  st[kRZ] = rz;
  st[kMuR] = mu;
  st[kMuZ] = muz;
  st[kRN2] = rn2;
  account(st, rn2, rz, start != 0);
}


// Chebyshev: mean and norm of the new residual (sums from k_update_xr_st<false>)
__global__ void __launch_bounds__(kThreads) k_fin_resid(const double* __restrict__ partial, int nblocks,
                                                        double* __restrict__ st, int start) {
  double v[2];
  block_sums<2>(partial, nblocks, v);
  const double Sr = v[0], Srr = v[1];
  if (threadIdx.x != 0) return;
  if (!start && st[kDone] != 0.0) return;
  const double n = st[kN];
  const double mu = st[kProj] != 0.0 ? Sr / n : 0.0;
  const double rn2 = Srr - 2.0 * mu * Sr + n * mu * mu;
  st[kMuR] = mu;
  st[kRN2] = rn2;
  st[kSumRp] = Sr - n * mu;
  account(st, rn2, 1.0, start != 0);
}

// p = D^-1 (r - mu) - mu_z + beta p
__global__ void __launch_bounds__(kThreads) k_update_p_jacobi(const double* __restrict__ r, double* __restrict__ p,
                                                              const double* __restrict__ dinv, int n3,
                                                              const double* __restrict__ st, long long n) {
  const double mu = st[kMuR], muz = st[kMuZ], beta = st[kBeta];
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
    const double zi = fma(dinv[i % n3], r[i] - mu, -muz);
    p[i] = beta != 0.0 ? zi + beta * p[i] : zi;   // a zero beta never reads the old direction
  }
}

// p = (z - mu_z) + beta p, z the FP32 smoother output
__global__ void __launch_bounds__(kThreads) k_update_p_cheb(const float* __restrict__ z, double* __restrict__ p,
                                                            const double* __restrict__ st, long long n) {
  const double muz = st[kMuZ], beta = st[kBeta];
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
    const double zi = (double)z[i] - muz;
    p[i] = beta != 0.0 ? zi + beta * p[i] : zi;
  }
}

// Chebyshev degree 1 (no operator apply): z = D^-1 r' / theta and the
// partials sum z, r'.z, r'.(zprev - mu_z_prev) of the flexible beta
__global__ void __launch_bounds__(kThreads) k_cheb1(const double* __restrict__ r, float* __restrict__ z,
                                                    const float* __restrict__ zprev,
                                                    const float* __restrict__ dinv32, int n3,
                                                    const double* __restrict__ st, float inv_theta, long long n,
                                                    double* partial) {
  const double mu = st[kMuR], muzp = st[kMuZ];
  double v[3] = {0, 0, 0};
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
    const double rp = r[i] - mu;
    const float zf = dinv32[i % n3] * (float)rp * inv_theta;
    z[i] = zf;
    const double zd = (double)zf;
    v[0] += zd;
    v[1] += rp * zd;
    v[2] += rp * ((double)zprev[i] - muzp);
  }
  block_partials<3>(v, partial);
}

__global__ void __launch_bounds__(kThreads) k_fill32(float* __restrict__ y, float c, long long n) {
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads)
    y[i] = c;
}

// flexible beta = r'.(z' - zold) / rz with z' = z - mu_z
__global__ void __launch_bounds__(kThreads) k_fin_cheb(const double* __restrict__ partial, int nblocks,
                                                       double* __restrict__ st, int start) {
  double v[3];
  block_sums<3>(partial, nblocks, v);
  const double Sz = v[0], Srz = v[1], Srzo = v[2];
  if (threadIdx.x != 0) return;
  if (!start && st[kDone] != 0.0) return;
  const double muz = st[kProj] != 0.0 ? Sz / st[kN] : 0.0;
  const double rz = Srz - muz * st[kSumRp];
  st[kBeta] = start ? 0.0 : (rz - Srzo) / st[kRZ];
  st[kRZ] = rz;
  st[kMuZ] = muz;
  if (!isfinite(rz)) {
    st[kDone] = 1.0;
    st[kStatus] = 2.0;
  }
}

// Preconditioners that are a separate call (the multigrid V-cycle): the
// cycle's input r' = r - mu_r in the cycle's precision, the partials sum z,
// r'.z, r'.(zprev - mu_z_prev) of the flexible beta (k_fin_cheb), and
// p = (z - mu_z) + beta p, for an output z in either precision.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_rprime(const double* __restrict__ r, const double* __restrict__ st,
                                                     T* __restrict__ out, long long n) {
  const double mu = st[kMuR];
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads)
    out[i] = (T)(r[i] - mu);
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_zsums(const double* __restrict__ r, const T* __restrict__ z,
                                                    const T* __restrict__ zprev, const double* __restrict__ st,
                                                    long long n, double* partial) {
  const double mu = st[kMuR], muzp = st[kMuZ];
  double v[3] = {};
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
    const double rp = r[i] - mu, zi = (double)z[i];
    v[0] += zi;
    v[1] += rp * zi;
    v[2] += rp * ((double)zprev[i] - muzp);
  }
  block_partials<3>(v, partial);
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_update_p_z(const T* __restrict__ z, double* __restrict__ p,
                                                         const double* __restrict__ st, long long n) {
  const double muz = st[kMuZ], beta = st[kBeta];
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
    const double zi = (double)z[i] - muz;
    p[i] = beta != 0.0 ? zi + beta * p[i] : zi;   // a zero beta never reads the old direction
  }
}

// state set-up: zero, then the constants
__global__ void k_state_init(double* __restrict__ st, double tol2, double max_it, double sum_d, double n,
                             double proj) {
  if (threadIdx.x < kStateSize) st[threadIdx.x] = 0.0;
  __syncthreads();
  if (threadIdx.x == 0) {
    st[kTol2] = tol2;
    st[kMaxIt] = max_it;
    st[kSumD] = sum_d;
    st[kN] = n;
    st[kProj] = proj;
  }
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
hipError_t cg_hash_fill(double* v, unsigned long long seed, long long n, double* partial, hipStream_t s) {
  DG_LAUNCH(k_hash_fill, v, seed, n, partial);
}
hipError_t cg_axpb(double* y, const double* x, double a, double c, long long n, hipStream_t s) {
  DG_LAUNCH(k_axpb, y, x, a, c, n);
}
hipError_t cg_fill(double* y, double c, long long n, hipStream_t s) { DG_LAUNCH(k_fill, y, c, n); }
hipError_t cg_xpby(double* y, const double* x, double b, long long n, hipStream_t s) { DG_LAUNCH(k_xpby, y, x, b, n); }

hipError_t cg_state_init(double* st, double tol2, int max_it, double sum_d, long long n, bool proj, hipStream_t s) {
  hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, s, st, tol2, (double)max_it, sum_d, (double)n,
                     proj ? 1.0 : 0.0);
  return hipGetLastError();
}
hipError_t cg_fin_alpha(const double* partial, int nblocks, double* st, hipStream_t s) {
  hipLaunchKernelGGL(k_fin_alpha, dim3(1), dim3(kThreads), 0, s, partial, nblocks, st);
  return hipGetLastError();
}
hipError_t cg_update_xr_st(double* x, double* r, const double* p, const double* q, const double* dinv, int n3,
                           const double* st, bool jacobi, long long n, double* partial, hipStream_t s) {
  if (jacobi) DG_LAUNCH(k_update_xr_st<true>, x, r, p, q, dinv, n3, st, n, partial);
  DG_LAUNCH(k_update_xr_st<false>, x, r, p, q, dinv, n3, st, n, partial);
}
hipError_t cg_fin_jacobi(const double* partial, double* st, bool start, hipStream_t s) {
  hipLaunchKernelGGL(k_fin_jacobi, dim3(1), dim3(kThreads), 0, s, partial, kCgBlocks, st, start ? 1 : 0);
  return hipGetLastError();
}
hipError_t cg_fin_resid(const double* partial, double* st, bool start, hipStream_t s) {
  hipLaunchKernelGGL(k_fin_resid, dim3(1), dim3(kThreads), 0, s, partial, kCgBlocks, st, start ? 1 : 0);
  return hipGetLastError();
}
hipError_t cg_fin_cheb(const double* partial, int nblocks, double* st, bool start, hipStream_t s) {
  hipLaunchKernelGGL(k_fin_cheb, dim3(1), dim3(kThreads), 0, s, partial, nblocks, st, start ? 1 : 0);
  return hipGetLastError();
}
hipError_t cg_cheb1(const double* r, float* z, const float* zprev, const float* dinv32, int n3, const double* st,
                    float inv_theta, long long n, double* partial, hipStream_t s) {
  DG_LAUNCH(k_cheb1, r, z, zprev, dinv32, n3, st, inv_theta, n, partial);
}
hipError_t cg_fill32(float* y, float c, long long n, hipStream_t s) { DG_LAUNCH(k_fill32, y, c, n); }
hipError_t cg_update_p_jacobi(const double* r, double* p, const double* dinv, int n3, const double* st, long long n,
                              hipStream_t s) {
  DG_LAUNCH(k_update_p_jacobi, r, p, dinv, n3, st, n);
}
template <typename T>
static hipError_t rprime_t(const double* r, const double* st, T* out, long long n, hipStream_t s) {
  DG_LAUNCH(k_rprime<T>, r, st, out, n);
}
hipError_t cg_rprime(const double* r, const double* st, double* out, long long n, hipStream_t s) {
  return rprime_t(r, st, out, n, s);
}
hipError_t cg_rprime(const double* r, const double* st, float* out, long long n, hipStream_t s) {
  return rprime_t(r, st, out, n, s);
}
template <typename T>
static hipError_t zsums_t(const double* r, const T* z, const T* zprev, const double* st, long long n,
                          double* partial, hipStream_t s) {
  DG_LAUNCH(k_zsums<T>, r, z, zprev, st, n, partial);
}
hipError_t cg_zsums(const double* r, const double* z, const double* zprev, const double* st, long long n,
                    double* partial, hipStream_t s) {
  return zsums_t(r, z, zprev, st, n, partial, s);
}
hipError_t cg_zsums(const double* r, const float* z, const float* zprev, const double* st, long long n,
                    double* partial, hipStream_t s) {
  return zsums_t(r, z, zprev, st, n, partial, s);
}
template <typename T>
static hipError_t update_p_z_t(const T* z, double* p, const double* st, long long n, hipStream_t s) {
  DG_LAUNCH(k_update_p_z<T>, z, p, st, n);
}
hipError_t cg_update_p_z(const double* z, double* p, const double* st, long long n, hipStream_t s) {
  return update_p_z_t(z, p, st, n, s);
}
hipError_t cg_update_p_z(const float* z, double* p, const double* st, long long n, hipStream_t s) {
  return update_p_z_t(z, p, st, n, s);
}
hipError_t cg_update_p_cheb(const float* z, double* p, const double* st, long long n, hipStream_t s) {
  DG_LAUNCH(k_update_p_cheb, z, p, st, n);
}

}  // namespace dgmf
