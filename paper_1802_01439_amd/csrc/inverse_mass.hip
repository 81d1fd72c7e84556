// Inverse mass matrix of the DG space (Sec. 3.3: block-diagonal, inverted
// element by element by sum factorisation), FP64 and FP32, degrees 1..11.
//
// On an affine Cartesian cell with the LGL nodal basis and k+1 Gauss points
// per direction (exact), the element mass matrix is h_x h_y h_z M1(x)M1(x)M1
// with M1 the 1D mass on [0,1], so
//   M_e^-1 = (1 / (h_x h_y h_z)) M1^-1 (x) M1^-1 (x) M1^-1,
// three dense 1D sweeps with the host-computed M1^-1.  Element-local: no
// neighbour data, input read once and output written once (memory bound,
// Sec. 4.4).
//
// Mapping: one workgroup per batch of E = floor(256/n^2) consecutive element
// blocks (components are further blocks of the component-major layout);
// n^2 threads per element.  Each thread loads its z column (consecutive
// threads read consecutive addresses), sweeps it in registers, and the y and
// x sweeps run on LDS pencils in place; each thread then stores its z column
// from LDS.  3 barriers.  Because every block is read completely before any
// of it is written, src == dst (in place) is allowed.
#include "api_internal.h"
#include "cg_kernels.h"
#include "common.h"
#include "laplace_kernels.h"
#include "ops.h"

namespace dgmf {

namespace {

template <int N, typename T>
struct InvMassTab {
  T A[N][N];   // M1^-1 (times 1/(h_x h_y h_z) in the x sweep)
  T scale;     // 1 / (h_x h_y h_z)
};

template <int N, typename T, typename Mat>
__device__ __forceinline__ void mv(const Mat& A, const T* x, T* y) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T s = A[i][0] * x[0];
#pragma unroll
    for (int j = 1; j < N; ++j) s = fmadd(A[i][j], x[j], s);
    y[i] = s;
  }
}

template <int N, typename T>
__global__ void __launch_bounds__(LapCfgB<N>::THREADS)
inverse_mass_kernel(const T* src, T* dst, long long nblocks, const InvMassTab<N, T>* __restrict__ tab) {
  using C = LapCfgB<N>;
  constexpr int N2 = N * N, N3 = N * N * N, E = C::E, ES = C::ES, PX = C::PX, PY = C::PY;
  __shared__ T U[E * ES];
  const int tid = threadIdx.x;
  const int le = tid / N2, p = tid - le * N2;
  const int p0 = p % N, p1 = p / N;
  const long long blk = (long long)blockIdx.x * E + le;
  const bool active = blk < nblocks;
  T* Ue = U + le * ES;
  T x[N], y[N];
  // z: own column in registers
  if (active) {
    const auto& t = *fresh(tab);
    const T* g = src + blk * N3 + p0 + N * p1;
#pragma unroll
    for (int c = 0; c < N; ++c) x[c] = g[N2 * c];
    mv<N, T>(t.A, x, y);
    const int base = p0 + PX * p1;
#pragma unroll
    for (int c = 0; c < N; ++c) Ue[base + PY * c] = y[c];
  }
  __syncthreads();
  // y: pencil (a, c) = (p0, p1), in place
  if (active) {
    const auto& t = *fresh(tab);
    const int base = p0 + PY * p1;
#pragma unroll
    for (int b = 0; b < N; ++b) x[b] = Ue[base + PX * b];
    mv<N, T>(t.A, x, y);
#pragma unroll
    for (int b = 0; b < N; ++b) Ue[base + PX * b] = y[b];
  }
  __syncthreads();
  // x: pencil (b, c) = (p0, p1), in place, with the cell scaling
  if (active) {
    const auto& t = *fresh(tab);
    const int base = PX * p0 + PY * p1;
#pragma unroll
    for (int a = 0; a < N; ++a) x[a] = Ue[base + a];
    mv<N, T>(t.A, x, y);
#pragma unroll
    for (int a = 0; a < N; ++a) Ue[base + a] = t.scale * y[a];
  }
  __syncthreads();
  // store the z column
  if (active) {
    T* g = dst + blk * N3 + p0 + N * p1;
    const int base = p0 + PX * p1;
#pragma unroll
    for (int c = 0; c < N; ++c) g[N2 * c] = Ue[base + PY * c];
  }
}

// One step of the inverse-mass-preconditioned CG on element blocks (FP64):
// x += alpha p and r -= alpha q (alpha from the solver state; nothing is
// written while it is 0), z = M^-1 r, and the block sums of r.r and r.z into
// partial[blockIdx.x] and partial[gridDim.x + blockIdx.x].  Each thread keeps
// its updated r column in registers for r.z.
template <int N>
__global__ void __launch_bounds__(LapCfgB<N>::THREADS)
pcg_precond_kernel(double* __restrict__ x, double* __restrict__ r, const double* __restrict__ p,
                   const double* __restrict__ q, double* __restrict__ z, const double* __restrict__ st,
                   long long nblocks, const InvMassTab<N, double>* __restrict__ tab, double* __restrict__ partial) {
  using C = LapCfgB<N>;
  constexpr int N2 = N * N, N3 = N * N * N, E = C::E, ES = C::ES, PX = C::PX, PY = C::PY;
  __shared__ double U[E * ES];
  __shared__ double red[2][C::THREADS];
  const int tid = threadIdx.x;
  const int le = tid / N2, pp = tid - le * N2;
  const int p0 = pp % N, p1 = pp / N;
  const long long blk = (long long)blockIdx.x * E + le;
  const bool active = blk < nblocks;
  double* Ue = U + le * ES;
  double rc[N], y[N];
  double rr = 0, rz = 0;
  if (active) {
    const double alpha = st[kAlpha];
    const size_t o = blk * N3 + p0 + N * p1;
#pragma unroll
    for (int c = 0; c < N; ++c) rc[c] = r[o + N2 * c];
    if (alpha != 0.0) {
#pragma unroll
      for (int c = 0; c < N; ++c) {
        x[o + N2 * c] += alpha * p[o + N2 * c];
        rc[c] -= alpha * q[o + N2 * c];
        r[o + N2 * c] = rc[c];
      }
    }
#pragma unroll
    for (int c = 0; c < N; ++c) rr = fmadd(rc[c], rc[c], rr);
    const auto& t = *fresh(tab);
    mv<N, double>(t.A, rc, y);
    const int base = p0 + PX * p1;
#pragma unroll
    for (int c = 0; c < N; ++c) Ue[base + PY * c] = y[c];
  }
  __syncthreads();
  if (active) {
    const auto& t = *fresh(tab);
    const int base = p0 + PY * p1;
    double v[N];
#pragma unroll
    for (int b = 0; b < N; ++b) v[b] = Ue[base + PX * b];
    mv<N, double>(t.A, v, y);
#pragma unroll
    for (int b = 0; b < N; ++b) Ue[base + PX * b] = y[b];
  }
  __syncthreads();
  if (active) {
    const auto& t = *fresh(tab);
    const int base = PX * p0 + PY * p1;
    double v[N];
#pragma unroll
    for (int a = 0; a < N; ++a) v[a] = Ue[base + a];
    mv<N, double>(t.A, v, y);
#pragma unroll
    for (int a = 0; a < N; ++a) Ue[base + a] = t.scale * y[a];
  }
  __syncthreads();
  if (active) {
    double* g = z + blk * N3 + p0 + N * p1;
    const int base = p0 + PX * p1;
#pragma unroll
    for (int c = 0; c < N; ++c) {
      const double zc = Ue[base + PY * c];
      g[N2 * c] = zc;
      rz = fmadd(rc[c], zc, rz);
    }
  }
  red[0][tid] = rr;
  red[1][tid] = rz;
  __syncthreads();
  if (tid == 0) {
    double a = 0, b = 0;
    for (int i = 0; i < C::THREADS; ++i) {
      a += red[0][i];
      b += red[1][i];
    }
    partial[blockIdx.x] = a;
    partial[gridDim.x + blockIdx.x] = b;
  }
}

template <int N>
hipError_t launch_pcg_n(const std::vector<double>& Minv, double scale, long long nblocks, double* x, double* r,
                        const double* p, const double* q, double* z, const double* st, double* partial,
                        hipStream_t s) {
  InvMassTab<N, double> t;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) t.A[i][j] = Minv[i * N + j];
  t.scale = scale;
  hipError_t err;
  const InvMassTab<N, double>* dt = device_table_of("inverse_mass", t, &err);
  if (!dt) return err;
  using C = LapCfgB<N>;
  const long long grid = (nblocks + C::E - 1) / C::E;
  if (grid > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL((pcg_precond_kernel<N>), dim3((unsigned)grid), dim3(C::THREADS), 0, s, x, r, p, q, z, st,
                     nblocks, dt, partial);
  return hipGetLastError();
}

// Convective substep of the dual-splitting scheme in one pass (FP64):
//   C = b0 cn + b1 cm (cm optional),  C' = M^-1 C,
//   uhat = a0 un + a1 unm1 + a2 C' (unm1 optional),
// each combination with the operations of the step's separate linear
// combination kernel (a product, then fused multiply-adds), so the result is
// the one of the three separate passes; C and C' never go to memory.
template <int N>
__global__ void __launch_bounds__(LapCfgB<N>::THREADS)
conv_substep_kernel(const double* __restrict__ cn, const double* __restrict__ cm, double b0, double b1,
                    const double* __restrict__ un, const double* __restrict__ unm1, double a0, double a1, double a2,
                    double* __restrict__ uhat, long long nblocks, const InvMassTab<N, double>* __restrict__ tab) {
  using C = LapCfgB<N>;
  constexpr int N2 = N * N, N3 = N * N * N, E = C::E, ES = C::ES, PX = C::PX, PY = C::PY;
  __shared__ double U[E * ES];
  const int tid = threadIdx.x;
  const int le = tid / N2, p = tid - le * N2;
  const int p0 = p % N, p1 = p / N;
  const long long blk = (long long)blockIdx.x * E + le;
  const bool active = blk < nblocks;
  double* Ue = U + le * ES;
  double x[N], y[N];
  if (active) {
    const auto& t = *fresh(tab);
    const size_t o = blk * N3 + p0 + N * p1;
#pragma unroll
    for (int c = 0; c < N; ++c) {
      if (cm) {
        double v = b0 * cn[o + N2 * c];
        x[c] = fma(b1, cm[o + N2 * c], v);
      } else {
        x[c] = cn[o + N2 * c];
      }
    }
    mv<N, double>(t.A, x, y);
    const int base = p0 + PX * p1;
#pragma unroll
    for (int c = 0; c < N; ++c) Ue[base + PY * c] = y[c];
  }
  __syncthreads();
  if (active) {
    const auto& t = *fresh(tab);
    const int base = p0 + PY * p1;
#pragma unroll
    for (int b = 0; b < N; ++b) x[b] = Ue[base + PX * b];
    mv<N, double>(t.A, x, y);
#pragma unroll
    for (int b = 0; b < N; ++b) Ue[base + PX * b] = y[b];
  }
  __syncthreads();
  if (active) {
    const auto& t = *fresh(tab);
    const int base = PX * p0 + PY * p1;
#pragma unroll
    for (int a = 0; a < N; ++a) x[a] = Ue[base + a];
    mv<N, double>(t.A, x, y);
#pragma unroll
    for (int a = 0; a < N; ++a) Ue[base + a] = t.scale * y[a];
  }
  __syncthreads();
  if (active) {
    const size_t o = blk * N3 + p0 + N * p1;
    const int base = p0 + PX * p1;
#pragma unroll
    for (int c = 0; c < N; ++c) {
      double v = a0 * un[o + N2 * c];
      if (unm1) v = fma(a1, unm1[o + N2 * c], v);
      uhat[o + N2 * c] = fma(a2, Ue[base + PY * c], v);
    }
  }
}

template <int N>
hipError_t launch_substep_n(const std::vector<double>& Minv, double scale, long long nblocks, const double* cn,
                            const double* cm, double b0, double b1, const double* un, const double* unm1, double a0,
                            double a1, double a2, double* uhat, hipStream_t s) {
  InvMassTab<N, double> t;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) t.A[i][j] = Minv[i * N + j];
  t.scale = scale;
  hipError_t err;
  const InvMassTab<N, double>* dt = device_table_of("inverse_mass", t, &err);
  if (!dt) return err;
  using C = LapCfgB<N>;
  const long long grid = (nblocks + C::E - 1) / C::E;
  if (grid > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL((conv_substep_kernel<N>), dim3((unsigned)grid), dim3(C::THREADS), 0, s, cn, cm, b0, b1, un, unm1,
                     a0, a1, a2, uhat, nblocks, dt);
  return hipGetLastError();
}

template <int N, typename T>
hipError_t launch_n(const std::vector<double>& Minv, double scale, long long nblocks, const void* src, void* dst,
                    hipStream_t s) {
  InvMassTab<N, T> t;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) t.A[i][j] = (T)Minv[i * N + j];
  t.scale = (T)scale;
  hipError_t err;
  const InvMassTab<N, T>* dt = device_table_of("inverse_mass", t, &err);
  if (!dt) return err;
  using C = LapCfgB<N>;
  const long long grid = (nblocks + C::E - 1) / C::E;
  if (grid > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL((inverse_mass_kernel<N, T>), dim3((unsigned)grid), dim3(C::THREADS), 0, s, (const T*)src,
                     (T*)dst, nblocks, dt);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_t(int k, const std::vector<double>& Minv, double scale, long long nblocks, const void* src,
                    void* dst, hipStream_t s) {
  switch (k) {
    case 1: return launch_n<2, T>(Minv, scale, nblocks, src, dst, s);
    case 2: return launch_n<3, T>(Minv, scale, nblocks, src, dst, s);
    case 3: return launch_n<4, T>(Minv, scale, nblocks, src, dst, s);
    case 4: return launch_n<5, T>(Minv, scale, nblocks, src, dst, s);
    case 5: return launch_n<6, T>(Minv, scale, nblocks, src, dst, s);
    case 6: return launch_n<7, T>(Minv, scale, nblocks, src, dst, s);
    case 7: return launch_n<8, T>(Minv, scale, nblocks, src, dst, s);
    case 8: return launch_n<9, T>(Minv, scale, nblocks, src, dst, s);
    case 9: return launch_n<10, T>(Minv, scale, nblocks, src, dst, s);
    case 10: return launch_n<11, T>(Minv, scale, nblocks, src, dst, s);
    case 11: return launch_n<12, T>(Minv, scale, nblocks, src, dst, s);
    default: return hipErrorInvalidValue;
  }
}

template <int N>
long long pcg_grid_n(long long nblocks) {
  return (nblocks + LapCfgB<N>::E - 1) / LapCfgB<N>::E;
}

}  // namespace

long long pcg_precond_grid(int k, long long nblocks) {
  switch (k) {
    case 1: return pcg_grid_n<2>(nblocks);
    case 2: return pcg_grid_n<3>(nblocks);
    case 3: return pcg_grid_n<4>(nblocks);
    case 4: return pcg_grid_n<5>(nblocks);
    case 5: return pcg_grid_n<6>(nblocks);
    case 6: return pcg_grid_n<7>(nblocks);
    case 7: return pcg_grid_n<8>(nblocks);
    case 8: return pcg_grid_n<9>(nblocks);
    case 9: return pcg_grid_n<10>(nblocks);
    case 10: return pcg_grid_n<11>(nblocks);
    case 11: return pcg_grid_n<12>(nblocks);
    default: return 0;
  }
}

hipError_t launch_pcg_precond(int k, const std::vector<double>& Minv, double scale, long long nblocks, double* x,
                              double* r, const double* p, const double* q, double* z, const double* st,
                              double* partial, hipStream_t s) {
  switch (k) {
    case 1: return launch_pcg_n<2>(Minv, scale, nblocks, x, r, p, q, z, st, partial, s);
    case 2: return launch_pcg_n<3>(Minv, scale, nblocks, x, r, p, q, z, st, partial, s);
    case 3: return launch_pcg_n<4>(Minv, scale, nblocks, x, r, p, q, z, st, partial, s);
    case 4: return launch_pcg_n<5>(Minv, scale, nblocks, x, r, p, q, z, st, partial, s);
    case 5: return launch_pcg_n<6>(Minv, scale, nblocks, x, r, p, q, z, st, partial, s);
    case 6: return launch_pcg_n<7>(Minv, scale, nblocks, x, r, p, q, z, st, partial, s);
    case 7: return launch_pcg_n<8>(Minv, scale, nblocks, x, r, p, q, z, st, partial, s);
    case 8: return launch_pcg_n<9>(Minv, scale, nblocks, x, r, p, q, z, st, partial, s);
    case 9: return launch_pcg_n<10>(Minv, scale, nblocks, x, r, p, q, z, st, partial, s);
    case 10: return launch_pcg_n<11>(Minv, scale, nblocks, x, r, p, q, z, st, partial, s);
    case 11: return launch_pcg_n<12>(Minv, scale, nblocks, x, r, p, q, z, st, partial, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_convective_substep(int k, const std::vector<double>& Minv, double scale, long long nblocks,
                                    const double* cn, const double* cm, double b0, double b1, const double* un,
                                    const double* unm1, double a0, double a1, double a2, double* uhat,
                                    hipStream_t s) {
  switch (k) {
#define DG_SUBSTEP_CASE(K) \
  case K: return launch_substep_n<K + 1>(Minv, scale, nblocks, cn, cm, b0, b1, un, unm1, a0, a1, a2, uhat, s);
    DG_SUBSTEP_CASE(1) DG_SUBSTEP_CASE(2) DG_SUBSTEP_CASE(3) DG_SUBSTEP_CASE(4) DG_SUBSTEP_CASE(5)
    DG_SUBSTEP_CASE(6) DG_SUBSTEP_CASE(7) DG_SUBSTEP_CASE(8) DG_SUBSTEP_CASE(9) DG_SUBSTEP_CASE(10)
    DG_SUBSTEP_CASE(11)
#undef DG_SUBSTEP_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_inverse_mass(int k, const std::vector<double>& Minv, double scale, long long nblocks, bool f32,
                               const void* src, void* dst, hipStream_t s) {
  return f32 ? launch_t<float>(k, Minv, scale, nblocks, src, dst, s)
             : launch_t<double>(k, Minv, scale, nblocks, src, dst, s);
}

}  // namespace dgmf
