// SIPG negative Laplacian (Sec. 3.2, weak form of l_h) by sum factorisation
// on periodic Cartesian meshes, FP64 and FP32, degrees 1..11.
//
// Method.  On an affine, axis-aligned cell the Gauss sums of the SIPG form
// factor by direction (Sec. 3.4: sum factorisation over the tensor-product
// basis and quadrature), and after collapsing "interpolate to Gauss points,
// weight, integrate back" into 1D matrices the operator is
//
//   A = c_x Kx(x)My(x)Mz + c_y Mx(x)Ky(x)Mz + c_z Mx(x)My(x)Kz,
//   c_d = scale * (h_x h_y h_z) / h_d^2,
//
// with M the 1D mass matrix on [0,1] and K the 1D SIPG operator on [0,1]
// (cell stiffness plus the own-side face terms of both ends, penalty
// sigma = penalty_factor (k+1)^2), which couples the two end nodes of each
// pencil to the neighbour element through its end value and end slope only
// (LGL nodes include the end points, Sec. 3.4).  Evaluated as
//
//   y = Mz (c_x My Kx u + c_y Mx Ky u) + c_z Mx My Kz u,
//
// i.e. eight 1D sweeps per element (3 K, 5 M) instead of the twelve of a
// general-geometry evaluation; every neighbour coupling acts on raw u.
//
// GPU mapping.  One workgroup per batch of E = floor(256/n^2) consecutive
// elements, n^2 threads per element.  The batch's n^3*E values are staged in
// LDS once (coalesced); each phase gives every thread one pencil in one
// direction, held in registers while the 1D matrices (kernel arguments, read
// through the scalar unit) are applied; intermediate fields go back to LDS
// between phases.  Neighbour pencils for the face terms are read straight
// from global memory, where neighbouring batches keep them in L2.  Each DoF is
// written once; no atomics.
#include "common.h"
#include "ops.h"

namespace dgmf {

template <int N, typename T>
struct LapTab {
  T M[N][N];
  T K[N][N];
  T hd0[N];   // 1/2 l_b'(0)
  T hd1[N];   // 1/2 l_b'(1)
  T c[3];     // scale * vol / h_d^2
  T sigma;    // penalty_factor * (k+1)^2
};

template <int N>
struct LapCfg {
  static constexpr int N2 = N * N, N3 = N * N * N;
  static constexpr int E = (256 / N2) > 0 ? 256 / N2 : 1;
  static constexpr int THREADS = E * N2;
};

template <int N, typename T>
__device__ __forceinline__ void matvec(const T (&A)[N][N], const T* x, T* y) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T s = A[i][0] * x[0];
#pragma unroll
    for (int j = 1; j < N; ++j) s = fmadd(A[i][j], x[j], s);
    y[i] = s;
  }
}

// 1D SIPG along one pencil: y = Kown u + couplings to the left (uL) and
// right (uR) neighbour pencils through their end value and end slope.
template <int N, typename T>
__device__ __forceinline__ void sipg_pencil(const LapTab<N, T>& t, const T* u, const T* uL,
                                            const T* uR, T* y) {
  matvec<N, T>(t.K, u, y);
  T gR = 0, gL = 0;   // half slopes of the neighbours at the shared faces
#pragma unroll
  for (int j = 0; j < N; ++j) {
    gR = fmadd(t.hd0[j], uR[j], gR);
    gL = fmadd(t.hd1[j], uL[j], gL);
  }
  const T vR = uR[0], vL = uL[N - 1];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    y[i] = fmadd(t.hd1[i], vR, y[i]);
    y[i] = fmadd(-t.hd0[i], vL, y[i]);
  }
  y[N - 1] -= gR + t.sigma * vR;
  y[0] += gL - t.sigma * vL;
}

template <int N, typename T>
__global__ void __launch_bounds__(LapCfg<N>::THREADS)
laplace_kernel(const T* __restrict__ src, T* __restrict__ dst, MeshArgs mesh, int n_total,
               LapTab<N, T> t) {
  using C = LapCfg<N>;
  constexpr int N2 = C::N2, N3 = C::N3, E = C::E;
  __shared__ T U[E * N3];
  __shared__ T B1[E * N3];
  __shared__ T B2[E * N3];
  __shared__ T B3[E * N3];

  const int tid = threadIdx.x;
  const int e0 = blockIdx.x * E;
  const int ne = min(E, n_total - e0);
  {
    const T* g = src + (size_t)e0 * N3;
    for (int i = tid; i < ne * N3; i += C::THREADS) U[i] = g[i];
  }
  __syncthreads();

  const int le = tid / N2, p = tid - le * N2;
  const int p0 = p % N, p1 = p / N;
  const bool active = le < ne;
  const int eg = e0 + le;
  const int comp = eg / mesh.n_el;
  const int e = eg - comp * mesh.n_el;
  const int ex = e % mesh.nx, ey = (e / mesh.nx) % mesh.ny, ez = e / (mesh.nx * mesh.ny);
  const T* csrc = src + (size_t)comp * mesh.n_el * N3;
  T* Ue = U + le * N3;
  T* B1e = B1 + le * N3;
  T* B2e = B2 + le * N3;
  T* B3e = B3 + le * N3;
  T in[N], out[N], nl[N], nr[N], tmp[N];

  // Z: pencil (a,b) = (p0,p1) along z: R = Kz u
  if (active) {
    const int base = p0 + N * p1;
    const T* gl = csrc + (size_t)neighbor(mesh, ex, ey, ez, 2, 0) * N3 + base;
    const T* gr = csrc + (size_t)neighbor(mesh, ex, ey, ez, 2, 1) * N3 + base;
#pragma unroll
    for (int c = 0; c < N; ++c) {
      in[c] = Ue[base + N2 * c];
      nl[c] = gl[N2 * c];
      nr[c] = gr[N2 * c];
    }
    sipg_pencil<N, T>(t, in, nl, nr, out);
#pragma unroll
    for (int c = 0; c < N; ++c) B1e[base + N2 * c] = out[c];
  }
  __syncthreads();

  // Y: pencil (a,c) = (p0,p1) along y: Q = Ky u; R <- My R
  if (active) {
    const int base = p0 + N2 * p1;
    const T* gl = csrc + (size_t)neighbor(mesh, ex, ey, ez, 1, 0) * N3 + base;
    const T* gr = csrc + (size_t)neighbor(mesh, ex, ey, ez, 1, 1) * N3 + base;
#pragma unroll
    for (int b = 0; b < N; ++b) {
      in[b] = Ue[base + N * b];
      nl[b] = gl[N * b];
      nr[b] = gr[N * b];
      tmp[b] = B1e[base + N * b];
    }
    sipg_pencil<N, T>(t, in, nl, nr, out);
#pragma unroll
    for (int b = 0; b < N; ++b) B2e[base + N * b] = out[b];
    matvec<N, T>(t.M, tmp, out);
#pragma unroll
    for (int b = 0; b < N; ++b) B1e[base + N * b] = out[b];
  }
  __syncthreads();

  // X: pencil (b,c) = (p0,p1) along x: P = Kx u; Q <- Mx Q; R <- Mx R
  if (active) {
    const int base = N * p0 + N2 * p1;
    const T* gl = csrc + (size_t)neighbor(mesh, ex, ey, ez, 0, 0) * N3 + base;
    const T* gr = csrc + (size_t)neighbor(mesh, ex, ey, ez, 0, 1) * N3 + base;
#pragma unroll
    for (int a = 0; a < N; ++a) {
      in[a] = Ue[base + a];
      nl[a] = gl[a];
      nr[a] = gr[a];
    }
    sipg_pencil<N, T>(t, in, nl, nr, out);
#pragma unroll
    for (int a = 0; a < N; ++a) tmp[a] = B2e[base + a];
#pragma unroll
    for (int a = 0; a < N; ++a) B2e[base + a] = t.c[0] * out[a];
    matvec<N, T>(t.M, tmp, out);
#pragma unroll
    for (int a = 0; a < N; ++a) {
      B3e[base + a] = t.c[1] * out[a];
      tmp[a] = B1e[base + a];
    }
    matvec<N, T>(t.M, tmp, out);
#pragma unroll
    for (int a = 0; a < N; ++a) B1e[base + a] = t.c[2] * out[a];
  }
  __syncthreads();

  // Y again: S = My (c_x P) + c_y Q
  if (active) {
    const int base = p0 + N2 * p1;
#pragma unroll
    for (int b = 0; b < N; ++b) tmp[b] = B2e[base + N * b];
    matvec<N, T>(t.M, tmp, out);
#pragma unroll
    for (int b = 0; b < N; ++b) B3e[base + N * b] += out[b];
  }
  __syncthreads();

  // Z again: y = Mz S + c_z R, written once
  if (active) {
    const int base = p0 + N * p1;
#pragma unroll
    for (int c = 0; c < N; ++c) tmp[c] = B3e[base + N2 * c];
    matvec<N, T>(t.M, tmp, out);
    T* g = dst + (size_t)eg * N3 + base;
#pragma unroll
    for (int c = 0; c < N; ++c) g[N2 * c] = out[c] + B1e[base + N2 * c];
  }
}

template <int N, typename T>
static hipError_t launch_laplace_n(const LaplacePlan& P, const void* src, void* dst,
                                   hipStream_t stream) {
  using C = LapCfg<N>;
  LapTab<N, T> t;
  for (int i = 0; i < N; ++i) {
    for (int j = 0; j < N; ++j) {
      t.M[i][j] = (T)P.Mref[i * N + j];
      t.K[i][j] = (T)P.Kown[i * N + j];
    }
    t.hd0[i] = (T)(0.5 * P.D[i]);
    t.hd1[i] = (T)(0.5 * P.D[(N - 1) * N + i]);
  }
  for (int d = 0; d < 3; ++d) t.c[d] = (T)P.c[d];
  t.sigma = (T)P.sigma;
  const int total = P.n_comp * P.mesh.n_el;
  const int grid = (total + C::E - 1) / C::E;
  hipLaunchKernelGGL((laplace_kernel<N, T>), dim3(grid), dim3(C::THREADS), 0, stream,
                     (const T*)src, (T*)dst, P.mesh, total, t);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_laplace_t(const LaplacePlan& P, const void* src, void* dst,
                                   hipStream_t s) {
  switch (P.k) {
    case 1: return launch_laplace_n<2, T>(P, src, dst, s);
    case 2: return launch_laplace_n<3, T>(P, src, dst, s);
    case 3: return launch_laplace_n<4, T>(P, src, dst, s);
    case 4: return launch_laplace_n<5, T>(P, src, dst, s);
    case 5: return launch_laplace_n<6, T>(P, src, dst, s);
    case 6: return launch_laplace_n<7, T>(P, src, dst, s);
    case 7: return launch_laplace_n<8, T>(P, src, dst, s);
    case 8: return launch_laplace_n<9, T>(P, src, dst, s);
    case 9: return launch_laplace_n<10, T>(P, src, dst, s);
    case 10: return launch_laplace_n<11, T>(P, src, dst, s);
    case 11: return launch_laplace_n<12, T>(P, src, dst, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_laplace(const LaplacePlan& P, bool f32, const void* src, void* dst,
                          hipStream_t stream) {
  return f32 ? launch_laplace_t<float>(P, src, dst, stream)
             : launch_laplace_t<double>(P, src, dst, stream);
}

}  // namespace dgmf
