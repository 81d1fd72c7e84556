// Pressure gradient with central flux (Sec. 3.2, weak form of g_h), the
// pressure term of the projection step's right-hand side, FP64 and FP32:
//
//   y_j,i = -(d_j phi_i, p)_K + sum over the faces normal to e_j of
//           n_j (phi_i, 1/2 (p- + p+))
//
// On an affine, axis-aligned cell component j factors by direction:
//   y_j = c_j (G along j) (x) (M along the other two) p,   c_j = vol/h_j,
// with the 1D operator G[i][l] = -sum_q w_q l_i'(z_q) l_l(z_q) + 1/2 l_i(1) l_l(1)
// - 1/2 l_i(0) l_l(0) and the neighbour couplings 1/2 pR(0) at the right end,
// -1/2 pL(1) at the left.  Integration by parts shows G = -B^T for the
// divergence's 1D operator B (exact Gauss integration), so the divergence
// plan's tables serve both.  The G sweep of each component comes first (the
// neighbour terms enter there), then the two mass sweeps:
//   Z   Rz = Gz p
//   Y   Ry = Gy p;  Rz <- My Rz
//   X   Rx = Gx p;  Ry <- Mx Ry;  y_z = c_z Mx Rz (stored)
//   Y   Rx <- My Rx
//   Z   y_x = c_x Mz Rx, y_y = c_y Mz Ry (stored)
// E elements per workgroup, one pencil per thread per phase, LDS between
// (three arrays of E n^3 values: Rx takes the place of p in the X phase).
#include "api_internal.h"
#include "common.h"
#include "ops.h"

namespace dgmf {

namespace {

template <int N, typename T>
struct GradTab {
  T M[N][N];
  T G[N][N];
};

template <int N>
struct GradCfg {
  static constexpr int N2 = N * N, N3 = N * N * N;
  static constexpr int E = (256 / N2) > 0 ? 256 / N2 : 1;
  static constexpr int THREADS = E * N2;
};

template <int N, typename T, typename Mat>
__device__ __forceinline__ void gmv(const Mat& A, const T* x, T* y) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T s = A[i][0] * x[0];
#pragma unroll
    for (int l = 1; l < N; ++l) s = fmadd(A[i][l], x[l], s);
    y[i] = s;
  }
}

template <int N, typename T>
__global__ void __launch_bounds__(GradCfg<N>::THREADS)
gradient_kernel(const T* __restrict__ p, T* __restrict__ y, MeshArgs mesh, const GradTab<N, T>* __restrict__ tab,
                T cx, T cy, T cz) {
  using C = GradCfg<N>;
  constexpr int N2 = C::N2, N3 = C::N3, E = C::E;
  // RX overwrites P pencil by pencil in the X phase (each thread reads its
  // whole x pencil of P before writing it), so three arrays suffice
  __shared__ T P[E * N3];
  __shared__ T RY[E * N3];
  __shared__ T RZ[E * N3];
  T* RX = P;
  const int tid = threadIdx.x;
  const int e0 = xcd_remap(blockIdx.x, gridDim.x) * E;
  const int ne = min(E, mesh.n_el - e0);
  const size_t cs = (size_t)mesh.n_el * N3;
  const int le = tid / N2, q = tid - le * N2;
  const int q0 = q % N, q1 = q / N;
  const bool active = le < ne;
  const int e = e0 + le;
  const int ex = active ? e % mesh.nx : 0, ey = active ? (e / mesh.nx) % mesh.ny : 0;
  const int ez = active ? e / (mesh.nx * mesh.ny) : 0;
  const int off = le * N3;
  T in[N], out[N];
  // Z: own z column of p from global memory (consecutive threads, consecutive
  // addresses) into registers and LDS; Rz = Gz p, neighbour layers along z
  if (active) {
    const auto& t = *fresh(tab);
    const int base = q0 + N * q1;
    const T* gc = p + (size_t)e * N3 + base;
    const T* gl = p + (size_t)neighbor(mesh, ex, ey, ez, 2, 0) * N3 + base;
    const T* gr = p + (size_t)neighbor(mesh, ex, ey, ez, 2, 1) * N3 + base;
#pragma unroll
    for (int c = 0; c < N; ++c) in[c] = gc[N2 * c];
#pragma unroll
    for (int c = 0; c < N; ++c) P[off + base + N2 * c] = in[c];
    gmv<N, T>(t.G, in, out);
    out[N - 1] += T(0.5) * gr[0];
    out[0] -= T(0.5) * gl[N2 * (N - 1)];
#pragma unroll
    for (int c = 0; c < N; ++c) RZ[off + base + N2 * c] = out[c];
  }
  __syncthreads();
  // Y: Ry = Gy p; Rz <- My Rz
  if (active) {
    const auto& t = *fresh(tab);
    const int base = q0 + N2 * q1;
    const T* gl = p + (size_t)neighbor(mesh, ex, ey, ez, 1, 0) * N3 + base;
    const T* gr = p + (size_t)neighbor(mesh, ex, ey, ez, 1, 1) * N3 + base;
#pragma unroll
    for (int b = 0; b < N; ++b) in[b] = P[off + base + N * b];
    gmv<N, T>(t.G, in, out);
    out[N - 1] += T(0.5) * gr[0];
    out[0] -= T(0.5) * gl[N * (N - 1)];
#pragma unroll
    for (int b = 0; b < N; ++b) RY[off + base + N * b] = out[b];
#pragma unroll
    for (int b = 0; b < N; ++b) in[b] = RZ[off + base + N * b];
    gmv<N, T>(t.M, in, out);
#pragma unroll
    for (int b = 0; b < N; ++b) RZ[off + base + N * b] = out[b];
  }
  __syncthreads();
  // X: Rx = Gx p; Ry <- Mx Ry; y_z = c_z Mx Rz
  if (active) {
    const auto& t = *fresh(tab);
    const int base = N * q0 + N2 * q1;
    const T* gl = p + (size_t)neighbor(mesh, ex, ey, ez, 0, 0) * N3 + base;
    const T* gr = p + (size_t)neighbor(mesh, ex, ey, ez, 0, 1) * N3 + base;
#pragma unroll
    for (int a = 0; a < N; ++a) in[a] = P[off + base + a];
    gmv<N, T>(t.G, in, out);
    out[N - 1] += T(0.5) * gr[0];
    out[0] -= T(0.5) * gl[N - 1];
#pragma unroll
    for (int a = 0; a < N; ++a) RX[off + base + a] = out[a];
#pragma unroll
    for (int a = 0; a < N; ++a) in[a] = RY[off + base + a];
    gmv<N, T>(t.M, in, out);
#pragma unroll
    for (int a = 0; a < N; ++a) RY[off + base + a] = out[a];
#pragma unroll
    for (int a = 0; a < N; ++a) in[a] = RZ[off + base + a];
    gmv<N, T>(t.M, in, out);
    T* g = y + 2 * cs + (size_t)e * N3 + base;
#pragma unroll
    for (int a = 0; a < N; ++a) g[a] = cz * out[a];
  }
  __syncthreads();
  // Y again: Rx <- My Rx
  if (active) {
    const auto& t = *fresh(tab);
    const int base = q0 + N2 * q1;
#pragma unroll
    for (int b = 0; b < N; ++b) in[b] = RX[off + base + N * b];
    gmv<N, T>(t.M, in, out);
#pragma unroll
    for (int b = 0; b < N; ++b) RX[off + base + N * b] = out[b];
  }
  __syncthreads();
  // Z again: y_x = c_x Mz Rx, y_y = c_y Mz Ry
  if (active) {
    const auto& t = *fresh(tab);
    const int base = q0 + N * q1;
#pragma unroll
    for (int c = 0; c < N; ++c) in[c] = RX[off + base + N2 * c];
    gmv<N, T>(t.M, in, out);
    T* gx = y + (size_t)e * N3 + base;
#pragma unroll
    for (int c = 0; c < N; ++c) gx[N2 * c] = cx * out[c];
#pragma unroll
    for (int c = 0; c < N; ++c) in[c] = RY[off + base + N2 * c];
    gmv<N, T>(t.M, in, out);
    T* gy = y + cs + (size_t)e * N3 + base;
#pragma unroll
    for (int c = 0; c < N; ++c) gy[N2 * c] = cy * out[c];
  }
}

template <int N, typename T>
hipError_t launch_grad_n(const DivPlan& P, const void* p, void* y, hipStream_t s) {
  using C = GradCfg<N>;
  GradTab<N, T> t;
  for (int i = 0; i < N; ++i)
    for (int l = 0; l < N; ++l) {
      t.M[i][l] = (T)P.Mref[i * N + l];
      t.G[i][l] = (T)(-P.Bown[l * N + i]);
    }
  hipError_t err;
  const GradTab<N, T>* dt = device_table_of("gradient", t, &err);
  if (!dt) return err;
  const long long grid = ((long long)P.mesh.n_el + C::E - 1) / C::E;
  if (grid > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((gradient_kernel<N, T>), dim3((unsigned)grid), dim3(C::THREADS), 0, s, (const T*)p, (T*)y,
                     P.mesh, dt, (T)P.c[0], (T)P.c[1], (T)P.c[2]);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_grad_t(const DivPlan& P, const void* p, void* y, hipStream_t s) {
  switch (P.k) {
    case 1: return launch_grad_n<2, T>(P, p, y, s);
    case 2: return launch_grad_n<3, T>(P, p, y, s);
    case 3: return launch_grad_n<4, T>(P, p, y, s);
    case 4: return launch_grad_n<5, T>(P, p, y, s);
    case 5: return launch_grad_n<6, T>(P, p, y, s);
    case 6: return launch_grad_n<7, T>(P, p, y, s);
    case 7: return launch_grad_n<8, T>(P, p, y, s);
    case 8: return launch_grad_n<9, T>(P, p, y, s);
    case 9: return launch_grad_n<10, T>(P, p, y, s);
    case 10: return launch_grad_n<11, T>(P, p, y, s);
    case 11: return launch_grad_n<12, T>(P, p, y, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_gradient(const DivPlan& P, bool f32, const void* p, void* y, hipStream_t s) {
  return f32 ? launch_grad_t<float>(P, p, y, s) : launch_grad_t<double>(P, p, y, s);
}

}  // namespace dgmf
