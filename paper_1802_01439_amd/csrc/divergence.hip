// Velocity divergence with central flux (Sec. 3.2, weak form of d_h): the
// right-hand side of the pressure Poisson step, FP64 and FP32.
//
//   b_i = -(grad phi_i, u)_K + sum_faces (phi_i, 1/2 (u- + u+) . n)
//
// On an affine, axis-aligned cell each term involves one velocity component
// and factors by direction like the SIPG form:
//   b = c_x Bx(x)My(x)Mz u_x + c_y Mx(x)By(x)Mz u_y + c_z Mx(x)My(x)Bz u_z,
//   c_d = vol/h_d,
// with B the 1D operator on [0,1]: B[i][j] = -sum_q w_q l_i'(z_q) l_j(z_q) plus
// the own-side central-flux terms 1/2 l_i(1) l_j(1) - 1/2 l_i(0) l_j(0), and
// the neighbour coupling 1/2 uR(0) at the right end, -1/2 uL(1) at the left.
// GPU mapping: E elements per workgroup, one pencil per thread per phase,
// LDS between phases; each thread loads its own z columns straight into
// registers, and four LDS arrays of E n^3 values carry the rest.
#include "api_internal.h"
#include "common.h"
#include "ops.h"

namespace dgmf {

template <int N, typename T>
struct DivTab {
  T M[N][N];
  T B[N][N];
};

template <typename T>
struct DivScal {
  T c[3];   // vol/h_d
};

template <int N>
struct DivCfg {
  static constexpr int N2 = N * N, N3 = N * N * N;
  // one element per workgroup from n = 10 on: two would need 64-85 KB of LDS
  // per workgroup and leave fewer waves per CU than single elements
  // (measured: k = 9, 10 FP64 17 % and 30 % faster)
  static constexpr int E = (N >= 10 || 256 / N2 < 1) ? 1 : 256 / N2;
  static constexpr int THREADS = E * N2;
};

template <int N, typename T, typename Mat>
__device__ __forceinline__ void dmv(const Mat& A, const T* x, T* y) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T s = A[i][0] * x[0];
#pragma unroll
    for (int j = 1; j < N; ++j) s = fmadd(A[i][j], x[j], s);
    y[i] = s;
  }
}

template <int N, typename T>
__global__ void __launch_bounds__(DivCfg<N>::THREADS)
divergence_kernel(const T* __restrict__ u, T* __restrict__ b, MeshArgs mesh,
                  const DivTab<N, T>* __restrict__ tab, DivScal<T> sc) {
  using C = DivCfg<N>;
  constexpr int N2 = C::N2, N3 = C::N3, E = C::E;
  // u_x and u_y columns; P = c_x Bx u_x later takes the place of u_x and
  // c_y Mx Q the place of Q (pencil by pencil: each thread reads its whole
  // pencil before writing it); u_z stays in registers
  __shared__ T UX[E * N3];
  __shared__ T UY[E * N3];
  __shared__ T B1[E * N3];
  __shared__ T B2[E * N3];
  const int tid = threadIdx.x;
  const int e0 = xcd_remap(blockIdx.x, gridDim.x) * E;
  const int ne = min(E, mesh.n_el - e0);
  const size_t cs = (size_t)mesh.n_el * N3;
  const int le = tid / N2, p = tid - le * N2;
  const int p0 = p % N, p1 = p / N;
  const bool active = le < ne;
  const int e = e0 + le;
  const int ex = active ? e % mesh.nx : 0, ey = active ? (e / mesh.nx) % mesh.ny : 0;
  const int ez = active ? e / (mesh.nx * mesh.ny) : 0;
  T in[N], out[N], tmp[N];
  const int off = le * N3;

  // Z: own z columns of the three components from global memory (consecutive
  // threads, consecutive addresses); R = Bz u_z
  if (active) {
    const auto& t = *fresh(tab);
    const int base = p0 + N * p1;
    const T* gc = u + (size_t)e * N3 + base;
#pragma unroll
    for (int c = 0; c < N; ++c) {
      UX[off + base + N2 * c] = gc[N2 * c];
      UY[off + base + N2 * c] = gc[cs + N2 * c];
      in[c] = gc[2 * cs + N2 * c];
    }
    const T* gl = u + 2 * cs + (size_t)neighbor(mesh, ex, ey, ez, 2, 0) * N3 + base;
    const T* gr = u + 2 * cs + (size_t)neighbor(mesh, ex, ey, ez, 2, 1) * N3 + base;
    dmv<N, T>(t.B, in, out);
    out[N - 1] += T(0.5) * gr[0];
    out[0] -= T(0.5) * gl[N2 * (N - 1)];
#pragma unroll
    for (int c = 0; c < N; ++c) B1[off + base + N2 * c] = out[c];
  }
  __syncthreads();
  // Y: Q = By u_y; R <- My R
  if (active) {
    const auto& t = *fresh(tab);
    const int base = p0 + N2 * p1;
    const T* gl = u + 1 * cs + (size_t)neighbor(mesh, ex, ey, ez, 1, 0) * N3 + base;
    const T* gr = u + 1 * cs + (size_t)neighbor(mesh, ex, ey, ez, 1, 1) * N3 + base;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      in[j] = UY[off + base + N * j];
      tmp[j] = B1[off + base + N * j];
    }
    dmv<N, T>(t.B, in, out);
    out[N - 1] += T(0.5) * gr[0];
    out[0] -= T(0.5) * gl[N * (N - 1)];
#pragma unroll
    for (int j = 0; j < N; ++j) B2[off + base + N * j] = out[j];
    dmv<N, T>(t.M, tmp, out);
#pragma unroll
    for (int j = 0; j < N; ++j) B1[off + base + N * j] = out[j];
  }
  __syncthreads();
  // X: UX <- c_x Bx u_x; B2 <- c_y Mx Q; B1 <- c_z Mx R
  if (active) {
    const auto& t = *fresh(tab);
    const int base = N * p0 + N2 * p1;
    const T* gl = u + (size_t)neighbor(mesh, ex, ey, ez, 0, 0) * N3 + base;
    const T* gr = u + (size_t)neighbor(mesh, ex, ey, ez, 0, 1) * N3 + base;
#pragma unroll
    for (int a = 0; a < N; ++a) in[a] = UX[off + base + a];
    dmv<N, T>(t.B, in, out);
    out[N - 1] += T(0.5) * gr[0];
    out[0] -= T(0.5) * gl[N - 1];
#pragma unroll
    for (int a = 0; a < N; ++a) {
      UX[off + base + a] = sc.c[0] * out[a];
      tmp[a] = B2[off + base + a];
    }
    dmv<N, T>(t.M, tmp, out);
#pragma unroll
    for (int a = 0; a < N; ++a) {
      B2[off + base + a] = sc.c[1] * out[a];
      tmp[a] = B1[off + base + a];
    }
    dmv<N, T>(t.M, tmp, out);
#pragma unroll
    for (int a = 0; a < N; ++a) B1[off + base + a] = sc.c[2] * out[a];
  }
  __syncthreads();
  // Y again: S = My (c_x P) + c_y Q
  if (active) {
    const auto& t = *fresh(tab);
    const int base = p0 + N2 * p1;
#pragma unroll
    for (int j = 0; j < N; ++j) tmp[j] = UX[off + base + N * j];
    dmv<N, T>(t.M, tmp, out);
#pragma unroll
    for (int j = 0; j < N; ++j) B2[off + base + N * j] += out[j];
  }
  __syncthreads();
  // Z again: b = Mz S + c_z R
  if (active) {
    const auto& t = *fresh(tab);
    const int base = p0 + N * p1;
#pragma unroll
    for (int c = 0; c < N; ++c) tmp[c] = B2[off + base + N2 * c];
    dmv<N, T>(t.M, tmp, out);
    T* g = b + (size_t)e * N3 + base;
#pragma unroll
    for (int c = 0; c < N; ++c) g[N2 * c] = out[c] + B1[off + base + N2 * c];
  }
}

template <int N, typename T>
static hipError_t launch_div_n(const DivPlan& P, const void* u, void* b, hipStream_t s) {
  using C = DivCfg<N>;
  DivTab<N, T> t;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      t.M[i][j] = (T)P.Mref[i * N + j];
      t.B[i][j] = (T)P.Bown[i * N + j];
    }
  DivScal<T> sc;
  for (int d = 0; d < 3; ++d) sc.c[d] = (T)P.c[d];
  hipError_t err;
  const DivTab<N, T>* dt = device_table_of("divergence", t, &err);
  if (!dt) return err;
  const int grid = (P.mesh.n_el + C::E - 1) / C::E;
  hipLaunchKernelGGL((divergence_kernel<N, T>), dim3(grid), dim3(C::THREADS), 0, s, (const T*)u, (T*)b,
                     P.mesh, dt, sc);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_div_t(const DivPlan& P, const void* u, void* b, hipStream_t s) {
  switch (P.k) {
    case 1: return launch_div_n<2, T>(P, u, b, s);
    case 2: return launch_div_n<3, T>(P, u, b, s);
    case 3: return launch_div_n<4, T>(P, u, b, s);
    case 4: return launch_div_n<5, T>(P, u, b, s);
    case 5: return launch_div_n<6, T>(P, u, b, s);
    case 6: return launch_div_n<7, T>(P, u, b, s);
    case 7: return launch_div_n<8, T>(P, u, b, s);
    case 8: return launch_div_n<9, T>(P, u, b, s);
    case 9: return launch_div_n<10, T>(P, u, b, s);
    case 10: return launch_div_n<11, T>(P, u, b, s);
    case 11: return launch_div_n<12, T>(P, u, b, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_divergence(const DivPlan& P, bool f32, const void* u, void* b, hipStream_t s) {
  return f32 ? launch_div_t<float>(P, u, b, s) : launch_div_t<double>(P, u, b, s);
}

}  // namespace dgmf
