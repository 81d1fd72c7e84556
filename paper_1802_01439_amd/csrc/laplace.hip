// SIPG negative Laplacian (Sec. 3.2, weak form of l_h) by sum factorisation
// on periodic Cartesian meshes, FP64 and FP32, degrees 1..11.
//
// Method.  On an affine, axis-aligned cell the Gauss sums of the SIPG form
// factor by direction (sum factorisation over the tensor-product basis and
// quadrature, Sec. 3.4).  Collapsing "interpolate to Gauss points, weight,
// integrate back" into 1D matrices on [0,1] gives
//
//   A = c_x Kx(x)My(x)Mz + c_y Mx(x)Ky(x)Mz + c_z Mx(x)My(x)Kz,
//   c_d = scale * (h_x h_y h_z) / h_d^2,
//
// with M the 1D mass matrix and K the 1D SIPG operator (cell stiffness plus
// the own-side face terms of both ends, penalty sigma = penalty_factor
// (k+1)^2).  K couples each pencil to its neighbour pencils only through
// their end value and end slope (LGL nodes include the end points).  Since
// the three terms share the mass factors,
//
//   A = (Mx(x)My(x)Mz) (c_x Lx + c_y Ly + c_z Lz),   L = M^-1 K,
//
// which the kernel evaluates as three L sweeps (one per direction, with the
// neighbour couplings turned into dense vectors M^-1 e by the host) followed
// by three M sweeps: six 1D sweeps per element instead of the eight of the
// unfactored form.
//
// GPU mapping.  One workgroup per batch of E = floor(256/n^2) consecutive
// elements (n^2 threads per element), batches walked strip by strip, XCD by
// XCD.  Each thread first issues all of its global loads (its own z-column
// and the six neighbour pencils, reduced at once to end values and slopes);
// then phase Z (Lz, own column in registers), Y (Ly), X (Lx then Mx), Y (My),
// Z (Mz, written once) hand pencils over through two LDS buffers (4 barriers).
// The 1D tables are a small device table read through the scalar unit.  No
// atomics.
#include <algorithm>

#include "api_internal.h"
#include "common.h"
#include "ops.h"

namespace dgmf {

template <int N, typename T>
struct LapTab {
  T M[N][N];      // 1D mass matrix on [0,1]
  T L[3][N][N];   // c_d M^-1 Kown, per direction d
  T aR[3][N];     // c_d M^-1 (coefficient of the right neighbour's end value)
  T aL[3][N];     // c_d M^-1 (coefficient of the left neighbour's end value)
  T eR[3][N];     // c_d M^-1 (coefficient of the right neighbour's half slope)
  T eL[3][N];     // c_d M^-1 (coefficient of the left neighbour's half slope)
  T hd0[N];       // 1/2 l_b'(0)
  T hd1[N];       // 1/2 l_b'(1)
};

// LDS layout of one element's n^3 block: node (a,b,c) at a + PX*b + PY*c,
// elements ES apart.  The paddings (per n) keep the three pencil access
// patterns of a wavefront free of bank conflicts for 32 and 64 banks.
template <int N>
struct LapPad {
  static constexpr int px = (N == 6 || N == 8 || N == 12) ? 1 : 0;
  static constexpr int py = (N == 2) ? 1 : (N == 4 ? 3 : (N == 10 ? 1 : 0));
  static constexpr int pe = (N == 2) ? 2 : (N == 4 ? 4 : 0);
};

template <int N>
struct LapCfg {
  static constexpr int N2 = N * N, N3 = N * N * N;
  static constexpr int E = (256 / N2) > 0 ? 256 / N2 : 1;
  static constexpr int THREADS = E * N2;
  static constexpr int PX = N + LapPad<N>::px;
  static constexpr int PY = PX * N + LapPad<N>::py;
  static constexpr int ES = PY * N + LapPad<N>::pe;
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

// Face data of the two neighbours of one pencil: end values and half slopes
// at the shared faces (the only neighbour quantities the SIPG form needs).
template <typename T>
struct NbrFace {
  T vL, gL, vR, gR;
};

template <int N, typename T>
__device__ __forceinline__ NbrFace<T> nbr_face(const LapTab<N, T>& t, const T* uL, const T* uR) {
  NbrFace<T> f;
  T gR = 0, gL = 0;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    gR = fmadd(t.hd0[j], uR[j], gR);
    gL = fmadd(t.hd1[j], uL[j], gL);
  }
  f.vL = uL[N - 1];
  f.gL = gL;
  f.vR = uR[0];
  f.gR = gR;
  return f;
}

// y (+)= c_d M^-1 (1D SIPG of one pencil in direction d, with the couplings
// to the neighbours' end values and half slopes).
template <int N, typename T, bool ACC>
__device__ __forceinline__ void l_pencil(const LapTab<N, T>& t, int d, const T* u, const NbrFace<T>& f, T* y) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T s = ACC ? fmadd(t.L[d][i][0], u[0], y[i]) : t.L[d][i][0] * u[0];
#pragma unroll
    for (int j = 1; j < N; ++j) s = fmadd(t.L[d][i][j], u[j], s);
    s = fmadd(t.aR[d][i], f.vR, s);
    s = fmadd(t.aL[d][i], f.vL, s);
    s = fmadd(t.eR[d][i], f.gR, s);
    s = fmadd(t.eL[d][i], f.gL, s);
    y[i] = s;
  }
}

// Position of this thread's element in logical batch L of the traversal.
struct BatchPos {
  int ne;       // elements in the batch
  int ex, ey, ez, comp;
  int eg;       // element index including the component offset
  bool active;  // this thread's element exists
};

__device__ __forceinline__ BatchPos batch_pos(int L, const Traversal& tv, const MeshArgs& mesh, int E,
                                              int le) {
  BatchPos b;
  int jrun, pz;
  strip_order(L, tv, jrun, pz);
  const int nxy = mesh.nx * mesh.ny;
  b.comp = pz / mesh.nz;   // uniform: scalar unit
  b.ez = pz - b.comp * mesh.nz;
  b.ne = min(E, nxy - jrun * E);
  b.active = le < b.ne;
  // (ex, ey): start of the run (uniform division) plus le, wrapped row by row
  const int ey0 = (jrun * E) / mesh.nx, ex0 = jrun * E - ey0 * mesh.nx;
  int ex = ex0 + le, ey = ey0;
  while (ex >= mesh.nx) {
    ex -= mesh.nx;
    ++ey;
  }
  b.ex = ex;
  b.ey = ey;
  b.eg = b.comp * mesh.n_el + b.ez * nxy + ex + mesh.nx * ey;
  return b;
}

// The seven pencils one thread reads from global memory for one batch.
template <int N, typename T>
struct Pencils {
  T own[N];          // own z-column (a,b) = (p0,p1)
  T zl[N], zr[N];    // z-neighbours, same column
  T yl[N], yr[N];    // y-neighbours, y-pencil (a,c) = (p0,p1)
  T xl[N], xr[N];    // x-neighbours, x-pencil (b,c) = (p0,p1)
};

template <int N, typename T>
__device__ __forceinline__ void load_pencils(const T* __restrict__ src, const MeshArgs& mesh,
                                             const BatchPos& b, int p0, int p1, Pencils<N, T>& P) {
  constexpr int N2 = N * N, N3 = N * N * N;
  const T* csrc = src + (size_t)b.comp * mesh.n_el * N3;
  const int e = b.eg - b.comp * mesh.n_el;
  const T* own = csrc + (size_t)e * N3 + p0 + N * p1;
  const T* zl = csrc + (size_t)neighbor(mesh, b.ex, b.ey, b.ez, 2, 0) * N3 + p0 + N * p1;
  const T* zr = csrc + (size_t)neighbor(mesh, b.ex, b.ey, b.ez, 2, 1) * N3 + p0 + N * p1;
  const T* yl = csrc + (size_t)neighbor(mesh, b.ex, b.ey, b.ez, 1, 0) * N3 + p0 + N2 * p1;
  const T* yr = csrc + (size_t)neighbor(mesh, b.ex, b.ey, b.ez, 1, 1) * N3 + p0 + N2 * p1;
  const T* xl = csrc + (size_t)neighbor(mesh, b.ex, b.ey, b.ez, 0, 0) * N3 + N * p0 + N2 * p1;
  const T* xr = csrc + (size_t)neighbor(mesh, b.ex, b.ey, b.ez, 0, 1) * N3 + N * p0 + N2 * p1;
#pragma unroll
  for (int c = 0; c < N; ++c) {
    P.own[c] = own[N2 * c];
    P.zl[c] = zl[N2 * c];
    P.zr[c] = zr[N2 * c];
    P.yl[c] = yl[N * c];
    P.yr[c] = yr[N * c];
    P.xl[c] = xl[c];
    P.xr[c] = xr[c];
  }
}

// One batch: the five phases of the factorised operator.  Starts and ends
// with LDS free (the caller puts a barrier between batches).
// What one thread keeps of a batch's loads: its own z-column and the end
// values / half slopes of the six neighbour pencils.
template <int N, typename T>
struct BatchIn {
  T own[N];
  NbrFace<T> fx, fy, fz;
};

template <int N, typename T>
__device__ __forceinline__ void reduce_pencils(const LapTab<N, T>& t, const Pencils<N, T>& P, BatchIn<N, T>& I) {
#pragma unroll
  for (int c = 0; c < N; ++c) I.own[c] = P.own[c];
  I.fz = nbr_face<N, T>(t, P.zl, P.zr);
  I.fy = nbr_face<N, T>(t, P.yl, P.yr);
  I.fx = nbr_face<N, T>(t, P.xl, P.xr);
}

template <int N, typename T>
__device__ __forceinline__ void laplace_batch(const LapTab<N, T>& t, const BatchPos& b, const BatchIn<N, T>& I,
                                              T* __restrict__ dst, T* Ue, T* Ve, int p0, int p1) {
  using C = LapCfg<N>;
  constexpr int N2 = C::N2, N3 = C::N3, PX = C::PX, PY = C::PY;
  T in[N], v[N], out[N];
  // Z: V = c_z Lz u (own column in registers)
  if (b.active) {
    l_pencil<N, T, false>(t, 2, I.own, I.fz, v);
    const int base = p0 + PX * p1;
#pragma unroll
    for (int c = 0; c < N; ++c) {
      Ue[base + PY * c] = I.own[c];
      Ve[base + PY * c] = v[c];
    }
  }
  __syncthreads();
  // Y: pencil (a,c) = (p0,p1): V += c_y Ly u
  if (b.active) {
    const int base = p0 + PY * p1;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      in[j] = Ue[base + PX * j];
      v[j] = Ve[base + PX * j];
    }
    l_pencil<N, T, true>(t, 1, in, I.fy, v);
#pragma unroll
    for (int j = 0; j < N; ++j) Ve[base + PX * j] = v[j];
  }
  __syncthreads();
  // X: pencil (b,c) = (p0,p1): V += c_x Lx u, then V <- Mx V
  if (b.active) {
    const int base = PX * p0 + PY * p1;
#pragma unroll
    for (int a = 0; a < N; ++a) {
      in[a] = Ue[base + a];
      v[a] = Ve[base + a];
    }
    l_pencil<N, T, true>(t, 0, in, I.fx, v);
    matvec<N, T>(t.M, v, out);
#pragma unroll
    for (int a = 0; a < N; ++a) Ve[base + a] = out[a];
  }
  __syncthreads();
  // Y again: V <- My V
  if (b.active) {
    const int base = p0 + PY * p1;
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] = Ve[base + PX * j];
    matvec<N, T>(t.M, v, out);
#pragma unroll
    for (int j = 0; j < N; ++j) Ve[base + PX * j] = out[j];
  }
  __syncthreads();
  // Z again: y = Mz V, written once
  if (b.active) {
    const int base = p0 + PX * p1;
#pragma unroll
    for (int c = 0; c < N; ++c) v[c] = Ve[base + PY * c];
    matvec<N, T>(t.M, v, out);
    T* g = dst + (size_t)b.eg * N3 + p0 + N * p1;
#pragma unroll
    for (int c = 0; c < N; ++c) g[N2 * c] = out[c];
  }
}

// One workgroup per batch, batches in traversal order (XCD by XCD).  All
// global loads of the batch are issued first and reduced to the own column
// plus the neighbours' end values and slopes; then the five phases run.
template <int N, typename T>
__global__ void __launch_bounds__(LapCfg<N>::THREADS)
laplace_kernel(const T* __restrict__ src, T* __restrict__ dst, MeshArgs mesh, Traversal tv,
               const LapTab<N, T>* __restrict__ tab) {
  const LapTab<N, T>& t = *tab;
  using C = LapCfg<N>;
  constexpr int N2 = C::N2, E = C::E, ES = C::ES;
  __shared__ T U[E * ES];
  __shared__ T V[E * ES];

  const int tid = threadIdx.x;
  const int le = tid / N2, p = tid - le * N2;
  const int p0 = p % N, p1 = p / N;
  const BatchPos b = batch_pos(xcd_remap(blockIdx.x, gridDim.x), tv, mesh, E, le);
  BatchIn<N, T> I;
  if (b.active) {
    Pencils<N, T> P;
    load_pencils<N, T>(src, mesh, b, p0, p1, P);
    reduce_pencils<N, T>(t, P, I);
  }
  laplace_batch<N, T>(t, b, I, dst, U + le * ES, V + le * ES, p0, p1);
}

template <int N, typename T>
static hipError_t launch_laplace_n(const LaplacePlan& P, const void* src, void* dst,
                                   hipStream_t stream) {
  using C = LapCfg<N>;
  LapTab<N, T> t;
  for (int i = 0; i < N; ++i) {
    for (int j = 0; j < N; ++j) {
      t.M[i][j] = (T)P.Mref[i * N + j];
      for (int d = 0; d < 3; ++d) t.L[d][i][j] = (T)(P.c[d] * P.Lown[i * N + j]);
    }
    for (int d = 0; d < 3; ++d) {
      t.aR[d][i] = (T)(P.c[d] * P.cR[i]);
      t.aL[d][i] = (T)(P.c[d] * P.cL[i]);
      t.eR[d][i] = (T)(P.c[d] * P.gR[i]);
      t.eL[d][i] = (T)(P.c[d] * P.gL[i]);
    }
    t.hd0[i] = (T)(0.5 * P.D[i]);
    t.hd1[i] = (T)(0.5 * P.D[(N - 1) * N + i]);
  }
  hipError_t err;
  const LapTab<N, T>* dt = device_table_of("laplace", t, &err);
  if (!dt) return err;
  Traversal tv;
  tv.PB = (P.mesh.nx * P.mesh.ny + C::E - 1) / C::E;
  tv.PZ = P.n_comp * P.mesh.nz;
  tv.S = std::max(1, std::min(tv.PB, (16 * P.mesh.nx + C::E / 2) / C::E));
  const int grid = tv.PB * tv.PZ;
  hipLaunchKernelGGL((laplace_kernel<N, T>), dim3(grid), dim3(C::THREADS), 0, stream,
                     (const T*)src, (T*)dst, P.mesh, tv, dt);
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
