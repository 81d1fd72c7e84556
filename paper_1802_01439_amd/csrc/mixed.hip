// Kernels of the dual-splitting time step (Sec. 3.1) beyond the operators
// of the other files, FP64 (divergence and gradient also FP32):
//
// * divergence d_h(q, u) and gradient g_h(v, p) between the degree-k
//   velocity (NU = k+1 LGL nodes per direction) and the degree-(k-1)
//   pressure (NP = k nodes), the mixed-order pair of Sec. 3.2, central
//   fluxes, k+1 Gauss points (exact).  On an axis-aligned affine cell each
//   term factors by direction:
//     b   = c_x Bx(x)My(x)Mz u_x + c_y Mx(x)By(x)Mz u_y + c_z Mx(x)My(x)Bz u_z,
//     y_j = c_j (G along j)(x)(M^T along the other two) p,   c_d = vol/h_d,
//   with rectangular 1D tables on [0,1] (rows: test functions): the mass
//   M[i][a] = (l^p_i, l^u_a) (NP x NU), B[i][a] = -(l^p_i', l^u_a) plus the
//   own-side central-flux ends 1/2 l^p_i(1) l^u_a(1) - 1/2 l^p_i(0) l^u_a(0),
//   and G = -B^T (exact integration by parts); the neighbour couplings are
//   1/2 of the neighbour's end value at the end test functions, applied in
//   the sweep along the face normal, before the mass sweeps of the other
//   directions.  Five sweep phases per element, pencils through LDS, every
//   output written once, no atomics.
// * per-element penalty parameters of the projection step from the
//   extrapolated velocity (Sec. 3.2): tau_D = zeta_D |u|_e h/(k+1) dt,
//   tau_C = zeta_C |u|_e dt, |u|_e the volume average of the velocity
//   magnitude (k+1 Gauss points), h = vol^(1/3);
// * the Taylor-Green diagnostics (Sec. 4.2): per-workgroup partial sums of
//   int u.u and int grad u : grad u (k+1 Gauss points, exact), reduced in a
//   fixed order;
// * y = a0 x0 + a1 x1 + a2 x2 (vector combinations of the step).
#include <cmath>
#include <vector>

#include "api_internal.h"
#include "common.h"
#include "ops.h"

namespace dgmf {

namespace {

// element index, batch layout: E elements per workgroup, THREADS = E NU^2
template <int NU>
struct MixCfg {
  static constexpr int U2 = NU * NU, U3 = NU * NU * NU;
  static constexpr int E = 256 / U2 > 0 ? 256 / U2 : 1;
  static constexpr int THREADS = E * U2;
};

template <int NU, int NP, typename T>
struct MixTab {
  T M[NP][NU];   // (l^p_i, l^u_a)
  T B[NP][NU];   // divergence, own element
  T MT[NU][NP];  // M^T
  T G[NU][NP];   // gradient, own element (= -B^T)
};

// out[r] = sum_c A[r][c] in[c]
template <int R, int C, typename T, typename Mat>
__device__ __forceinline__ void rmv(const Mat& A, const T* in, T* out) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
    T s = A[r][0] * in[0];
#pragma unroll
    for (int c = 1; c < C; ++c) s = fmadd(A[r][c], in[c], s);
    out[r] = s;
  }
}

// position of element e
struct ElPos {
  int ex, ey, ez;
};
__device__ __forceinline__ ElPos el_pos(const MeshArgs& m, int e) {
  ElPos p;
  p.ex = e % m.nx;
  p.ey = (e / m.nx) % m.ny;
  p.ez = e / (m.nx * m.ny);
  return p;
}

// LDS arrays of one element: [i0 + NU (i1 + NU i2)] with NU strides whatever
// the extents (a sweep along a direction changes its extent in place).
template <int NU>
__device__ __forceinline__ int ix(int i0, int i1, int i2) {
  return i0 + NU * (i1 + NU * i2);
}

// b = D u: u [3][N_el][NU^3] -> b [N_el][NP^3], times `scale`
template <int NU, int NP, typename T>
__global__ void __launch_bounds__(MixCfg<NU>::THREADS)
mixed_divergence_kernel(const T* __restrict__ u, T* __restrict__ b, MeshArgs mesh,
                        const MixTab<NU, NP, T>* __restrict__ tab, T cx, T cy, T cz) {
  using C = MixCfg<NU>;
  constexpr int U2 = C::U2, U3 = C::U3, E = C::E, P3 = NP * NP * NP;
  __shared__ T UX[E * U3];
  __shared__ T UY[E * U3];
  __shared__ T B1[E * U3];
  __shared__ T B2[E * U3];
  const int tid = threadIdx.x;
  const int e0 = xcd_remap(blockIdx.x, gridDim.x) * E;
  const int le = tid / U2, p = tid - le * U2;
  const int p0 = p % NU, p1 = p / NU;
  const bool active = e0 + le < mesh.n_el;
  const int e = e0 + le;
  const size_t cs = (size_t)mesh.n_el * U3;
  const ElPos ep = active ? el_pos(mesh, e) : ElPos{0, 0, 0};
  T* ux = UX + le * U3;
  T* uy = UY + le * U3;
  T* b1 = B1 + le * U3;
  T* b2 = B2 + le * U3;
  T in[NU], out[NU];

  // Z: raw u_x, u_y columns to LDS; R = Bz u_z (+ z neighbours) -> b1[a, b, k]
  if (active) {
    const auto& t = *fresh(tab);
    const int a = p0, bb = p1;
    const T* g = u + (size_t)e * U3 + ix<NU>(a, bb, 0);
#pragma unroll
    for (int c = 0; c < NU; ++c) {
      ux[ix<NU>(a, bb, c)] = g[U2 * c];
      uy[ix<NU>(a, bb, c)] = g[cs + U2 * c];
      in[c] = g[2 * cs + U2 * c];
    }
    const T vl = u[2 * cs + (size_t)neighbor(mesh, ep.ex, ep.ey, ep.ez, 2, 0) * U3 + ix<NU>(a, bb, NU - 1)];
    const T vr = u[2 * cs + (size_t)neighbor(mesh, ep.ex, ep.ey, ep.ez, 2, 1) * U3 + ix<NU>(a, bb, 0)];
    rmv<NP, NU, T>(t.B, in, out);
    out[NP - 1] += T(0.5) * vr;
    out[0] -= T(0.5) * vl;
#pragma unroll
    for (int k = 0; k < NP; ++k) b1[ix<NU>(a, bb, k)] = out[k];
  }
  __syncthreads();
  // Y: Q = By u_y (+ y neighbours) -> b2[a, j, c]; R <- My R -> b1[a, j, k]
  if (active) {
    const auto& t = *fresh(tab);
    const int a = p0, c = p1;
#pragma unroll
    for (int bb = 0; bb < NU; ++bb) in[bb] = uy[ix<NU>(a, bb, c)];
    const T vl = u[cs + (size_t)neighbor(mesh, ep.ex, ep.ey, ep.ez, 1, 0) * U3 + ix<NU>(a, NU - 1, c)];
    const T vr = u[cs + (size_t)neighbor(mesh, ep.ex, ep.ey, ep.ez, 1, 1) * U3 + ix<NU>(a, 0, c)];
    rmv<NP, NU, T>(t.B, in, out);
    out[NP - 1] += T(0.5) * vr;
    out[0] -= T(0.5) * vl;
#pragma unroll
    for (int j = 0; j < NP; ++j) b2[ix<NU>(a, j, c)] = out[j];
    if (c < NP) {   // pencil (a, k = c) of R
#pragma unroll
      for (int bb = 0; bb < NU; ++bb) in[bb] = b1[ix<NU>(a, bb, c)];
      rmv<NP, NU, T>(t.M, in, out);
#pragma unroll
      for (int j = 0; j < NP; ++j) b1[ix<NU>(a, j, c)] = out[j];
    }
  }
  __syncthreads();
  // X: ux <- c_x Bx u_x (+ x neighbours) [i, b, c]; b2 <- c_y Mx Q [i, j, c];
  // b1 <- c_z Mx R [i, j, k]
  if (active) {
    const auto& t = *fresh(tab);
    {
      const int bb = p0, c = p1;
#pragma unroll
      for (int a = 0; a < NU; ++a) in[a] = ux[ix<NU>(a, bb, c)];
      const T vl = u[(size_t)neighbor(mesh, ep.ex, ep.ey, ep.ez, 0, 0) * U3 + ix<NU>(NU - 1, bb, c)];
      const T vr = u[(size_t)neighbor(mesh, ep.ex, ep.ey, ep.ez, 0, 1) * U3 + ix<NU>(0, bb, c)];
      rmv<NP, NU, T>(t.B, in, out);
      out[NP - 1] += T(0.5) * vr;
      out[0] -= T(0.5) * vl;
#pragma unroll
      for (int i = 0; i < NP; ++i) ux[ix<NU>(i, bb, c)] = cx * out[i];
    }
    if (p0 < NP) {   // pencil (j = p0, c = p1) of Q
      const int j = p0, c = p1;
#pragma unroll
      for (int a = 0; a < NU; ++a) in[a] = b2[ix<NU>(a, j, c)];
      rmv<NP, NU, T>(t.M, in, out);
#pragma unroll
      for (int i = 0; i < NP; ++i) b2[ix<NU>(i, j, c)] = cy * out[i];
    }
    if (p0 < NP && p1 < NP) {   // pencil (j, k) of R
      const int j = p0, k = p1;
#pragma unroll
      for (int a = 0; a < NU; ++a) in[a] = b1[ix<NU>(a, j, k)];
      rmv<NP, NU, T>(t.M, in, out);
#pragma unroll
      for (int i = 0; i < NP; ++i) b1[ix<NU>(i, j, k)] = cz * out[i];
    }
  }
  __syncthreads();
  // Y again: b2[i, j, c] += My (c_x P)[i, j, c]
  if (active && p0 < NP) {
    const auto& t = *fresh(tab);
    const int i = p0, c = p1;
#pragma unroll
    for (int bb = 0; bb < NU; ++bb) in[bb] = ux[ix<NU>(i, bb, c)];
    rmv<NP, NU, T>(t.M, in, out);
#pragma unroll
    for (int j = 0; j < NP; ++j) b2[ix<NU>(i, j, c)] += out[j];
  }
  __syncthreads();
  // Z again: b = Mz S + c_z R, written once
  if (active && p0 < NP && p1 < NP) {
    const auto& t = *fresh(tab);
    const int i = p0, j = p1;
#pragma unroll
    for (int c = 0; c < NU; ++c) in[c] = b2[ix<NU>(i, j, c)];
    rmv<NP, NU, T>(t.M, in, out);
    T* g = b + (size_t)e * P3 + i + NP * j;
#pragma unroll
    for (int k = 0; k < NP; ++k) g[NP * NP * k] = out[k] + b1[ix<NU>(i, j, k)];
  }
}

// y = G p: p [N_el][NP^3] -> y [3][N_el][NU^3]
template <int NU, int NP, typename T>
__global__ void __launch_bounds__(MixCfg<NU>::THREADS)
mixed_gradient_kernel(const T* __restrict__ pr, T* __restrict__ y, MeshArgs mesh,
                      const MixTab<NU, NP, T>* __restrict__ tab, T cx, T cy, T cz) {
  using C = MixCfg<NU>;
  constexpr int U2 = C::U2, U3 = C::U3, E = C::E, P2 = NP * NP, P3 = NP * NP * NP;
  __shared__ T P0[E * U3];
  __shared__ T A1[E * U3];
  __shared__ T A2[E * U3];
  const int tid = threadIdx.x;
  const int e0 = xcd_remap(blockIdx.x, gridDim.x) * E;
  const int le = tid / U2, p = tid - le * U2;
  const int p0 = p % NU, p1 = p / NU;
  const bool active = e0 + le < mesh.n_el;
  const int e = e0 + le;
  const size_t cs = (size_t)mesh.n_el * U3;
  const ElPos ep = active ? el_pos(mesh, e) : ElPos{0, 0, 0};
  T* q0 = P0 + le * U3;
  T* a1 = A1 + le * U3;
  T* a2 = A2 + le * U3;
  T in[NU], out[NU];
  auto pidx = [](int a, int b, int c) { return a + NP * (b + NP * c); };

  // Z: raw p columns to LDS; Tz = Gz p (+ z neighbours) -> a1[a, b, k]
  if (active && p0 < NP && p1 < NP) {
    const auto& t = *fresh(tab);
    const int a = p0, bb = p1;
    const T* g = pr + (size_t)e * P3 + pidx(a, bb, 0);
#pragma unroll
    for (int c = 0; c < NP; ++c) {
      in[c] = g[P2 * c];
      q0[ix<NU>(a, bb, c)] = in[c];
    }
    const T vl = pr[(size_t)neighbor(mesh, ep.ex, ep.ey, ep.ez, 2, 0) * P3 + pidx(a, bb, NP - 1)];
    const T vr = pr[(size_t)neighbor(mesh, ep.ex, ep.ey, ep.ez, 2, 1) * P3 + pidx(a, bb, 0)];
    rmv<NU, NP, T>(t.G, in, out);
    out[NU - 1] += T(0.5) * vr;
    out[0] -= T(0.5) * vl;
#pragma unroll
    for (int k = 0; k < NU; ++k) a1[ix<NU>(a, bb, k)] = out[k];
  }
  __syncthreads();
  // Y: Ty = Gy p (+ y neighbours) -> a2[a, j, c]; a1 <- My^T a1 [a, j, k]
  if (active && p0 < NP) {
    const auto& t = *fresh(tab);
    const int a = p0;
    if (p1 < NP) {   // pencil (a, c) of p
      const int c = p1;
#pragma unroll
      for (int bb = 0; bb < NP; ++bb) in[bb] = q0[ix<NU>(a, bb, c)];
      const T vl = pr[(size_t)neighbor(mesh, ep.ex, ep.ey, ep.ez, 1, 0) * P3 + pidx(a, NP - 1, c)];
      const T vr = pr[(size_t)neighbor(mesh, ep.ex, ep.ey, ep.ez, 1, 1) * P3 + pidx(a, 0, c)];
      rmv<NU, NP, T>(t.G, in, out);
      out[NU - 1] += T(0.5) * vr;
      out[0] -= T(0.5) * vl;
#pragma unroll
      for (int j = 0; j < NU; ++j) a2[ix<NU>(a, j, c)] = out[j];
    }
    {   // pencil (a, k = p1) of Tz
      const int k = p1;
#pragma unroll
      for (int bb = 0; bb < NP; ++bb) in[bb] = a1[ix<NU>(a, bb, k)];
      rmv<NU, NP, T>(t.MT, in, out);
#pragma unroll
      for (int j = 0; j < NU; ++j) a1[ix<NU>(a, j, k)] = out[j];
    }
  }
  __syncthreads();
  // X: q0 <- c_x Gx p (+ x neighbours) [i, b, c]; a2 <- c_y Mx^T a2 [i, j, c];
  // a1 <- c_z Mx^T a1 [i, j, k]
  if (active) {
    const auto& t = *fresh(tab);
    if (p0 < NP && p1 < NP) {   // pencil (b, c) of p
      const int bb = p0, c = p1;
#pragma unroll
      for (int a = 0; a < NP; ++a) in[a] = q0[ix<NU>(a, bb, c)];
      const T vl = pr[(size_t)neighbor(mesh, ep.ex, ep.ey, ep.ez, 0, 0) * P3 + pidx(NP - 1, bb, c)];
      const T vr = pr[(size_t)neighbor(mesh, ep.ex, ep.ey, ep.ez, 0, 1) * P3 + pidx(0, bb, c)];
      rmv<NU, NP, T>(t.G, in, out);
      out[NU - 1] += T(0.5) * vr;
      out[0] -= T(0.5) * vl;
#pragma unroll
      for (int i = 0; i < NU; ++i) q0[ix<NU>(i, bb, c)] = cx * out[i];
    }
    if (p1 < NP) {   // pencil (j = p0, c = p1) of Ty
      const int j = p0, c = p1;
#pragma unroll
      for (int a = 0; a < NP; ++a) in[a] = a2[ix<NU>(a, j, c)];
      rmv<NU, NP, T>(t.MT, in, out);
#pragma unroll
      for (int i = 0; i < NU; ++i) a2[ix<NU>(i, j, c)] = cy * out[i];
    }
    {   // pencil (j, k) of Tz
      const int j = p0, k = p1;
#pragma unroll
      for (int a = 0; a < NP; ++a) in[a] = a1[ix<NU>(a, j, k)];
      rmv<NU, NP, T>(t.MT, in, out);
#pragma unroll
      for (int i = 0; i < NU; ++i) a1[ix<NU>(i, j, k)] = cz * out[i];
    }
  }
  __syncthreads();
  // Y again: q0[i, j, c] = My^T (c_x Gx p)[i, j, c]
  if (active && p1 < NP) {
    const auto& t = *fresh(tab);
    const int i = p0, c = p1;
#pragma unroll
    for (int bb = 0; bb < NP; ++bb) in[bb] = q0[ix<NU>(i, bb, c)];
    rmv<NU, NP, T>(t.MT, in, out);
#pragma unroll
    for (int j = 0; j < NU; ++j) q0[ix<NU>(i, j, c)] = out[j];
  }
  __syncthreads();
  // Z again: y_x = Mz^T q0, y_y = Mz^T a2, y_z = a1; written once
  if (active) {
    const auto& t = *fresh(tab);
    const int i = p0, j = p1;
    T* g = y + (size_t)e * U3 + i + NU * j;
#pragma unroll
    for (int c = 0; c < NP; ++c) in[c] = q0[ix<NU>(i, j, c)];
    rmv<NU, NP, T>(t.MT, in, out);
#pragma unroll
    for (int k = 0; k < NU; ++k) g[U2 * k] = out[k];
#pragma unroll
    for (int c = 0; c < NP; ++c) in[c] = a2[ix<NU>(i, j, c)];
    rmv<NU, NP, T>(t.MT, in, out);
#pragma unroll
    for (int k = 0; k < NU; ++k) g[cs + U2 * k] = out[k];
#pragma unroll
    for (int k = 0; k < NU; ++k) g[2 * cs + U2 * k] = a1[ix<NU>(i, j, k)];
  }
}

template <int N>
struct GaussTab {
  double S[N][N];   // l_a(z_q): LGL nodes -> Gauss points
  double G[N][N];   // l_a'(z_q)
  double w[N];      // Gauss weights on [0,1]
};

// The tables a Gauss-point kernel reads: from N = 6 on (72 doubles or more)
// a copy in LDS, which all lanes read entry by entry at once (a broadcast),
// so that they stay out of the scalar registers (at k = 7 the diagnostics
// ran 2.6x faster, at k = 5 25 %); below, the device table itself, which the
// scalar registers hold (the LDS copy was 5 % slower at k = 4 and 36 % at
// k = 3).  Every thread of the workgroup calls it; it synchronises.
template <int N>
__device__ __forceinline__ const GaussTab<N>& gauss_tables(const GaussTab<N>* __restrict__ tab, GaussTab<N>& tl) {
  if constexpr (N >= 6) {
    for (int i = threadIdx.x; i < (int)(sizeof(GaussTab<N>) / sizeof(double)); i += blockDim.x)
      reinterpret_cast<double*>(&tl)[i] = reinterpret_cast<const double*>(tab)[i];
    __syncthreads();
    return tl;
  } else {
    return *tab;
  }
}

// Values of the three components at the N^3 Gauss points by sum
// factorisation (one element per workgroup, thread (p0, p1) < N); work: 3 N^3
// doubles of LDS.  f(q1, q2, q3, v) is called once per point by the thread
// owning the (q2, q3) pencil, v[j] = u_j there.
template <int N, typename F>
__device__ __forceinline__ void gauss_values3(const GaussTab<N>& t, const double* __restrict__ u, size_t cs,
                                              size_t eoff, int p0, int p1, double* work, F&& f) {
  constexpr int N2 = N * N, N3 = N2 * N;
  double in[N], out[N];
  for (int j = 0; j < 3; ++j) {   // z: column (a, b)
#pragma unroll
    for (int c = 0; c < N; ++c) in[c] = u[j * cs + eoff + p0 + N * p1 + N2 * c];
    rmv<N, N, double>(t.S, in, out);
#pragma unroll
    for (int q = 0; q < N; ++q) work[j * N3 + p0 + N * (p1 + N * q)] = out[q];
  }
  __syncthreads();
  for (int j = 0; j < 3; ++j) {   // y: pencil (a, q3), in place
#pragma unroll
    for (int b = 0; b < N; ++b) in[b] = work[j * N3 + p0 + N * (b + N * p1)];
    rmv<N, N, double>(t.S, in, out);
#pragma unroll
    for (int q = 0; q < N; ++q) work[j * N3 + p0 + N * (q + N * p1)] = out[q];
  }
  __syncthreads();
  double a[3][N];   // x: pencil (q2, q3)
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int i = 0; i < N; ++i) a[j][i] = work[j * N3 + i + N * (p0 + N * p1)];
#pragma unroll
  for (int q = 0; q < N; ++q) {
    double v[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double s = 0;
#pragma unroll
      for (int i = 0; i < N; ++i) s = fma(t.S[q][i], a[j][i], s);
      v[j] = s;
    }
    f(q, p0, p1, v);
  }
}

// Value and reference gradient of component u_j (pointer to its element) at
// the N^3 Gauss points; work: 3 N^3 doubles.  f(q1, q2, q3, v, gx, gy, gz).
template <int N, typename F>
__device__ __forceinline__ void gauss_grad1(const GaussTab<N>& t, const double* __restrict__ ue, int p0, int p1,
                                            double* work, F&& f) {
  constexpr int N2 = N * N, N3 = N2 * N;
  double* W0 = work;            // S_z u, then S_y S_z u
  double* W1 = work + N3;       // G_z u, then S_y G_z u
  double* W2 = work + 2 * N3;   // G_y S_z u
  double in[N], o1[N], o2[N];
#pragma unroll
  for (int c = 0; c < N; ++c) in[c] = ue[p0 + N * p1 + N2 * c];
  rmv<N, N, double>(t.S, in, o1);
  rmv<N, N, double>(t.G, in, o2);
#pragma unroll
  for (int q = 0; q < N; ++q) {
    W0[p0 + N * (p1 + N * q)] = o1[q];
    W1[p0 + N * (p1 + N * q)] = o2[q];
  }
  __syncthreads();
  {   // y: pencil (a, q3)
    double b0[N], b1[N];
#pragma unroll
    for (int b = 0; b < N; ++b) {
      b0[b] = W0[p0 + N * (b + N * p1)];
      b1[b] = W1[p0 + N * (b + N * p1)];
    }
    rmv<N, N, double>(t.S, b0, o1);
    rmv<N, N, double>(t.G, b0, o2);
    rmv<N, N, double>(t.S, b1, in);
#pragma unroll
    for (int q = 0; q < N; ++q) {
      W0[p0 + N * (q + N * p1)] = o1[q];
      W2[p0 + N * (q + N * p1)] = o2[q];
      W1[p0 + N * (q + N * p1)] = in[q];
    }
  }
  __syncthreads();
  double a0[N], a1[N], a2[N];   // x: pencil (q2, q3)
#pragma unroll
  for (int i = 0; i < N; ++i) {
    a0[i] = W0[i + N * (p0 + N * p1)];
    a1[i] = W2[i + N * (p0 + N * p1)];
    a2[i] = W1[i + N * (p0 + N * p1)];
  }
#pragma unroll
  for (int q = 0; q < N; ++q) {
    double v = 0, gx = 0, gy = 0, gz = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      v = fma(t.S[q][i], a0[i], v);
      gx = fma(t.G[q][i], a0[i], gx);
      gy = fma(t.S[q][i], a1[i], gy);
      gz = fma(t.S[q][i], a2[i], gz);
    }
    f(q, p0, p1, v, gx, gy, gz);
  }
  __syncthreads();   // the caller's next component reuses work
}

// tau_D, tau_C per element from u_ex (one element per workgroup, N^2 threads)
template <int N>
__global__ void __launch_bounds__(N* N)
penalty_kernel(const double* __restrict__ u, double* __restrict__ tau_d, double* __restrict__ tau_c,
               MeshArgs mesh, const GaussTab<N>* __restrict__ tab, double fd, double fc) {
  constexpr int N3 = N * N * N;
  __shared__ double work[3 * N3];
  __shared__ double red[N * N];
  __shared__ GaussTab<N> tl;
  const int e = blockIdx.x;
  const int p0 = threadIdx.x % N, p1 = threadIdx.x / N;
  const GaussTab<N>& t = gauss_tables<N>(tab, tl);
  double acc = 0;
  gauss_values3<N>(t, u, (size_t)mesh.n_el * N3, (size_t)e * N3, p0, p1, work,
                   [&](int q1, int q2, int q3, const double (&v)[3]) {
                     acc += t.w[q1] * t.w[q2] * t.w[q3] * sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                   });
  red[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0;
    for (int i = 0; i < N * N; ++i) s += red[i];
    tau_d[e] = fd * s;
    tau_c[e] = fc * s;
  }
}

// per-workgroup partials of sum_e vol sum_q W |u|^2 and of
// sum_e vol sum_q W sum_{j,d} (d_d u_j / h_d)^2; partial[2 * blockIdx.x + {0, 1}]
template <int N>
__global__ void __launch_bounds__(N* N)
diagnostics_kernel(const double* __restrict__ u, double* __restrict__ partial, MeshArgs mesh,
                   const GaussTab<N>* __restrict__ tab, double vol, double ih0, double ih1, double ih2) {
  constexpr int N3 = N * N * N;
  __shared__ double work[3 * N3];
  __shared__ double red[2 * N * N];
  __shared__ GaussTab<N> tl;
  const int e = blockIdx.x;
  const int p0 = threadIdx.x % N, p1 = threadIdx.x / N;
  const GaussTab<N>& t = gauss_tables<N>(tab, tl);
  double uu = 0, gg = 0;
  for (int j = 0; j < 3; ++j)
    gauss_grad1<N>(t, u + ((size_t)j * mesh.n_el + e) * N3, p0, p1, work,
                   [&](int q1, int q2, int q3, double v, double gx, double gy, double gz) {
                     const double w = t.w[q1] * t.w[q2] * t.w[q3];
                     const double a = gx * ih0, b = gy * ih1, c = gz * ih2;
                     uu += w * v * v;
                     gg += w * (a * a + b * b + c * c);
                   });
  red[threadIdx.x] = uu;
  red[N * N + threadIdx.x] = gg;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s0 = 0, s1 = 0;
    for (int i = 0; i < N * N; ++i) {
      s0 += red[i];
      s1 += red[N * N + i];
    }
    partial[2 * (size_t)e] = vol * s0;
    partial[2 * (size_t)e + 1] = vol * s1;
  }
}

// out[q] = sum over the n partials of quantity q (stride 2), fixed order
__global__ void __launch_bounds__(256) reduce2_kernel(const double* __restrict__ partial, long n,
                                                      double* __restrict__ out) {
  __shared__ double sh[2][256];
  double s0 = 0, s1 = 0;
  for (long i = threadIdx.x; i < n; i += 256) {
    s0 += partial[2 * i];
    s1 += partial[2 * i + 1];
  }
  sh[0][threadIdx.x] = s0;
  sh[1][threadIdx.x] = s1;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0, b = 0;
    for (int i = 0; i < 256; ++i) {
      a += sh[0][i];
      b += sh[1][i];
    }
    out[0] = a;
    out[1] = b;
  }
}

__global__ void __launch_bounds__(256) lincomb_kernel(double* __restrict__ y, const double* __restrict__ x0,
                                                      const double* __restrict__ x1, const double* __restrict__ x2,
                                                      double a0, double a1, double a2, long long n) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    double v = a0 * x0[i];
    if (x1) v = fma(a1, x1[i], v);
    if (x2) v = fma(a2, x2[i], v);
    y[i] = v;
  }
}

// 1D tables of the mixed pair on [0,1] with k+1 Gauss points
template <int NU, int NP, typename T>
MixTab<NU, NP, T> make_mix_tab(int k) {
  const Basis1D& bu = basis(k, k + 1);
  const Basis1D& bp = basis(k - 1, k + 1);
  MixTab<NU, NP, T> t{};
  const int m = k + 1;
  for (int i = 0; i < NP; ++i)
    for (int a = 0; a < NU; ++a) {
      double s = 0, d = 0;
      for (int q = 0; q < m; ++q) {
        s += bu.wq[q] * bp.S[q * NP + i] * bu.S[q * NU + a];
        d -= bu.wq[q] * bp.G[q * NP + i] * bu.S[q * NU + a];
      }
      // own-side central-flux ends: l^p_i(1) = [i = NP-1], l^u_a(1) = [a = NU-1]
      if (i == NP - 1 && a == NU - 1) d += 0.5;
      if (i == 0 && a == 0) d -= 0.5;
      t.M[i][a] = (T)s;
      t.B[i][a] = (T)d;
      t.MT[a][i] = (T)s;
      t.G[a][i] = (T)(-d);
    }
  return t;
}

template <int NU, typename T>
hipError_t launch_mix(const DivPlan& P, bool grad, const void* src, void* dst, double scale, hipStream_t s) {
  constexpr int NP = NU - 1;
  using C = MixCfg<NU>;
  hipError_t err;
  const MixTab<NU, NP, T>* dt = device_table_of("mixed", make_mix_tab<NU, NP, T>(P.k), &err);
  if (!dt) return err;
  const int grid = (P.mesh.n_el + C::E - 1) / C::E;
  const T cx = (T)(scale * P.c[0]), cy = (T)(scale * P.c[1]), cz = (T)(scale * P.c[2]);
  if (grad)
    hipLaunchKernelGGL((mixed_gradient_kernel<NU, NP, T>), dim3(grid), dim3(C::THREADS), 0, s, (const T*)src,
                       (T*)dst, P.mesh, dt, cx, cy, cz);
  else
    hipLaunchKernelGGL((mixed_divergence_kernel<NU, NP, T>), dim3(grid), dim3(C::THREADS), 0, s, (const T*)src,
                       (T*)dst, P.mesh, dt, cx, cy, cz);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mix_t(const DivPlan& P, bool grad, const void* src, void* dst, double scale, hipStream_t s) {
  switch (P.k) {
    case 2: return launch_mix<3, T>(P, grad, src, dst, scale, s);
    case 3: return launch_mix<4, T>(P, grad, src, dst, scale, s);
    case 4: return launch_mix<5, T>(P, grad, src, dst, scale, s);
    case 5: return launch_mix<6, T>(P, grad, src, dst, scale, s);
    case 6: return launch_mix<7, T>(P, grad, src, dst, scale, s);
    case 7: return launch_mix<8, T>(P, grad, src, dst, scale, s);
    case 8: return launch_mix<9, T>(P, grad, src, dst, scale, s);
    case 9: return launch_mix<10, T>(P, grad, src, dst, scale, s);
    case 10: return launch_mix<11, T>(P, grad, src, dst, scale, s);
    case 11: return launch_mix<12, T>(P, grad, src, dst, scale, s);
    default: return hipErrorInvalidValue;
  }
}

template <int N>
const GaussTab<N>* gauss_tab(int k, hipError_t* err) {
  const Basis1D& b = basis(k, N);
  GaussTab<N> t{};
  for (int q = 0; q < N; ++q) {
    t.w[q] = b.wq[q];
    for (int a = 0; a < N; ++a) {
      t.S[q][a] = b.S[q * N + a];
      t.G[q][a] = b.G[q * N + a];
    }
  }
  return device_table_of("gauss", t, err);
}

template <int N>
hipError_t launch_gauss_n(int which, const MeshArgs& mesh, const double* u, double* a, double* b, double fd,
                          double fc, const double* scal, hipStream_t s) {
  hipError_t err;
  const GaussTab<N>* t = gauss_tab<N>(N - 1, &err);
  if (!t) return err;
  if (which == 0)
    hipLaunchKernelGGL((penalty_kernel<N>), dim3(mesh.n_el), dim3(N * N), 0, s, u, a, b, mesh, t, fd, fc);
  else
    hipLaunchKernelGGL((diagnostics_kernel<N>), dim3(mesh.n_el), dim3(N * N), 0, s, u, a, mesh, t, scal[0],
                       scal[1], scal[2], scal[3]);
  return hipGetLastError();
}

hipError_t launch_gauss(int k, int which, const MeshArgs& mesh, const double* u, double* a, double* b, double fd,
                        double fc, const double* scal, hipStream_t s) {
  switch (k) {
    case 1: return launch_gauss_n<2>(which, mesh, u, a, b, fd, fc, scal, s);
    case 2: return launch_gauss_n<3>(which, mesh, u, a, b, fd, fc, scal, s);
    case 3: return launch_gauss_n<4>(which, mesh, u, a, b, fd, fc, scal, s);
    case 4: return launch_gauss_n<5>(which, mesh, u, a, b, fd, fc, scal, s);
    case 5: return launch_gauss_n<6>(which, mesh, u, a, b, fd, fc, scal, s);
    case 6: return launch_gauss_n<7>(which, mesh, u, a, b, fd, fc, scal, s);
    case 7: return launch_gauss_n<8>(which, mesh, u, a, b, fd, fc, scal, s);
    case 8: return launch_gauss_n<9>(which, mesh, u, a, b, fd, fc, scal, s);
    case 9: return launch_gauss_n<10>(which, mesh, u, a, b, fd, fc, scal, s);
    case 10: return launch_gauss_n<11>(which, mesh, u, a, b, fd, fc, scal, s);
    case 11: return launch_gauss_n<12>(which, mesh, u, a, b, fd, fc, scal, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_mixed(const DivPlan& P, bool grad, bool f32, const void* src, void* dst, double scale,
                        hipStream_t s) {
  return f32 ? launch_mix_t<float>(P, grad, src, dst, scale, s) : launch_mix_t<double>(P, grad, src, dst, scale, s);
}

hipError_t launch_penalty(int k, const MeshArgs& mesh, const double* u, double* tau_d, double* tau_c, double fd,
                          double fc, hipStream_t s) {
  return launch_gauss(k, 0, mesh, u, tau_d, tau_c, fd, fc, nullptr, s);
}

hipError_t launch_diagnostics(int k, const MeshArgs& mesh, const double* u, double* partial, double* out2,
                              double vol, const double ih[3], hipStream_t s) {
  const double scal[4] = {vol, ih[0], ih[1], ih[2]};
  hipError_t e = launch_gauss(k, 1, mesh, u, partial, nullptr, 0, 0, scal, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reduce2_kernel, dim3(1), dim3(256), 0, s, partial, (long)mesh.n_el, out2);
  return hipGetLastError();
}

hipError_t launch_lincomb(double* y, const double* x0, const double* x1, const double* x2, double a0, double a1,
                          double a2, long long n, hipStream_t s) {
  const long long want = (n + 255) / 256;
  const int grid = (int)std::min<long long>(std::max<long long>(want, 1), 8192);
  hipLaunchKernelGGL(lincomb_kernel, dim3(grid), dim3(256), 0, s, y, x0, x1, x2, a0, a1, a2, n);
  return hipGetLastError();
}

}  // namespace dgmf
