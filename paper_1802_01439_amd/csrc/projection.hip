// Operator of the projection step (Sec. 3.3: (M + A_D + A_C) u; the penalty
// terms of Sec. 3.2): mass, divergence penalty (div v, tau_D div u)_K and
// continuity penalty (v . n, {tau_C} [[u]] . n) on the faces, for a velocity
// field, FP64 and FP32, degrees 1..11, k+1 Gauss points per direction.
//
// Work in the Lagrange basis of the Gauss points (the k+1 point rule makes
// the interpolation S: LGL -> Gauss square and the quadrature exact):
//   ug_j = (S (x) S (x) S) u_j,
//   div  = sum_j (1/h_j) Dg_j ug_j         (Dg: collocation derivative),
//   z_j  = vol W ug_j + (1/h_j) Dg_j^T (tau_D vol W div),
//   y_j  = (S^T (x) S^T (x) S^T) z_j  + continuity term,
// where W is the tensor Gauss weight.  On a face normal to e_d only the
// normal component couples: y_d gains area {tau_C} (M1 (x) M1)(u^-_d - u^+_d)
// on the face layer (LGL face nodes, M1 the 1D mass on [0,1]).
//
// Mapping: one workgroup per batch of E elements, 3 n^2 threads per element
// (component j, pencil); batches are mapped XCD-aware, so that the
// neighbours' facing layers are mostly found in the same L2.  The z sweeps
// of S and S^T run in registers on the loaded and stored z columns; the other
// sweeps run on LDS pencils in place; 8 barriers.  Both point sets are
// symmetric about 1/2, so S and S^T are centrosymmetric and Dg, Dg^T
// centro-antisymmetric: every 1D sweep runs in even-odd form, about half the
// multiply-adds of the dense product.
#include <algorithm>
#include <cmath>

#include "api_internal.h"
#include "common.h"
#include "laplace_kernels.h"
#include "ops.h"

namespace dgmf {

namespace {

// Even-odd form of an n x n matrix A with A[n-1-i][n-1-j] = SIG A[i][j]
// (H = n/2): P[i][j] = (A[i][j] + A[i][n-1-j]) / 2, Q[i][j] = (A[i][j] -
// A[i][n-1-j]) / 2 for i, j < H; for odd n also the middle column, row and
// entry.
template <int N, typename T>
struct EOMat {
  static constexpr int H = N / 2;
  T P[H][H], Q[H][H];
  T col[H], row[H], mid;
};

// y = A x for such a matrix, from the even and odd halves of x.
template <int N, int SIG, typename T, typename M>
__device__ __forceinline__ void eo_apply(const M& A, const T* x, T* y) {
  constexpr int H = N / 2;
  T e[H], o[H];
#pragma unroll
  for (int j = 0; j < H; ++j) {
    e[j] = x[j] + x[N - 1 - j];
    o[j] = x[j] - x[N - 1 - j];
  }
#pragma unroll
  for (int i = 0; i < H; ++i) {
    T P = A.P[i][0] * e[0];
#pragma unroll
    for (int j = 1; j < H; ++j) P = fmadd(A.P[i][j], e[j], P);
    if constexpr (N % 2) P = fmadd(A.col[i], x[H], P);
    T Q = A.Q[i][0] * o[0];
#pragma unroll
    for (int j = 1; j < H; ++j) Q = fmadd(A.Q[i][j], o[j], Q);
    y[i] = P + Q;
    y[N - 1 - i] = SIG > 0 ? P - Q : Q - P;
  }
  if constexpr (N % 2) {
    T m = A.mid * x[H];
#pragma unroll
    for (int j = 0; j < H; ++j) m = fmadd(A.row[j], SIG > 0 ? e[j] : o[j], m);
    y[H] = m;
  }
}

template <int N, typename T>
struct ProjTab {
  EOMat<N, T> S, St, Dg, Dt;   // S[q][a] = l_a(z_q); Dg[q][r] = derivative of
                               // the Gauss Lagrange basis r at z_q; St, Dt transposed
  T M1[N][N];                  // 1D mass on [0,1]
  T w[N];                      // Gauss weights on [0,1]
  T vol, ih[3], area[3];
};

template <int N>
struct ProjCfg {
  static constexpr int N2 = N * N, N3 = N * N * N;
  static constexpr int E = (256 / (3 * N2)) > 0 ? 256 / (3 * N2) : 1;
  static constexpr int THREADS = E * 3 * N2;
  static constexpr int PX = LapCfgB<N>::PX, PY = LapCfgB<N>::PY, ES = LapCfgB<N>::ES;
  // per element: 3 components + div, then 6 own and 6 neighbour face layers
  static constexpr int PER = 4 * ES + 12 * N2;
};

// From n = 9 on, at least 4 waves per SIMD (at most 128 VGPRs): at n = 12
// in FP64 the compiler would otherwise take 129 and halve the resident
// workgroups.
template <int N, typename T>
__global__ void __launch_bounds__(ProjCfg<N>::THREADS) __attribute__((amdgpu_waves_per_eu(N >= 9 ? 4 : 1, 8)))
projection_kernel(const T* __restrict__ u, T* __restrict__ y, const T* __restrict__ tau_d,
                  const T* __restrict__ tau_c, MeshArgs mesh, const ProjTab<N, T>* __restrict__ tab,
                  T* __restrict__ dot) {
  using C = ProjCfg<N>;
  constexpr int N2 = C::N2, N3 = C::N3, E = C::E, PX = C::PX, PY = C::PY, ES = C::ES, PER = C::PER;
  __shared__ T lds[E * PER];
  const int tid = threadIdx.x;
  const int le = tid / (3 * N2);
  const int rem = tid - le * 3 * N2;
  const int j = rem / N2, p = rem - j * N2;
  const int p0 = p % N, p1 = p / N;
  const long long e = (long long)xcd_remap(blockIdx.x, gridDim.x) * E + le;
  const bool active = e < mesh.n_el;
  const size_t cs = (size_t)mesh.n_el * N3;
  T* L = lds + le * PER;
  T* A = L + j * ES;              // this thread's component
  T* DV = L + 3 * ES;
  T* GF = L + 4 * ES;             // own face layers, then half-applied face mass  [d][s][t0 + N t1]
  T* FF = GF + 6 * N2;            // neighbour layers, then jumps, then face terms [d][s][t0 + N t1]
  const int nxy = mesh.nx * mesh.ny;
  const int ez = active ? (int)(e / nxy) : 0, exy = active ? (int)(e - (long long)ez * nxy) : 0;
  const int ey = exy / (mesh.nx > 0 ? mesh.nx : 1), ex = exy - ey * mesh.nx;
  // pencil base and stride in direction dd for this thread's (p0, p1)
  auto pencil = [&](int dd, int& base, int& str) {
    if (dd == 0) { base = PX * p0 + PY * p1; str = 1; }
    else if (dd == 1) { base = p0 + PY * p1; str = PX; }
    else { base = p0 + PX * p1; str = PY; }
  };
  const int zcol = p0 + PX * p1;   // this thread's z column (a, b) = (p0, p1)
  T acc = 0;                       // this thread's part of u.y (dot only)
  // ---- P0: own z column of component j, its face values, the neighbours'
  //      facing layers of component j = d; S along z in registers
  if (active) {
    const T* g = u + j * cs + (size_t)e * N3 + p0 + N * p1;
    T x[N], v[N];
#pragma unroll
    for (int c = 0; c < N; ++c) x[c] = g[N2 * c];
    if (j == 0 && (p0 == 0 || p0 == N - 1)) {   // x faces: (t0, t1) = (b, c)
#pragma unroll
      for (int c = 0; c < N; ++c) GF[(0 * 2 + (p0 ? 1 : 0)) * N2 + p1 + N * c] = x[c];
    }
    if (j == 1 && (p1 == 0 || p1 == N - 1)) {   // y faces: (t0, t1) = (a, c)
#pragma unroll
      for (int c = 0; c < N; ++c) GF[(1 * 2 + (p1 ? 1 : 0)) * N2 + p0 + N * c] = x[c];
    }
    if (j == 2) {                                // z faces: (t0, t1) = (a, b)
      GF[(2 * 2 + 0) * N2 + p] = x[0];
      GF[(2 * 2 + 1) * N2 + p] = x[N - 1];
    }
    // neighbour across (d = j, s): its facing layer at tangential (t0, t1) = (p0, p1)
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int nb = neighbor(mesh, ex, ey, ez, j, s);
      const int lay = s ? 0 : N - 1;
      int idx;
      if (j == 0) idx = lay + N * p0 + N2 * p1;
      else if (j == 1) idx = p0 + N * lay + N2 * p1;
      else idx = p0 + N * p1 + N2 * lay;
      FF[(j * 2 + s) * N2 + p] = u[j * cs + (size_t)nb * N3 + idx];
    }
    eo_apply<N, 1>(fresh(tab)->S, x, v);
#pragma unroll
    for (int c = 0; c < N; ++c) A[zcol + PY * c] = v[c];
  }
  __syncthreads();
  // ---- P1, P2: S along x and y on LDS pencils.  Before the x sweep the face
  //      jumps u^- - u^+ of this thread's face nodes go into FF; before the
  //      y sweep the first factor of (M1 (x) M1) is applied to them:
  //      GF[d][s][p0 + N p1] = sum_t0 M1[p0][t0] jump[t0 + N p1]
#pragma unroll
  for (int dd = 0; dd < 2; ++dd) {
    if (active && dd == 0) {
#pragma unroll
      for (int s = 0; s < 2; ++s) FF[(j * 2 + s) * N2 + p] = GF[(j * 2 + s) * N2 + p] - FF[(j * 2 + s) * N2 + p];
    }
    if (active && dd == 1) {
      T m0[N];
#pragma unroll
      for (int i = 0; i < N; ++i) m0[i] = tab->M1[p0][i];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const T* df = FF + (j * 2 + s) * N2 + N * p1;
        T r = 0;
#pragma unroll
        for (int t0 = 0; t0 < N; ++t0) r = fmadd(m0[t0], df[t0], r);
        GF[(j * 2 + s) * N2 + p] = r;
      }
    }
    if (active) {
      int base, str;
      pencil(dd, base, str);
      T x[N], v[N];
#pragma unroll
      for (int a = 0; a < N; ++a) x[a] = A[base + str * a];
      eo_apply<N, 1>(fresh(tab)->S, x, v);
#pragma unroll
      for (int q = 0; q < N; ++q) A[base + str * q] = v[q];
    }
    __syncthreads();
  }
  // ---- P3: along direction j: keep vol W ug_j in registers, overwrite
  //      ug_j with its derivative (1/h_j) Dg_j ug_j
  int base, str;
  pencil(j, base, str);
  T mw[N];
  if (active) {
    const auto& t = *fresh(tab);
    T x[N], v[N];
#pragma unroll
    for (int r = 0; r < N; ++r) x[r] = A[base + str * r];
    // tensor weight along the pencil: the two fixed indices are (p0, p1)
    const T w2 = t.vol * t.w[p0] * t.w[p1];
#pragma unroll
    for (int r = 0; r < N; ++r) mw[r] = w2 * t.w[r] * x[r];
    eo_apply<N, -1>(t.Dg, x, v);
#pragma unroll
    for (int q = 0; q < N; ++q) A[base + str * q] = t.ih[j] * v[q];
  }
  __syncthreads();
  // ---- P4: DV <- tau_D vol W div on z-column nodes c = j, j+3, ...;
  //      second factor of (M1 (x) M1) and the penalty factor: continuity term
  //      of face node (p0, p1) of the faces normal to e_j into FF
  if (active) {
    const auto& t = *fresh(tab);
    const T td = tau_d[e] * t.vol;
    const T wab = t.w[p0] * t.w[p1];
    const T* A0 = L;
#pragma unroll
    for (int c = 0; c < N; ++c) {
      if (c % 3 != j) continue;
      const int i = zcol + PY * c;
      DV[i] = td * wab * t.w[c] * (A0[i] + A0[i + ES] + A0[i + 2 * ES]);
    }
    T m1[N];
#pragma unroll
    for (int i = 0; i < N; ++i) m1[i] = tab->M1[p1][i];
    const T tce = tau_c[e], area = t.area[j];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int nb = neighbor(mesh, ex, ey, ez, j, s);
      const T* r = GF + (j * 2 + s) * N2 + p0;
      T acc = 0;
#pragma unroll
      for (int t1 = 0; t1 < N; ++t1) acc = fmadd(m1[t1], r[N * t1], acc);
      FF[(j * 2 + s) * N2 + p] = T(0.5) * (tce + tau_c[nb]) * area * acc;
    }
  }
  __syncthreads();
  // ---- P5: z_j = vol W ug_j + (1/h_j) Dg_j^T DV along direction j
  if (active) {
    const auto& t = *fresh(tab);
    T x[N], v[N];
#pragma unroll
    for (int q = 0; q < N; ++q) x[q] = DV[base + str * q];
    eo_apply<N, -1>(t.Dt, x, v);
#pragma unroll
    for (int r = 0; r < N; ++r) A[base + str * r] = fmadd(t.ih[j], v[r], mw[r]);
  }
  __syncthreads();
  // ---- P6, P7: S^T along x and y
#pragma unroll
  for (int dd = 0; dd < 2; ++dd) {
    if (active) {
      int b2, s2;
      pencil(dd, b2, s2);
      T x[N], v[N];
#pragma unroll
      for (int q = 0; q < N; ++q) x[q] = A[b2 + s2 * q];
      eo_apply<N, 1>(fresh(tab)->St, x, v);
#pragma unroll
      for (int a = 0; a < N; ++a) A[b2 + s2 * a] = v[a];
    }
    __syncthreads();
  }
  // ---- P8: S^T along z in registers, the continuity terms of this column's
  //      face nodes, store
  if (active) {
    T x[N], v[N];
#pragma unroll
    for (int c = 0; c < N; ++c) x[c] = A[zcol + PY * c];
    eo_apply<N, 1>(fresh(tab)->St, x, v);
    if (j == 0 && (p0 == 0 || p0 == N - 1)) {
#pragma unroll
      for (int c = 0; c < N; ++c) v[c] += FF[(0 * 2 + (p0 ? 1 : 0)) * N2 + p1 + N * c];
    }
    if (j == 1 && (p1 == 0 || p1 == N - 1)) {
#pragma unroll
      for (int c = 0; c < N; ++c) v[c] += FF[(1 * 2 + (p1 ? 1 : 0)) * N2 + p0 + N * c];
    }
    if (j == 2) {
      v[0] += FF[(2 * 2 + 0) * N2 + p];
      v[N - 1] += FF[(2 * 2 + 1) * N2 + p];
    }
    T* g = y + j * cs + (size_t)e * N3 + p0 + N * p1;
#pragma unroll
    for (int c = 0; c < N; ++c) g[N2 * c] = v[c];
    if (dot) {   // u.y of this column (the input column again, from cache)
      const T* gu = u + j * cs + (size_t)e * N3 + p0 + N * p1;
      T sdot = 0;
#pragma unroll
      for (int c = 0; c < N; ++c) sdot = fmadd(gu[N2 * c], v[c], sdot);
      acc = sdot;
    }
  }
  // ---- optional: workgroup sum of u.y into dot[blockIdx.x] (fixed order)
  if (dot) {
    __syncthreads();
    lds[tid] = acc;
    __syncthreads();
    if (tid == 0) {
      T s = 0;
      for (int i = 0; i < C::THREADS; ++i) s += lds[i];
      dot[blockIdx.x] = s;
    }
  }
}

// Even-odd tables of the n x n row-major matrix A (parity sig); false if A
// lacks that parity.
template <int N, typename T>
bool make_eo(const double* A, int sig, EOMat<N, T>& m) {
  constexpr int H = N / 2;
  double amax = 0;
  for (int i = 0; i < N * N; ++i) amax = std::max(amax, std::fabs(A[i]));
  for (int i = 0; i < N; ++i)
    for (int k = 0; k < N; ++k)
      if (std::fabs(A[(N - 1 - i) * N + (N - 1 - k)] - sig * A[i * N + k]) > 1e-11 * amax) return false;
  for (int i = 0; i < H; ++i) {
    for (int k = 0; k < H; ++k) {
      m.P[i][k] = (T)(0.5 * (A[i * N + k] + A[i * N + N - 1 - k]));
      m.Q[i][k] = (T)(0.5 * (A[i * N + k] - A[i * N + N - 1 - k]));
    }
    m.col[i] = (T)(N % 2 ? A[i * N + H] : 0.0);
    m.row[i] = (T)(N % 2 ? A[H * N + i] : 0.0);
  }
  m.mid = (T)(N % 2 ? A[H * N + H] : 0.0);
  return true;
}

template <int N, typename T>
hipError_t launch_n(const ProjPlan& P, const void* u, void* yv, const void* td, const void* tc, hipStream_t s,
                    void* dot) {
  ProjTab<N, T> t{};
  double St[N * N], Dt[N * N];
  for (int i = 0; i < N; ++i) {
    for (int a = 0; a < N; ++a) {
      St[a * N + i] = P.S[i * N + a];
      Dt[a * N + i] = P.Dg[i * N + a];
      t.M1[i][a] = (T)P.M1[i * N + a];
    }
    t.w[i] = (T)P.w[i];
  }
  if (!make_eo<N, T>(P.S.data(), 1, t.S) || !make_eo<N, T>(St, 1, t.St) || !make_eo<N, T>(P.Dg.data(), -1, t.Dg) ||
      !make_eo<N, T>(Dt, -1, t.Dt))
    return hipErrorInvalidValue;
  t.vol = (T)P.vol;
  for (int d = 0; d < 3; ++d) {
    t.ih[d] = (T)P.ih[d];
    t.area[d] = (T)P.area[d];
  }
  hipError_t err;
  const ProjTab<N, T>* dt = device_table_of("projection", t, &err);
  if (!dt) return err;
  using C = ProjCfg<N>;
  const long long grid = ((long long)P.mesh.n_el + C::E - 1) / C::E;
  if (grid > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((projection_kernel<N, T>), dim3((unsigned)grid), dim3(C::THREADS), 0, s, (const T*)u,
                     (T*)yv, (const T*)td, (const T*)tc, P.mesh, dt, (T*)dot);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_t(const ProjPlan& P, const void* u, void* y, const void* td, const void* tc, hipStream_t s,
                    void* dot) {
  switch (P.k) {
    case 1: return launch_n<2, T>(P, u, y, td, tc, s, dot);
    case 2: return launch_n<3, T>(P, u, y, td, tc, s, dot);
    case 3: return launch_n<4, T>(P, u, y, td, tc, s, dot);
    case 4: return launch_n<5, T>(P, u, y, td, tc, s, dot);
    case 5: return launch_n<6, T>(P, u, y, td, tc, s, dot);
    case 6: return launch_n<7, T>(P, u, y, td, tc, s, dot);
    case 7: return launch_n<8, T>(P, u, y, td, tc, s, dot);
    case 8: return launch_n<9, T>(P, u, y, td, tc, s, dot);
    case 9: return launch_n<10, T>(P, u, y, td, tc, s, dot);
    case 10: return launch_n<11, T>(P, u, y, td, tc, s, dot);
    case 11: return launch_n<12, T>(P, u, y, td, tc, s, dot);
    default: return hipErrorInvalidValue;
  }
}

template <int N>
long long grid_n(long long n_el) {
  return (n_el + ProjCfg<N>::E - 1) / ProjCfg<N>::E;
}

}  // namespace

hipError_t launch_projection(const ProjPlan& P, bool f32, const void* u, void* y, const void* tau_d,
                             const void* tau_c, hipStream_t s, void* dot_partial) {
  return f32 ? launch_t<float>(P, u, y, tau_d, tau_c, s, dot_partial)
             : launch_t<double>(P, u, y, tau_d, tau_c, s, dot_partial);
}

long long projection_grid(const ProjPlan& P) {
  const long long n = P.mesh.n_el;
  switch (P.k) {
    case 1: return grid_n<2>(n);
    case 2: return grid_n<3>(n);
    case 3: return grid_n<4>(n);
    case 4: return grid_n<5>(n);
    case 5: return grid_n<6>(n);
    case 6: return grid_n<7>(n);
    case 7: return grid_n<8>(n);
    case 8: return grid_n<9>(n);
    case 9: return grid_n<10>(n);
    case 10: return grid_n<11>(n);
    case 11: return grid_n<12>(n);
    default: return 0;
  }
}

}  // namespace dgmf
