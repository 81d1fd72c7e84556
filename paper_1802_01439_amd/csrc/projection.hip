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
// neighbours' facing layers are mostly found in the same L2.  Own data and
// the neighbours' facing layers of the normal components are loaded first;
// the sweeps run on LDS pencils in place; 13 barriers.
#include "api_internal.h"
#include "common.h"
#include "laplace_kernels.h"
#include "ops.h"

namespace dgmf {

namespace {

template <int N, typename T>
struct ProjTab {
  T S[N][N];    // S[q][a] = l_a(z_q)
  T Dg[N][N];   // Dg[q][r] = derivative of the Gauss Lagrange basis r at z_q
  T M1[N][N];   // 1D mass on [0,1]
  T w[N];       // Gauss weights on [0,1]
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

template <int N, typename T>
__global__ void __launch_bounds__(ProjCfg<N>::THREADS)
projection_kernel(const T* __restrict__ u, T* __restrict__ y, const T* __restrict__ tau_d,
                  const T* __restrict__ tau_c, MeshArgs mesh, const ProjTab<N, T>* __restrict__ tab) {
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
  T* GF = L + 4 * ES;             // own face layers   [d][s][t0 + N t1]
  T* FF = GF + 6 * N2;            // neighbour layers  [d][s][t0 + N t1]
  const int nxy = mesh.nx * mesh.ny;
  const int ez = active ? (int)(e / nxy) : 0, exy = active ? (int)(e - (long long)ez * nxy) : 0;
  const int ey = exy / (mesh.nx > 0 ? mesh.nx : 1), ex = exy - ey * mesh.nx;
  // pencil base and stride in direction dd for this thread's (p0, p1)
  auto pencil = [&](int dd, int& base, int& str) {
    if (dd == 0) { base = PX * p0 + PY * p1; str = 1; }
    else if (dd == 1) { base = p0 + PY * p1; str = PX; }
    else { base = p0 + PX * p1; str = PY; }
  };
  // ---- P0: own z column of component j; own face layers of the normal
  //      component; the neighbours' facing layers of component j = d
  if (active) {
    const T* g = u + j * cs + (size_t)e * N3 + p0 + N * p1;
    T x[N];
#pragma unroll
    for (int c = 0; c < N; ++c) x[c] = g[N2 * c];
#pragma unroll
    for (int c = 0; c < N; ++c) A[p0 + PX * p1 + PY * c] = x[c];
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
  }
  __syncthreads();
  // ---- P1..P3: ug = S (x) S (x) S u, in place, all components; first the
  //      face jumps u^- - u^+ of this thread's face nodes into FF
#pragma unroll
  for (int dd = 0; dd < 3; ++dd) {
    if (active && dd == 0) {
#pragma unroll
      for (int s = 0; s < 2; ++s) FF[(j * 2 + s) * N2 + p] = GF[(j * 2 + s) * N2 + p] - FF[(j * 2 + s) * N2 + p];
    }
    if (active) {
      const auto& t = *fresh(tab);
      int base, str;
      pencil(dd, base, str);
      T x[N], v[N];
#pragma unroll
      for (int a = 0; a < N; ++a) x[a] = A[base + str * a];
#pragma unroll
      for (int q = 0; q < N; ++q) {
        T s = t.S[q][0] * x[0];
#pragma unroll
        for (int a = 1; a < N; ++a) s = fmadd(t.S[q][a], x[a], s);
        v[q] = s;
      }
#pragma unroll
      for (int q = 0; q < N; ++q) A[base + str * q] = v[q];
    }
    __syncthreads();
  }
  // ---- P4: div = sum_j (1/h_j) Dg_j ug_j, one component after the other
#pragma unroll
  for (int jj = 0; jj < 3; ++jj) {
    if (active && j == jj) {
      const auto& t = *fresh(tab);
      int base, str;
      pencil(jj, base, str);
      T x[N];
#pragma unroll
      for (int r = 0; r < N; ++r) x[r] = A[base + str * r];
#pragma unroll
      for (int q = 0; q < N; ++q) {
        T s = t.Dg[q][0] * x[0];
#pragma unroll
        for (int r = 1; r < N; ++r) s = fmadd(t.Dg[q][r], x[r], s);
        s *= t.ih[jj];
        DV[base + str * q] = jj == 0 ? s : DV[base + str * q] + s;
      }
    }
    __syncthreads();
  }
  // ---- P5: pointwise weights: DV <- tau_D vol W div, A_j <- vol W ug_j
  if (active) {
    const auto& t = *fresh(tab);
    const T td = tau_d[e] * t.vol;
    int base, str;
    pencil(2, base, str);   // this thread's z column (p0, p1) = (a, b)
    const T wab = t.w[p0] * t.w[p1];
#pragma unroll
    for (int c = 0; c < N; ++c) {
      const T wq = wab * t.w[c];
      A[base + str * c] *= t.vol * wq;
      if (j == 0) DV[base + str * c] *= td * wq;
    }
  }
  __syncthreads();
  // ---- P6: A_j += (1/h_j) Dg_j^T DV
  if (active) {
    const auto& t = *fresh(tab);
    int base, str;
    pencil(j, base, str);
    T x[N];
#pragma unroll
    for (int q = 0; q < N; ++q) x[q] = DV[base + str * q];
#pragma unroll
    for (int r = 0; r < N; ++r) {
      T s = t.Dg[0][r] * x[0];
#pragma unroll
      for (int q = 1; q < N; ++q) s = fmadd(t.Dg[q][r], x[q], s);
      A[base + str * r] = fmadd(t.ih[j], s, A[base + str * r]);
    }
  }
  __syncthreads();
  // ---- P7..P9: y = S^T (x) S^T (x) S^T z, in place
#pragma unroll
  for (int dd = 0; dd < 3; ++dd) {
    if (active) {
      const auto& t = *fresh(tab);
      int base, str;
      pencil(dd, base, str);
      T x[N], v[N];
#pragma unroll
      for (int q = 0; q < N; ++q) x[q] = A[base + str * q];
#pragma unroll
      for (int a = 0; a < N; ++a) {
        T s = t.S[0][a] * x[0];
#pragma unroll
        for (int q = 1; q < N; ++q) s = fmadd(t.S[q][a], x[q], s);
        v[a] = s;
      }
#pragma unroll
      for (int a = 0; a < N; ++a) A[base + str * a] = v[a];
    }
    __syncthreads();
  }
  // ---- P10: continuity penalty on component j = d, face node (t0, t1) = (p0, p1):
  //      (M1 (x) M1) applied to the jump layer; the M1 rows of p0 and p1 are
  //      held in registers and the t1 loop is not unrolled, so that the jump
  //      layer is read one row at a time
  if (active) {
    const int d = j;
    T m0[N];
#pragma unroll
    for (int i = 0; i < N; ++i) m0[i] = tab->M1[p0][i];
    const T* m1 = &tab->M1[p1][0];
#pragma unroll 1
    for (int s = 0; s < 2; ++s) {
      const int nb = neighbor(mesh, ex, ey, ez, d, s);
      const T tau = T(0.5) * (tau_c[e] + tau_c[nb]) * tab->area[d];
      const T* df = FF + (d * 2 + s) * N2;
      T acc = 0;
#pragma unroll 1
      for (int t1 = 0; t1 < N; ++t1) {
        T row = 0;
#pragma unroll
        for (int t0 = 0; t0 < N; ++t0) row = fmadd(m0[t0], df[t0 + N * t1], row);
        acc = fmadd(m1[t1], row, acc);
      }
      const int lay = s ? N - 1 : 0;
      int idx;
      if (d == 0) idx = lay + PX * p0 + PY * p1;
      else if (d == 1) idx = p0 + PX * lay + PY * p1;
      else idx = p0 + PX * p1 + PY * lay;
      A[idx] += tau * acc;
    }
  }
  __syncthreads();
  // ---- P11: store the z column of component j
  if (active) {
    T* g = y + j * cs + (size_t)e * N3 + p0 + N * p1;
#pragma unroll
    for (int c = 0; c < N; ++c) g[N2 * c] = A[p0 + PX * p1 + PY * c];
  }
}

template <int N, typename T>
hipError_t launch_n(const ProjPlan& P, const void* u, void* yv, const void* td, const void* tc, hipStream_t s) {
  ProjTab<N, T> t;
  for (int i = 0; i < N; ++i) {
    for (int a = 0; a < N; ++a) {
      t.S[i][a] = (T)P.S[i * N + a];
      t.Dg[i][a] = (T)P.Dg[i * N + a];
      t.M1[i][a] = (T)P.M1[i * N + a];
    }
    t.w[i] = (T)P.w[i];
  }
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
                     (T*)yv, (const T*)td, (const T*)tc, P.mesh, dt);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_t(const ProjPlan& P, const void* u, void* y, const void* td, const void* tc, hipStream_t s) {
  switch (P.k) {
    case 1: return launch_n<2, T>(P, u, y, td, tc, s);
    case 2: return launch_n<3, T>(P, u, y, td, tc, s);
    case 3: return launch_n<4, T>(P, u, y, td, tc, s);
    case 4: return launch_n<5, T>(P, u, y, td, tc, s);
    case 5: return launch_n<6, T>(P, u, y, td, tc, s);
    case 6: return launch_n<7, T>(P, u, y, td, tc, s);
    case 7: return launch_n<8, T>(P, u, y, td, tc, s);
    case 8: return launch_n<9, T>(P, u, y, td, tc, s);
    case 9: return launch_n<10, T>(P, u, y, td, tc, s);
    case 10: return launch_n<11, T>(P, u, y, td, tc, s);
    case 11: return launch_n<12, T>(P, u, y, td, tc, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_projection(const ProjPlan& P, bool f32, const void* u, void* y, const void* tau_d,
                             const void* tau_c, hipStream_t s) {
  return f32 ? launch_t<float>(P, u, y, tau_d, tau_c, s) : launch_t<double>(P, u, y, tau_d, tau_c, s);
}

}  // namespace dgmf
