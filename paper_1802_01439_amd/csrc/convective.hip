// Convective term c_h with the local Lax-Friedrichs flux (Sec. 3.2, weak form
// of c_h, F_c(u) = u (x) u), by sum factorisation on periodic Cartesian meshes,
// FP64 and FP32, degrees 1..11 with floor(3k/2)+1 Gauss points (3/2 rule).
//
//   R_c = -sum_j s_j (d_j phi, u_c u_j)_K + sum_faces (phi, F*_c),   s_j = vol/h_j
//   F*_c = 1/2 (u-_c u-.n + u+_c u+.n) + lf * max(|u-.n|, |u+.n|) (u-_c - u+_c)
//
// Sum factorisation with S (m x n, LGL -> Gauss interpolation) and G (m x n,
// derivatives of the LGL basis at the Gauss points):
//   cell:  u -> Sx -> Sy -> [Sz, flux W u_c u_j, S^T_z / G^T_z fused per
//          z-pencil in registers] -> y back-sweep -> x back-sweep
//          R_c = G^T_x S^T_y S^T_z F_cx + S^T_x G^T_y S^T_z F_cy + S^T_x S^T_y G^T_z F_cz
//   faces: per direction, own (from LDS) and neighbour (from global) face
//          layers are interpolated to the m x m face Gauss points (t1 then t2),
//          the flux is formed pointwise and integrated back (t2 then t1) onto
//          the n x n face nodes; the LGL basis makes the face layer the only
//          non-zero trace.  Each element does its own six faces (no atomics).
//
// GPU mapping: one workgroup per batch of E consecutive elements; every phase
// is a loop of the workgroup's threads over the pencils of that phase, with
// LDS buffers between phases (aliased by lifetime so that even k = 11 in FP64
// fits one element in the 160 KB LDS).
#include "api_internal.h"
#include "common.h"
#include "ops.h"

namespace dgmf {

template <int N, int Q, typename T>
struct ConvTab {
  T S[Q][N];   // l_a(z_q)
  T G[Q][N];   // l_a'(z_q)
  T w[Q];      // Gauss weights on [0,1]
};

template <typename T>
struct ConvScal {
  T cell[3];   // -vol/h_j
  T area[3];   // vol/h_d
  T lf;
};

template <int N, int Q, typename T>
struct ConvCfg {
  static constexpr int N2 = N * N, N3 = N * N * N;
  static constexpr int RA = (3 * Q * Q * N > 3 * N3 + 18 * Q * N) ? 3 * Q * Q * N : 3 * N3 + 18 * Q * N;
  static constexpr int RB = 3 * Q * N2;
  static constexpr int FR = 18 * N2;
  static constexpr int PER_ELEM = RA + RB + FR;
  static constexpr int BUDGET = 64 * 1024 / (int)sizeof(T);
  static constexpr int LDS_MAX = 160 * 1024 / (int)sizeof(T);
  static constexpr int E = (PER_ELEM <= BUDGET) ? (BUDGET / PER_ELEM) : 1;
  static constexpr int THREADS = (Q * Q * E > 256) ? 512 : 256;
  static constexpr int PPT = (E * Q * Q + THREADS - 1) / THREADS;   // z-pencils per thread
  static_assert(E * PER_ELEM <= LDS_MAX, "convective LDS footprint exceeds 160 KB");
};

// node index of (value along d, t1, t2) for face direction d
template <int N>
__device__ __forceinline__ int face_node(int d, int dv, int t1, int t2) {
  return d == 0 ? dv + N * (t1 + N * t2) : (d == 1 ? t1 + N * (dv + N * t2) : t1 + N * (t2 + N * dv));
}

template <int N, int Q, typename T>
__global__ void __launch_bounds__((ConvCfg<N, Q, T>::THREADS))
convective_kernel(const T* __restrict__ u, T* __restrict__ r, MeshArgs mesh,
                  const ConvTab<N, Q, T>* __restrict__ tab, ConvScal<T> sc) {
  const ConvTab<N, Q, T>& t = *tab;
  using C = ConvCfg<N, Q, T>;
  constexpr int N2 = C::N2, N3 = C::N3, E = C::E, TH = C::THREADS;
  __shared__ T RA[E * C::RA];
  __shared__ T RB[E * C::RB];
  __shared__ T FRb[E * C::FR];

  const int tid = threadIdx.x;
  const int e0 = xcd_remap(blockIdx.x, gridDim.x) * E;
  const int ne = min(E, mesh.n_el - e0);
  const size_t cstride = (size_t)mesh.n_el * N3;   // component stride in global arrays

  // stage the batch: A[le][c][node] at RA + le*RA
  for (int i = tid; i < ne * 3 * N3; i += TH) {
    const int le = i / (3 * N3), rem = i - le * 3 * N3, c = rem / N3, node = rem - c * N3;
    RA[le * C::RA + c * N3 + node] = u[c * cstride + (size_t)(e0 + le) * N3 + node];
  }
  __syncthreads();

  // ---------------- faces, one direction at a time ----------------
  for (int d = 0; d < 3; ++d) {
    // F1: interpolate face layers along t1 (own from LDS, neighbour from global)
    for (int w = tid; w < ne * 12 * N; w += TH) {
      const int le = w / (12 * N);
      int rem = w - le * 12 * N;
      const int j = rem % N; rem /= N;
      const int side = rem % 2; rem /= 2;
      const int c = rem % 3;
      const int s = rem / 3;
      const int e = e0 + le;
      T in[N];
      if (side == 0) {
        const T* A = RA + le * C::RA + c * N3;
#pragma unroll
        for (int i = 0; i < N; ++i) in[i] = A[face_node<N>(d, s ? N - 1 : 0, i, j)];
      } else {
        const int ex = e % mesh.nx, ey = (e / mesh.nx) % mesh.ny, ez = e / (mesh.nx * mesh.ny);
        const T* g = u + c * cstride + (size_t)neighbor(mesh, ex, ey, ez, d, s) * N3;
#pragma unroll
        for (int i = 0; i < N; ++i) in[i] = g[face_node<N>(d, s ? 0 : N - 1, i, j)];
      }
      T* FA = RA + le * C::RA + 3 * N3 + (((s * 3 + c) * 2 + side) * N + j) * Q;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        T acc = t.S[q][0] * in[0];
#pragma unroll
        for (int i = 1; i < N; ++i) acc = fmadd(t.S[q][i], in[i], acc);
        FA[q] = acc;
      }
    }
    __syncthreads();
    // F2: per face column q1: interpolate along t2, flux, integrate along t2
    for (int w = tid; w < ne * 2 * Q; w += TH) {
      const int le = w / (2 * Q);
      const int rem = w - le * 2 * Q;
      const int s = rem / Q, q1 = rem - (rem / Q) * Q;
      const T* FA = RA + le * C::RA + 3 * N3;
      T tr[3][2][N];
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int side = 0; side < 2; ++side)
#pragma unroll
          for (int j = 0; j < N; ++j) tr[c][side][j] = FA[(((s * 3 + c) * 2 + side) * N + j) * Q + q1];
      T acc[3][N];
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int j = 0; j < N; ++j) acc[c][j] = 0;
      const T sgn = s ? T(1) : T(-1);
      const T wq1 = t.w[q1] * sc.area[d];
#pragma unroll
      for (int q2 = 0; q2 < Q; ++q2) {
        T um[3], up[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          T a = t.S[q2][0] * tr[c][0][0], b = t.S[q2][0] * tr[c][1][0];
#pragma unroll
          for (int j = 1; j < N; ++j) {
            a = fmadd(t.S[q2][j], tr[c][0][j], a);
            b = fmadd(t.S[q2][j], tr[c][1][j], b);
          }
          um[c] = a;
          up[c] = b;
        }
        const T unm = sgn * um[d], unp = sgn * up[d];
        const T lam = fmax(fabs(unm), fabs(unp));
        const T wgt = wq1 * t.w[q2];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const T F = wgt * (T(0.5) * (um[c] * unm + up[c] * unp) + sc.lf * lam * (um[c] - up[c]));
#pragma unroll
          for (int j = 0; j < N; ++j) acc[c][j] = fmadd(t.S[q2][j], F, acc[c][j]);
        }
      }
      T* FB = RA + le * C::RA + 3 * N3 + 12 * Q * N;
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int j = 0; j < N; ++j) FB[((s * 3 + c) * Q + q1) * N + j] = acc[c][j];
    }
    __syncthreads();
    // F3: integrate along t1 onto the face nodes
    for (int w = tid; w < ne * 6 * N; w += TH) {
      const int le = w / (6 * N);
      int rem = w - le * 6 * N;
      const int j = rem % N;
      rem /= N;
      const int c = rem % 3, s = rem / 3;
      const T* FB = RA + le * C::RA + 3 * N3 + 12 * Q * N + ((s * 3 + c) * Q) * N + j;
      T in[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) in[q] = FB[q * N];
      T* FR = FRb + le * C::FR + ((d * 2 + s) * 3 + c) * N2 + N * j;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        T acc = t.S[0][i] * in[0];
#pragma unroll
        for (int q = 1; q < Q; ++q) acc = fmadd(t.S[q][i], in[q], acc);
        FR[i] = acc;
      }
    }
    __syncthreads();
  }

  // ---------------- cell: forward interpolation ----------------
  // X: A[c][a,b,cz] -> B[c][q1 + Q(b + N cz)]
  for (int w = tid; w < ne * 3 * N2; w += TH) {
    const int le = w / (3 * N2);
    const int rem = w - le * 3 * N2;
    const int c = rem / N2, bc = rem - c * N2;
    const T* A = RA + le * C::RA + c * N3 + N * bc;
    T in[N];
#pragma unroll
    for (int a = 0; a < N; ++a) in[a] = A[a];
    T* B = RB + le * C::RB + c * Q * N2 + Q * bc;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      T acc = t.S[q][0] * in[0];
#pragma unroll
      for (int a = 1; a < N; ++a) acc = fmadd(t.S[q][a], in[a], acc);
      B[q] = acc;
    }
  }
  __syncthreads();
  // Y: B[c][q1 + Q(b + N cz)] -> Cb[c][q1 + Q(q2 + Q cz)]   (Cb aliases A's region)
  for (int w = tid; w < ne * 3 * Q * N; w += TH) {
    const int le = w / (3 * Q * N);
    int rem = w - le * 3 * Q * N;
    const int c = rem / (Q * N);
    rem -= c * Q * N;
    const int cz = rem / Q, q1 = rem - cz * Q;
    const T* B = RB + le * C::RB + c * Q * N2 + q1 + Q * N * cz;
    T in[N];
#pragma unroll
    for (int b = 0; b < N; ++b) in[b] = B[Q * b];
    T* Cb = RA + le * C::RA + c * Q * Q * N + q1 + Q * Q * cz;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      T acc = t.S[q][0] * in[0];
#pragma unroll
      for (int b = 1; b < N; ++b) acc = fmadd(t.S[q][b], in[b], acc);
      Cb[Q * q] = acc;
    }
  }
  __syncthreads();
  // Z: each thread takes whole (q1,q2) z-pencils into registers and
  // interpolates them to the Gauss points in z: U[j][q3]
  T Uz[C::PPT][3][Q];
#pragma unroll
  for (int pp = 0; pp < C::PPT; ++pp) {
    const int w = tid + pp * TH;
    if (w < ne * Q * Q) {
      const int le = w / (Q * Q), qq = w - le * Q * Q;
      const T* Cb = RA + le * C::RA + qq;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        T in[N];
#pragma unroll
        for (int cz = 0; cz < N; ++cz) in[cz] = Cb[c * Q * Q * N + Q * Q * cz];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          T acc = t.S[q][0] * in[0];
#pragma unroll
          for (int cz = 1; cz < N; ++cz) acc = fmadd(t.S[q][cz], in[cz], acc);
          Uz[pp][c][q] = acc;
        }
      }
    }
  }
  __syncthreads();

  // ---------------- cell: flux and back-contraction, per component ----------------
  for (int c = 0; c < 3; ++c) {
    // Zc: T_x = S^T_z F_cx, T_y = S^T_z F_cy, T_z = G^T_z F_cz  -> Tb[f][q1 + Q(q2 + Q cz)]
#pragma unroll
    for (int pp = 0; pp < C::PPT; ++pp) {
      const int w = tid + pp * TH;
      if (w < ne * Q * Q) {
        const int le = w / (Q * Q), qq = w - le * Q * Q;
        const int q2 = qq / Q, q1 = qq - q2 * Q;
        const T w12 = t.w[q1] * t.w[q2];
        T ox[N], oy[N], oz[N];
#pragma unroll
        for (int cz = 0; cz < N; ++cz) ox[cz] = oy[cz] = oz[cz] = 0;
#pragma unroll
        for (int q3 = 0; q3 < Q; ++q3) {
          const T uc = w12 * t.w[q3] * Uz[pp][c][q3];
          const T fx = sc.cell[0] * uc * Uz[pp][0][q3];
          const T fy = sc.cell[1] * uc * Uz[pp][1][q3];
          const T fz = sc.cell[2] * uc * Uz[pp][2][q3];
#pragma unroll
          for (int cz = 0; cz < N; ++cz) {
            ox[cz] = fmadd(t.S[q3][cz], fx, ox[cz]);
            oy[cz] = fmadd(t.S[q3][cz], fy, oy[cz]);
            oz[cz] = fmadd(t.G[q3][cz], fz, oz[cz]);
          }
        }
        T* Tb = RA + le * C::RA + qq;
#pragma unroll
        for (int cz = 0; cz < N; ++cz) {
          Tb[0 * Q * Q * N + Q * Q * cz] = ox[cz];
          Tb[1 * Q * Q * N + Q * Q * cz] = oy[cz];
          Tb[2 * Q * Q * N + Q * Q * cz] = oz[cz];
        }
      }
    }
    __syncthreads();
    // Yc: V1 = S^T_y T_x, V2 = G^T_y T_y + S^T_y T_z  -> Vb[f][q1 + Q(b + N cz)]
    for (int w = tid; w < ne * Q * N; w += TH) {
      const int le = w / (Q * N);
      const int rem = w - le * Q * N;
      const int cz = rem / Q, q1 = rem - cz * Q;
      const T* Tb = RA + le * C::RA + q1 + Q * Q * cz;
      T v1[N], v2[N];
#pragma unroll
      for (int b = 0; b < N; ++b) v1[b] = v2[b] = 0;
#pragma unroll
      for (int q2 = 0; q2 < Q; ++q2) {
        const T tx = Tb[Q * q2], ty = Tb[Q * Q * N + Q * q2], tz = Tb[2 * Q * Q * N + Q * q2];
#pragma unroll
        for (int b = 0; b < N; ++b) {
          v1[b] = fmadd(t.S[q2][b], tx, v1[b]);
          v2[b] = fmadd(t.G[q2][b], ty, fmadd(t.S[q2][b], tz, v2[b]));
        }
      }
      T* Vb = RB + le * C::RB + q1 + Q * N * cz;
#pragma unroll
      for (int b = 0; b < N; ++b) {
        Vb[Q * b] = v1[b];
        Vb[Q * N2 + Q * b] = v2[b];
      }
    }
    __syncthreads();
    // Xc: R_c = G^T_x V1 + S^T_x V2 + face terms, written once
    for (int w = tid; w < ne * N2; w += TH) {
      const int le = w / N2, bc = w - le * N2;
      const int b = bc % N, cz = bc / N;
      const T* Vb = RB + le * C::RB + Q * bc;
      T o[N];
#pragma unroll
      for (int a = 0; a < N; ++a) o[a] = 0;
#pragma unroll
      for (int q1 = 0; q1 < Q; ++q1) {
        const T v1 = Vb[q1], v2 = Vb[Q * N2 + q1];
#pragma unroll
        for (int a = 0; a < N; ++a) o[a] = fmadd(t.G[q1][a], v1, fmadd(t.S[q1][a], v2, o[a]));
      }
      const T* FR = FRb + le * C::FR;
      // x faces: nodes a = 0 / N-1, face index (t1,t2) = (b,cz)
      o[0] += FR[((0 * 2 + 0) * 3 + c) * N2 + b + N * cz];
      o[N - 1] += FR[((0 * 2 + 1) * 3 + c) * N2 + b + N * cz];
      if (b == 0 || b == N - 1) {   // y faces: (t1,t2) = (a,cz)
        const T* F = FR + ((1 * 2 + (b == 0 ? 0 : 1)) * 3 + c) * N2 + N * cz;
#pragma unroll
        for (int a = 0; a < N; ++a) o[a] += F[a];
      }
      if (cz == 0 || cz == N - 1) { // z faces: (t1,t2) = (a,b)
        const T* F = FR + ((2 * 2 + (cz == 0 ? 0 : 1)) * 3 + c) * N2 + N * b;
#pragma unroll
        for (int a = 0; a < N; ++a) o[a] += F[a];
      }
      T* g = r + c * cstride + (size_t)(e0 + le) * N3 + N * bc;
#pragma unroll
      for (int a = 0; a < N; ++a) g[a] = o[a];
    }
    __syncthreads();
  }
}

template <int N, int Q, typename T>
static hipError_t launch_conv_nq(const ConvPlan& P, const void* u, void* r, hipStream_t s) {
  using C = ConvCfg<N, Q, T>;
  ConvTab<N, Q, T> t;
  for (int q = 0; q < Q; ++q) {
    for (int a = 0; a < N; ++a) {
      t.S[q][a] = (T)P.S[q * N + a];
      t.G[q][a] = (T)P.G[q * N + a];
    }
    t.w[q] = (T)P.w[q];
  }
  ConvScal<T> sc;
  for (int d = 0; d < 3; ++d) {
    sc.cell[d] = (T)P.cell[d];
    sc.area[d] = (T)P.area[d];
  }
  sc.lf = (T)P.lf;
  hipError_t err;
  const ConvTab<N, Q, T>* dt = device_table_of("convective", t, &err);
  if (!dt) return err;
  const int grid = (P.mesh.n_el + C::E - 1) / C::E;
  hipLaunchKernelGGL((convective_kernel<N, Q, T>), dim3(grid), dim3(C::THREADS), 0, s,
                     (const T*)u, (T*)r, P.mesh, dt, sc);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_conv_t(const ConvPlan& P, const void* u, void* r, hipStream_t s) {
  switch (P.k) {
    case 1: return launch_conv_nq<2, 2, T>(P, u, r, s);
    case 2: return launch_conv_nq<3, 4, T>(P, u, r, s);
    case 3: return launch_conv_nq<4, 5, T>(P, u, r, s);
    case 4: return launch_conv_nq<5, 7, T>(P, u, r, s);
    case 5: return launch_conv_nq<6, 8, T>(P, u, r, s);
    case 6: return launch_conv_nq<7, 10, T>(P, u, r, s);
    case 7: return launch_conv_nq<8, 11, T>(P, u, r, s);
    case 8: return launch_conv_nq<9, 13, T>(P, u, r, s);
    case 9: return launch_conv_nq<10, 14, T>(P, u, r, s);
    case 10: return launch_conv_nq<11, 16, T>(P, u, r, s);
    case 11: return launch_conv_nq<12, 17, T>(P, u, r, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_convective(const ConvPlan& P, bool f32, const void* u, void* r, hipStream_t s) {
  return f32 ? launch_conv_t<float>(P, u, r, s) : launch_conv_t<double>(P, u, r, s);
}

}  // namespace dgmf
