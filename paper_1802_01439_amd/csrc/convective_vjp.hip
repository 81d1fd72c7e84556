// Vector-Jacobian product of the convective term: g = J(u)^T w, by sum
// factorisation, FP64 (k <= 7) and FP32 (k <= 9), floor(3k/2)+1 Gauss points.
//
// Linearising R_c = -sum_j s_j (d_j phi, u_c u_j) + faces (Sec. 3.2, weak
// form of c_h) and transposing against the coefficient vector w gives
//   cell:  g_k = (phi, P_k),  P_k = sum_j c_j u_j d_j w_k + c_k sum_c u_c d_k w_c,
//          c_j = -vol/h_j (reference derivatives), W the Gauss weights,
//   faces: g_k += area * (phi, sum_i (w-_i - w+_i) dF*_i/du-_k), with
//          dF*_i/du-_k = 1/2 (delta_ik u-.n + u-_i n_k)
//                      + lf [ L delta_ik + (u-_i - u+_i) s- sign(u-.n) n_k ],
//          L = max(|u-.n|, |u+.n|), s- = 1, 1/2, 0 as |u-.n| >, =, < |u+.n|.
// Each element differentiates only through its own traces u-, so every
// element writes its own coefficients (no atomics).
//
// Sum factorisation: u -> Sx Sy (3 fields), w -> (Sx,Gx) then (Sy,Gy) giving
// the partial fields of d_x w, d_y w and the Sx Sy w field that G_z turns into
// d_z w (9 fields); per (x,y) Gauss pencil the z-direction interpolation, P_k
// and the S^T_z back-contraction run in registers; then S^T_y and S^T_x.
// Faces as in the forward operator: per direction, own/neighbour traces of u
// and w are interpolated to the face Gauss points, combined pointwise and
// integrated back onto the face nodes.
#include "api_internal.h"
#include "common.h"
#include "ops.h"

namespace dgmf {

template <int N, int Q, typename T>
struct VjpTab {
  T S[Q][N];
  T G[Q][N];
  T w[Q];
};

template <typename T>
struct VjpScal {
  T cell[3];   // -vol/h_j
  T area[3];   // vol/h_d
  T lf;
};

template <int N, int Q, typename T>
struct VjpCfg {
  static constexpr int N2 = N * N, N3 = N * N * N;
  static constexpr int RA0 = 6 * N3 + 30 * N * Q;
  static constexpr int RA1 = 12 * Q * Q * N;
  static constexpr int RA2 = 3 * Q * N2;
  static constexpr int RA = RA0 > RA1 ? (RA0 > RA2 ? RA0 : RA2) : (RA1 > RA2 ? RA1 : RA2);
  static constexpr int RB = (9 * Q * N2 > 3 * Q * Q * N) ? 9 * Q * N2 : 3 * Q * Q * N;
  static constexpr int FR = 18 * N2;
  static constexpr int PER_ELEM = RA + RB + FR;
  static constexpr int BUDGET = 80 * 1024 / (int)sizeof(T);
  static constexpr int LDS_MAX = 160 * 1024 / (int)sizeof(T);
  static constexpr int E = (PER_ELEM <= BUDGET) ? (BUDGET / PER_ELEM) : 1;
  static constexpr int THREADS = 256;
  static constexpr bool FITS = E * PER_ELEM <= LDS_MAX;
};

template <int N>
__device__ __forceinline__ int vface_node(int d, int dv, int t1, int t2) {
  return d == 0 ? dv + N * (t1 + N * t2) : (d == 1 ? t1 + N * (dv + N * t2) : t1 + N * (t2 + N * dv));
}

template <int N, int Q, typename T>
__global__ void __launch_bounds__(256)
convective_vjp_kernel(const T* __restrict__ u, const T* __restrict__ wv, T* __restrict__ g,
                      MeshArgs mesh, const VjpTab<N, Q, T>* __restrict__ tab, VjpScal<T> sc) {
  const VjpTab<N, Q, T>& t = *tab;
  using C = VjpCfg<N, Q, T>;
  constexpr int N2 = C::N2, N3 = C::N3, E = C::E, TH = C::THREADS;
  __shared__ T RA[E * C::RA];
  __shared__ T RB[E * C::RB];
  __shared__ T FRb[E * C::FR];

  const int tid = threadIdx.x;
  const int e0 = xcd_remap(blockIdx.x, gridDim.x) * E;
  const int ne = min(E, mesh.n_el - e0);
  const size_t cs = (size_t)mesh.n_el * N3;

  // stage u (fields 0..2) and w (fields 3..5)
  for (int i = tid; i < ne * 6 * N3; i += TH) {
    const int le = i / (6 * N3), rem = i - le * 6 * N3, f = rem / N3, node = rem - f * N3;
    const T* src = f < 3 ? u : wv;
    RA[le * C::RA + f * N3 + node] = src[(f % 3) * cs + (size_t)(e0 + le) * N3 + node];
  }
  __syncthreads();

  // ---------------- faces ----------------
  for (int d = 0; d < 3; ++d) {
    // F1: field f = (kind*2 + side)*3 + c, kind 0 = u, 1 = w; side 0 own, 1 neighbour
    for (int it = tid; it < ne * 24 * N; it += TH) {
      const int le = it / (24 * N);
      int rem = it - le * 24 * N;
      const int j = rem % N;
      rem /= N;
      const int f = rem % 12, s = rem / 12;
      const int c = f % 3, side = (f / 3) % 2, kind = f / 6;
      T in[N];
      if (side == 0) {
        const T* A = RA + le * C::RA + (kind * 3 + c) * N3;
#pragma unroll
        for (int i = 0; i < N; ++i) in[i] = A[vface_node<N>(d, s ? N - 1 : 0, i, j)];
      } else {
        const int e = e0 + le;
        const int ex = e % mesh.nx, ey = (e / mesh.nx) % mesh.ny, ez = e / (mesh.nx * mesh.ny);
        const T* src = (kind == 0 ? u : wv) + c * cs + (size_t)neighbor(mesh, ex, ey, ez, d, s) * N3;
#pragma unroll
        for (int i = 0; i < N; ++i) in[i] = src[vface_node<N>(d, s ? 0 : N - 1, i, j)];
      }
      T* FA = RA + le * C::RA + 6 * N3 + ((s * 12 + f) * N + j) * Q;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        T acc = t.S[q][0] * in[0];
#pragma unroll
        for (int i = 1; i < N; ++i) acc = fmadd(t.S[q][i], in[i], acc);
        FA[q] = acc;
      }
    }
    __syncthreads();
    // F2: per face column q1: along t2, pointwise adjoint flux, back along t2
    for (int it = tid; it < ne * 2 * Q; it += TH) {
      const int le = it / (2 * Q);
      const int rem = it - le * 2 * Q;
      const int s = rem / Q, q1 = rem % Q;
      const T* FA = RA + le * C::RA + 6 * N3 + (s * 12) * N * Q + q1;
      T acc[3][N];
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int j = 0; j < N; ++j) acc[k][j] = 0;
      const T sgn = s ? T(1) : T(-1);
      const T wq1 = t.w[q1] * sc.area[d];
#pragma unroll 1
      for (int q2 = 0; q2 < Q; ++q2) {
        T v[12];
#pragma unroll
        for (int f = 0; f < 12; ++f) {
          T a = 0;
#pragma unroll
          for (int j = 0; j < N; ++j) a = fmadd(t.S[q2][j], FA[(f * N + j) * Q], a);
          v[f] = a;
        }
        // v[0..2] u-, v[3..5] u+, v[6..8] w-, v[9..11] w+
        const T unm = sgn * v[d], unp = sgn * v[3 + d];
        const T am = fabs(unm), ap = fabs(unp);
        const T lam = fmax(am, ap);
        const T sm = am > ap ? T(1) : (am == ap ? T(0.5) : T(0));
        const T sg = unm > 0 ? T(1) : (unm < 0 ? T(-1) : T(0));
        T dw[3], sdu = 0, sdj = 0;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          dw[i] = v[6 + i] - v[9 + i];
          sdu = fmadd(dw[i], v[i], sdu);
          sdj = fmadd(dw[i], v[i] - v[3 + i], sdj);
        }
        const T wgt = wq1 * t.w[q2];
        const T diag = T(0.5) * unm + sc.lf * lam;
        const T extra = sgn * (T(0.5) * sdu + sc.lf * sm * sg * sdj);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const T Gk = wgt * (dw[k] * diag + (k == d ? extra : T(0)));
#pragma unroll
          for (int j = 0; j < N; ++j) acc[k][j] = fmadd(t.S[q2][j], Gk, acc[k][j]);
        }
      }
      T* FB = RA + le * C::RA + 6 * N3 + 24 * N * Q;
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int j = 0; j < N; ++j) FB[((s * 3 + k) * Q + q1) * N + j] = acc[k][j];
    }
    __syncthreads();
    // F3: back along t1 onto the face nodes
    for (int it = tid; it < ne * 6 * N; it += TH) {
      const int le = it / (6 * N);
      int rem = it - le * 6 * N;
      const int j = rem % N;
      rem /= N;
      const int k = rem % 3, s = rem / 3;
      const T* FB = RA + le * C::RA + 6 * N3 + 24 * N * Q + ((s * 3 + k) * Q) * N + j;
      T in[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) in[q] = FB[q * N];
      T* FR = FRb + le * C::FR + ((d * 2 + s) * 3 + k) * N2 + N * j;
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

  // ---------------- cell forward ----------------
  // X: fields XB[0..2] = Sx u_c, XB[3..5] = Sx w_c, XB[6..8] = Gx w_c, layout q1 + Q(b + N cz)
  for (int it = tid; it < ne * 6 * N2; it += TH) {
    const int le = it / (6 * N2);
    const int rem = it - le * 6 * N2;
    const int f = rem / N2, bc = rem - f * N2;
    const T* A = RA + le * C::RA + f * N3 + N * bc;
    T in[N];
#pragma unroll
    for (int a = 0; a < N; ++a) in[a] = A[a];
    T* XB = RB + le * C::RB + Q * bc;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      T sv = t.S[q][0] * in[0], gv = t.G[q][0] * in[0];
#pragma unroll
      for (int a = 1; a < N; ++a) {
        sv = fmadd(t.S[q][a], in[a], sv);
        gv = fmadd(t.G[q][a], in[a], gv);
      }
      XB[f * Q * N2 + q] = sv;
      if (f >= 3) XB[(f + 3) * Q * N2 + q] = gv;
    }
  }
  __syncthreads();
  // Y: YC fields (layout q1 + Q(q2 + Q cz)):
  //   0..2 Sy Sx u_c; 3..5 Sy Sx w_c (-> d_z w); 6..8 Gy Sx w_c (d_y w); 9..11 Sy Gx w_c (d_x w)
  for (int it = tid; it < ne * 9 * Q * N; it += TH) {
    const int le = it / (9 * Q * N);
    int rem = it - le * 9 * Q * N;
    const int f = rem / (Q * N);
    rem -= f * Q * N;
    const int cz = rem / Q, q1 = rem - cz * Q;
    const T* XB = RB + le * C::RB + f * Q * N2 + q1 + Q * N * cz;
    T in[N];
#pragma unroll
    for (int b = 0; b < N; ++b) in[b] = XB[Q * b];
    T* YC = RA + le * C::RA + q1 + Q * Q * cz;
    // f 0..2 -> out 0..2 (S); f 3..5 -> out 3..5 (S) and 6..8 (G); f 6..8 -> out 9..11 (S)
    const int fo = f < 3 ? f : (f < 6 ? f : f + 3);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      T sv = t.S[q][0] * in[0], gv = t.G[q][0] * in[0];
#pragma unroll
      for (int b = 1; b < N; ++b) {
        sv = fmadd(t.S[q][b], in[b], sv);
        gv = fmadd(t.G[q][b], in[b], gv);
      }
      YC[fo * Q * Q * N + Q * q] = sv;
      if (f >= 3 && f < 6) YC[(f + 3) * Q * Q * N + Q * q] = gv;
    }
  }
  __syncthreads();
  // Z (fused): per (q1,q2) pencil: values at z Gauss points, P_k, S^T_z -> ZT[k] in RB
  for (int it = tid; it < ne * Q * Q; it += TH) {
    const int le = it / (Q * Q), qq = it - le * Q * Q;
    const int q2 = qq / Q, q1 = qq - q2 * Q;
    const T* YC = RA + le * C::RA + qq;
    T o[3][N];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int cz = 0; cz < N; ++cz) o[k][cz] = 0;
    const T w12 = t.w[q1] * t.w[q2];
#pragma unroll 1
    for (int q3 = 0; q3 < Q; ++q3) {
      T uu[3], dx[3], dy[3], dz[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll
        for (int cz = 0; cz < N; ++cz) {
          const T sq = t.S[q3][cz];
          a0 = fmadd(sq, YC[(0 + c) * Q * Q * N + Q * Q * cz], a0);
          a1 = fmadd(sq, YC[(9 + c) * Q * Q * N + Q * Q * cz], a1);
          a2 = fmadd(sq, YC[(6 + c) * Q * Q * N + Q * Q * cz], a2);
          a3 = fmadd(t.G[q3][cz], YC[(3 + c) * Q * Q * N + Q * Q * cz], a3);
        }
        uu[c] = a0;
        dx[c] = a1;
        dy[c] = a2;
        dz[c] = a3;
      }
      const T wq = w12 * t.w[q3];
      const T cu[3] = {sc.cell[0] * uu[0], sc.cell[1] * uu[1], sc.cell[2] * uu[2]};
      // sum_c u_c d_k w_c for k = x, y, z
      const T ux = uu[0] * dx[0] + uu[1] * dx[1] + uu[2] * dx[2];
      const T uy = uu[0] * dy[0] + uu[1] * dy[1] + uu[2] * dy[2];
      const T uz = uu[0] * dz[0] + uu[1] * dz[1] + uu[2] * dz[2];
      T P[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) P[k] = cu[0] * dx[k] + cu[1] * dy[k] + cu[2] * dz[k];
      P[0] += sc.cell[0] * ux;
      P[1] += sc.cell[1] * uy;
      P[2] += sc.cell[2] * uz;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const T pk = wq * P[k];
#pragma unroll
        for (int cz = 0; cz < N; ++cz) o[k][cz] = fmadd(t.S[q3][cz], pk, o[k][cz]);
      }
    }
    T* ZT = RB + le * C::RB + qq;
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int cz = 0; cz < N; ++cz) ZT[k * Q * Q * N + Q * Q * cz] = o[k][cz];
  }
  __syncthreads();
  // back Y: V[k][q1 + Q(b + N cz)] = S^T_y ZT[k]
  for (int it = tid; it < ne * 3 * Q * N; it += TH) {
    const int le = it / (3 * Q * N);
    int rem = it - le * 3 * Q * N;
    const int k = rem / (Q * N);
    rem -= k * Q * N;
    const int cz = rem / Q, q1 = rem - cz * Q;
    const T* ZT = RB + le * C::RB + k * Q * Q * N + q1 + Q * Q * cz;
    T in[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) in[q] = ZT[Q * q];
    T* V = RA + le * C::RA + k * Q * N2 + q1 + Q * N * cz;
#pragma unroll
    for (int b = 0; b < N; ++b) {
      T acc = t.S[0][b] * in[0];
#pragma unroll
      for (int q = 1; q < Q; ++q) acc = fmadd(t.S[q][b], in[q], acc);
      V[Q * b] = acc;
    }
  }
  __syncthreads();
  // back X + faces: g_k = S^T_x V[k] + face terms, written once
  for (int it = tid; it < ne * 3 * N2; it += TH) {
    const int le = it / (3 * N2);
    const int rem = it - le * 3 * N2;
    const int k = rem / N2, bc = rem - k * N2;
    const int b = bc % N, cz = bc / N;
    const T* V = RA + le * C::RA + k * Q * N2 + Q * bc;
    T in[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) in[q] = V[q];
    T o[N];
#pragma unroll
    for (int a = 0; a < N; ++a) {
      T acc = t.S[0][a] * in[0];
#pragma unroll
      for (int q = 1; q < Q; ++q) acc = fmadd(t.S[q][a], in[q], acc);
      o[a] = acc;
    }
    const T* FR = FRb + le * C::FR;
    o[0] += FR[((0 * 2 + 0) * 3 + k) * N2 + b + N * cz];
    o[N - 1] += FR[((0 * 2 + 1) * 3 + k) * N2 + b + N * cz];
    if (b == 0 || b == N - 1) {
      const T* F = FR + ((1 * 2 + (b == 0 ? 0 : 1)) * 3 + k) * N2 + N * cz;
#pragma unroll
      for (int a = 0; a < N; ++a) o[a] += F[a];
    }
    if (cz == 0 || cz == N - 1) {
      const T* F = FR + ((2 * 2 + (cz == 0 ? 0 : 1)) * 3 + k) * N2 + N * b;
#pragma unroll
      for (int a = 0; a < N; ++a) o[a] += F[a];
    }
    T* out = g + k * cs + (size_t)(e0 + le) * N3 + N * bc;
#pragma unroll
    for (int a = 0; a < N; ++a) out[a] = o[a];
  }
}

template <int N, int Q, typename T>
static hipError_t launch_vjp_nq(const ConvPlan& P, const void* u, const void* w, void* g,
                                hipStream_t s) {
  using C = VjpCfg<N, Q, T>;
  if constexpr (!C::FITS) {
    return hipErrorInvalidConfiguration;
  } else {
    VjpTab<N, Q, T> t;
    for (int q = 0; q < Q; ++q) {
      for (int a = 0; a < N; ++a) {
        t.S[q][a] = (T)P.S[q * N + a];
        t.G[q][a] = (T)P.G[q * N + a];
      }
      t.w[q] = (T)P.w[q];
    }
    VjpScal<T> sc;
    for (int d = 0; d < 3; ++d) {
      sc.cell[d] = (T)P.cell[d];
      sc.area[d] = (T)P.area[d];
    }
    sc.lf = (T)P.lf;
    hipError_t err;
    const VjpTab<N, Q, T>* dt = device_table_of("convective_vjp", t, &err);
    if (!dt) return err;
    const int grid = (P.mesh.n_el + C::E - 1) / C::E;
    hipLaunchKernelGGL((convective_vjp_kernel<N, Q, T>), dim3(grid), dim3(C::THREADS), 0, s,
                       (const T*)u, (const T*)w, (T*)g, P.mesh, dt, sc);
    return hipGetLastError();
  }
}

template <typename T>
static hipError_t launch_vjp_t(const ConvPlan& P, const void* u, const void* w, void* g,
                               hipStream_t s) {
  switch (P.k) {
    case 1: return launch_vjp_nq<2, 2, T>(P, u, w, g, s);
    case 2: return launch_vjp_nq<3, 4, T>(P, u, w, g, s);
    case 3: return launch_vjp_nq<4, 5, T>(P, u, w, g, s);
    case 4: return launch_vjp_nq<5, 7, T>(P, u, w, g, s);
    case 5: return launch_vjp_nq<6, 8, T>(P, u, w, g, s);
    case 6: return launch_vjp_nq<7, 10, T>(P, u, w, g, s);
    case 7: return launch_vjp_nq<8, 11, T>(P, u, w, g, s);
    case 8: return launch_vjp_nq<9, 13, T>(P, u, w, g, s);
    case 9: return launch_vjp_nq<10, 14, T>(P, u, w, g, s);
    default: return hipErrorInvalidConfiguration;
  }
}

int vjp_max_degree(bool f32) { return f32 ? 9 : 7; }

hipError_t launch_convective_vjp(const ConvPlan& P, bool f32, const void* u, const void* w,
                                 void* g, hipStream_t s) {
  return f32 ? launch_vjp_t<float>(P, u, w, g, s) : launch_vjp_t<double>(P, u, w, g, s);
}

}  // namespace dgmf
