// Level transfers of the h-multigrid hierarchy (Sec. 3.3: geometric
// multigrid with matrix-free transfers), FP64 and FP32, degrees 1..11.
//
// The fine mesh splits every element of the coarse one in two per direction
// (same degree).  Prolongation embeds the coarse DG space: the fine element
// with child index (cx, cy, cz) gets
//   u_f = (P_cx (x) P_cy (x) P_cz) u_parent,   P_c[i][a] = l_a((xi_i + c)/2);
// restriction is the transpose, summed over the eight children:
//   r_c = sum_children (P_cx^T (x) P_cy^T (x) P_cz^T) r_child.
// Element-local apart from the parent/child gather; memory bound.
//
// Both run one workgroup per batch of E = floor(256/n^2) coarse elements,
// n^2 threads each, and loop over the eight children, so the child's 1D
// matrices are uniform (scalar loads).  Prolongation: the parent's column is
// read once into registers; per child the z sweep runs on it, the y and x
// sweeps on LDS pencils in place, and the child's z columns are stored
// (3 barriers per child).  Where that launch would have fewer than 1024
// workgroups (about four per CU: the coarse levels of a V-cycle, the high
// degrees) the eight children of a batch go to eight workgroups instead,
// which shortens each workgroup's chain of barriers eightfold; the parent's
// column is then read by each of them (from L2: they run on one XCD).  Restriction: per child a z sweep from the child's
// column, a y sweep in LDS, and an x sweep whose result each thread
// accumulates in registers for its own x pencil of the coarse element
// (3 barriers per child).
#include "api_internal.h"
#include "common.h"
#include "laplace_kernels.h"
#include "ops.h"

namespace dgmf {

namespace {

// The restriction applies P transposed: with R it walks rows in memory order,
// as the prolongation does with P.  Walking P by columns made the compiler
// keep the whole table in scalar registers, which spilled into vector lanes
// at n = 9..12 in FP64 (the FP64 restriction at n = 9 and 11 ran 2.2-2.6x
// slower).
template <int N, typename T>
struct TransferTab {
  T P[2][N][N];   // P[c][i][a] = l_a((xi_i + c)/2)
  T R[2][N][N];   // R[c][a][i] = P[c][i][a]
};

struct LevelArgs {
  int nxc, nyc, nzc;   // coarse elements per direction (fine: twice as many)
  long long ncoarse;   // nxc * nyc * nzc
};

// ACC: uf += the prolongation (the coarse-grid correction of a V-cycle)
// instead of uf = it.
template <int N, typename T, bool CP, bool ACC>
__global__ void __launch_bounds__(LapCfgB<N>::THREADS)
prolongate_kernel(const T* __restrict__ uc, T* __restrict__ uf, LevelArgs lv,
                  const TransferTab<N, T>* __restrict__ tab) {
  using C = LapCfgB<N>;
  constexpr int N2 = N * N, N3 = N * N * N, E = C::E, ES = C::ES, PX = C::PX, PY = C::PY;
  __shared__ T U[E * ES];
  const int tid = threadIdx.x;
  const int le = tid / N2, p = tid - le * N2;
  const int p0 = p % N, p1 = p / N;
  // CP: one child per workgroup, logical id = batch * 8 + child, so that
  // the eight children of a batch run on one XCD
  const int lid = xcd_remap(blockIdx.x, gridDim.x);
  const int ch0 = CP ? (lid & 7) : 0, ch1 = CP ? ch0 + 1 : 8;
  const long long e = (long long)(CP ? lid >> 3 : lid) * E + le;
  const bool active = e < lv.ncoarse;
  const int comp = blockIdx.y;
  const long long nfine = 8 * lv.ncoarse;
  const int nxf = 2 * lv.nxc, nyf = 2 * lv.nyc;
  int ex = 0, ey = 0, ez = 0;
  T xp[N], x[N], y[N];
  if (active) {
    ez = (int)(e / ((long long)lv.nxc * lv.nyc));
    const long long r = e - (long long)ez * lv.nxc * lv.nyc;
    ey = (int)(r / lv.nxc);
    ex = (int)(r - (long long)ey * lv.nxc);
    // the parent's column (a, b) = (p0, p1), read once for this workgroup's children
    const T* g = uc + (size_t)comp * lv.ncoarse * N3 + (size_t)e * N3 + p0 + N * p1;
#pragma unroll
    for (int c = 0; c < N; ++c) xp[c] = g[N2 * c];
  }
  T* Ue = U + le * ES;
  for (int ch = ch0; ch < ch1; ++ch) {
    const int cx = ch & 1, cy = (ch >> 1) & 1, cz = ch >> 2;
    // z: P_cz on the parent column in registers.  The previous child's store
    // read only this thread's own column, so no barrier is needed before it.
    if (active) {
      const int base = p0 + PX * p1;
#pragma unroll
      for (int l = 0; l < N; ++l) {
        T s = tab->P[cz][l][0] * xp[0];
#pragma unroll
        for (int c = 1; c < N; ++c) s = fmadd(tab->P[cz][l][c], xp[c], s);
        Ue[base + PY * l] = s;
      }
    }
    __syncthreads();
    // y: pencil (a, l) = (p0, p1), P_cy, in place
    if (active) {
      const int base = p0 + PY * p1;
#pragma unroll
      for (int b = 0; b < N; ++b) x[b] = Ue[base + PX * b];
#pragma unroll
      for (int j = 0; j < N; ++j) {
        T s = tab->P[cy][j][0] * x[0];
#pragma unroll
        for (int b = 1; b < N; ++b) s = fmadd(tab->P[cy][j][b], x[b], s);
        y[j] = s;
      }
#pragma unroll
      for (int j = 0; j < N; ++j) Ue[base + PX * j] = y[j];
    }
    __syncthreads();
    // x: pencil (j, l) = (p0, p1), P_cx, in place
    if (active) {
      const int base = PX * p0 + PY * p1;
#pragma unroll
      for (int a = 0; a < N; ++a) x[a] = Ue[base + a];
#pragma unroll
      for (int i = 0; i < N; ++i) {
        T s = tab->P[cx][i][0] * x[0];
#pragma unroll
        for (int a = 1; a < N; ++a) s = fmadd(tab->P[cx][i][a], x[a], s);
        y[i] = s;
      }
#pragma unroll
      for (int i = 0; i < N; ++i) Ue[base + i] = y[i];
    }
    __syncthreads();
    // store the child's z column (i, j) = (p0, p1)
    if (active) {
      const long long f = (2 * ex + cx) + (long long)nxf * ((2 * ey + cy) + (long long)nyf * (2 * ez + cz));
      T* g = uf + (size_t)comp * nfine * N3 + (size_t)f * N3 + p0 + N * p1;
      const int base = p0 + PX * p1;
#pragma unroll
      for (int l = 0; l < N; ++l) {
        if constexpr (ACC) g[N2 * l] += Ue[base + PY * l];
        else g[N2 * l] = Ue[base + PY * l];
      }
    }
  }
}

// First step of a zero-start Chebyshev smoother on the coarse level, taken
// in the restriction's store: d = x = s D^-1 r_c (one component).
template <typename T>
struct ChebFirst {
  const T* dinv;   // D^-1 at the n^3 nodes, the same in every element
  T s;             // 1 / theta
  T* d;
  T* x;
};

template <int N, typename T, bool CF>
__global__ void __launch_bounds__(LapCfgB<N>::THREADS)
restrict_kernel(const T* __restrict__ rf, T* __restrict__ rc, LevelArgs lv,
                const TransferTab<N, T>* __restrict__ tab, ChebFirst<T> cf) {
  using C = LapCfgB<N>;
  constexpr int N2 = N * N, N3 = N * N * N, E = C::E, ES = C::ES, PX = C::PX, PY = C::PY;
  __shared__ T U[E * ES];
  const int tid = threadIdx.x;
  const int le = tid / N2, p = tid - le * N2;
  const int p0 = p % N, p1 = p / N;
  const long long e = (long long)xcd_remap(blockIdx.x, gridDim.x) * E + le;
  const bool active = e < lv.ncoarse;
  const int comp = blockIdx.y;
  const long long nfine = 8 * lv.ncoarse;
  const int nxf = 2 * lv.nxc, nyf = 2 * lv.nyc;
  int ex = 0, ey = 0, ez = 0;
  if (active) {
    ez = (int)(e / ((long long)lv.nxc * lv.nyc));
    const long long r = e - (long long)ez * lv.nxc * lv.nyc;
    ey = (int)(r / lv.nxc);
    ex = (int)(r - (long long)ey * lv.nxc);
  }
  T* Ue = U + le * ES;
  T x[N], y[N], acc[N];
#pragma unroll
  for (int a = 0; a < N; ++a) acc[a] = 0;
  for (int ch = 0; ch < 8; ++ch) {
    const int cx = ch & 1, cy = (ch >> 1) & 1, cz = ch >> 2;
    // z: the child's column (i, j) = (p0, p1), P_cz^T
    if (active) {
      const long long f = (2 * ex + cx) + (long long)nxf * ((2 * ey + cy) + (long long)nyf * (2 * ez + cz));
      const T* g = rf + (size_t)comp * nfine * N3 + (size_t)f * N3 + p0 + N * p1;
#pragma unroll
      for (int l = 0; l < N; ++l) x[l] = g[N2 * l];
#pragma unroll
      for (int c = 0; c < N; ++c) {
        T s = tab->R[cz][c][0] * x[0];
#pragma unroll
        for (int l = 1; l < N; ++l) s = fmadd(tab->R[cz][c][l], x[l], s);
        y[c] = s;
      }
      const int base = p0 + PX * p1;
#pragma unroll
      for (int c = 0; c < N; ++c) Ue[base + PY * c] = y[c];
    }
    __syncthreads();
    // y: pencil (i, c) = (p0, p1), P_cy^T, in place
    if (active) {
      const int base = p0 + PY * p1;
#pragma unroll
      for (int j = 0; j < N; ++j) x[j] = Ue[base + PX * j];
#pragma unroll
      for (int b = 0; b < N; ++b) {
        T s = tab->R[cy][b][0] * x[0];
#pragma unroll
        for (int j = 1; j < N; ++j) s = fmadd(tab->R[cy][b][j], x[j], s);
        y[b] = s;
      }
#pragma unroll
      for (int b = 0; b < N; ++b) Ue[base + PX * b] = y[b];
    }
    __syncthreads();
    // x: pencil (b, c) = (p0, p1), P_cx^T, accumulated in registers
    if (active) {
      const int base = PX * p0 + PY * p1;
#pragma unroll
      for (int i = 0; i < N; ++i) x[i] = Ue[base + i];
#pragma unroll
      for (int a = 0; a < N; ++a) {
        T s = tab->R[cx][a][0] * x[0];
#pragma unroll
        for (int i = 1; i < N; ++i) s = fmadd(tab->R[cx][a][i], x[i], s);
        acc[a] += s;
      }
    }
    __syncthreads();
  }
  // store the coarse x pencil (b, c) = (p0, p1)
  if (active) {
    const size_t o = (size_t)comp * lv.ncoarse * N3 + (size_t)e * N3 + N * p0 + N2 * p1;
#pragma unroll
    for (int a = 0; a < N; ++a) {
      rc[o + a] = acc[a];
      if constexpr (CF) {
        const T v = cf.s * cf.dinv[N * p0 + N2 * p1 + a] * acc[a];
        cf.d[o + a] = v;
        cf.x[o + a] = v;
      }
    }
  }
}

template <int N, typename T, bool ACC>
hipError_t launch_prolong(const TransferPlan& P, const void* src, void* dst, long long grid, const TransferTab<N, T>* dt,
                          LevelArgs lv, hipStream_t s) {
  using C = LapCfgB<N>;
  // one child per workgroup below 1024 workgroups (measured: the V-cycle
  // BDF2 step at k = 7, 24^3 1.5 % faster, the prolongation at k = 8, 10, 11
  // on the sweep meshes 3-22 %; on larger grids the loop is 0-60 % faster)
  if (grid * P.n_comp < 1024)
    hipLaunchKernelGGL((prolongate_kernel<N, T, true, ACC>), dim3((unsigned)(8 * grid), (unsigned)P.n_comp),
                       dim3(C::THREADS), 0, s, (const T*)src, (T*)dst, lv, dt);
  else
    hipLaunchKernelGGL((prolongate_kernel<N, T, false, ACC>), dim3((unsigned)grid, (unsigned)P.n_comp),
                       dim3(C::THREADS), 0, s, (const T*)src, (T*)dst, lv, dt);
  return hipGetLastError();
}

struct ChebFirstArgs {
  const void* dinv;
  double s;
  void* d;
  void* x;
};

template <int N, typename T>
hipError_t launch_n(const TransferPlan& P, int mode, const void* src, void* dst, const ChebFirstArgs* cfa,
                    hipStream_t s) {
  TransferTab<N, T> t;
  for (int c = 0; c < 2; ++c)
    for (int i = 0; i < N; ++i)
      for (int a = 0; a < N; ++a) t.R[c][a][i] = t.P[c][i][a] = (T)P.P[c][i * N + a];
  hipError_t err;
  const TransferTab<N, T>* dt = device_table_of("transfer", t, &err);
  if (!dt) return err;
  LevelArgs lv{P.nxc, P.nyc, P.nzc, (long long)P.nxc * P.nyc * P.nzc};
  using C = LapCfgB<N>;
  const long long grid = (lv.ncoarse + C::E - 1) / C::E;
  if (8 * grid > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  if (grid == 0) return hipSuccess;
  if (mode == 1) return launch_prolong<N, T, false>(P, src, dst, grid, dt, lv, s);
  if (mode == 2) return launch_prolong<N, T, true>(P, src, dst, grid, dt, lv, s);
  const dim3 g((unsigned)grid, (unsigned)P.n_comp);
  if (mode == 3) {
    if (P.n_comp != 1 || !cfa) return hipErrorInvalidValue;
    const ChebFirst<T> cf{(const T*)cfa->dinv, (T)cfa->s, (T*)cfa->d, (T*)cfa->x};
    hipLaunchKernelGGL((restrict_kernel<N, T, true>), g, dim3(C::THREADS), 0, s, (const T*)src, (T*)dst, lv, dt, cf);
  } else {
    hipLaunchKernelGGL((restrict_kernel<N, T, false>), g, dim3(C::THREADS), 0, s, (const T*)src, (T*)dst, lv, dt,
                       ChebFirst<T>{});
  }
  return hipGetLastError();
}

// mode 0: restriction, 1: prolongation, 2: prolongation added to dst,
// 3: restriction and the first Chebyshev step on the coarse level
template <typename T>
hipError_t launch_t(const TransferPlan& P, int mode, const void* src, void* dst, const ChebFirstArgs* cf,
                    hipStream_t s) {
  switch (P.k) {
    case 1: return launch_n<2, T>(P, mode, src, dst, cf, s);
    case 2: return launch_n<3, T>(P, mode, src, dst, cf, s);
    case 3: return launch_n<4, T>(P, mode, src, dst, cf, s);
    case 4: return launch_n<5, T>(P, mode, src, dst, cf, s);
    case 5: return launch_n<6, T>(P, mode, src, dst, cf, s);
    case 6: return launch_n<7, T>(P, mode, src, dst, cf, s);
    case 7: return launch_n<8, T>(P, mode, src, dst, cf, s);
    case 8: return launch_n<9, T>(P, mode, src, dst, cf, s);
    case 9: return launch_n<10, T>(P, mode, src, dst, cf, s);
    case 10: return launch_n<11, T>(P, mode, src, dst, cf, s);
    case 11: return launch_n<12, T>(P, mode, src, dst, cf, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_transfer(const TransferPlan& P, bool prolong, bool f32, const void* src, void* dst,
                           hipStream_t s) {
  const int mode = prolong ? 1 : 0;
  return f32 ? launch_t<float>(P, mode, src, dst, nullptr, s) : launch_t<double>(P, mode, src, dst, nullptr, s);
}

hipError_t launch_prolongate_add(const TransferPlan& P, bool f32, const void* src, void* dst, hipStream_t s) {
  return f32 ? launch_t<float>(P, 2, src, dst, nullptr, s) : launch_t<double>(P, 2, src, dst, nullptr, s);
}

hipError_t launch_restrict_cheb_first(const TransferPlan& P, bool f32, const void* rf, void* rc, const void* dinv,
                                      double scale, void* d, void* x, hipStream_t s) {
  const ChebFirstArgs cf{dinv, scale, d, x};
  return f32 ? launch_t<float>(P, 3, rf, rc, &cf, s) : launch_t<double>(P, 3, rf, rc, &cf, s);
}

}  // namespace dgmf
