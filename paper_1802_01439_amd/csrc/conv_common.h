// Pieces shared by the convective kernel and its vector-Jacobian product:
// the 1D tables of the LGL basis at the Gauss points in even-odd form, where
// the kernels read them from, and the 1D sweeps.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "basis_ct.h"
#include "common.h"

namespace dgmf {

// Workgroup barrier for LDS traffic only: waits for this wave's LDS (and
// scalar) operations, not for its global loads, so loads issued before it
// stay in flight across it.  The memory clobber keeps the compiler from
// moving shared-memory accesses across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Index of the first item of a second kind of work that follows n0 items
// of a first kind in a loop over items by th threads: the next wavefront
// boundary when that adds no round of th items, so that no wavefront runs the
// (divergent) code of both kinds one after the other.
constexpr int wave_split(int n0, int n1, int th) {
  const int p = (n0 + 63) / 64 * 64;
  return (p + n1 + th - 1) / th == (n0 + n1 + th - 1) / th ? p : n0;
}

// 1D tables in even-odd form.  The LGL nodes and the Gauss points are
// symmetric about 1/2, so S[m-1-q][n-1-a] = S[q][a] and
// G[m-1-q][n-1-a] = -G[q][a].  With x_e[a] = x[a] + x[n-1-a] and
// x_o[a] = x[a] - x[n-1-a] (a < n/2):
//   y = S x:      y[q] = E_q + O_q,  y[m-1-q] = E_q - O_q   (q < ceil(m/2))
//                 E_q = sum_a Sp[q][a] x_e[a] + Sc[q] x[n/2] (n odd),
//                 O_q = sum_a Sm[q][a] x_o[a],
//                 Sp/Sm = half sum/difference of S[q][a] and S[q][n-1-a];
//   y = A^T x     (A = S, sign +1; A = G, sign -1), inputs taken in mirrored
//                 pairs (x[q], x[m-1-q]), q < m/2, and the middle x[m/2]:
//                 y[a] = E_a + O_a,  y[n-1-a] = sign (E_a - O_a)  (a < ceil(n/2)),
//                 E_a = sum_q Tp[q][a] (x[q] + x[m-1-q]) + Tc[a] x[m/2] (m odd),
//                 O_a = sum_q Tm[q][a] (x[q] - x[m-1-q]),
//                 Tp/Tm = half sum/difference of A[q][a] and A[m-1-q][a];
//   y = G x:      as for S with Gp/Gm/Gc, except y[m-1-q] = O_q - E_q.
// Each sweep thus takes about half the multiply-adds of the plain product.
template <int N, int Q, typename T>
struct ConvTab {
  static constexpr int NH = N / 2, NC = (N + 1) / 2, QH = Q / 2, QC = (Q + 1) / 2;
  T Sp[QC][NH], Sm[QC][NH], Sc[QC];   // S, rows q < ceil(m/2)
  T Gp[QC][NH], Gm[QC][NH], Gc[QC];   // G, rows q < ceil(m/2)
  T Tp[QH][NC], Tm[QH][NC], Tc[NC];   // S^T, by input pair q < m/2
  T Hp[QH][NC], Hm[QH][NC], Hc[NC];   // G^T, by input pair q < m/2
  T w[Q];                             // Gauss weights on [0,1]
};

// Even-odd tables from plain row-major S, G (m x n) and w.
template <int N, int Q, typename T>
constexpr ConvTab<N, Q, T> make_conv_tab(const double* S, const double* G, const double* w) {
  using Tb = ConvTab<N, Q, T>;
  Tb t{};
  for (int q = 0; q < Tb::QC; ++q) {
    for (int a = 0; a < Tb::NH; ++a) {
      t.Sp[q][a] = (T)(0.5 * (S[q * N + a] + S[q * N + N - 1 - a]));
      t.Sm[q][a] = (T)(0.5 * (S[q * N + a] - S[q * N + N - 1 - a]));
    }
    t.Sc[q] = (N % 2) ? (T)S[q * N + Tb::NH] : T(0);
    for (int a = 0; a < Tb::NH; ++a) {
      t.Gp[q][a] = (T)(0.5 * (G[q * N + a] + G[q * N + N - 1 - a]));
      t.Gm[q][a] = (T)(0.5 * (G[q * N + a] - G[q * N + N - 1 - a]));
    }
    t.Gc[q] = (N % 2) ? (T)G[q * N + Tb::NH] : T(0);
  }
  for (int q = 0; q < Tb::QH; ++q)
    for (int a = 0; a < Tb::NC; ++a) {
      t.Tp[q][a] = (T)(0.5 * (S[q * N + a] + S[(Q - 1 - q) * N + a]));
      t.Tm[q][a] = (T)(0.5 * (S[q * N + a] - S[(Q - 1 - q) * N + a]));
      t.Hp[q][a] = (T)(0.5 * (G[q * N + a] + G[(Q - 1 - q) * N + a]));
      t.Hm[q][a] = (T)(0.5 * (G[q * N + a] - G[(Q - 1 - q) * N + a]));
    }
  for (int a = 0; a < Tb::NC; ++a) {
    t.Tc[a] = (Q % 2) ? (T)S[Tb::QH * N + a] : T(0);
    t.Hc[a] = (Q % 2) ? (T)G[Tb::QH * N + a] : T(0);
  }
  for (int q = 0; q < Q; ++q) t.w[q] = (T)w[q];
  return t;
}

// The tables of degree N-1 with Q Gauss points as compile-time constants.
template <int N, int Q, typename T>
constexpr ConvTab<N, Q, T> conv_tab_ct() {
  constexpr ct::Tables<N, Q> d{};
  double S[Q * N] = {}, G[Q * N] = {};
  for (int q = 0; q < Q; ++q)
    for (int a = 0; a < N; ++a) {
      S[q * N + a] = d.S[q][a];
      G[q * N + a] = d.G[q][a];
    }
  return make_conv_tab<N, Q, T>(S, G, d.w);
}

// Where the kernels read the tables from.  FP32: compile-time constants, which
// become literal operands of the FMAs.  FP64: a table in device memory read
// through fresh() (common.h) in every phase (64-bit constants would each take
// a scalar register pair and spill at high degree).
template <int N, int Q, typename T>
__device__ __forceinline__ decltype(auto) conv_pick(const ConvTab<N, Q, T>& ct, const ConvTab<N, Q, T>* tab) {
  if constexpr (sizeof(T) == 4) return (ct);
  else return *fresh(tab);
}

// Declares `t`, the tables of the current phase.  The compile-time copy is a
// constexpr local so that its entries fold into the instructions.
#define CONV_TABLES(t)                                              \
  constexpr ConvTab<N, Q, T> t##_ct =                               \
      sizeof(T) == 4 ? conv_tab_ct<N, Q, T>() : ConvTab<N, Q, T>{}; \
  const auto& t = conv_pick<N, Q, T>(t##_ct, tab)

template <typename T>
struct ConvScal {
  T cell[3];   // -vol/h_j
  T area[3];   // vol/h_d
  T lf;
};

template <int N, int Q, typename T>
__device__ __forceinline__ void load_pencil(const T* __restrict__ p, int stride, T (&in)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) in[i] = p[i * stride];
}

// A pencil of n contiguous values in 16-byte loads; n values fill whole
// 16-byte words and p is 16-byte aligned (the caller guarantees both).
template <int N, typename T>
__device__ __forceinline__ void load_pencil16(const T* __restrict__ p, T (&in)[N]) {
  constexpr int V = 16 / (int)sizeof(T);
  static_assert((N * sizeof(T)) % 16 == 0, "pencil does not fill whole 16-byte words");
  typedef T vec __attribute__((ext_vector_type(V)));
  const vec* q = reinterpret_cast<const vec*>(__builtin_assume_aligned(p, 16));
#pragma unroll
  for (int i = 0; i < N / V; ++i) {
    const vec x = q[i];
#pragma unroll
    for (int c = 0; c < V; ++c) in[i * V + c] = x[c];
  }
}

// load_pencil, in 16-byte loads where they apply: n values fill whole 16-byte
// words, the pencil is contiguous (stride 1) and a16 says it is 16-byte aligned.
template <int N, int Q, typename T>
__device__ __forceinline__ void load_pencil_a16(const T* __restrict__ p, int stride, bool a16, T (&in)[N]) {
  if constexpr ((N * sizeof(T)) % 16 == 0) {
    if (a16 && stride == 1) {
      load_pencil16<N, T>(p, in);
      return;
    }
  }
  load_pencil<N, Q, T>(p, stride, in);
}

// y = S x in even-odd form; st(q, y[q]) receives every output.
template <int N, int Q, typename T, typename Tab, typename St>
__device__ __forceinline__ void eo_interp(const Tab& t, const T (&x)[N], St&& st) {
  constexpr int NH = N / 2, QH = Q / 2, QC = (Q + 1) / 2;
  T xe[NH], xo[NH];
#pragma unroll
  for (int a = 0; a < NH; ++a) {
    xe[a] = x[a] + x[N - 1 - a];
    xo[a] = x[a] - x[N - 1 - a];
  }
#pragma unroll
  for (int q = 0; q < QC; ++q) {
    T e = t.Sp[q][0] * xe[0], o = t.Sm[q][0] * xo[0];
#pragma unroll
    for (int a = 1; a < NH; ++a) {
      e = fmadd(t.Sp[q][a], xe[a], e);
      o = fmadd(t.Sm[q][a], xo[a], o);
    }
    if constexpr (N % 2 == 1) e = fmadd(t.Sc[q], x[NH], e);
    st(q, e + o);
    if (q < QH) st(Q - 1 - q, e - o);
  }
}

// y = G x in even-odd form (the derivatives of the LGL basis at the Gauss
// points); st(q, y[q]) receives every output.
template <int N, int Q, typename T, typename Tab, typename St>
__device__ __forceinline__ void eo_interp_g(const Tab& t, const T (&x)[N], St&& st) {
  constexpr int NH = N / 2, QH = Q / 2, QC = (Q + 1) / 2;
  T xe[NH], xo[NH];
#pragma unroll
  for (int a = 0; a < NH; ++a) {
    xe[a] = x[a] + x[N - 1 - a];
    xo[a] = x[a] - x[N - 1 - a];
  }
#pragma unroll
  for (int q = 0; q < QC; ++q) {
    T e = t.Gp[q][0] * xe[0], o = t.Gm[q][0] * xo[0];
#pragma unroll
    for (int a = 1; a < NH; ++a) {
      e = fmadd(t.Gp[q][a], xe[a], e);
      o = fmadd(t.Gm[q][a], xo[a], o);
    }
    if constexpr (N % 2 == 1) e = fmadd(t.Gc[q], x[NH], e);
    st(q, e + o);
    if (q < QH) st(Q - 1 - q, o - e);
  }
}

// y = A^T x in even-odd form (A = S: SIGN = +1, A = G: SIGN = -1), fed with
// mirrored input pairs and, for odd m, the middle input.
template <int N, typename T, int SIGN>
struct EoT {
  static constexpr int NH = N / 2, NC = (N + 1) / 2;
  T e[NC], o[NC];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int a = 0; a < NC; ++a) e[a] = o[a] = T(0);
  }
  template <typename Row>
  __device__ __forceinline__ void pair(const Row& p, const Row& m, T xq, T xr) {
    const T xe = xq + xr, xo = xq - xr;
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      e[a] = fmadd(p[a], xe, e[a]);
      o[a] = fmadd(m[a], xo, o[a]);
    }
  }
  template <typename Row>
  __device__ __forceinline__ void mid(const Row& c, T x) {
#pragma unroll
    for (int a = 0; a < NC; ++a) e[a] = fmadd(c[a], x, e[a]);
  }
  // output a (a compile-time index after unrolling)
  __device__ __forceinline__ T out(int a) const {
    if (a < NC) return e[a] + o[a];
    const int b = N - 1 - a;
    return SIGN > 0 ? e[b] - o[b] : o[b] - e[b];
  }
};

// LLF flux of component values um/up (own/neighbour) with normal velocities
// unm/unp (already signed by the outward normal), scaled by wgt.
template <typename T>
__device__ __forceinline__ T llf(T um, T up, T unm, T unp, T lam, T lf, T wgt) {
  return wgt * (T(0.5) * (um * unm + up * unp) + lf * lam * (um - up));
}

}  // namespace dgmf
