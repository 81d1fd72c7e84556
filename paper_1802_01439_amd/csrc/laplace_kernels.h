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
// GPU mapping, FP64 n <= 5 and FP32 n = 3, 5.  A workgroup owns an x-y tile
// of TX x TY elements (n^2 threads per element) and marches through a segment
// of consecutive z layers.  Every element column is loaded from global memory
// once, one layer ahead: when a thread reaches layer ez it already holds its
// column of layer ez+1, whose end value and half slope are the z face data
// above, while those of layer ez-1 were kept from the previous step.  x- and
// y-neighbours inside the tile are read from LDS; only pencils across the
// tile boundary come from global memory (L2).  Per layer: phase Z (Lz, own
// column in registers), Y (Ly), X (Lx then Mx), Y (My), Z (Mz, written once),
// with pencils handed over through two LDS buffers (4 barriers).
//
// GPU mapping, n >= 6 and FP32 n = 2, 4 (measured: there the march's serial
// layer steps and register pressure cost more than the neighbour loads it
// saves): one workgroup per batch of E = floor(256/n^2) consecutive
// elements, batches walked strip by strip, XCD by XCD; each thread first
// issues all of its global loads (own z column and the six neighbour pencils,
// reduced at once to end values and slopes), then the same five phases.
//
// The 1D tables are a small device table read through the scalar unit.  No
// atomics.
//
// Input and output go through an IO policy, so that the same kernels serve
// the plain apply y = A x and the CG applies with fused vector work:
//   io.begin()                     per thread, at kernel start
//   io.load(i, loc)                value of the operand at global index i
//                                  (local node loc of its element); called
//                                  for own and neighbour DoFs alike
//   io.store(i, loc, in, out)      once per own DoF: in = operand value,
//                                  out = (A in) at that DoF
//   io.finish<THREADS, BYTES>(lds) all threads at kernel end; lds (BYTES of
//                                  LDS, free at that point) may serve a
//                                  workgroup reduction
#pragma once

#include <algorithm>

#include "api_internal.h"
#include "common.h"
#include "ops.h"

namespace dgmf {


// Even-odd form of the 1D operators (used for n >= kLapEvenOddFrom).  M and
// L = M^-1 K are centro-symmetric (A[n-1-i][n-1-j] = A[i][j]: the LGL nodes
// are symmetric and the SIPG form is invariant under x -> 1-x), and the neighbour couplings
// are mirror images (left = reflected right for the end values, negated for
// the half slopes).  With e_j = u_j + u_{n-1-j}, o_j = u_j - u_{n-1-j}
// (j < h = n/2) and, for odd n, the middle value u_h:
//   y_i = E_i + O_i,  y_{n-1-i} = E_i - O_i  (i < h),
//   E_i = sum_j Ep[i][j] e_j + Em[i] u_h,  O_i = sum_j Op[i][j] o_j,
//   y_h = sum_j Mr[j] e_j + Mc u_h,
// Ep = (A[i][j] + A[i][n-1-j]) / 2, Op = (A[i][j] - A[i][n-1-j]) / 2,
// Em[i] = A[i][h], Mr[j] = A[h][j], Mc = A[h][h]; the couplings enter E with
// (vR + vL), (gR - gL) and O with (vR - vL), (gR + gL).  Half the
// multiply-adds of the plain matrix-vector products.
template <int N, typename T>
struct LapEO {
  static constexpr int H = N / 2, HM = H > 0 ? H : 1;
  T MEp[HM][HM], MOp[HM][HM], MEm[HM], MMr[HM], MMc;          // mass
  T LEp[3][HM][HM], LOp[3][HM][HM], LEm[3][HM], LMr[3][HM], LMc[3];
  T cvE[3][HM], cgE[3][HM], cvO[3][HM], cgO[3][HM];            // couplings
  T cvM[3], cgM[3];                                            // middle node
};

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
  LapEO<N, T> eo;
};

// Sweeps in even-odd form from this n on (measured: -6..-10 % at n = 4, 5
// and up to -29 % at n = 11; nothing at n = 3).
constexpr int kLapEvenOddFrom = 4;

// LDS layout of one element's n^3 block: node (a,b,c) at a + PX*b + PY*c,
// elements ES apart.  The paddings (per n) keep the three pencil access
// patterns of a wavefront free of bank conflicts for 32 and 64 banks.
template <int N>
struct LapPad {
  static constexpr int px = (N == 6 || N == 8 || N == 12) ? 1 : 0;
  static constexpr int py = (N == 2) ? 1 : (N == 4 ? 3 : (N == 10 ? 1 : 0));
  static constexpr int pe = (N == 2) ? 2 : (N == 4 ? 4 : 0);
};

// Element tile of a marching workgroup (about 256 threads, n^2 per
// element) and the padded LDS layout of one element.
template <int N>
struct LapCfg {
  static constexpr int N2 = N * N, N3 = N * N * N;
  static constexpr int TX = N == 2 ? 8 : N == 3 ? 7 : N == 4 ? 4 : N == 5 ? 5 : N == 6 ? 7 : N == 7 ? 5
                            : N == 8 ? 2 : N == 9 ? 3 : N == 12 ? 1 : 2;
  static constexpr int TY = N == 2 ? 8 : N == 3 ? 4 : N == 4 ? 4 : N == 5 ? 2 : N == 8 ? 2 : 1;
  static constexpr int E = TX * TY;
  static constexpr int THREADS = E * N2;
  static constexpr int PX = N + LapPad<N>::px;
  static constexpr int PY = PX * N + LapPad<N>::py;
  static constexpr int ES = PY * N + LapPad<N>::pe;
};

// E = floor(256/n^2) consecutive elements per batch workgroup.
template <int N>
struct LapCfgB {
  static constexpr int N2 = N * N, N3 = N * N * N;
  static constexpr int E = (256 / N2) > 0 ? 256 / N2 : 1;
  static constexpr int THREADS = E * N2;
  static constexpr int PX = N + LapPad<N>::px;
  static constexpr int PY = PX * N + LapPad<N>::py;
  static constexpr int ES = PY * N + LapPad<N>::pe;
};

// Traversal of the element batches.  A batch is a run of E consecutive
// elements inside one z-plane (plane-linear index j*E .. j*E+E-1, so only the
// last batch of a plane can be short); planes are numbered pz = comp*Nz + ez.
// Batches are grouped into strips of S consecutive runs (a few element rows)
// and a strip is walked plane by plane: logical id L -> (strip, pz, run in
// strip).  Consecutive ids are x-neighbours, ids S apart are z-neighbours and
// y-neighbours sit within the same strip, so the neighbour data an element
// needs was loaded a few dozen workgroups earlier and is still in L2.
struct Traversal {
  int PB;   // batches per plane
  int PZ;   // planes (n_comp * Nz)
  int S;    // runs per strip
};

__device__ __forceinline__ void strip_order(int L, const Traversal& t, int& j, int& pz) {
  const int F = t.PB / t.S, R = t.PB - F * t.S;
  const int full = F * t.S * t.PZ;
  if (L < full) {
    const int s = L / (t.S * t.PZ), rem = L - s * t.S * t.PZ;
    pz = rem / t.S;
    j = s * t.S + (rem - pz * t.S);
  } else {
    const int rem = L - full;
    pz = rem / R;
    j = F * t.S + (rem - pz * R);
  }
}

template <int N, typename T, typename Mat>
__device__ __forceinline__ void matvec(const Mat& A, const T* x, T* y) {
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

template <int N, typename T, typename Tab>
__device__ __forceinline__ NbrFace<T> nbr_face(const Tab& t, const T* uL, const T* uR) {
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
template <int N, typename T, bool ACC, typename Tab>
__device__ __forceinline__ void l_pencil(const Tab& t, int d, const T* u, const NbrFace<T>& f, T* y) {
  if constexpr (N >= kLapEvenOddFrom) {
    constexpr int H = N / 2;
    const auto& q = t.eo;
    T e[H], o[H];
#pragma unroll
    for (int j = 0; j < H; ++j) {
      e[j] = u[j] + u[N - 1 - j];
      o[j] = u[j] - u[N - 1 - j];
    }
    const T sv = f.vR + f.vL, dv = f.vR - f.vL, sg = f.gR - f.gL, dg = f.gR + f.gL;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      T E = q.cvE[d][i] * sv;
      E = fmadd(q.cgE[d][i], sg, E);
#pragma unroll
      for (int j = 0; j < H; ++j) E = fmadd(q.LEp[d][i][j], e[j], E);
      if constexpr (N % 2) E = fmadd(q.LEm[d][i], u[H], E);
      T O = q.cvO[d][i] * dv;
      O = fmadd(q.cgO[d][i], dg, O);
#pragma unroll
      for (int j = 0; j < H; ++j) O = fmadd(q.LOp[d][i][j], o[j], O);
      y[i] = ACC ? y[i] + (E + O) : E + O;
      y[N - 1 - i] = ACC ? y[N - 1 - i] + (E - O) : E - O;
    }
    if constexpr (N % 2) {
      T m = q.cvM[d] * sv;
      m = fmadd(q.cgM[d], sg, m);
      m = fmadd(q.LMc[d], u[H], m);
#pragma unroll
      for (int j = 0; j < H; ++j) m = fmadd(q.LMr[d][j], e[j], m);
      y[H] = ACC ? y[H] + m : m;
    }
    return;
  }
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

// y = M x along one pencil (even-odd from kLapEvenOddFrom on)
template <int N, typename T, typename Tab>
__device__ __forceinline__ void mass_pencil(const Tab& t, const T* x, T* y) {
  if constexpr (N >= kLapEvenOddFrom) {
    constexpr int H = N / 2;
    const auto& q = t.eo;
    T e[H], o[H];
#pragma unroll
    for (int j = 0; j < H; ++j) {
      e[j] = x[j] + x[N - 1 - j];
      o[j] = x[j] - x[N - 1 - j];
    }
#pragma unroll
    for (int i = 0; i < H; ++i) {
      T E = q.MEp[i][0] * e[0];
#pragma unroll
      for (int j = 1; j < H; ++j) E = fmadd(q.MEp[i][j], e[j], E);
      if constexpr (N % 2) E = fmadd(q.MEm[i], x[H], E);
      T O = q.MOp[i][0] * o[0];
#pragma unroll
      for (int j = 1; j < H; ++j) O = fmadd(q.MOp[i][j], o[j], O);
      y[i] = E + O;
      y[N - 1 - i] = E - O;
    }
    if constexpr (N % 2) {
      T m = q.MMc * x[H];
#pragma unroll
      for (int j = 0; j < H; ++j) m = fmadd(q.MMr[j], e[j], m);
      y[H] = m;
    }
  } else {
    matvec<N, T>(t.M, x, y);
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

template <int N, typename T, typename IO>
__device__ __forceinline__ void load_pencils(const IO& io, const MeshArgs& mesh, const BatchPos& b, int p0, int p1,
                                             Pencils<N, T>& P) {
  constexpr int N2 = N * N, N3 = N * N * N;
  const size_t cs = (size_t)b.comp * mesh.n_el * N3;
  const int e = b.eg - b.comp * mesh.n_el;
  // local node of entry c of the z-, y- and x-pencils through (p0, p1)
  const int lz = p0 + N * p1, ly = p0 + N2 * p1, lx = N * p0 + N2 * p1;
  const size_t own = cs + (size_t)e * N3 + lz;
  const size_t zl = cs + (size_t)neighbor(mesh, b.ex, b.ey, b.ez, 2, 0) * N3 + lz;
  const size_t zr = cs + (size_t)neighbor(mesh, b.ex, b.ey, b.ez, 2, 1) * N3 + lz;
  const size_t yl = cs + (size_t)neighbor(mesh, b.ex, b.ey, b.ez, 1, 0) * N3 + ly;
  const size_t yr = cs + (size_t)neighbor(mesh, b.ex, b.ey, b.ez, 1, 1) * N3 + ly;
  const size_t xl = cs + (size_t)neighbor(mesh, b.ex, b.ey, b.ez, 0, 0) * N3 + lx;
  const size_t xr = cs + (size_t)neighbor(mesh, b.ex, b.ey, b.ez, 0, 1) * N3 + lx;
#pragma unroll
  for (int c = 0; c < N; ++c) {
    P.own[c] = io.load(own + N2 * c, lz + N2 * c);
    P.zl[c] = io.load(zl + N2 * c, lz + N2 * c);
    P.zr[c] = io.load(zr + N2 * c, lz + N2 * c);
    P.yl[c] = io.load(yl + N * c, ly + N * c);
    P.yr[c] = io.load(yr + N * c, ly + N * c);
    P.xl[c] = io.load(xl + c, lx + c);
    P.xr[c] = io.load(xr + c, lx + c);
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

template <int N, typename T, typename IO>
__device__ __forceinline__ void laplace_batch(const LapTab<N, T>& t, const BatchPos& b, const BatchIn<N, T>& I,
                                              IO& io, T* Ue, T* Ve, int p0, int p1) {
  using C = LapCfgB<N>;
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
    mass_pencil<N, T>(t, v, out);
#pragma unroll
    for (int a = 0; a < N; ++a) Ve[base + a] = out[a];
  }
  __syncthreads();
  // Y again: V <- My V
  if (b.active) {
    const int base = p0 + PY * p1;
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] = Ve[base + PX * j];
    mass_pencil<N, T>(t, v, out);
#pragma unroll
    for (int j = 0; j < N; ++j) Ve[base + PX * j] = out[j];
  }
  __syncthreads();
  // Z again: y = Mz V, written once
  if (b.active) {
    const int base = p0 + PX * p1;
#pragma unroll
    for (int c = 0; c < N; ++c) v[c] = Ve[base + PY * c];
    mass_pencil<N, T>(t, v, out);
    const size_t g = (size_t)b.eg * N3 + p0 + N * p1;
#pragma unroll
    for (int c = 0; c < N; ++c) io.store(g + N2 * c, p0 + N * p1 + N2 * c, Ue[base + PY * c], out[c]);
  }
}

// Batch kernel: one workgroup per batch, batches in traversal order (XCD by XCD).  All
// global loads of the batch are issued first and reduced to the own column
// plus the neighbours' end values and slopes; then the five phases run.
template <int N, typename T, typename IO>
__global__ void __launch_bounds__(LapCfgB<N>::THREADS)
laplace_batch_kernel(IO io, MeshArgs mesh, Traversal tv, const LapTab<N, T>* __restrict__ tab) {
  const LapTab<N, T>& t = *tab;
  using C = LapCfgB<N>;
  constexpr int N2 = C::N2, E = C::E, ES = C::ES;
  __shared__ __attribute__((aligned(16))) T UV[2 * E * ES];
  T* U = UV;
  T* V = UV + E * ES;

  io.begin();
  const int tid = threadIdx.x;
  const int le = tid / N2, p = tid - le * N2;
  const int p0 = p % N, p1 = p / N;
  const BatchPos b = batch_pos(xcd_remap(blockIdx.x, gridDim.x), tv, mesh, E, le);
  BatchIn<N, T> I;
  if (b.active) {
    Pencils<N, T> P;
    load_pencils<N, T>(io, mesh, b, p0, p1, P);
    reduce_pencils<N, T>(t, P, I);
  }
  laplace_batch<N, T>(t, b, I, io, U + le * ES, V + le * ES, p0, p1);
  io.template finish<C::THREADS, sizeof(UV)>(UV);
}

// Element rows per strip of the batch traversal (measured over 4..32: short
// strips keep the previous plane in L2 up to n = 8, -3..-10 %; beyond that
// long strips re-read fewer y-neighbour rows, -4..-6 %).
template <int N>
constexpr int lap_strip_rows() {
  return N <= 8 ? 4 : 32;
}

// Workgroups a march launch aims at (z segments are sized for it).
constexpr long kLapMarchWGs = 2048;

// Work of one marching workgroup: tile (tx, ty) of component comp, z layers [z0, z1).
struct LapWork {
  int ntx, nty, nseg, lz;   // tiles per direction, z segments, layers per segment
};

// N values at offsets off + stride*i (local nodes loc + stride*i) through the IO
template <int N, typename T, typename IO>
__device__ __forceinline__ void load_line(const IO& io, size_t off, int loc, int stride, T (&c)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) c[i] = io.load(off + (size_t)stride * i, loc + stride * i);
}

template <int N, typename T, typename Vec>
__device__ __forceinline__ T dot(const Vec& a, const T (&b)[N]) {
  T s = a[0] * b[0];
#pragma unroll
  for (int i = 1; i < N; ++i) s = fmadd(a[i], b[i], s);
  return s;
}

template <int N, typename T, typename IO>
__global__ void __launch_bounds__(LapCfg<N>::THREADS)
laplace_march_kernel(IO io, MeshArgs mesh, LapWork wk, const LapTab<N, T>* __restrict__ tab) {
  using C = LapCfg<N>;
  constexpr int N2 = C::N2, N3 = C::N3, TX = C::TX, TY = C::TY, E = C::E, ES = C::ES, PX = C::PX, PY = C::PY;
  __shared__ __attribute__((aligned(16))) T UV[2 * E * ES];
  T* U = UV;
  T* V = UV + E * ES;
  io.begin();

  // workgroup -> (tile, segment, component), XCD by XCD
  int w = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = w % wk.ntx;
  w /= wk.ntx;
  const int ty = w % wk.nty;
  w /= wk.nty;
  const int seg = w % wk.nseg, comp = w / wk.nseg;
  const int z0 = seg * wk.lz, z1 = min(mesh.nz, z0 + wk.lz);

  const int tid = threadIdx.x;
  const int le = tid / N2, p = tid - le * N2;
  const int p0 = p % N, p1 = p / N;
  const int ix = le % TX, iy = le / TX;
  const int ex = tx * TX + ix, ey = ty * TY + iy;
  const bool active = ex < mesh.nx && ey < mesh.ny;
  const size_t cs = (size_t)comp * mesh.n_el * N3;
  const int nxy = mesh.nx * mesh.ny;
  // neighbours inside the tile (same layer) are read from LDS
  const bool inXL = ix > 0, inXR = ix + 1 < TX && ex + 1 < mesh.nx;
  const bool inYL = iy > 0, inYR = iy + 1 < TY && ey + 1 < mesh.ny;
  const int exl = ex == 0 ? mesh.nx - 1 : ex - 1, exr = ex + 1 == mesh.nx ? 0 : ex + 1;
  const int eyl = ey == 0 ? mesh.ny - 1 : ey - 1, eyr = ey + 1 == mesh.ny ? 0 : ey + 1;
  auto zwrap = [&](int ez) { return ez < 0 ? ez + mesh.nz : (ez >= mesh.nz ? ez - mesh.nz : ez); };
  // local nodes of entry 0 of this thread's z-, y- and x-pencils
  const int lz = p0 + N * p1, ly = p0 + N2 * p1, lx = N * p0 + N2 * p1;
  // column (p0,p1) of element (ex, ey, ez)
  auto col_off = [&](int ez) { return cs + ((size_t)ez * nxy + ex + (size_t)mesh.nx * ey) * N3 + lz; };

  T cur[N], nxt[N];
  T zvL = 0, zgL = 0;   // end value and half slope at the top of the layer below
  if (active) {
    const auto& t = *fresh(tab);
    T below[N];
    load_line<N, T>(io, col_off(zwrap(z0 - 1)), lz, N2, below);
    load_line<N, T>(io, col_off(z0), lz, N2, cur);
    load_line<N, T>(io, col_off(zwrap(z0 + 1)), lz, N2, nxt);
    zvL = below[N - 1];
    zgL = dot<N, T>(t.hd1, below);
  }
  T* Ue = U + le * ES;
  T* Ve = V + le * ES;
  for (int ez = z0; ez < z1; ++ez) {
    // Global loads are issued one phase before the phase that needs them and
    // reduced to end values and half slopes as soon as they are used: the
    // tile-boundary y pencils now (reduced after Z), the x pencils after Z
    // (reduced after Y), the column two layers up after Y (next step's face
    // data above).
    const size_t lay = (size_t)ez * nxy;
    NbrFace<T> fy{}, fx{};
    T v[N];
    // FP32 has the registers to issue every load of the step at its start
    constexpr bool EARLY = sizeof(T) == 4;
    T xl[N], xr[N], nn[N];
    {
      // in order of use: vector loads return in order, so waiting for the y
      // pencils leaves the later loads in flight
      T yl[N], yr[N];
      if (active) {
        if (!inYL) load_line<N, T>(io, cs + (lay + ex + (size_t)mesh.nx * eyl) * N3 + ly, ly, N, yl);
        if (!inYR) load_line<N, T>(io, cs + (lay + ex + (size_t)mesh.nx * eyr) * N3 + ly, ly, N, yr);
      }
      if (EARLY && active) {
        if (!inXL) load_line<N, T>(io, cs + (lay + exl + (size_t)mesh.nx * ey) * N3 + lx, lx, 1, xl);
        if (!inXR) load_line<N, T>(io, cs + (lay + exr + (size_t)mesh.nx * ey) * N3 + lx, lx, 1, xr);
        if (ez + 1 < z1) load_line<N, T>(io, col_off(zwrap(ez + 2)), lz, N2, nn);
      }
      // Z: V = c_z Lz u (own column in registers); U = u
      if (active) {
        const auto& t = *fresh(tab);
        NbrFace<T> fz;
        fz.vL = zvL;
        fz.gL = zgL;
        fz.vR = nxt[0];
        fz.gR = dot<N, T>(t.hd0, nxt);
        l_pencil<N, T, false>(t, 2, cur, fz, v);
        const int base = p0 + PX * p1;
#pragma unroll
        for (int c = 0; c < N; ++c) {
          Ue[base + PY * c] = cur[c];
          Ve[base + PY * c] = v[c];
        }
        zvL = cur[N - 1];
        zgL = dot<N, T>(t.hd1, cur);
        if (!inYL) {
          fy.vL = yl[N - 1];
          fy.gL = dot<N, T>(t.hd1, yl);
        }
        if (!inYR) {
          fy.vR = yr[0];
          fy.gR = dot<N, T>(t.hd0, yr);
        }
      }
    }
    if (!EARLY && active) {
      if (!inXL) load_line<N, T>(io, cs + (lay + exl + (size_t)mesh.nx * ey) * N3 + lx, lx, 1, xl);
      if (!inXR) load_line<N, T>(io, cs + (lay + exr + (size_t)mesh.nx * ey) * N3 + lx, lx, 1, xr);
    }
    __syncthreads();
    // Y: pencil (a,c) = (p0,p1): V += c_y Ly u
    if (active) {
      const auto& t = *fresh(tab);
      const int base = p0 + PY * p1;
      if (inYL) {   // neighbour pencil in LDS: end value and half slope at its right end
        T g = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) g = fmadd(t.hd1[j], Ue[base + PX * j - TX * ES], g);
        fy.vL = Ue[base + PX * (N - 1) - TX * ES];
        fy.gL = g;
      }
      if (inYR) {
        T g = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) g = fmadd(t.hd0[j], Ue[base + PX * j + TX * ES], g);
        fy.vR = Ue[base + TX * ES];
        fy.gR = g;
      }
      T in[N];
#pragma unroll
      for (int j = 0; j < N; ++j) {
        in[j] = Ue[base + PX * j];
        v[j] = Ve[base + PX * j];
      }
      l_pencil<N, T, true>(t, 1, in, fy, v);
#pragma unroll
      for (int j = 0; j < N; ++j) Ve[base + PX * j] = v[j];
      if (!inXL) {
        fx.vL = xl[N - 1];
        fx.gL = dot<N, T>(t.hd1, xl);
      }
      if (!inXR) {
        fx.vR = xr[0];
        fx.gR = dot<N, T>(t.hd0, xr);
      }
      if (!EARLY && ez + 1 < z1) load_line<N, T>(io, col_off(zwrap(ez + 2)), lz, N2, nn);
    }
    __syncthreads();
    // X: pencil (b,c) = (p0,p1): V += c_x Lx u, then V <- Mx V
    if (active) {
      const auto& t = *fresh(tab);
      const int base = PX * p0 + PY * p1;
      if (inXL) {
        T g = 0;
#pragma unroll
        for (int a = 0; a < N; ++a) g = fmadd(t.hd1[a], Ue[base + a - ES], g);
        fx.vL = Ue[base + N - 1 - ES];
        fx.gL = g;
      }
      if (inXR) {
        T g = 0;
#pragma unroll
        for (int a = 0; a < N; ++a) g = fmadd(t.hd0[a], Ue[base + a + ES], g);
        fx.vR = Ue[base + ES];
        fx.gR = g;
      }
      T in[N], out[N];
#pragma unroll
      for (int a = 0; a < N; ++a) {
        in[a] = Ue[base + a];
        v[a] = Ve[base + a];
      }
      l_pencil<N, T, true>(t, 0, in, fx, v);
      mass_pencil<N, T>(t, v, out);
#pragma unroll
      for (int a = 0; a < N; ++a) Ve[base + a] = out[a];
    }
    __syncthreads();
    // Y again: V <- My V
    if (active) {
      const auto& t = *fresh(tab);
      const int base = p0 + PY * p1;
      T out[N];
#pragma unroll
      for (int j = 0; j < N; ++j) v[j] = Ve[base + PX * j];
      mass_pencil<N, T>(t, v, out);
#pragma unroll
      for (int j = 0; j < N; ++j) Ve[base + PX * j] = out[j];
    }
    __syncthreads();
    // Z again: y = Mz V, written once.  The next layer's Z phase touches only
    // this thread's own column of U and V, so no barrier is needed before it.
    if (active) {
      const auto& t = *fresh(tab);
      const int base = p0 + PX * p1;
      T out[N];
#pragma unroll
      for (int c = 0; c < N; ++c) v[c] = Ve[base + PY * c];
      mass_pencil<N, T>(t, v, out);
      const size_t g = col_off(ez);
#pragma unroll
      for (int c = 0; c < N; ++c) io.store(g + N2 * c, lz + N2 * c, cur[c], out[c]);
#pragma unroll
      for (int c = 0; c < N; ++c) {
        cur[c] = nxt[c];
        nxt[c] = nn[c];
      }
    }
  }
  io.template finish<C::THREADS, sizeof(UV)>(UV);
}


// Sums v[q] over the workgroup (THREADS threads) in a fixed order; thread 0
// writes partial[q * gridDim.x + blockIdx.x].  lds: BYTES of free LDS.
template <int THREADS, size_t BYTES, int NQ>
__device__ __forceinline__ void wg_partials(const double (&v)[NQ], double* __restrict__ partial, void* lds) {
  static_assert(THREADS >= 64 && THREADS <= 1024 && BYTES >= THREADS * sizeof(double), "reduction scratch");
  double* sh = static_cast<double*>(lds);
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    __syncthreads();
    sh[tid] = v[q];
    __syncthreads();
    if (tid < 64) {   // one full wavefront
      double s = sh[tid];
      for (int j = tid + 64; j < THREADS; j += 64) s += sh[j];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
      if (tid == 0) partial[(size_t)q * gridDim.x + blockIdx.x] = s;
    }
  }
}

// y = A x
template <typename T>
struct LapPlainIO {
  const T* __restrict__ src;
  T* __restrict__ dst;
  __device__ __forceinline__ void begin() {}
  __device__ __forceinline__ T load(size_t i, int) const { return src[i]; }
  __device__ __forceinline__ void store(size_t i, int, T, T out) { dst[i] = out; }
  template <int THREADS, size_t BYTES>
  __device__ __forceinline__ void finish(void*) {}
};

template <int N, typename T>
LapTab<N, T> make_lap_tab(const LaplacePlan& P) {
  LapTab<N, T> t;
  for (int i = 0; i < N; ++i) {
    for (int j = 0; j < N; ++j) {
      t.M[i][j] = (T)P.Mref[i * N + j];
      for (int d = 0; d < 3; ++d)
        t.L[d][i][j] = (T)(P.c[d] * P.Lown[i * N + j] + (d == 2 && i == j ? P.shift : 0.0));
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
  // even-odd form, from the symmetrised double-precision matrices
  constexpr int H = N / 2;
  auto fill = [&](auto A, auto& Ep, auto& Op, auto& Em, auto& Mr, auto& Mc) {
    // A(i, j) in double; centro-symmetric average first
    auto S = [&](int i, int j) { return 0.5 * (A(i, j) + A(N - 1 - i, N - 1 - j)); };
    for (int i = 0; i < H; ++i) {
      for (int j = 0; j < H; ++j) {
        Ep[i][j] = (T)(0.5 * (S(i, j) + S(i, N - 1 - j)));
        Op[i][j] = (T)(0.5 * (S(i, j) - S(i, N - 1 - j)));
      }
      Em[i] = (T)(N % 2 ? S(i, H) : 0.0);
      Mr[i] = (T)(N % 2 ? S(H, i) : 0.0);
    }
    Mc = (T)(N % 2 ? S(H, H) : 0.0);
  };
  fill([&](int i, int j) { return P.Mref[i * N + j]; }, t.eo.MEp, t.eo.MOp, t.eo.MEm, t.eo.MMr, t.eo.MMc);
  for (int d = 0; d < 3; ++d) {
    // the mass term of a Helmholtz operator is a diagonal shift of the z matrix
    fill([&](int i, int j) { return P.c[d] * P.Lown[i * N + j] + (d == 2 && i == j ? P.shift : 0.0); },
         t.eo.LEp[d], t.eo.LOp[d], t.eo.LEm[d], t.eo.LMr[d], t.eo.LMc[d]);
    // mirrored couplings: aL[i] = aR[n-1-i], eL[i] = -eR[n-1-i] (averaged)
    auto aR = [&](int i) { return 0.5 * P.c[d] * (P.cR[i] + P.cL[N - 1 - i]); };
    auto eR = [&](int i) { return 0.5 * P.c[d] * (P.gR[i] - P.gL[N - 1 - i]); };
    for (int i = 0; i < H; ++i) {
      const double aRi = aR(i), aLi = aR(N - 1 - i), eRi = eR(i), eLi = -eR(N - 1 - i);
      t.eo.cvE[d][i] = (T)(0.5 * (aRi + aLi));
      t.eo.cgE[d][i] = (T)(0.5 * (eRi - eLi));
      t.eo.cvO[d][i] = (T)(0.5 * (aRi - aLi));
      t.eo.cgO[d][i] = (T)(0.5 * (eRi + eLi));
    }
    t.eo.cvM[d] = (T)(N % 2 ? aR(H) : 0.0);
    t.eo.cgM[d] = (T)(N % 2 ? eR(H) : 0.0);
  }
  return t;
}

// Device copy of the plan's table (uploaded once per content and device).
template <int N, typename T>
const LapTab<N, T>* lap_device_tab(const LaplacePlan& P, hipError_t* err) {
  return device_table_of("laplace", make_lap_tab<N, T>(P), err);
}

// measured choice: the march wins for FP64 up to n = 5 and for FP32 at
// n = 3 and 5; the batch kernel is faster everywhere else
template <int N, typename T>
constexpr bool lap_march() {
  return sizeof(T) == 8 ? N <= 5 : (N == 3 || N == 5);
}

// Workgroups of one launch (for the size of a partial-sum buffer).
template <int N, typename T>
long lap_grid(const LaplacePlan& P) {
  if constexpr (!lap_march<N, T>()) {
    using CB = LapCfgB<N>;
    const long PB = (P.mesh.nx * (long)P.mesh.ny + CB::E - 1) / CB::E;
    return PB * P.n_comp * P.mesh.nz;
  } else {
    using C = LapCfg<N>;
    const long ntx = (P.mesh.nx + C::TX - 1) / C::TX, nty = (P.mesh.ny + C::TY - 1) / C::TY;
    const long tiles = ntx * nty * P.n_comp;
    const long want = std::max(1L, std::min<long>(P.mesh.nz, (kLapMarchWGs + tiles - 1) / tiles));
    const long lz = (P.mesh.nz + want - 1) / want;
    return tiles * ((P.mesh.nz + lz - 1) / lz);
  }
}

// Launch y = A x through io.  tab: device table from lap_device_tab (or
// nullptr to look it up here).
template <int N, typename T, typename IO>
hipError_t launch_laplace_io(const LaplacePlan& P, const IO& io, const LapTab<N, T>* tab, hipStream_t stream) {
  hipError_t err;
  if (!tab && !(tab = lap_device_tab<N, T>(P, &err))) return err;
  if constexpr (!lap_march<N, T>()) {
    using CB = LapCfgB<N>;
    Traversal tv;
    tv.PB = (P.mesh.nx * P.mesh.ny + CB::E - 1) / CB::E;
    tv.PZ = P.n_comp * P.mesh.nz;
    tv.S = std::max(1, std::min(tv.PB, (lap_strip_rows<N>() * P.mesh.nx + CB::E / 2) / CB::E));
    const long grid = (long)tv.PB * tv.PZ;
    if (grid > 0x7fffffffL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((laplace_batch_kernel<N, T, IO>), dim3((unsigned)grid), dim3(CB::THREADS), 0, stream, io,
                       P.mesh, tv, tab);
  } else {
    // tiles x z segments x components, about kLapMarchWGs workgroups
    using C = LapCfg<N>;
    LapWork wk;
    wk.ntx = (P.mesh.nx + C::TX - 1) / C::TX;
    wk.nty = (P.mesh.ny + C::TY - 1) / C::TY;
    const long tiles = (long)wk.ntx * wk.nty * P.n_comp;
    const int want = (int)std::max(1L, std::min<long>(P.mesh.nz, (kLapMarchWGs + tiles - 1) / tiles));
    wk.lz = (P.mesh.nz + want - 1) / want;
    wk.nseg = (P.mesh.nz + wk.lz - 1) / wk.lz;
    const long grid = tiles * wk.nseg;
    if (grid > 0x7fffffffL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((laplace_march_kernel<N, T, IO>), dim3((unsigned)grid), dim3(C::THREADS), 0, stream, io,
                       P.mesh, wk, tab);
  }
  return hipGetLastError();
}

}  // namespace dgmf
