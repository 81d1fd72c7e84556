// Convective term c_h with the local Lax-Friedrichs flux (Sec. 3.2, weak form
// of c_h, F_c(u) = u (x) u), by sum factorisation on periodic Cartesian meshes,
// FP64 and FP32, degrees 1..11 with floor(3k/2)+1 Gauss points (3/2 rule).
//
//   R_c = -sum_j s_j (d_j phi, u_c u_j)_K + sum_faces (phi, F*_c),   s_j = vol/h_j
//   F*_c = 1/2 (u-_c u-.n + u+_c u+.n) + lf * max(|u-.n|, |u+.n|) (u-_c - u+_c)
//
// 1D tables: S (m x n, LGL -> Gauss interpolation), G (m x n, derivatives of
// the LGL basis at the Gauss points), Gauss weights w.
//
// Cell term: u -> S_x -> S_y -> S_z gives u at the m^3 points; the flux
// F_cj = s_j W u_c u_j is contracted back as
//   R_c = G^T_x S^T_y (S^T_z F_cx) + S^T_x [G^T_y (S^T_z F_cy) + S^T_y (G^T_z F_cz)].
//
// Face terms ride along with the cell sweeps.  With LGL nodes the trace of u on
// a face is the face layer of nodes, and its test functions are the face layer:
//   z faces: the neighbours' facing layers are carried as two extra z layers
//            through the x and y sweeps, so after them both traces sit at the
//            face points (q1,q2) of the z pencil that a thread owns; the face
//            flux is added to the G^T_z F_cz pencil at its end nodes, where the
//            following S^T_y, S^T_x sweeps integrate it over the face.
//   y faces: own and neighbour layers are swept in x (own ones come out of the
//            cell x sweep), then one thread per (side, q1) interpolates them in
//            z, forms the flux at the m face points and integrates it back in
//            z; the result joins the y back sweep at the end nodes.
//   x faces: own and neighbour layers are swept in y, then in z per (side, q2)
//            as for y; the result is integrated in y and added at the end
//            nodes after the x back sweep.
// Each element does its own six faces (each face flux is formed twice, no
// atomics, every output written once).
//
// GPU mapping: one workgroup per batch of E consecutive elements.  Phases
// (barriers between them):
//   P1  x sweep of the cell (3n^2 pencils per element) and of the y/z
//       neighbour layers, y sweep of the x-face layers; all inputs straight
//       from global memory into registers.
//   P2  y sweep, in place in LDS, of the cell and the two extra z layers.
//   P3  per (q1,q2): z sweep into registers, z-face flux, cell flux and the
//       z back sweep; per (side, q): y- and x-face flux pencils.
//   Y   y back sweep (in place) and the y integral of the x-face terms.
//   X   x back sweep, face end-node terms, write-out.
// Small degrees keep the back sweeps of all three components in LDS at once
// (5 phases); large ones run the Z/Y/X back sweeps per component from the z
// pencils held in registers (11 phases, a third of the LDS).
#include <cmath>

#include "api_internal.h"
#include "basis_ct.h"
#include "common.h"
#include "ops.h"

namespace dgmf {

template <int N, int Q, typename T>
struct ConvTab {
  T S[Q][N];   // l_a(z_q)
  T G[Q][N];   // l_a'(z_q)
  T w[Q];      // Gauss weights on [0,1]
};

// The tables of degree N-1 with Q Gauss points as compile-time constants.
template <int N, int Q, typename T>
constexpr ConvTab<N, Q, T> conv_tab_ct() {
  constexpr ct::Tables<N, Q> d{};
  ConvTab<N, Q, T> t{};
  for (int q = 0; q < Q; ++q) {
    for (int a = 0; a < N; ++a) {
      t.S[q][a] = (T)d.S[q][a];
      t.G[q][a] = (T)d.G[q][a];
    }
    t.w[q] = (T)d.w[q];
  }
  return t;
}

// Where the kernels read the tables from.  FP32: compile-time constants, which
// become literal operands of the FMAs.  FP64: a table in device memory, read
// with scalar loads through a pointer laundered by an empty asm (and returned
// in the constant address space), so that loads issued after it cannot be
// merged with loads of the same entries elsewhere in the kernel: each phase
// loads the rows it uses when it uses them instead of keeping the table live
// in scalar registers (64-bit constants would each take a scalar register pair
// and spill at high degree).
template <typename P>
using const_ptr = const __attribute__((address_space(4))) P*;

template <typename P>
__device__ __forceinline__ const_ptr<P> fresh(const P* p) {
  uint64_t x = (uint64_t)p;
  asm volatile("" : "+v"(x));
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
  return (const_ptr<P>)(((uint64_t)hi << 32) | lo);
}

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

// LDS layout of one element (units of T).
//  Column block: a (q1, q2) grid with q1 pitch MP (odd, against bank
//  conflicts); "slots" are stacked column blocks.
//   forward:  slot j*(n+2) + c+1 holds component j at z layer c in -1..n
//             (-1 and n: the z neighbours' facing layers), first as (q1, b)
//             after the x sweep, then as (q1, q2) after the in-place y sweep.
//   backward: slot (jj*3 + f)*n + cz holds S^T_z F_jx, S^T_z F_jy, G^T_z F_jz
//             (f = 0, 1, 2) at (q1, q2); the y back sweep overwrites f = 0, 1
//             in place with (q1, b).  A thread only overwrites the column it
//             has itself read, so no barrier separates those steps.
//  Face layers FY (y faces) and FX (x faces): [sigma][s][j][c][q] with sigma
//  0 = own, 1 = neighbour, s the side, c the z node, q = q1 (FY) or q2 (FX);
//  the face-flux pencils overwrite their own sigma = 0 entries with the z back
//  sweep result (cz in place of c).
//  XR: the x-face terms after the y integral, [jj][s][cz][b].
template <int N, int Q, int SZ>
struct ConvShape {
  static constexpr int N2 = N * N, N3 = N * N * N;
  static constexpr int MP = Q | 1;
  static constexpr int COLS = MP * Q;
  static constexpr int LAYER = N * Q;
  static constexpr int FL = 12 * LAYER;
  static constexpr int slots(bool allc) { return allc ? (9 * N > 3 * (N + 2) ? 9 * N : 3 * (N + 2)) : 3 * (N + 2); }
  static constexpr int per(bool allc) { return slots(allc) * COLS + 2 * FL + (allc ? 3 : 1) * 2 * N2; }
  // all components' back sweeps at once while an element needs <= 24 KB
  static constexpr bool ALLC = per(true) * SZ <= 24 * 1024;
  static constexpr int PER = per(ALLC);
  static constexpr int BYTES = PER * SZ;
  // about 52 KB per workgroup (three per CU), 1..16 elements
  static constexpr int E0 = (52 * 1024) / BYTES;
  static constexpr int E = E0 < 1 ? 1 : (E0 > 16 ? 16 : E0);
  // per-component mode keeps one z pencil per thread in registers
  static constexpr int TH = (E * Q * Q > 256) ? ((E * Q * Q + 63) / 64) * 64 : 256;
  static_assert(E * PER * SZ <= 160 * 1024, "convective LDS footprint exceeds 160 KB");
};

template <int N, int Q, typename T>
__device__ __forceinline__ void load_pencil(const T* __restrict__ p, int stride, T (&in)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) in[i] = p[i * stride];
}

// dst[q*stride] = sum_a S[q][a] in[a]   (and the same into dst2 if given)
template <int N, int Q, typename T, typename Tab>
__device__ __forceinline__ void interp_store(const Tab& t, const T (&in)[N], T* dst, int stride, T* dst2) {
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    T acc = t.S[q][0] * in[0];
#pragma unroll
    for (int a = 1; a < N; ++a) acc = fmadd(t.S[q][a], in[a], acc);
    dst[q * stride] = acc;
    if (dst2) dst2[q] = acc;
  }
}

// LLF flux of component values um/up (own/neighbour) with normal velocities
// unm/unp (already signed by the outward normal), scaled by wgt.
template <typename T>
__device__ __forceinline__ T llf(T um, T up, T unm, T unp, T lam, T lf, T wgt) {
  return wgt * (T(0.5) * (um * unm + up * unp) + lf * lam * (um - up));
}

template <int N, int Q, typename T, int E, int TH, bool ALLC>
__global__ void __launch_bounds__(TH)
convective_kernel(const T* __restrict__ u, T* __restrict__ r, MeshArgs mesh,
                  const ConvTab<N, Q, T>* __restrict__ tab, ConvScal<T> sc) {
  using Sh = ConvShape<N, Q, (int)sizeof(T)>;
  constexpr int N2 = Sh::N2, N3 = Sh::N3, MP = Sh::MP, COLS = Sh::COLS, LAYER = Sh::LAYER;
  constexpr int PER = Sh::per(ALLC);
  constexpr int FYo = Sh::slots(ALLC) * COLS;
  constexpr int FXo = FYo + Sh::FL;
  constexpr int XRo = FXo + Sh::FL;
  __shared__ T lds[E * PER];
  const int tid = threadIdx.x;
  const int e0 = xcd_remap(blockIdx.x, gridDim.x) * E;
  const int ne = min(E, mesh.n_el - e0);   // elements of this batch; items of le >= ne are skipped
  const size_t cs = (size_t)mesh.n_el * N3;
  // grid position of element e0 + le from that of e0 (uniform)
  const int nxy = mesh.nx * mesh.ny;
  const int ez0 = e0 / nxy, exy0 = e0 - ez0 * nxy, ey0 = exy0 / mesh.nx, ex0 = exy0 - ey0 * mesh.nx;
  auto nbr = [&](int le, int d, int s) {
    int ex = ex0 + le, ey = ey0, ez = ez0;
    while (ex >= mesh.nx) {
      ex -= mesh.nx;
      if (++ey == mesh.ny) {
        ey = 0;
        ++ez;
      }
    }
    return neighbor(mesh, ex, ey, ez, d, s);
  };

  // ---------------- P1: x sweeps (and y sweeps of x-face layers) from global ----------------
  // An item is one pencil position taken for all three components, which
  // share its index arithmetic; all of a thread's loads are issued before any
  // sweep, so the global load latency is paid once per thread.
  {
    constexpr int nM = E * N2, nL = E * 4 * N, nX = E * 4 * N;   // cell, y/z neighbour, x-face items
    constexpr int total = nM + nL + nX;
    constexpr int D1S = (N + 2) * COLS;   // component stride of the BC slots
    // item w -> source pencil of component 0 (src, stride), LDS destination of
    // component 0 (d1) with its component stride (dstr), second destination d2
    auto item = [&](int w, const T*& src, int& sstride, int& d1, int& dstr, int& d2) {
      sstride = 1;
      d1 = -1;
      d2 = -1;
      dstr = D1S;
      if (w < nM) {   // cell pencil (b, c)
        const int le = w / N2, bc = w - le * N2;
        if (le >= ne) return;
        const int b = bc % N, c = bc / N;
        src = u + (size_t)(e0 + le) * N3 + N * bc;
        const int L = le * PER;
        d1 = L + (c + 1) * COLS + MP * b;
        if (b == 0) d2 = L + FYo + (0 * 2 + 0) * 3 * LAYER + c * Q;
        else if (b == N - 1) d2 = L + FYo + (0 * 2 + 1) * 3 * LAYER + c * Q;
      } else if (w < nM + nL) {   // y or z neighbour layer pencil, swept in x
        const int v = w - nM;
        const int le = v / (4 * N);
        if (le >= ne) return;
        const int rem = v - le * 4 * N;
        const int isz = rem / (2 * N), r2 = rem - isz * 2 * N;
        const int s = r2 / N, p = r2 - s * N;
        const int nb = nbr(le, isz ? 2 : 1, s);
        const int lay = s ? 0 : N - 1;   // neighbour's facing layer
        const int L = le * PER;
        if (isz) {   // pencil b = p of z layer lay -> extra z slot
          src = u + (size_t)nb * N3 + N * (p + N * lay);
          d1 = L + (s ? N + 1 : 0) * COLS + MP * p;
        } else {     // pencil c = p of y layer lay -> FY neighbour entry
          src = u + (size_t)nb * N3 + N * (lay + N * p);
          d1 = L + FYo + (1 * 2 + s) * 3 * LAYER + p * Q;
          dstr = LAYER;
        }
      } else {        // x-face layer (own or neighbour), swept in y
        const int v = w - nM - nL;
        const int le = v / (4 * N);
        if (le >= ne) return;
        const int rem = v - le * 4 * N;
        const int sg = rem / (2 * N), r2 = rem - sg * 2 * N;
        const int s = r2 / N, c = r2 - s * N;
        int e = e0 + le, a = s ? N - 1 : 0;
        if (sg) {
          e = nbr(le, 0, s);
          a = s ? 0 : N - 1;
        }
        src = u + (size_t)e * N3 + a + N2 * c;
        sstride = N;
        d1 = le * PER + FXo + (sg * 2 + s) * 3 * LAYER + c * Q;
        dstr = LAYER;
      }
    };
    constexpr int NI1 = (total + TH - 1) / TH;
    T in[NI1][3][N];
    int d1[NI1], ds[NI1], d2[NI1];
#pragma unroll
    for (int i = 0; i < NI1; ++i) {
      const int w = tid + i * TH;
      d1[i] = -1;
      if (w < total) {
        const T* src;
        int sstride;
        item(w, src, sstride, d1[i], ds[i], d2[i]);
        if (d1[i] >= 0) {
#pragma unroll
          for (int j = 0; j < 3; ++j) load_pencil<N, Q, T>(src + j * cs, sstride, in[i][j]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NI1; ++i) {
      if (d1[i] >= 0) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          CONV_TABLES(t);
          interp_store<N, Q, T>(t, in[i][j], lds + d1[i] + j * ds[i], 1,
                                d2[i] >= 0 ? lds + d2[i] + j * LAYER : (T*)nullptr);
        }
      }
    }
  }
  __syncthreads();

  // ---------------- P2: y sweep in place (cell and extra z layers) ----------------
  {
    constexpr int n2 = 3 * E * (N + 2) * Q;
    for (int w = tid; w < n2; w += TH) {
      const int q1 = w % Q, rest = w / Q;           // rest = (j*E + le)*(N+2) + c'
      const int cl = rest % (N + 2), jl = rest / (N + 2);
      const int le = jl % E, j = jl / E;
      if (le >= ne) continue;
      CONV_TABLES(t);
      T* p = lds + le * PER + (j * (N + 2) + cl) * COLS + q1;
      T in[N];
#pragma unroll
      for (int b = 0; b < N; ++b) in[b] = p[MP * b];
      interp_store<N, Q, T>(t, in, p, MP, (T*)nullptr);
    }
  }
  __syncthreads();

  // ---------------- P3: z sweeps, fluxes, z back sweep ----------------
  constexpr int nCell = E * Q * Q;
  bool own_cell = false;   // this thread holds the z pencil of cell item tid
  T Uz[3][Q];
  T Fz[2][3];
  T w12 = 0;
  T* colp = lds;   // this thread's column (per-component mode)
  {
    constexpr int nH = E * 4 * Q;
    for (int w = tid; w < nCell + nH; w += TH) {
      CONV_TABLES(t);
      if (w < nCell) {
        const int le = w / (Q * Q), qq = w - le * (Q * Q);
        if (le >= ne) continue;
        own_cell = true;
        const int q2 = qq / Q, q1 = qq - q2 * Q;
        T* col = lds + le * PER + q1 + MP * q2;
        T v[3][N + 2];
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
          for (int c = 0; c < N + 2; ++c) v[j][c] = col[(j * (N + 2) + c) * COLS];
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            T acc = t.S[q][0] * v[j][1];
#pragma unroll
            for (int c = 1; c < N; ++c) acc = fmadd(t.S[q][c], v[j][c + 1], acc);
            Uz[j][q] = acc;
          }
        w12 = t.w[q1] * t.w[q2];
        const T wz = w12 * sc.area[2];
        {   // z faces: side 0 (own layer c=0, neighbour below), side 1 (c=n-1, above)
          const T unm0 = -v[2][1], unp0 = -v[2][0];
          const T lam0 = fmax(fabs(unm0), fabs(unp0));
          const T unm1 = v[2][N], unp1 = v[2][N + 1];
          const T lam1 = fmax(fabs(unm1), fabs(unp1));
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            Fz[0][j] = llf(v[j][1], v[j][0], unm0, unp0, lam0, sc.lf, wz);
            Fz[1][j] = llf(v[j][N], v[j][N + 1], unm1, unp1, lam1, sc.lf, wz);
          }
        }
        colp = col;
        // z back sweep: all components (ALLC) or component 0
#pragma unroll
        for (int j = 0; j < (ALLC ? 3 : 1); ++j) {
          T ox[N], oy[N], oz[N];
#pragma unroll
          for (int c = 0; c < N; ++c) ox[c] = oy[c] = oz[c] = 0;
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            const T uc = t.w[q] * Uz[j][q];
            const T fx = uc * Uz[0][q], fy = uc * Uz[1][q], fz = uc * Uz[2][q];
#pragma unroll
            for (int c = 0; c < N; ++c) {
              ox[c] = fmadd(t.S[q][c], fx, ox[c]);
              oy[c] = fmadd(t.S[q][c], fy, oy[c]);
              oz[c] = fmadd(t.G[q][c], fz, oz[c]);
            }
          }
          {   // cell scalings s_d w_q1 w_q2 applied once per output
            const T s0 = sc.cell[0] * w12, s1 = sc.cell[1] * w12, s2 = sc.cell[2] * w12;
#pragma unroll
            for (int c = 0; c < N; ++c) {
              ox[c] *= s0;
              oy[c] *= s1;
              oz[c] *= s2;
            }
          }
          oz[0] += Fz[0][j];
          oz[N - 1] += Fz[1][j];
#pragma unroll
          for (int c = 0; c < N; ++c) {
            col[((j * 3 + 0) * N + c) * COLS] = ox[c];
            col[((j * 3 + 1) * N + c) * COLS] = oy[c];
            col[((j * 3 + 2) * N + c) * COLS] = oz[c];
          }
        }
      } else {   // face-flux pencil: fam 0 = y face (q = q1), 1 = x face (q = q2)
        const int h = w - nCell;
        const int le = h / (4 * Q);
        if (le >= ne) continue;
        int rem = h - le * 4 * Q;
        const int fam = rem / (2 * Q);
        rem -= fam * 2 * Q;
        const int s = rem / Q, q = rem - s * Q;
        T* F = lds + le * PER + (fam ? FXo : FYo) + q;
        T own[3][N], nbr[3][N], acc[3][N];
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
          for (int c = 0; c < N; ++c) {
            own[j][c] = F[((0 * 2 + s) * 3 + j) * LAYER + c * Q];
            nbr[j][c] = F[((1 * 2 + s) * 3 + j) * LAYER + c * Q];
            acc[j][c] = 0;
          }
        const T sgn = s ? T(1) : T(-1);
        const T wq = t.w[q] * (fam ? sc.area[0] : sc.area[1]);
#pragma unroll
        for (int q3 = 0; q3 < Q; ++q3) {
          T um[3], up[3];
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            T a = t.S[q3][0] * own[j][0], b = t.S[q3][0] * nbr[j][0];
#pragma unroll
            for (int c = 1; c < N; ++c) {
              a = fmadd(t.S[q3][c], own[j][c], a);
              b = fmadd(t.S[q3][c], nbr[j][c], b);
            }
            um[j] = a;
            up[j] = b;
          }
          const T unm = sgn * (fam ? um[0] : um[1]), unp = sgn * (fam ? up[0] : up[1]);
          const T lam = fmax(fabs(unm), fabs(unp));
          const T wgt = wq * t.w[q3];
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            const T f = llf(um[j], up[j], unm, unp, lam, sc.lf, wgt);
#pragma unroll
            for (int c = 0; c < N; ++c) acc[j][c] = fmadd(t.S[q3][c], f, acc[j][c]);
          }
        }
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
          for (int c = 0; c < N; ++c) F[((0 * 2 + s) * 3 + j) * LAYER + c * Q] = acc[j][c];
      }
    }
  }
  __syncthreads();

  // ---------------- Y and X back sweeps ----------------
  // component range [j0, j1) uses slot set jj = ALLC ? j : 0
  auto back_y = [&](int j0, int j1) {
    const int nc = j1 - j0;
    const int nYc = nc * E * N * Q, nXf = nc * E * 2 * N;
    for (int w = tid; w < nYc + nXf; w += TH) {
      CONV_TABLES(t);
      if (w < nYc) {
        const int q1 = w % Q, rest = w / Q;
        const int cz = rest % N, jl = rest / N;
        const int le = jl % E, j = j0 + jl / E;
        if (le >= ne) continue;
        const int jj = ALLC ? j : 0;
        T* L = lds + le * PER;
        T* tb = L + q1;
        const int sx = ((jj * 3 + 0) * N + cz) * COLS, sy = sx + N * COLS, sz = sx + 2 * N * COLS;
        T v1[N], v2[N];
#pragma unroll
        for (int b = 0; b < N; ++b) v1[b] = v2[b] = 0;
#pragma unroll
        for (int q2 = 0; q2 < Q; ++q2) {
          const T tx = tb[sx + MP * q2], ty = tb[sy + MP * q2], tz = tb[sz + MP * q2];
#pragma unroll
          for (int b = 0; b < N; ++b) {
            v1[b] = fmadd(t.S[q2][b], tx, v1[b]);
            v2[b] = fmadd(t.G[q2][b], ty, fmadd(t.S[q2][b], tz, v2[b]));
          }
        }
        v2[0] += L[FYo + ((0 * 2 + 0) * 3 + j) * LAYER + cz * Q + q1];
        v2[N - 1] += L[FYo + ((0 * 2 + 1) * 3 + j) * LAYER + cz * Q + q1];
#pragma unroll
        for (int b = 0; b < N; ++b) {
          tb[sx + MP * b] = v1[b];
          tb[sy + MP * b] = v2[b];
        }
      } else {   // x-face terms: integrate in y
        const int v = w - nYc;
        const int cz = v % N, rest = v / N;
        const int s = rest % 2, jl = rest / 2;
        const int le = jl % E, j = j0 + jl / E;
        if (le >= ne) continue;
        const int jj = ALLC ? j : 0;
        T* L = lds + le * PER;
        const T* xf = L + FXo + ((0 * 2 + s) * 3 + j) * LAYER + cz * Q;
        T o[N];
#pragma unroll
        for (int b = 0; b < N; ++b) o[b] = 0;
#pragma unroll
        for (int q2 = 0; q2 < Q; ++q2) {
          const T x = xf[q2];
#pragma unroll
          for (int b = 0; b < N; ++b) o[b] = fmadd(t.S[q2][b], x, o[b]);
        }
        T* xr = L + XRo + ((jj * 2 + s) * N + cz) * N;
#pragma unroll
        for (int b = 0; b < N; ++b) xr[b] = o[b];
      }
    }
  };
  auto back_x = [&](int j0, int j1) {
    const int nXc = (j1 - j0) * E * N2;
    for (int w = tid; w < nXc; w += TH) {
      CONV_TABLES(t);
      const int bc = w % N2, jl = w / N2;
      const int le = jl % E, j = j0 + jl / E;
      if (le >= ne) continue;
      const int jj = ALLC ? j : 0;
      const int b = bc % N, cz = bc / N;
      const T* L = lds + le * PER;
      const T* v1 = L + ((jj * 3 + 0) * N + cz) * COLS + MP * b;
      const T* v2 = v1 + N * COLS;
      T o[N];
#pragma unroll
      for (int a = 0; a < N; ++a) o[a] = 0;
#pragma unroll
      for (int q1 = 0; q1 < Q; ++q1) {
        const T x1 = v1[q1], x2 = v2[q1];
#pragma unroll
        for (int a = 0; a < N; ++a) o[a] = fmadd(t.G[q1][a], x1, fmadd(t.S[q1][a], x2, o[a]));
      }
      const T* xr = L + XRo + (jj * 2 * N + cz) * N + b;
      o[0] += xr[0];
      o[N - 1] += xr[N2];
      T* g = r + j * cs + (size_t)(e0 + le) * N3 + N * bc;
#pragma unroll
      for (int a = 0; a < N; ++a) g[a] = o[a];
    }
  };

  if constexpr (ALLC) {
    back_y(0, 3);
    __syncthreads();
    back_x(0, 3);
  } else {
    // per component: the thread's own z pencil (tid < nCell) is still in registers
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      if (j > 0) {
        if (own_cell) {
          CONV_TABLES(t);
          T ox[N], oy[N], oz[N];
#pragma unroll
          for (int c = 0; c < N; ++c) ox[c] = oy[c] = oz[c] = 0;
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            const T uc = t.w[q] * Uz[j][q];
            const T fx = uc * Uz[0][q], fy = uc * Uz[1][q], fz = uc * Uz[2][q];
#pragma unroll
            for (int c = 0; c < N; ++c) {
              ox[c] = fmadd(t.S[q][c], fx, ox[c]);
              oy[c] = fmadd(t.S[q][c], fy, oy[c]);
              oz[c] = fmadd(t.G[q][c], fz, oz[c]);
            }
          }
          {   // cell scalings s_d w_q1 w_q2 applied once per output
            const T s0 = sc.cell[0] * w12, s1 = sc.cell[1] * w12, s2 = sc.cell[2] * w12;
#pragma unroll
            for (int c = 0; c < N; ++c) {
              ox[c] *= s0;
              oy[c] *= s1;
              oz[c] *= s2;
            }
          }
          oz[0] += Fz[0][j];
          oz[N - 1] += Fz[1][j];
#pragma unroll
          for (int c = 0; c < N; ++c) {
            colp[(0 * N + c) * COLS] = ox[c];
            colp[(1 * N + c) * COLS] = oy[c];
            colp[(2 * N + c) * COLS] = oz[c];
          }
        }
        __syncthreads();
      }
      back_y(j, j + 1);
      __syncthreads();
      back_x(j, j + 1);
      if (j < 2) __syncthreads();
    }
  }
}

template <int N, int Q, typename T>
static hipError_t launch_conv_nq(const ConvPlan& P, const void* u, void* r, hipStream_t s) {
  using Sh = ConvShape<N, Q, (int)sizeof(T)>;
  // the kernel's compile-time tables must be the plan's tables
  constexpr ct::Tables<N, Q> C{};
  for (int q = 0; q < Q; ++q) {
    if (std::fabs(C.w[q] - P.w[q]) > 1e-13) return hipErrorInvalidValue;
    for (int a = 0; a < N; ++a)
      if (std::fabs(C.S[q][a] - P.S[q * N + a]) > 1e-13 || std::fabs(C.G[q][a] - P.G[q * N + a]) > 1e-11)
        return hipErrorInvalidValue;
  }
  ConvScal<T> sc;
  for (int d = 0; d < 3; ++d) {
    sc.cell[d] = (T)P.cell[d];
    sc.area[d] = (T)P.area[d];
  }
  sc.lf = (T)P.lf;
  const ConvTab<N, Q, T>* dt = nullptr;   // FP32 kernels use the compile-time tables
  if (sizeof(T) == 8) {
    ConvTab<N, Q, T> t;
    for (int q = 0; q < Q; ++q) {
      for (int a = 0; a < N; ++a) {
        t.S[q][a] = (T)P.S[q * N + a];
        t.G[q][a] = (T)P.G[q * N + a];
      }
      t.w[q] = (T)P.w[q];
    }
    hipError_t err;
    dt = device_table_of("convective", t, &err);
    if (!dt) return err;
  }
  const int grid = (P.mesh.n_el + Sh::E - 1) / Sh::E;
  hipLaunchKernelGGL((convective_kernel<N, Q, T, Sh::E, Sh::TH, Sh::ALLC>), dim3(grid), dim3(Sh::TH), 0, s,
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
