// Convective term c_h with the local Lax-Friedrichs flux (Sec. 3.2, weak form
// of c_h, F_c(u) = u (x) u), by sum factorisation on periodic Cartesian meshes,
// FP64 and FP32, degrees 1..11 with floor(3k/2)+1 Gauss points (3/2 rule).
//
//   R_c = -sum_j s_j (d_j phi, u_c u_j)_K + sum_faces (phi, F*_c),   s_j = vol/h_j
//   F*_c = 1/2 (u-_c u-.n + u+_c u+.n) + lf * max(|u-.n|, |u+.n|) (u-_c - u+_c)
//
// 1D tables: S (m x n, LGL -> Gauss interpolation), G (m x n, derivatives of
// the LGL basis at the Gauss points), Gauss weights w.  Every 1D sweep runs in
// even-odd form (see ConvTab), which halves its multiply-adds.
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
//   P1  x sweep of the cell (n^2 pencil positions per element, three
//       components each) and of the y/z neighbour layers, y sweep of the
//       x-face layers; all inputs straight from global memory into registers.
//   P2  y sweep, in place in LDS, of the cell and the two extra z layers.
//   P3  per (q1,q2): z sweep into registers, z-face flux, cell flux and the
//       z back sweep; per (side, q): y- and x-face flux pencils.
//   Y   y back sweep (in place) and the y integral of the x-face terms.
//   X   x back sweep, face end-node terms, write-out.
// Small degrees keep the back sweeps of all three components in LDS at once
// (5 phases); large ones run the Z/Y/X back sweeps per component from the z
// pencils held in registers (11 phases, a third of the LDS).  Where a phase
// has two kinds of items (cell and face pencils), the second kind starts at a
// wavefront boundary, so that no wavefront runs both codes one after the
// other.  FP64 k=11 runs in persistent form: one workgroup per CU walks a
// share of the batches and loads the next batch during the last back pass.
#include <algorithm>
#include <atomic>
#include <cmath>

#include "api_internal.h"
#include "common.h"
#include "conv_common.h"
#include "ops.h"

namespace dgmf {

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
  // about 52 KB per workgroup (three per CU), 1..16 elements; FP64 k=6
  // takes two (76 KB, two workgroups per CU): 10 % faster than three
  // elements in one 512-thread workgroup per CU, once cell and face pencils
  // no longer share wavefronts (before that, three measured 14 % faster)
  static constexpr int E0 = (52 * 1024) / BYTES;
  static constexpr int E = (N == 7 && SZ == 8) ? 2 : (E0 < 1 ? 1 : (E0 > 16 ? 16 : E0));
  // per-component mode keeps one z pencil per thread in registers.  Where
  // one workgroup fills a CU's LDS (the highest degrees) 512 threads hide
  // more latency; below that a larger group only lowers the register limit.
  // FP64 k=7 (121 z pencils, 44 face pencils) runs three wavefronts, the
  // face pencils in the third: 10 % faster than two wavefronts (two rounds
  // of items) and than four; elsewhere fewer threads than 256 cost
  // occupancy (the freed register budget gets used), and 320-thread groups
  // measured slower (FP64 k=4: 2x, FP32 k=9: 33 %)
  static constexpr int TH0 = (N == 8 && SZ == 8) ? 192 : (E * Q * Q > 256) ? ((E * Q * Q + 63) / 64) * 64 : 256;
  static constexpr int TH = ((E == 1 && Q >= 16) || E * BYTES > 80 * 1024) ? (TH0 > 512 ? TH0 : 512) : TH0;
  // minimum wavefronts per SIMD (register cap) where registers, not LDS,
  // limited the groups per CU: at 128 VGPRs FP32 k=11 fits two 512-thread
  // groups (33 % faster despite a small spill) and FP32 k=6 four 256-thread
  // groups (15 % faster)
  static constexpr int MINW = (N == 12 && SZ == 4) ? 4 : (N == 7 && SZ == 4) ? 4 : 1;
  // persistent form: one workgroup per CU walks its batches and loads the
  // next one while finishing the current.  Measured only at FP64 k=11 faster
  // (5 %); at FP64 k=6, 9, 10, also one workgroup per CU, 0 to 5 % slower
  static constexpr bool PERS = N == 12 && SZ == 8;
  // 16-byte loads of contiguous pencils (where n values fill whole 16-byte
  // words; the launch uses them only for a 16-byte aligned input): 2 % (FP64
  // k=9) to 11 % (FP32 k=7) faster; at FP64 k=11 (persistent) 40 % slower
  static constexpr bool VEC = !PERS && (N * SZ) % 16 == 0;
  static_assert(E * PER * SZ <= 160 * 1024, "convective LDS footprint exceeds 160 KB");
};

template <int N, int Q, typename T, int E, int TH, bool ALLC, bool PERS>
__global__ void __launch_bounds__(TH) __attribute__((amdgpu_waves_per_eu(ConvShape<N, Q, (int)sizeof(T)>::MINW, 8)))
convective_kernel(const T* __restrict__ u, T* __restrict__ r, MeshArgs mesh,
                  const ConvTab<N, Q, T>* __restrict__ tab, ConvScal<T> sc, bool u16) {
  using Sh = ConvShape<N, Q, (int)sizeof(T)>;
  static_assert(!(PERS && ALLC), "the persistent form prefetches during the per-component back sweeps");
  static_assert(ALLC || TH >= E * Q * Q, "per-component mode keeps one z pencil per thread in registers");
  constexpr int N2 = Sh::N2, N3 = Sh::N3, MP = Sh::MP, COLS = Sh::COLS, LAYER = Sh::LAYER;
  constexpr int NH = N / 2, QH = Q / 2;
  constexpr int PER = Sh::per(ALLC);
  constexpr int FYo = Sh::slots(ALLC) * COLS;
  constexpr int FXo = FYo + Sh::FL;
  constexpr int XRo = FXo + Sh::FL;
  __shared__ T lds[E * PER];
  // the thread index; in the persistent form opaque to the compiler (its
  // range restated) and taken afresh in each loop step: otherwise the index
  // arithmetic of every phase, which depends on it alone, is hoisted out of
  // the batch loop and held in registers throughout
  auto thread_index = []() {
    int t = threadIdx.x;
    if constexpr (PERS) {
      asm volatile("" : "+v"(t));
      __builtin_assume(t >= 0 && t < TH);
    }
    return t;
  };
  const size_t cs = (size_t)mesh.n_el * N3;
  const int nxy = mesh.nx * mesh.ny;
  // Batches of E consecutive elements taken by this workgroup: one, or in the
  // persistent form every bstep-th batch of its XCD's contiguous share from
  // its index on that XCD (workgroups go round-robin to the 8 XCDs; a grid of
  // fewer than 8 workgroups splits the batches among as many shares), the
  // pencils of the next batch loaded while the current one finishes.
  int bt, bend, bstep;
  if constexpr (PERS) {
    const int nbt = (mesh.n_el + E - 1) / E, G = gridDim.x, x = blockIdx.x & 7;
    const int nx = G < 8 ? G : 8;
    bstep = (G >> 3) + (x < (G & 7) ? 1 : 0);
    bt = (int)((long)nbt * x / nx) + (blockIdx.x >> 3);
    bend = (int)((long)nbt * (x + 1) / nx);
  } else {
    bt = xcd_remap(blockIdx.x, gridDim.x);
    bend = bt + 1;
    bstep = 1;
  }
  // first element of a batch, its element count and the grid position of
  // its first element; element e0 + le lies le steps further along x
  struct Bat {
    int e0, ne, ex, ey, ez;
  };
  auto batch = [&](int b) {
    Bat p;
    p.e0 = b * E;
    p.ne = min(E, mesh.n_el - p.e0);
    p.ez = p.e0 / nxy;
    const int exy = p.e0 - p.ez * nxy;
    p.ey = exy / mesh.nx;
    p.ex = exy - p.ey * mesh.nx;
    return p;
  };
  auto nbr = [&](const Bat& p, int le, int d, int s) {
    int ex = p.ex + le, ey = p.ey, ez = p.ez;
    while (ex >= mesh.nx) {
      ex -= mesh.nx;
      if (++ey == mesh.ny) {
        ey = 0;
        ++ez;
      }
    }
    return neighbor(mesh, ex, ey, ez, d, s);
  };
  auto bar = [&]() {
    if constexpr (PERS) lds_barrier();   // keeps the next batch's loads in flight
    else __syncthreads();
  };

  // ---------------- P1: x sweeps (and y sweeps of x-face layers) from global ----------------
  // An item is one pencil position taken for all three components, which
  // share its index arithmetic; all of a thread's loads are issued before any
  // sweep, so the global load latency is paid once per thread.
  constexpr int nM = E * N2, nL = E * 4 * N, nX = E * 4 * N;   // cell, y/z neighbour, x-face items
  // first x-face item: its strided loads start a wavefront where the others take 16-byte loads
  constexpr int FXI = Sh::VEC ? wave_split(nM + nL, nX, TH) : nM + nL;
  constexpr int total = FXI + nX;
  constexpr int D1S = (N + 2) * COLS;   // component stride of the BC slots
  // item w of batch p -> source pencil of component 0 (src, stride), LDS
  // destination of component 0 (d1) with its component stride (dstr), second
  // destination d2
  auto item = [&](const Bat& p, int w, const T*& src, int& sstride, int& d1, int& dstr, int& d2) {
    sstride = 1;
    d1 = -1;
    d2 = -1;
    dstr = D1S;
    if (w < nM) {   // cell pencil (b, c)
      const int le = w / N2, bc = w - le * N2;
      if (le >= p.ne) return;
      const int b = bc % N, c = bc / N;
      src = u + (size_t)(p.e0 + le) * N3 + N * bc;
      const int L = le * PER;
      d1 = L + (c + 1) * COLS + MP * b;
      if (b == 0) d2 = L + FYo + (0 * 2 + 0) * 3 * LAYER + c * Q;
      else if (b == N - 1) d2 = L + FYo + (0 * 2 + 1) * 3 * LAYER + c * Q;
    } else if (w < nM + nL) {   // y or z neighbour layer pencil, swept in x
      const int v = w - nM;
      const int le = v / (4 * N);
      if (le >= p.ne) return;
      const int rem = v - le * 4 * N;
      const int isz = rem / (2 * N), r2 = rem - isz * 2 * N;
      const int s = r2 / N, q = r2 - s * N;
      const int nb = nbr(p, le, isz ? 2 : 1, s);
      const int lay = s ? 0 : N - 1;   // neighbour's facing layer
      const int L = le * PER;
      if (isz) {   // pencil b = q of z layer lay -> extra z slot
        src = u + (size_t)nb * N3 + N * (q + N * lay);
        d1 = L + (s ? N + 1 : 0) * COLS + MP * q;
      } else {     // pencil c = q of y layer lay -> FY neighbour entry
        src = u + (size_t)nb * N3 + N * (lay + N * q);
        d1 = L + FYo + (1 * 2 + s) * 3 * LAYER + q * Q;
        dstr = LAYER;
      }
    } else if (w >= FXI) {   // x-face layer (own or neighbour), swept in y
      const int v = w - FXI;
      const int le = v / (4 * N);
      if (le >= p.ne) return;
      const int rem = v - le * 4 * N;
      const int sg = rem / (2 * N), r2 = rem - sg * 2 * N;
      const int s = r2 / N, c = r2 - s * N;
      int e = p.e0 + le, a = s ? N - 1 : 0;
      if (sg) {
        e = nbr(p, le, 0, s);
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
  // issue every load of this thread's items of batch p (none if !valid);
  // items without loads get zeros, so that nothing of the previous batch
  // stays live across a loop step
  auto issue = [&](const Bat& p, bool valid) {
    const int tid = thread_index();
#pragma unroll
    for (int i = 0; i < NI1; ++i) {
      const int w = tid + i * TH;
      d1[i] = -1;
      if (valid && w < total) {
        const T* src;
        int sstride;
        item(p, w, src, sstride, d1[i], ds[i], d2[i]);
        if (d1[i] >= 0) {
          bool done = false;
          if constexpr (Sh::VEC) {
            if (u16 && sstride == 1) {
#pragma unroll
              for (int j = 0; j < 3; ++j) load_pencil16<N, T>(src + j * cs, in[i][j]);
              done = true;
            }
          }
          if (!done) {
#pragma unroll
            for (int j = 0; j < 3; ++j) load_pencil<N, Q, T>(src + j * cs, sstride, in[i][j]);
          }
        }
      }
      if constexpr (PERS) {
        if (d1[i] < 0) {
#pragma unroll
          for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int c = 0; c < N; ++c) in[i][j][c] = T(0);
        }
      }
    }
  };
  issue(batch(bt), bt < bend);
  for (; bt < bend; bt += bstep) {
    const int tid = thread_index();
    const Bat cur = batch(bt);
    const int e0 = cur.e0, ne = cur.ne;   // items of le >= ne are skipped
#pragma unroll
    for (int i = 0; i < NI1; ++i) {
      if (d1[i] >= 0) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          CONV_TABLES(t);
          // the second destination, where there is none, repeats the first:
          // one sweep for every item, no divergent copy of it
          T* dst = lds + d1[i] + j * ds[i];
          T* dst2 = d2[i] >= 0 ? lds + d2[i] + j * LAYER : dst;
          eo_interp<N, Q, T>(t, in[i][j], [&](int q, T v) {
            dst[q] = v;
            dst2[q] = v;
          });
        }
      }
    }
    bar();

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
        eo_interp<N, Q, T>(t, in, [&](int q, T v) { p[MP * q] = v; });
      }
    }
    bar();

    // ---------------- P3: z sweeps, fluxes, z back sweep ----------------
    constexpr int nCell = E * Q * Q;
    bool own_cell = false;   // this thread holds the z pencil of cell item tid
    T Uz[3][Q];
    T Fz[2][3];
    T w12 = 0;
    T* colp = lds;   // this thread's column (per-component mode)
    if constexpr (PERS) {
      // defined on every path, so that the pencil of the previous batch is not
      // carried (and kept in registers) through the face-pencil branch below
#pragma unroll
      for (int j = 0; j < 3; ++j) {
#pragma unroll
        for (int q = 0; q < Q; ++q) Uz[j][q] = T(0);
        Fz[0][j] = Fz[1][j] = T(0);
      }
    }
    // z back sweep of component j of the thread's pencil into slot set jj:
    // S^T_z F_jx, S^T_z F_jy, G^T_z F_jz (+ z-face terms at the end nodes)
    auto zback = [&](int j, int jj, T* col) {
      CONV_TABLES(t);
      EoT<N, T, 1> ax, ay;
      EoT<N, T, -1> az;
      ax.zero();
      ay.zero();
      az.zero();
#pragma unroll
      for (int q = 0; q < QH; ++q) {
        const int rq = Q - 1 - q;
        const T uq = t.w[q] * Uz[j][q], ur = t.w[q] * Uz[j][rq];   // w[m-1-q] = w[q]
        ax.pair(t.Tp[q], t.Tm[q], uq * Uz[0][q], ur * Uz[0][rq]);
        ay.pair(t.Tp[q], t.Tm[q], uq * Uz[1][q], ur * Uz[1][rq]);
        az.pair(t.Hp[q], t.Hm[q], uq * Uz[2][q], ur * Uz[2][rq]);
      }
      if constexpr (Q % 2 == 1) {
        const T um = t.w[QH] * Uz[j][QH];
        ax.mid(t.Tc, um * Uz[0][QH]);
        ay.mid(t.Tc, um * Uz[1][QH]);
        az.mid(t.Hc, um * Uz[2][QH]);
      }
      // cell scalings s_d w_q1 w_q2 applied once per output
      const T s0 = sc.cell[0] * w12, s1 = sc.cell[1] * w12, s2 = sc.cell[2] * w12;
#pragma unroll
      for (int c = 0; c < N; ++c) {
        T oz = s2 * az.out(c);
        if (c == 0) oz += Fz[0][j];
        if (c == N - 1) oz += Fz[1][j];
        col[((jj * 3 + 0) * N + c) * COLS] = s0 * ax.out(c);
        col[((jj * 3 + 1) * N + c) * COLS] = s1 * ay.out(c);
        col[((jj * 3 + 2) * N + c) * COLS] = oz;
      }
    };
    {
      constexpr int nH = E * 4 * Q;
      constexpr int FO = wave_split(nCell, nH, TH);   // first face-pencil item
      for (int w = tid; w < FO + nH; w += TH) {
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
          {
            CONV_TABLES(t);
#pragma unroll
            for (int j = 0; j < 3; ++j) {
              T x[N];
#pragma unroll
              for (int c = 0; c < N; ++c) x[c] = v[j][c + 1];
              eo_interp<N, Q, T>(t, x, [&](int q, T val) { Uz[j][q] = val; });
            }
            w12 = t.w[q1] * t.w[q2];
          }
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
          for (int j = 0; j < (ALLC ? 3 : 1); ++j) zback(j, j, col);
        } else if (w >= FO) {   // face-flux pencil: fam 0 = y face (q = q1), 1 = x face (q = q2)
          const int h = w - FO;
          const int le = h / (4 * Q);
          if (le >= ne) continue;
          CONV_TABLES(t);
          int rem = h - le * 4 * Q;
          const int fam = rem / (2 * Q);
          rem -= fam * 2 * Q;
          const int s = rem / Q, q = rem - s * Q;
          T* F = lds + le * PER + (fam ? FXo : FYo) + q;
          // even-odd parts of the own (0) and neighbour (1) pencils of each component
          T xe[2][3][NH], xo[2][3][NH], xm[2][3];
#pragma unroll
          for (int sg = 0; sg < 2; ++sg)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
              T x[N];
#pragma unroll
              for (int c = 0; c < N; ++c) x[c] = F[((sg * 2 + s) * 3 + j) * LAYER + c * Q];
#pragma unroll
              for (int a = 0; a < NH; ++a) {
                xe[sg][j][a] = x[a] + x[N - 1 - a];
                xo[sg][j][a] = x[a] - x[N - 1 - a];
              }
              xm[sg][j] = (N % 2) ? x[NH] : T(0);
            }
          EoT<N, T, 1> acc[3];
#pragma unroll
          for (int j = 0; j < 3; ++j) acc[j].zero();
          const T sgn = s ? T(1) : T(-1);
          const T wq = t.w[q] * (fam ? sc.area[0] : sc.area[1]);
          // fluxes f[j] at a face point with traces um (own), up (neighbour)
          auto flux = [&](const T (&um)[3], const T (&up)[3], T wgt, T (&f)[3]) {
            const T unm = sgn * (fam ? um[0] : um[1]), unp = sgn * (fam ? up[0] : up[1]);
            const T lam = fmax(fabs(unm), fabs(unp));
#pragma unroll
            for (int j = 0; j < 3; ++j) f[j] = llf(um[j], up[j], unm, unp, lam, sc.lf, wgt);
          };
#pragma unroll
          for (int q3 = 0; q3 < (Q + 1) / 2; ++q3) {
            // traces at q3 and at its mirror m-1-q3
            T umq[3], upq[3], umr[3], upr[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
              T e0v = t.Sp[q3][0] * xe[0][j][0], o0v = t.Sm[q3][0] * xo[0][j][0];
              T e1v = t.Sp[q3][0] * xe[1][j][0], o1v = t.Sm[q3][0] * xo[1][j][0];
#pragma unroll
              for (int a = 1; a < NH; ++a) {
                e0v = fmadd(t.Sp[q3][a], xe[0][j][a], e0v);
                o0v = fmadd(t.Sm[q3][a], xo[0][j][a], o0v);
                e1v = fmadd(t.Sp[q3][a], xe[1][j][a], e1v);
                o1v = fmadd(t.Sm[q3][a], xo[1][j][a], o1v);
              }
              if constexpr (N % 2 == 1) {
                e0v = fmadd(t.Sc[q3], xm[0][j], e0v);
                e1v = fmadd(t.Sc[q3], xm[1][j], e1v);
              }
              umq[j] = e0v + o0v;
              upq[j] = e1v + o1v;
              umr[j] = e0v - o0v;
              upr[j] = e1v - o1v;
            }
            const T wgt = wq * t.w[q3];
            T fq[3];
            flux(umq, upq, wgt, fq);
            if (q3 < QH) {
              T fr[3];
              flux(umr, upr, wgt, fr);
#pragma unroll
              for (int j = 0; j < 3; ++j) acc[j].pair(t.Tp[q3], t.Tm[q3], fq[j], fr[j]);
            } else {
#pragma unroll
              for (int j = 0; j < 3; ++j) acc[j].mid(t.Tc, fq[j]);
            }
          }
#pragma unroll
          for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int c = 0; c < N; ++c) F[((0 * 2 + s) * 3 + j) * LAYER + c * Q] = acc[j].out(c);
        }
      }
    }
    bar();

    // ---------------- Y and X back sweeps ----------------
    // component range [j0, j1) uses slot set jj = ALLC ? j : 0
    auto back_y = [&](int j0, int j1) {
      const int nc = j1 - j0;
      const int nYc = nc * E * N * Q, nXf = nc * E * 2 * N;
      const int FX = wave_split(nYc, nXf, TH);   // first x-face item
      for (int w = tid; w < FX + nXf; w += TH) {
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
          // v1 = S^T_y T_x, v2 = G^T_y T_y + S^T_y T_z
          EoT<N, T, 1> v1, v2s;
          EoT<N, T, -1> v2g;
          v1.zero();
          v2s.zero();
          v2g.zero();
#pragma unroll
          for (int q2 = 0; q2 < QH; ++q2) {
            const int r2 = Q - 1 - q2;
            v1.pair(t.Tp[q2], t.Tm[q2], tb[sx + MP * q2], tb[sx + MP * r2]);
            v2g.pair(t.Hp[q2], t.Hm[q2], tb[sy + MP * q2], tb[sy + MP * r2]);
            v2s.pair(t.Tp[q2], t.Tm[q2], tb[sz + MP * q2], tb[sz + MP * r2]);
          }
          if constexpr (Q % 2 == 1) {
            v1.mid(t.Tc, tb[sx + MP * QH]);
            v2g.mid(t.Hc, tb[sy + MP * QH]);
            v2s.mid(t.Tc, tb[sz + MP * QH]);
          }
          const T f0 = L[FYo + ((0 * 2 + 0) * 3 + j) * LAYER + cz * Q + q1];
          const T f1 = L[FYo + ((0 * 2 + 1) * 3 + j) * LAYER + cz * Q + q1];
#pragma unroll
          for (int b = 0; b < N; ++b) {
            T o2 = v2g.out(b) + v2s.out(b);
            if (b == 0) o2 += f0;
            if (b == N - 1) o2 += f1;
            tb[sx + MP * b] = v1.out(b);
            tb[sy + MP * b] = o2;
          }
        } else if (w >= FX) {   // x-face terms: integrate in y
          const int v = w - FX;
          const int cz = v % N, rest = v / N;
          const int s = rest % 2, jl = rest / 2;
          const int le = jl % E, j = j0 + jl / E;
          if (le >= ne) continue;
          const int jj = ALLC ? j : 0;
          T* L = lds + le * PER;
          const T* xf = L + FXo + ((0 * 2 + s) * 3 + j) * LAYER + cz * Q;
          EoT<N, T, 1> o;
          o.zero();
#pragma unroll
          for (int q2 = 0; q2 < QH; ++q2) o.pair(t.Tp[q2], t.Tm[q2], xf[q2], xf[Q - 1 - q2]);
          if constexpr (Q % 2 == 1) o.mid(t.Tc, xf[QH]);
          T* xr = L + XRo + ((jj * 2 + s) * N + cz) * N;
#pragma unroll
          for (int b = 0; b < N; ++b) xr[b] = o.out(b);
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
        // o = G^T_x v1 + S^T_x v2
        EoT<N, T, -1> og;
        EoT<N, T, 1> os;
        og.zero();
        os.zero();
#pragma unroll
        for (int q1 = 0; q1 < QH; ++q1) {
          og.pair(t.Hp[q1], t.Hm[q1], v1[q1], v1[Q - 1 - q1]);
          os.pair(t.Tp[q1], t.Tm[q1], v2[q1], v2[Q - 1 - q1]);
        }
        if constexpr (Q % 2 == 1) {
          og.mid(t.Hc, v1[QH]);
          os.mid(t.Tc, v2[QH]);
        }
        const T* xr = L + XRo + (jj * 2 * N + cz) * N + b;
        const T x0 = xr[0], x1 = xr[N2];
        T* g = r + j * cs + (size_t)(e0 + le) * N3 + N * bc;
#pragma unroll
        for (int a = 0; a < N; ++a) {
          T o = og.out(a) + os.out(a);
          if (a == 0) o += x0;
          if (a == N - 1) o += x1;
          g[a] = o;
        }
      }
    };

    if constexpr (ALLC) {
      back_y(0, 3);
      bar();
      back_x(0, 3);
    } else {
      // per component: the thread's own z pencil (tid < nCell) is still in registers
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        if (j > 0) {
          if (own_cell) zback(j, 0, colp);
          bar();
        }
        // the z pencils are done with: load the next batch during the last pass
        if constexpr (PERS)
          if (j == 2) issue(batch(bt + bstep), bt + bstep < bend);
        back_y(j, j + 1);
        bar();
        back_x(j, j + 1);
        if (j < 2) bar();
      }
    }
    if constexpr (PERS) bar();   // the next batch's P1 overwrites the slots read above
  }
}

// compute units of the current device, cached per device
static hipError_t cu_count(int* n) {
  static std::atomic<int> cache[64];
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 64 && (*n = cache[dev].load(std::memory_order_relaxed)) > 0) return hipSuccess;
  e = hipDeviceGetAttribute(n, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess && *n < 1) e = hipErrorInvalidDevice;
  if (e == hipSuccess && dev < 64) cache[dev].store(*n, std::memory_order_relaxed);
  return e;
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
    const ConvTab<N, Q, T> t = make_conv_tab<N, Q, T>(P.S.data(), P.G.data(), P.w.data());
    hipError_t err;
    dt = device_table_of("convective", t, &err);
    if (!dt) return err;
  }
  int grid = (P.mesh.n_el + Sh::E - 1) / Sh::E;
  if (Sh::PERS) {
    int cus = 0;
    const hipError_t err = cu_count(&cus);
    if (err != hipSuccess) return err;
    grid = std::min(grid, cus);
  }
  // every pencil of n contiguous values starts at a multiple of n values
  // from u, so a 16-byte aligned u aligns them all where n values fill whole
  // 16-byte words
  const bool u16 = Sh::VEC && (reinterpret_cast<uintptr_t>(u) % 16) == 0;
  hipLaunchKernelGGL((convective_kernel<N, Q, T, Sh::E, Sh::TH, Sh::ALLC, Sh::PERS>), dim3(grid), dim3(Sh::TH), 0,
                     s, (const T*)u, (T*)r, P.mesh, dt, sc, u16);
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
