// Vector-Jacobian product of the convective term: g = J(u)^T w, by sum
// factorisation, FP64 and FP32, k <= 11, floor(3k/2)+1 Gauss points.
//
// Linearising R_c = -sum_j s_j (d_j phi, u_c u_j) + faces (Sec. 3.2, weak
// form of c_h) and transposing against the coefficient vector w gives
//   cell:  g_k = (phi, W P_k),  P_k = sum_j c_j u_j d_j w_k + c_k sum_c u_c d_k w_c,
//          c_j = -vol/h_j (reference derivatives), W the Gauss weights,
//   faces: g_k += area * (phi, sum_i (w-_i - w+_i) dF*_i/du-_k), with
//          dF*_i/du-_k = 1/2 (delta_ik u-.n + u-_i n_k)
//                      + lf [ L delta_ik + (u-_i - u+_i) s- sign(u-.n) n_k ],
//          L = max(|u-.n|, |u+.n|), s- = 1, 1/2, 0 as |u-.n| >, =, < |u+.n|.
// Each element differentiates only through its own traces u-, so every
// element writes its own coefficients (no atomics).
//
// Two kernels, both organised like the convective kernel (conv_common.h
// holds the even-odd tables and sweeps), both with the faces folded into
// the cell sweeps:
//
// One-pass kernel (k <= 7): all of u and w in LDS at once.
//   P1  x sweeps from global memory: u -> S_x u; w -> S_x w and G_x w; the
//       y/z neighbour layers of u and w -> S_x; the x-face layers -> S_y.
//   P2  y sweeps in place: S_y S_x u, S_y S_x w (and G_y S_x w beside it),
//       S_y G_x w; the two extra z layers of u and w come along.
//   P3  per (q1,q2) z pencil: u, d_x w, d_y w, d_z w at the m Gauss points
//       (S_z, S_z, S_z, G_z), P_k, and the back sweep S^T_z W P_k, with the
//       z-face terms added at the end nodes; per (side, q) face pencil of the
//       y and x faces: traces of u and w, the transposed flux derivative at
//       the m face points, and S^T_z.
//   Y   S^T_y (in place) plus the y-face terms; S^T_y of the x-face terms.
//   X   S^T_x plus the x-face terms, write-out.
//
// Per-component kernel (k >= 8): P_k is linear in w and the face terms are
// linear in w- - w+, so this kernel takes the components of w one at a time.
// u stays in LDS for the whole kernel, the sweeps of w_i replace those of
// w_{i-1}, and every pencil adds the share of w_i to accumulators it keeps in
// registers over the three passes.  Only one component of w is in LDS at a
// time, which about halves the LDS per element; the z pencils redo the
// sweeps of u in every pass, which is why the one-pass kernel is kept where
// it fits.
//   P1u  x sweeps of u as in P1.
//   per pass i = 0, 1, 2 (the loads of w_{i+1} stay in flight during the
//   sweeps of pass i):
//   P1w  the same x sweeps of w_i, and G_x w_i.
//   P2   y sweeps in place: S_y S_x u (first pass only); S_y S_x w_i, with
//        G_y S_x w_i beside it; S_y G_x w_i.
//   P3   as in the one-pass kernel with the share of w_i, accumulated in
//        registers.
//   Y, X as in the one-pass kernel.
// Where the G_x and G_y slots of w_i do not fit in LDS (FP64, k >= 10), the
// z pencils form d_x w_i and d_y w_i from S_y S_x w_i instead, by the
// collocation derivative at the Gauss points along q1 and q2.  That is exact:
// along each line the values are those of a polynomial of degree k < m.
// Where even that does not fit (FP64, k = 11), the x faces are taken after
// the three passes, in LDS the passes have freed.
// The back sweeps use S^T only, so all three components fit at once.
#include <cmath>

#include "api_internal.h"
#include "common.h"
#include "conv_common.h"
#include "ops.h"

namespace dgmf {

// Collocation derivative at the m Gauss points: d[q][p] = l_p'(z_q) for the
// Lagrange basis of the Gauss points (barycentric form).
template <int Q, typename T>
struct GaussDeriv {
  T d[Q][Q];
};

template <int N, int Q, typename T>
static GaussDeriv<Q, T> make_gauss_deriv() {
  constexpr ct::Tables<N, Q> C{};
  double lam[Q];
  for (int p = 0; p < Q; ++p) {
    double prod = 1.0;
    for (int r = 0; r < Q; ++r)
      if (r != p) prod *= C.z[p] - C.z[r];
    lam[p] = 1.0 / prod;
  }
  GaussDeriv<Q, T> D{};
  for (int q = 0; q < Q; ++q) {
    double diag = 0.0;
    for (int p = 0; p < Q; ++p) {
      if (p == q) continue;
      const double v = lam[p] / lam[q] / (C.z[q] - C.z[p]);
      D.d[q][p] = (T)v;
      diag -= v;
    }
    D.d[q][q] = (T)diag;
  }
  return D;
}

// ======================= one-pass kernel =======================
// LDS layout of one element (units of T); column blocks (q1, q2) with q1
// pitch MP as in the convective kernel.
//   slots [0, 3(n+2)):         U_j, S_y S_x u_j at z layer c in -1..n
//   slots [3(n+2), 6(n+2)):    WS_j, S_y S_x w_j at z layer c in -1..n
//   then 3n slots:             WGY_j, G_y S_x w_j
//   then 3n slots:             WGX_j, S_y G_x w_j
//   back sweep:                slot k*n + cz holds S^T_z W P_k (+ z faces),
//                              then S^T_y of it in place (own columns only)
//   face layers FY, FX:        [sigma][s][f][j][c][q], f = 0 (u), 1 (w); the
//                              face pencils overwrite (0, s, 0, k) with their
//                              S^T_z result for component k
//   XR:                        x-face terms after S^T_y, [k][s][cz][b]
template <int N, int Q, int SZ>
struct VjpShape1 {
  static constexpr int N2 = N * N, N3 = N * N * N;
  static constexpr int MP = Q | 1;
  static constexpr int COLS = MP * Q;
  static constexpr int LAYER = N * Q;
  static constexpr int SU = 0, SWS = 3 * (N + 2), SWGY = 6 * (N + 2), SWGX = 6 * (N + 2) + 3 * N;
  static constexpr int SLOTS = 6 * (N + 2) + 6 * N;
  static constexpr int FL = 24 * LAYER;
  static constexpr int PER = SLOTS * COLS + 2 * FL + 6 * N2;
  static constexpr int BYTES = PER * SZ;
  static constexpr int E0 = (52 * 1024) / BYTES;
  static constexpr int E = E0 < 1 ? 1 : (E0 > 16 ? 16 : E0);
  static constexpr int TH = (E * Q * Q >= 96) ? 256 : 128;
  static constexpr bool FITS = E * PER * SZ <= 160 * 1024;
};

template <int N, int Q, typename T, int E, int TH>
__global__ void __launch_bounds__(TH)
vjp_onepass_kernel(const T* __restrict__ u, const T* __restrict__ wv, T* __restrict__ g, MeshArgs mesh,
                   const ConvTab<N, Q, T>* __restrict__ tab, ConvScal<T> sc, bool a16) {
  using Sh = VjpShape1<N, Q, (int)sizeof(T)>;
  constexpr int N2 = Sh::N2, N3 = Sh::N3, MP = Sh::MP, COLS = Sh::COLS, LAYER = Sh::LAYER, PER = Sh::PER;
  constexpr int NH = N / 2, QH = Q / 2;
  constexpr int FYo = Sh::SLOTS * COLS, FXo = FYo + Sh::FL, XRo = FXo + Sh::FL;
  __shared__ T lds[E * PER];
  const int tid = threadIdx.x;
  const int e0 = xcd_remap(blockIdx.x, gridDim.x) * E;
  const int ne = min(E, mesh.n_el - e0);   // items of le >= ne are skipped
  const size_t cs = (size_t)mesh.n_el * N3;
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
  // offset of face-layer entry (sigma, s, f, j)
  auto fl = [](int sg, int s, int f, int j) { return (((sg * 2 + s) * 2 + f) * 3 + j) * LAYER; };

  // ---------------- P1: x sweeps from global (all loads first) ----------------
  {
    constexpr int nM = E * N2, nL = E * 4 * N, nX = E * 4 * N;
    constexpr int total = nM + nL + nX;
    constexpr int NI1 = (total + TH - 1) / TH;
    // kind 0: cell pencil, 1: y/z neighbour layer, 2: x-face layer
    T in[NI1][2][3][N];
    int kind[NI1], le_[NI1], a1[NI1], a2[NI1], a3[NI1];
#pragma unroll
    for (int i = 0; i < NI1; ++i) {
      const int w = tid + i * TH;
      kind[i] = -1;
      if (w >= total) continue;
      size_t off;
      int sstride = 1;
      if (w < nM) {
        const int le = w / N2, bc = w - le * N2;
        if (le >= ne) continue;
        kind[i] = 0;
        le_[i] = le;
        a1[i] = bc;
        off = (size_t)(e0 + le) * N3 + N * bc;
      } else if (w < nM + nL) {
        const int v = w - nM;
        const int le = v / (4 * N);
        if (le >= ne) continue;
        const int rem = v - le * 4 * N;
        const int isz = rem / (2 * N), r2 = rem - isz * 2 * N;
        const int s = r2 / N, p = r2 - s * N;
        kind[i] = 1;
        le_[i] = le;
        a1[i] = isz;
        a2[i] = s;
        a3[i] = p;
        const int nb = nbr(le, isz ? 2 : 1, s);
        const int lay = s ? 0 : N - 1;   // neighbour's facing layer
        off = (size_t)nb * N3 + (isz ? N * (p + N * lay) : N * (lay + N * p));
      } else {
        const int v = w - nM - nL;
        const int le = v / (4 * N);
        if (le >= ne) continue;
        const int rem = v - le * 4 * N;
        const int sg = rem / (2 * N), r2 = rem - sg * 2 * N;
        const int s = r2 / N, c = r2 - s * N;
        kind[i] = 2;
        le_[i] = le;
        a1[i] = sg;
        a2[i] = s;
        a3[i] = c;
        int e = e0 + le, a = s ? N - 1 : 0;
        if (sg) {
          e = nbr(le, 0, s);
          a = s ? 0 : N - 1;
        }
        sstride = N;
        off = (size_t)e * N3 + a + N2 * c;
      }
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        load_pencil_a16<N, Q, T>(u + j * cs + off, sstride, a16, in[i][0][j]);
        load_pencil_a16<N, Q, T>(wv + j * cs + off, sstride, a16, in[i][1][j]);
      }
    }
#pragma unroll
    for (int i = 0; i < NI1; ++i) {
      if (kind[i] < 0) continue;
      T* L = lds + le_[i] * PER;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        CONV_TABLES(t);
        if (kind[i] == 0) {
          const int bc = a1[i], b = bc % N, c = bc / N;
          T* du = L + (Sh::SU + j * (N + 2) + c + 1) * COLS + MP * b;
          T* dw = L + (Sh::SWS + j * (N + 2) + c + 1) * COLS + MP * b;
          T* dg = L + (Sh::SWGX + j * N + c) * COLS + MP * b;
          const int side = b == 0 ? 0 : (b == N - 1 ? 1 : -1);
          if (side >= 0) {   // own y-face layer: also into FY
            T* fu = L + FYo + fl(0, side, 0, j) + c * Q;
            T* fw = L + FYo + fl(0, side, 1, j) + c * Q;
            eo_interp<N, Q, T>(t, in[i][0][j], [&](int q, T val) {
              du[q] = val;
              fu[q] = val;
            });
            eo_interp<N, Q, T>(t, in[i][1][j], [&](int q, T val) {
              dw[q] = val;
              fw[q] = val;
            });
          } else {
            eo_interp<N, Q, T>(t, in[i][0][j], [&](int q, T val) { du[q] = val; });
            eo_interp<N, Q, T>(t, in[i][1][j], [&](int q, T val) { dw[q] = val; });
          }
          eo_interp_g<N, Q, T>(t, in[i][1][j], [&](int q, T val) { dg[q] = val; });
        } else if (kind[i] == 1) {
          const int isz = a1[i], s = a2[i], p = a3[i];
          T *du, *dw;
          if (isz) {   // pencil b = p of the neighbour's z layer -> extra z slot
            du = L + (Sh::SU + j * (N + 2) + (s ? N + 1 : 0)) * COLS + MP * p;
            dw = L + (Sh::SWS + j * (N + 2) + (s ? N + 1 : 0)) * COLS + MP * p;
          } else {     // pencil c = p of the neighbour's y layer -> FY
            du = L + FYo + fl(1, s, 0, j) + p * Q;
            dw = L + FYo + fl(1, s, 1, j) + p * Q;
          }
          eo_interp<N, Q, T>(t, in[i][0][j], [&](int q, T val) { du[q] = val; });
          eo_interp<N, Q, T>(t, in[i][1][j], [&](int q, T val) { dw[q] = val; });
        } else {
          const int sg = a1[i], s = a2[i], c = a3[i];
          T* du = L + FXo + fl(sg, s, 0, j) + c * Q;
          T* dw = L + FXo + fl(sg, s, 1, j) + c * Q;
          eo_interp<N, Q, T>(t, in[i][0][j], [&](int q, T val) { du[q] = val; });
          eo_interp<N, Q, T>(t, in[i][1][j], [&](int q, T val) { dw[q] = val; });
        }
      }
    }
  }
  __syncthreads();

  // ---------------- P2: y sweeps in place ----------------
  {
    constexpr int nUW = 2 * 3 * E * (N + 2) * Q, nG = 3 * E * N * Q;
    constexpr int FG = wave_split(nUW, nG, TH);   // first WGX item
    for (int w = tid; w < FG + nG; w += TH) {
      CONV_TABLES(t);
      if (w < nUW) {   // U or WS column block (q1, layer c')
        const int q1 = w % Q, rest = w / Q;
        const int cl = rest % (N + 2), r2 = rest / (N + 2);
        const int le = r2 % E, jw = r2 / E;   // jw = which*3 + j
        if (le >= ne) continue;
        const int which = jw / 3, j = jw - which * 3;
        T* L = lds + le * PER;
        T* p = L + ((which ? Sh::SWS : Sh::SU) + j * (N + 2) + cl) * COLS + q1;
        T x[N];
#pragma unroll
        for (int b = 0; b < N; ++b) x[b] = p[MP * b];
        if (which && cl >= 1 && cl <= N) {   // w: also G_y into WGY (interior layers)
          T* pg = L + (Sh::SWGY + j * N + cl - 1) * COLS + q1;
          eo_interp_g<N, Q, T>(t, x, [&](int q, T val) { pg[MP * q] = val; });
        }
        eo_interp<N, Q, T>(t, x, [&](int q, T val) { p[MP * q] = val; });
      } else if (w >= FG) {   // WGX column block: S_y in place
        const int v = w - FG;
        const int q1 = v % Q, rest = v / Q;
        const int c = rest % N, r2 = rest / N;
        const int le = r2 % E, j = r2 / E;
        if (le >= ne) continue;
        T* p = lds + le * PER + (Sh::SWGX + j * N + c) * COLS + q1;
        T x[N];
#pragma unroll
        for (int b = 0; b < N; ++b) x[b] = p[MP * b];
        eo_interp<N, Q, T>(t, x, [&](int q, T val) { p[MP * q] = val; });
      }
    }
  }
  __syncthreads();

  // transposed flux derivative at one face point from the own/neighbour
  // traces of u and w; normal index d, outward sign sgn; G_k weighted by wgt
  auto face_adj = [&](const T (&um)[3], const T (&up)[3], const T (&wm)[3], const T (&wp)[3], int d, T sgn,
                      T wgt, T (&G)[3]) {
    const T unm = sgn * (d == 0 ? um[0] : (d == 1 ? um[1] : um[2]));
    const T unp = sgn * (d == 0 ? up[0] : (d == 1 ? up[1] : up[2]));
    const T am = fabs(unm), ap = fabs(unp);
    const T lam = fmax(am, ap);
    const T sm = am > ap ? T(1) : (am == ap ? T(0.5) : T(0));
    const T sgu = unm > T(0) ? T(1) : (unm < T(0) ? T(-1) : T(0));
    T dw[3], sdu = 0, sdj = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      dw[i] = wm[i] - wp[i];
      sdu = fmadd(dw[i], um[i], sdu);
      sdj = fmadd(dw[i], um[i] - up[i], sdj);
    }
    const T diag = T(0.5) * unm + sc.lf * lam;
    const T extra = sgn * (T(0.5) * sdu + sc.lf * sm * sgu * sdj);
#pragma unroll
    for (int k = 0; k < 3; ++k) G[k] = wgt * (dw[k] * diag + (k == d ? extra : T(0)));
  };

  // ---------------- P3: z pencils and face pencils ----------------
  {
    constexpr int nCell = E * Q * Q, nH = E * 4 * Q;
    constexpr int FO = wave_split(nCell, nH, TH);   // first face-pencil item
    for (int w = tid; w < FO + nH; w += TH) {
      CONV_TABLES(t);
      if (w < nCell) {
        const int le = w / (Q * Q), qq = w - le * (Q * Q);
        if (le >= ne) continue;
        const int q2 = qq / Q, q1 = qq - q2 * Q;
        T* col = lds + le * PER + q1 + MP * q2;
        const T w12 = t.w[q1] * t.w[q2];
        // z faces from the layers -1, 0, n-1, n of U and WS
        T Gz[2][3];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          T um[3], up[3], wm[3], wp[3];
          const int own = s ? N : 1, nb = s ? N + 1 : 0;
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            um[j] = col[(Sh::SU + j * (N + 2) + own) * COLS];
            up[j] = col[(Sh::SU + j * (N + 2) + nb) * COLS];
            wm[j] = col[(Sh::SWS + j * (N + 2) + own) * COLS];
            wp[j] = col[(Sh::SWS + j * (N + 2) + nb) * COLS];
          }
          face_adj(um, up, wm, wp, 2, s ? T(1) : T(-1), w12 * sc.area[2], Gz[s]);
        }
        // even-odd parts of the interior columns: f = 0 U (S_z: u), 1 WGX
        // (S_z: d_x w), 2 WGY (S_z: d_y w), 3 WS (G_z: d_z w)
        T xe[4][3][NH], xo[4][3][NH], xm[4][3];
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            T x[N];
#pragma unroll
            for (int c = 0; c < N; ++c) {
              const int slot = f == 0   ? Sh::SU + j * (N + 2) + c + 1
                               : f == 1 ? Sh::SWGX + j * N + c
                               : f == 2 ? Sh::SWGY + j * N + c
                                        : Sh::SWS + j * (N + 2) + c + 1;
              x[c] = col[slot * COLS];
            }
#pragma unroll
            for (int a = 0; a < NH; ++a) {
              xe[f][j][a] = x[a] + x[N - 1 - a];
              xo[f][j][a] = x[a] - x[N - 1 - a];
            }
            xm[f][j] = (N % 2) ? x[NH] : T(0);
          }
        EoT<N, T, 1> acc[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) acc[k].zero();
        // W_q3 P_k at one point from u and d_x w, d_y w, d_z w
        auto pk = [&](const T (&uu)[3], const T (&dx)[3], const T (&dy)[3], const T (&dz)[3], T wq, T (&P)[3]) {
          const T cu0 = sc.cell[0] * uu[0], cu1 = sc.cell[1] * uu[1], cu2 = sc.cell[2] * uu[2];
          const T ux = uu[0] * dx[0] + uu[1] * dx[1] + uu[2] * dx[2];
          const T uy = uu[0] * dy[0] + uu[1] * dy[1] + uu[2] * dy[2];
          const T uz = uu[0] * dz[0] + uu[1] * dz[1] + uu[2] * dz[2];
#pragma unroll
          for (int k = 0; k < 3; ++k) P[k] = cu0 * dx[k] + cu1 * dy[k] + cu2 * dz[k];
          P[0] = wq * fmadd(sc.cell[0], ux, P[0]);
          P[1] = wq * fmadd(sc.cell[1], uy, P[1]);
          P[2] = wq * fmadd(sc.cell[2], uz, P[2]);
        };
#pragma unroll
        for (int q = 0; q < (Q + 1) / 2; ++q) {
          // the four fields at q and at its mirror m-1-q
          T vq[4][3], vr[4][3];
#pragma unroll
          for (int f = 0; f < 4; ++f)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
              T e, o;
              if (f == 3) {
                e = t.Gp[q][0] * xe[f][j][0];
                o = t.Gm[q][0] * xo[f][j][0];
#pragma unroll
                for (int a = 1; a < NH; ++a) {
                  e = fmadd(t.Gp[q][a], xe[f][j][a], e);
                  o = fmadd(t.Gm[q][a], xo[f][j][a], o);
                }
                if constexpr (N % 2 == 1) e = fmadd(t.Gc[q], xm[f][j], e);
                vq[f][j] = e + o;
                vr[f][j] = o - e;
              } else {
                e = t.Sp[q][0] * xe[f][j][0];
                o = t.Sm[q][0] * xo[f][j][0];
#pragma unroll
                for (int a = 1; a < NH; ++a) {
                  e = fmadd(t.Sp[q][a], xe[f][j][a], e);
                  o = fmadd(t.Sm[q][a], xo[f][j][a], o);
                }
                if constexpr (N % 2 == 1) e = fmadd(t.Sc[q], xm[f][j], e);
                vq[f][j] = e + o;
                vr[f][j] = e - o;
              }
            }
          T Pq[3];
          pk(vq[0], vq[1], vq[2], vq[3], t.w[q], Pq);
          if (q < QH) {
            T Pr[3];
            pk(vr[0], vr[1], vr[2], vr[3], t.w[q], Pr);   // w[m-1-q] = w[q]
#pragma unroll
            for (int k = 0; k < 3; ++k) acc[k].pair(t.Tp[q], t.Tm[q], Pq[k], Pr[k]);
          } else {
#pragma unroll
            for (int k = 0; k < 3; ++k) acc[k].mid(t.Tc, Pq[k]);
          }
        }
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
          for (int c = 0; c < N; ++c) {
            T o = w12 * acc[k].out(c);
            if (c == 0) o += Gz[0][k];
            if (c == N - 1) o += Gz[1][k];
            col[(k * N + c) * COLS] = o;
          }
      } else if (w >= FO) {   // face pencil: fam 0 = y face (q = q1), 1 = x face (q = q2)
        const int h = w - FO;
        const int le = h / (4 * Q);
        if (le >= ne) continue;
        int rem = h - le * 4 * Q;
        const int fam = rem / (2 * Q);
        rem -= fam * 2 * Q;
        const int s = rem / Q, q = rem - s * Q;
        T* F = lds + le * PER + (fam ? FXo : FYo) + q;
        // even-odd parts of the (sigma, f, j) pencils
        T xe[2][2][3][NH], xo[2][2][3][NH], xm[2][2][3];
#pragma unroll
        for (int sg = 0; sg < 2; ++sg)
#pragma unroll
          for (int f = 0; f < 2; ++f)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
              T x[N];
#pragma unroll
              for (int c = 0; c < N; ++c) x[c] = F[fl(sg, s, f, j) + c * Q];
#pragma unroll
              for (int a = 0; a < NH; ++a) {
                xe[sg][f][j][a] = x[a] + x[N - 1 - a];
                xo[sg][f][j][a] = x[a] - x[N - 1 - a];
              }
              xm[sg][f][j] = (N % 2) ? x[NH] : T(0);
            }
        EoT<N, T, 1> acc[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) acc[k].zero();
        const T sgn = s ? T(1) : T(-1);
        const int d = fam ? 0 : 1;
        const T wq = t.w[q] * (fam ? sc.area[0] : sc.area[1]);
#pragma unroll
        for (int q3 = 0; q3 < (Q + 1) / 2; ++q3) {
          T vq[2][2][3], vr[2][2][3];
#pragma unroll
          for (int sg = 0; sg < 2; ++sg)
#pragma unroll
            for (int f = 0; f < 2; ++f)
#pragma unroll
              for (int j = 0; j < 3; ++j) {
                T e = t.Sp[q3][0] * xe[sg][f][j][0], o = t.Sm[q3][0] * xo[sg][f][j][0];
#pragma unroll
                for (int a = 1; a < NH; ++a) {
                  e = fmadd(t.Sp[q3][a], xe[sg][f][j][a], e);
                  o = fmadd(t.Sm[q3][a], xo[sg][f][j][a], o);
                }
                if constexpr (N % 2 == 1) e = fmadd(t.Sc[q3], xm[sg][f][j], e);
                vq[sg][f][j] = e + o;
                vr[sg][f][j] = e - o;
              }
          const T wgt = wq * t.w[q3];
          T Gq[3];
          face_adj(vq[0][0], vq[1][0], vq[0][1], vq[1][1], d, sgn, wgt, Gq);
          if (q3 < QH) {
            T Gr[3];
            face_adj(vr[0][0], vr[1][0], vr[0][1], vr[1][1], d, sgn, wgt, Gr);
#pragma unroll
            for (int k = 0; k < 3; ++k) acc[k].pair(t.Tp[q3], t.Tm[q3], Gq[k], Gr[k]);
          } else {
#pragma unroll
            for (int k = 0; k < 3; ++k) acc[k].mid(t.Tc, Gq[k]);
          }
        }
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
          for (int c = 0; c < N; ++c) F[fl(0, s, 0, k) + c * Q] = acc[k].out(c);
      }
    }
  }
  __syncthreads();

  // ---------------- Y: S^T_y in place, y-face terms; S^T_y of the x-face terms ----------------
  {
    constexpr int nY = 3 * E * N * Q, nXf = 3 * E * 2 * N;
    constexpr int FX = wave_split(nY, nXf, TH);   // first x-face item
    for (int w = tid; w < FX + nXf; w += TH) {
      CONV_TABLES(t);
      if (w < nY) {
        const int q1 = w % Q, rest = w / Q;
        const int cz = rest % N, r2 = rest / N;
        const int le = r2 % E, k = r2 / E;
        if (le >= ne) continue;
        T* L = lds + le * PER;
        T* tb = L + (k * N + cz) * COLS + q1;
        EoT<N, T, 1> v;
        v.zero();
#pragma unroll
        for (int q2 = 0; q2 < QH; ++q2) v.pair(t.Tp[q2], t.Tm[q2], tb[MP * q2], tb[MP * (Q - 1 - q2)]);
        if constexpr (Q % 2 == 1) v.mid(t.Tc, tb[MP * QH]);
        const T f0 = L[FYo + fl(0, 0, 0, k) + cz * Q + q1];
        const T f1 = L[FYo + fl(0, 1, 0, k) + cz * Q + q1];
#pragma unroll
        for (int b = 0; b < N; ++b) {
          T o = v.out(b);
          if (b == 0) o += f0;
          if (b == N - 1) o += f1;
          tb[MP * b] = o;
        }
      } else if (w >= FX) {
        const int vv = w - FX;
        const int cz = vv % N, rest = vv / N;
        const int s = rest % 2, r2 = rest / 2;
        const int le = r2 % E, k = r2 / E;
        if (le >= ne) continue;
        T* L = lds + le * PER;
        const T* xf = L + FXo + fl(0, s, 0, k) + cz * Q;
        EoT<N, T, 1> o;
        o.zero();
#pragma unroll
        for (int q2 = 0; q2 < QH; ++q2) o.pair(t.Tp[q2], t.Tm[q2], xf[q2], xf[Q - 1 - q2]);
        if constexpr (Q % 2 == 1) o.mid(t.Tc, xf[QH]);
        T* xr = L + XRo + ((k * 2 + s) * N + cz) * N;
#pragma unroll
        for (int b = 0; b < N; ++b) xr[b] = o.out(b);
      }
    }
  }
  __syncthreads();

  // ---------------- X: S^T_x, x-face terms, write-out ----------------
  {
    constexpr int nX = 3 * E * N2;
    for (int w = tid; w < nX; w += TH) {
      CONV_TABLES(t);
      const int bc = w % N2, r2 = w / N2;
      const int le = r2 % E, k = r2 / E;
      if (le >= ne) continue;
      const int b = bc % N, cz = bc / N;
      const T* L = lds + le * PER;
      const T* v = L + (k * N + cz) * COLS + MP * b;
      EoT<N, T, 1> o;
      o.zero();
#pragma unroll
      for (int q1 = 0; q1 < QH; ++q1) o.pair(t.Tp[q1], t.Tm[q1], v[q1], v[Q - 1 - q1]);
      if constexpr (Q % 2 == 1) o.mid(t.Tc, v[QH]);
      const T* xr = L + XRo + (k * 2 * N + cz) * N + b;
      const T x0 = xr[0], x1 = xr[N2];
      T* out = g + k * cs + (size_t)(e0 + le) * N3 + N * bc;
#pragma unroll
      for (int a = 0; a < N; ++a) {
        T val = o.out(a);
        if (a == 0) val += x0;
        if (a == N - 1) val += x1;
        out[a] = val;
      }
    }
  }
}

// ======================= per-component kernel =======================
// LDS layout of one element (units of T); column blocks (q1, q2) with q1
// pitch MP as in the convective kernel.
//   slots [0, 3(n+2)):         U_j, S_y S_x u_j at z layer c in -1..n
//   slots [3(n+2), 4(n+2)):    WS, S_y S_x w_i at z layer c in -1..n
//   DER = 0, then n slots:     WGY, G_y S_x w_i
//            then n slots:     WGX, S_y G_x w_i
//   back sweep:                slot k*n + cz holds S^T_z W P_k (+ z faces),
//                              then S^T_y of it in place (own columns only)
//   face layers FY, FX:        [sigma][s][f][c][q], f = 0..2 (u_j), 3 (w_i);
//                              the face pencils overwrite (0, s, k) with their
//                              S^T_z result for component k
//   XR:                        x-face terms after S^T_y, [k][s][cz][b], in the
//                              sigma = 1 half of FX (free by then)
// FXL = 1 (FP64, k = 11): no FX during the passes.  The x faces are taken
// after them, in the slots [3n, SLOTS) that the passes leave free: the y
// sweeps of the x-face layers of u and of all three components of w,
// [sigma][s][f = u_0..2, w_0..2][c][q], then XR.
template <int N, int Q, int SZ, int DER, int FXL>
struct VjpShapeC {
  static constexpr int N2 = N * N, N3 = N * N * N;
  static constexpr int MP = Q | 1;
  static constexpr int COLS = MP * Q;
  static constexpr int LAYER = N * Q;
  static constexpr int SU = 0, SW = 3 * (N + 2), SWGY = 4 * (N + 2), SWGX = 4 * (N + 2) + N;
  static constexpr int SLOTS = 4 * (N + 2) + (DER ? 0 : 2 * N);
  static constexpr int FL = 16 * LAYER;
  static constexpr int XL = 3 * N * COLS;   // late x-face region (FXL)
  static constexpr int PER = SLOTS * COLS + (FXL ? 1 : 2) * FL;
  static constexpr int BYTES = PER * SZ;
  static constexpr int ITEMS = Q * Q + (FXL ? 2 : 4) * Q;   // z pencils and face pencils per element
  static constexpr int E0 = (56 * 1024) / BYTES;
  static constexpr int E = E0 < 1 ? 1 : (E0 > 8 ? 8 : E0);
  // one workgroup per CU (more than 80 KB): at most one wave per SIMD, which
  // then has the whole register file.  With the late x faces (FP64 k = 11)
  // the registers spill either way, and 512 threads (one z pencil each, two
  // wavefronts per SIMD) measured 5.5 % faster than 256.
  static constexpr int TH0 = (E * ITEMS + 63) / 64 * 64;
  static constexpr int TH = FXL                    ? 512
                            : E * BYTES > 80 * 1024 ? (TH0 > 256 ? 256 : TH0)
                                                    : (TH0 > 512 ? 512 : TH0);
  static constexpr bool FITS = E * BYTES <= 160 * 1024;
  static_assert(6 * N2 <= 8 * LAYER, "x-face results must fit in half of FX");
  static_assert(!FXL || 24 * LAYER + 6 * N2 <= (SLOTS - 3 * N) * COLS, "late x faces must fit in the free slots");
};

// DER = 0 where the derivative slots fit, else 1; FXL = 1 where even that
// does not fit.
template <int N, int Q, int SZ>
constexpr int vjp_der() {
  return VjpShapeC<N, Q, SZ, 0, 0>::FITS ? 0 : 1;
}
template <int N, int Q, int SZ>
constexpr int vjp_fxl() {
  return VjpShapeC<N, Q, SZ, vjp_der<N, Q, SZ>(), 0>::FITS ? 0 : 1;
}

template <int N, int Q, typename T, int E, int TH, int DER, int FXL>
__global__ void __launch_bounds__(TH) __attribute__((amdgpu_waves_per_eu(2)))
vjp_percomp_kernel(const T* __restrict__ u, const T* __restrict__ wv, T* __restrict__ g, MeshArgs mesh,
                      const ConvTab<N, Q, T>* __restrict__ tab, const GaussDeriv<Q, T>* __restrict__ gd,
                      ConvScal<T> sc, bool a16) {
  using Sh = VjpShapeC<N, Q, (int)sizeof(T), DER, FXL>;
  constexpr int N2 = Sh::N2, N3 = Sh::N3, MP = Sh::MP, COLS = Sh::COLS, LAYER = Sh::LAYER, PER = Sh::PER;
  constexpr int NH = N / 2, QH = Q / 2, QC = (Q + 1) / 2;
  // FP64 at the highest degree: Gauss-point loops not unrolled, so that the
  // table rows of one point are loaded when used (unrolled, the FP64 table
  // entries exhaust the scalar registers and spill)
  constexpr int RQ = (sizeof(T) == 8 && N >= 12) ? 1 : QC;
  constexpr int FYo = Sh::SLOTS * COLS, FXo = FYo + Sh::FL;
  constexpr int XRo = FXL ? Sh::XL + 24 * LAYER : FXo + 8 * LAYER;
  __shared__ T lds[E * PER];
  const int tid = threadIdx.x;
  const int e0 = xcd_remap(blockIdx.x, gridDim.x) * E;
  const int ne = min(E, mesh.n_el - e0);   // items of le >= ne are skipped
  const size_t cs = (size_t)mesh.n_el * N3;
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
  // offset of face-layer entry (sigma, s, f)
  auto fl = [](int sg, int s, int f) { return ((sg * 2 + s) * 4 + f) * LAYER; };

  // ---------------- P1 items ----------------
  // kind 0: x pencil (b, c) of the element; 1: x pencil p of the z neighbour's
  // facing layer (side s); 2: x pencil p of the y neighbour's facing layer;
  // 3: y pencil c of the x-face layer (own sigma = 0 / neighbour 1, side s).
  constexpr int nM = E * N2, nZ = E * 2 * N, nY = E * 2 * N, nX = FXL ? 0 : E * 4 * N;
  constexpr int P1N = nM + nZ + nY + nX;
  constexpr int NI1 = (P1N + TH - 1) / TH;
  int kd[NI1], ile[NI1], ia[NI1], ib[NI1], ic[NI1], ist[NI1];
  size_t ioff[NI1];
#pragma unroll
  for (int it = 0; it < NI1; ++it) {
    const int w = tid + it * TH;
    kd[it] = -1;
    ist[it] = 1;
    ioff[it] = 0;
    ile[it] = ia[it] = ib[it] = ic[it] = 0;
    if (w >= P1N) continue;
    if (w < nM) {
      const int le = w / N2;
      if (le >= ne) continue;
      const int bc = w - le * N2;
      kd[it] = 0;
      ile[it] = le;
      ia[it] = bc % N;
      ib[it] = bc / N;
      ioff[it] = (size_t)(e0 + le) * N3 + N * bc;
    } else if (w < nM + nZ + nY) {
      const int v = w - nM;
      const int isy = v >= nZ;
      const int v2 = isy ? v - nZ : v;
      const int le = v2 / (2 * N);
      if (le >= ne) continue;
      const int r = v2 - le * 2 * N, s = r / N, p = r - s * N;
      kd[it] = isy ? 2 : 1;
      ile[it] = le;
      ia[it] = s;
      ib[it] = p;
      const int nb = nbr(le, isy ? 1 : 2, s);
      const int lay = s ? 0 : N - 1;   // the neighbour's facing layer
      ioff[it] = (size_t)nb * N3 + (isy ? N * (lay + N * p) : N * (p + N * lay));
    } else {
      const int v = w - nM - nZ - nY;
      const int le = v / (4 * N);
      if (le >= ne) continue;
      const int r = v - le * 4 * N, sg = r / (2 * N), r2 = r - sg * 2 * N, s = r2 / N, c = r2 - s * N;
      kd[it] = 3;
      ile[it] = le;
      ia[it] = sg;
      ib[it] = s;
      ic[it] = c;
      int e = e0 + le, a = s ? N - 1 : 0;
      if (sg) {
        e = nbr(le, 0, s);
        a = s ? 0 : N - 1;
      }
      ist[it] = N;
      ioff[it] = (size_t)e * N3 + a + N2 * c;
    }
  }
  // x (or, kind 3, y) sweeps of one field into LDS: sb = slot base of its
  // S_y S_x layers, ff = face-layer field, gx = also G_x into WGX
  auto p1_store = [&](int it, const T (&x)[N], int sb, int ff, bool gx) {
    CONV_TABLES(t);
    T* L = lds + ile[it] * PER;
    if (kd[it] == 0) {
      const int b = ia[it], c = ib[it];
      T* d = L + (sb + c + 1) * COLS + MP * b;
      if (b == 0 || b == N - 1) {   // own y-face layer: also into FY
        T* f = L + FYo + fl(0, b ? 1 : 0, ff) + c * Q;
        eo_interp<N, Q, T>(t, x, [&](int q, T val) {
          d[q] = val;
          f[q] = val;
        });
      } else {
        eo_interp<N, Q, T>(t, x, [&](int q, T val) { d[q] = val; });
      }
      if (DER == 0 && gx) {
        T* dg = L + (Sh::SWGX + c) * COLS + MP * b;
        eo_interp_g<N, Q, T>(t, x, [&](int q, T val) { dg[q] = val; });
      }
    } else {
      T* d;
      if (kd[it] == 1) d = L + (sb + (ia[it] ? N + 1 : 0)) * COLS + MP * ib[it];
      else if (kd[it] == 2) d = L + FYo + fl(1, ia[it], ff) + ib[it] * Q;
      else d = L + FXo + fl(ia[it], ib[it], ff) + ic[it] * Q;
      eo_interp<N, Q, T>(t, x, [&](int q, T val) { d[q] = val; });
    }
  };

  // share of w_i in the transposed flux derivative at one face point from
  // the own (m) and neighbour (p) traces of u_d (normal component), u_i and
  // w_i; outward sign sgn; G_k weighted by wgt
  auto face_i = [&](T umd, T upd, T umi, T upi, T wm, T wp, int i, int d, T sgn, T wgt, T (&G)[3]) {
    const T unm = sgn * umd, unp = sgn * upd;
    const T am = fabs(unm), ap = fabs(unp);
    const T lam = fmax(am, ap);
    const T sm = am > ap ? T(1) : (am == ap ? T(0.5) : T(0));
    const T sgu = unm > T(0) ? T(1) : (unm < T(0) ? T(-1) : T(0));
    const T dw = wgt * (wm - wp);
    const T diag = dw * fmadd(T(0.5), unm, sc.lf * lam);
    const T ex = sgn * dw * fmadd(T(0.5), umi, sc.lf * sm * sgu * (umi - upi));
#pragma unroll
    for (int k = 0; k < 3; ++k) G[k] = (k == i ? diag : T(0)) + (k == d ? ex : T(0));
  };

  // loads of w_i, kept in registers until the LDS slots of w_{i-1} are free
  T pre[NI1][N];
  auto load_w = [&](int i) {
#pragma unroll
    for (int it = 0; it < NI1; ++it)
      if (kd[it] >= 0) load_pencil_a16<N, Q, T>(wv + i * cs + ioff[it], ist[it], a16, pre[it]);
  };
  load_w(0);

  // ---------------- P1u ----------------
  {
    T in[NI1][3][N];
#pragma unroll
    for (int it = 0; it < NI1; ++it)
      if (kd[it] >= 0)
#pragma unroll
        for (int j = 0; j < 3; ++j) load_pencil_a16<N, Q, T>(u + j * cs + ioff[it], ist[it], a16, in[it][j]);
#pragma unroll
    for (int it = 0; it < NI1; ++it)
      if (kd[it] >= 0)
#pragma unroll
        for (int j = 0; j < 3; ++j) p1_store(it, in[it][j], Sh::SU + j * (N + 2), j, false);
  }

  // ---------------- P3 state ----------------
  constexpr int FAM = FXL ? 1 : 2;   // face families taken in the passes
  constexpr int nCell = E * Q * Q, nH = E * FAM * 2 * Q;
  constexpr int FO = wave_split(nCell, nH, TH);   // first face-pencil item
  constexpr int NIT = (FO + nH + TH - 1) / TH;
  EoT<N, T, 1> acc[NIT][3];
  T gz[NIT][2][3];   // z-face terms of a z pencil at its two end nodes
#pragma unroll
  for (int it = 0; it < NIT; ++it)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      acc[it][k].zero();
      gz[it][0][k] = gz[it][1][k] = T(0);
    }

#pragma unroll 1
  for (int i = 0; i < 3; ++i) {
    if (i) lds_barrier();   // P3 of the previous pass is done with the slots of w
    // ---------------- P1w ----------------
#pragma unroll
    for (int it = 0; it < NI1; ++it)
      if (kd[it] >= 0) p1_store(it, pre[it], Sh::SW, 3, true);
    if (i < 2) load_w(i + 1);
    lds_barrier();

    // ---------------- P2: y sweeps in place ----------------
    {
      constexpr int nU = 3 * E * (N + 2) * Q, nW = E * (N + 2) * Q, nG = DER ? 0 : E * N * Q;
      for (int w = tid + (i ? nU : 0); w < nU + nW + nG; w += TH) {
        CONV_TABLES(t);
        T* p;
        bool gy = false;
        int cl = 0, le;
        if (w < nU) {   // U column block (q1, layer cl) of component j
          const int q1 = w % Q, rest = w / Q;
          cl = rest % (N + 2);
          const int r2 = rest / (N + 2);
          le = r2 % E;
          const int j = r2 / E;
          p = lds + le * PER + (Sh::SU + j * (N + 2) + cl) * COLS + q1;
        } else if (w < nU + nW) {   // WS column block; G_y of interior layers into WGY
          const int v = w - nU;
          const int q1 = v % Q, rest = v / Q;
          cl = rest % (N + 2);
          le = rest / (N + 2);
          p = lds + le * PER + (Sh::SW + cl) * COLS + q1;
          gy = DER == 0 && cl >= 1 && cl <= N;
        } else {        // WGX column block
          const int v = w - nU - nW;
          const int q1 = v % Q, rest = v / Q;
          const int c = rest % N;
          le = rest / N;
          p = lds + le * PER + (Sh::SWGX + c) * COLS + q1;
        }
        if (le >= ne) continue;
        T x[N];
#pragma unroll
        for (int b = 0; b < N; ++b) x[b] = p[MP * b];
        if (gy) {
          T* pg = p + (Sh::SWGY - 1 - Sh::SW) * COLS;   // WGY layer cl - 1
          eo_interp_g<N, Q, T>(t, x, [&](int q, T val) { pg[MP * q] = val; });
        }
        eo_interp<N, Q, T>(t, x, [&](int q, T val) { p[MP * q] = val; });
      }
    }
    lds_barrier();

    // W_q3 times the share of w_i in P_k at one point: v = u_0, u_1, u_2,
    // d_x w_i, d_y w_i, d_z w_i
    auto pk_i = [&](const T (&v)[6], T wq, T (&P)[3]) {
      const T ui = i == 0 ? v[0] : (i == 1 ? v[1] : v[2]);
      const T own = fmadd(sc.cell[0] * v[0], v[3], fmadd(sc.cell[1] * v[1], v[4], sc.cell[2] * v[2] * v[5]));
#pragma unroll
      for (int k = 0; k < 3; ++k) P[k] = wq * fmadd(sc.cell[k] * ui, v[3 + k], i == k ? own : T(0));
    };

    // ---------------- P3: z pencils and face pencils ----------------
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int w = tid + it * TH;
      if (w >= FO + nH || (w >= nCell && w < FO)) continue;
      CONV_TABLES(t);
      if (w < nCell) {
        const int le = w / (Q * Q), qq = w - le * (Q * Q);
        if (le >= ne) continue;
        const int q2 = qq / Q, q1 = qq - q2 * Q;
        const T* L = lds + le * PER;
        const T* col = L + q1 + MP * q2;
        const T w12 = t.w[q1] * t.w[q2];
        // z faces from the layers -1, 0, n-1, n of U and WS
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const int own = s ? N : 1, nb = s ? N + 1 : 0;
          const T* ud = col + (Sh::SU + 2 * (N + 2)) * COLS;
          const T* ui = col + (Sh::SU + i * (N + 2)) * COLS;
          const T* ws = col + Sh::SW * COLS;
          T G[3];
          face_i(ud[own * COLS], ud[nb * COLS], ui[own * COLS], ui[nb * COLS], ws[own * COLS], ws[nb * COLS], i, 2,
                 s ? T(1) : T(-1), w12 * sc.area[2], G);
#pragma unroll
          for (int k = 0; k < 3; ++k) gz[it][s][k] += G[k];
        }
        // even-odd parts of the interior columns: f = 0..2 u_j (S_z),
        // 3 d_x w_i (S_z), 4 d_y w_i (S_z), 5 w_i (G_z)
        T xe[6][NH], xo[6][NH], xm[6];
#pragma unroll
        for (int f = 0; f < 6; ++f) {
          T x[N];
          if (f == 3 && DER) {
            const T* dr = gd->d[q1];
            const T* ws = L + MP * q2 + (Sh::SW + 1) * COLS;
#pragma unroll
            for (int c = 0; c < N; ++c) x[c] = T(0);
            for (int qp = 0; qp < Q; ++qp) {
              const T dq = dr[qp];
#pragma unroll
              for (int c = 0; c < N; ++c) x[c] = fmadd(dq, ws[c * COLS + qp], x[c]);
            }
          } else if (f == 4 && DER) {
            const T* dr = gd->d[q2];
            const T* ws = L + q1 + (Sh::SW + 1) * COLS;
#pragma unroll
            for (int c = 0; c < N; ++c) x[c] = T(0);
            for (int qp = 0; qp < Q; ++qp) {
              const T dq = dr[qp];
#pragma unroll
              for (int c = 0; c < N; ++c) x[c] = fmadd(dq, ws[c * COLS + MP * qp], x[c]);
            }
          } else {
#pragma unroll
            for (int c = 0; c < N; ++c) {
              const int slot = f < 3    ? Sh::SU + f * (N + 2) + c + 1
                               : f == 3 ? Sh::SWGX + c
                               : f == 4 ? Sh::SWGY + c
                                        : Sh::SW + c + 1;
              x[c] = col[slot * COLS];
            }
          }
#pragma unroll
          for (int a = 0; a < NH; ++a) {
            xe[f][a] = x[a] + x[N - 1 - a];
            xo[f][a] = x[a] - x[N - 1 - a];
          }
          xm[f] = (N % 2) ? x[NH] : T(0);
        }
#pragma unroll RQ
        for (int q = 0; q < QC; ++q) {
          // the six fields at q and at its mirror m-1-q
          T vq[6], vr[6];
#pragma unroll
          for (int f = 0; f < 6; ++f) {
            T e, o;
            if (f == 5) {
              e = t.Gp[q][0] * xe[f][0];
              o = t.Gm[q][0] * xo[f][0];
#pragma unroll
              for (int a = 1; a < NH; ++a) {
                e = fmadd(t.Gp[q][a], xe[f][a], e);
                o = fmadd(t.Gm[q][a], xo[f][a], o);
              }
              if constexpr (N % 2 == 1) e = fmadd(t.Gc[q], xm[f], e);
              vq[f] = e + o;
              vr[f] = o - e;
            } else {
              e = t.Sp[q][0] * xe[f][0];
              o = t.Sm[q][0] * xo[f][0];
#pragma unroll
              for (int a = 1; a < NH; ++a) {
                e = fmadd(t.Sp[q][a], xe[f][a], e);
                o = fmadd(t.Sm[q][a], xo[f][a], o);
              }
              if constexpr (N % 2 == 1) e = fmadd(t.Sc[q], xm[f], e);
              vq[f] = e + o;
              vr[f] = e - o;
            }
          }
          T Pq[3];
          pk_i(vq, t.w[q], Pq);
          if (q < QH) {
            T Pr[3];
            pk_i(vr, t.w[q], Pr);   // w[m-1-q] = w[q]
#pragma unroll
            for (int k = 0; k < 3; ++k) acc[it][k].pair(t.Tp[q], t.Tm[q], Pq[k], Pr[k]);
          } else {
#pragma unroll
            for (int k = 0; k < 3; ++k) acc[it][k].mid(t.Tc, Pq[k]);
          }
        }
      } else {   // face pencil: fam 0 = y face (q = q1), 1 = x face (q = q2)
        const int h = w - FO;
        const int le = h / (FAM * 2 * Q);
        if (le >= ne) continue;
        int rem = h - le * FAM * 2 * Q;
        const int fam = FXL ? 0 : rem / (2 * Q);
        rem -= fam * 2 * Q;
        const int s = rem / Q, q = rem - s * Q;
        const T* F = lds + le * PER + (fam ? FXo : FYo) + q;
        const int d = fam ? 0 : 1;
        // even-odd parts of the pencils of u_d, u_i and w_i on both sides
        T xe[2][3][NH], xo[2][3][NH], xm[2][3];
#pragma unroll
        for (int sg = 0; sg < 2; ++sg)
#pragma unroll
          for (int f = 0; f < 3; ++f) {
            const T* src = F + fl(sg, s, f == 0 ? d : (f == 1 ? i : 3));
            T x[N];
#pragma unroll
            for (int c = 0; c < N; ++c) x[c] = src[c * Q];
#pragma unroll
            for (int a = 0; a < NH; ++a) {
              xe[sg][f][a] = x[a] + x[N - 1 - a];
              xo[sg][f][a] = x[a] - x[N - 1 - a];
            }
            xm[sg][f] = (N % 2) ? x[NH] : T(0);
          }
        const T sgn = s ? T(1) : T(-1);
        const T wq = t.w[q] * (fam ? sc.area[0] : sc.area[1]);
#pragma unroll RQ
        for (int q3 = 0; q3 < QC; ++q3) {
          T vq[2][3], vr[2][3];
#pragma unroll
          for (int sg = 0; sg < 2; ++sg)
#pragma unroll
            for (int f = 0; f < 3; ++f) {
              T e = t.Sp[q3][0] * xe[sg][f][0], o = t.Sm[q3][0] * xo[sg][f][0];
#pragma unroll
              for (int a = 1; a < NH; ++a) {
                e = fmadd(t.Sp[q3][a], xe[sg][f][a], e);
                o = fmadd(t.Sm[q3][a], xo[sg][f][a], o);
              }
              if constexpr (N % 2 == 1) e = fmadd(t.Sc[q3], xm[sg][f], e);
              vq[sg][f] = e + o;
              vr[sg][f] = e - o;
            }
          const T wgt = wq * t.w[q3];
          T Gq[3];
          face_i(vq[0][0], vq[1][0], vq[0][1], vq[1][1], vq[0][2], vq[1][2], i, d, sgn, wgt, Gq);
          if (q3 < QH) {
            T Gr[3];
            face_i(vr[0][0], vr[1][0], vr[0][1], vr[1][1], vr[0][2], vr[1][2], i, d, sgn, wgt, Gr);
#pragma unroll
            for (int k = 0; k < 3; ++k) acc[it][k].pair(t.Tp[q3], t.Tm[q3], Gq[k], Gr[k]);
          } else {
#pragma unroll
            for (int k = 0; k < 3; ++k) acc[it][k].mid(t.Tc, Gq[k]);
          }
        }
      }
    }
  }

  // P3 results: each pencil overwrites only entries of its own column or
  // face pencil, which no other pencil reads.
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int w = tid + it * TH;
    if (w >= FO + nH || (w >= nCell && w < FO)) continue;
    if (w < nCell) {
      const int le = w / (Q * Q), qq = w - le * (Q * Q);
      if (le >= ne) continue;
      const int q2 = qq / Q, q1 = qq - q2 * Q;
      CONV_TABLES(t);
      T* col = lds + le * PER + q1 + MP * q2;
      const T w12 = t.w[q1] * t.w[q2];
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int c = 0; c < N; ++c) {
          T o = w12 * acc[it][k].out(c);
          if (c == 0) o += gz[it][0][k];
          if (c == N - 1) o += gz[it][1][k];
          col[(k * N + c) * COLS] = o;
        }
    } else {
      const int h = w - FO;
      const int le = h / (FAM * 2 * Q);
      if (le >= ne) continue;
      int rem = h - le * FAM * 2 * Q;
      const int fam = FXL ? 0 : rem / (2 * Q);
      rem -= fam * 2 * Q;
      const int s = rem / Q, q = rem - s * Q;
      T* F = lds + le * PER + (fam ? FXo : FYo) + q;
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int c = 0; c < N; ++c) F[fl(0, s, k) + c * Q] = acc[it][k].out(c);
    }
  }
  lds_barrier();

  // late x faces (FXL): layer offset of (sigma, s, f), f = u_0..2, w_0..2
  auto fx = [](int sg, int s, int f) { return Sh::XL + ((sg * 2 + s) * 6 + f) * LAYER; };
  if constexpr (FXL) {
    // y sweeps of the x-face layers, one (pencil, field) per item
    constexpr int nXL = E * 4 * N * 6;
    for (int w = tid; w < nXL; w += TH) {
      CONV_TABLES(t);
      const int f = w % 6, v = w / 6;
      const int le = v / (4 * N);
      if (le >= ne) continue;
      const int r = v - le * 4 * N, sg = r / (2 * N), r2 = r - sg * 2 * N, s = r2 / N, c = r2 - s * N;
      int e = e0 + le, a = s ? N - 1 : 0;
      if (sg) {
        e = nbr(le, 0, s);
        a = s ? 0 : N - 1;
      }
      const T* src = (f < 3 ? u + f * cs : wv + (f - 3) * cs) + (size_t)e * N3 + a + N2 * c;
      T x[N];
      load_pencil<N, Q, T>(src, N, x);
      T* d = lds + le * PER + fx(sg, s, f) + c * Q;
      eo_interp<N, Q, T>(t, x, [&](int q, T val) { d[q] = val; });
    }
    lds_barrier();
    // x-face pencils (side s, point q), the three shares of w in turn
    constexpr int nF = E * 2 * Q;
    for (int w = tid; w < nF; w += TH) {
      CONV_TABLES(t);
      const int le = w / (2 * Q);
      if (le >= ne) continue;
      const int rem = w - le * 2 * Q, s = rem / Q, q = rem - s * Q;
      T* F = lds + le * PER + q;
      const T sgn = s ? T(1) : T(-1);
      const T wq = t.w[q] * sc.area[0];
      EoT<N, T, 1> fa[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) fa[k].zero();
#pragma unroll 1
      for (int i = 0; i < 3; ++i) {
        T xe[2][3][NH], xo[2][3][NH], xm[2][3];
#pragma unroll
        for (int sg = 0; sg < 2; ++sg)
#pragma unroll
          for (int f = 0; f < 3; ++f) {
            const T* src = F + fx(sg, s, f == 0 ? 0 : (f == 1 ? i : 3 + i));
            T x[N];
#pragma unroll
            for (int c = 0; c < N; ++c) x[c] = src[c * Q];
#pragma unroll
            for (int a = 0; a < NH; ++a) {
              xe[sg][f][a] = x[a] + x[N - 1 - a];
              xo[sg][f][a] = x[a] - x[N - 1 - a];
            }
            xm[sg][f] = (N % 2) ? x[NH] : T(0);
          }
#pragma unroll RQ
        for (int q3 = 0; q3 < QC; ++q3) {
          T vq[2][3], vr[2][3];
#pragma unroll
          for (int sg = 0; sg < 2; ++sg)
#pragma unroll
            for (int f = 0; f < 3; ++f) {
              T e = t.Sp[q3][0] * xe[sg][f][0], o = t.Sm[q3][0] * xo[sg][f][0];
#pragma unroll
              for (int a = 1; a < NH; ++a) {
                e = fmadd(t.Sp[q3][a], xe[sg][f][a], e);
                o = fmadd(t.Sm[q3][a], xo[sg][f][a], o);
              }
              if constexpr (N % 2 == 1) e = fmadd(t.Sc[q3], xm[sg][f], e);
              vq[sg][f] = e + o;
              vr[sg][f] = e - o;
            }
          const T wgt = wq * t.w[q3];
          T Gq[3];
          face_i(vq[0][0], vq[1][0], vq[0][1], vq[1][1], vq[0][2], vq[1][2], i, 0, sgn, wgt, Gq);
          if (q3 < QH) {
            T Gr[3];
            face_i(vr[0][0], vr[1][0], vr[0][1], vr[1][1], vr[0][2], vr[1][2], i, 0, sgn, wgt, Gr);
#pragma unroll
            for (int k = 0; k < 3; ++k) fa[k].pair(t.Tp[q3], t.Tm[q3], Gq[k], Gr[k]);
          } else {
#pragma unroll
            for (int k = 0; k < 3; ++k) fa[k].mid(t.Tc, Gq[k]);
          }
        }
      }
      // own u layers of this (s, q): read by no other pencil
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int c = 0; c < N; ++c) F[fx(0, s, k) + c * Q] = fa[k].out(c);
    }
    lds_barrier();
  }

  // ---------------- Y: S^T_y in place, y-face terms; S^T_y of the x-face terms ----------------
  {
    constexpr int nYs = 3 * E * N * Q, nXf = 3 * E * 2 * N;
    constexpr int FX = wave_split(nYs, nXf, TH);   // first x-face item
    for (int w = tid; w < FX + nXf; w += TH) {
      CONV_TABLES(t);
      if (w < nYs) {
        const int q1 = w % Q, rest = w / Q;
        const int cz = rest % N, r2 = rest / N;
        const int le = r2 % E, k = r2 / E;
        if (le >= ne) continue;
        T* L = lds + le * PER;
        T* tb = L + (k * N + cz) * COLS + q1;
        EoT<N, T, 1> v;
        v.zero();
#pragma unroll
        for (int q2 = 0; q2 < QH; ++q2) v.pair(t.Tp[q2], t.Tm[q2], tb[MP * q2], tb[MP * (Q - 1 - q2)]);
        if constexpr (Q % 2 == 1) v.mid(t.Tc, tb[MP * QH]);
        const T f0 = L[FYo + fl(0, 0, k) + cz * Q + q1];
        const T f1 = L[FYo + fl(0, 1, k) + cz * Q + q1];
#pragma unroll
        for (int b = 0; b < N; ++b) {
          T o = v.out(b);
          if (b == 0) o += f0;
          if (b == N - 1) o += f1;
          tb[MP * b] = o;
        }
      } else if (w >= FX) {
        const int vv = w - FX;
        const int cz = vv % N, rest = vv / N;
        const int s = rest % 2, r2 = rest / 2;
        const int le = r2 % E, k = r2 / E;
        if (le >= ne) continue;
        T* L = lds + le * PER;
        const T* xf = L + (FXL ? fx(0, s, k) : FXo + fl(0, s, k)) + cz * Q;
        EoT<N, T, 1> o;
        o.zero();
#pragma unroll
        for (int q2 = 0; q2 < QH; ++q2) o.pair(t.Tp[q2], t.Tm[q2], xf[q2], xf[Q - 1 - q2]);
        if constexpr (Q % 2 == 1) o.mid(t.Tc, xf[QH]);
        T* xr = L + XRo + ((k * 2 + s) * N + cz) * N;
#pragma unroll
        for (int b = 0; b < N; ++b) xr[b] = o.out(b);
      }
    }
  }
  lds_barrier();

  // ---------------- X: S^T_x, x-face terms, write-out ----------------
  {
    constexpr int nXo = 3 * E * N2;
    for (int w = tid; w < nXo; w += TH) {
      CONV_TABLES(t);
      const int bc = w % N2, r2 = w / N2;
      const int le = r2 % E, k = r2 / E;
      if (le >= ne) continue;
      const int b = bc % N, cz = bc / N;
      const T* L = lds + le * PER;
      const T* v = L + (k * N + cz) * COLS + MP * b;
      EoT<N, T, 1> o;
      o.zero();
#pragma unroll
      for (int q1 = 0; q1 < QH; ++q1) o.pair(t.Tp[q1], t.Tm[q1], v[q1], v[Q - 1 - q1]);
      if constexpr (Q % 2 == 1) o.mid(t.Tc, v[QH]);
      const T* xr = L + XRo + (k * 2 * N + cz) * N + b;
      const T x0 = xr[0], x1 = xr[N2];
      T* out = g + k * cs + (size_t)(e0 + le) * N3 + N * bc;
#pragma unroll
      for (int a = 0; a < N; ++a) {
        T val = o.out(a);
        if (a == 0) val += x0;
        if (a == N - 1) val += x1;
        out[a] = val;
      }
    }
  }
}

// The one-pass kernel where its LDS per element allows a few elements per
// CU (k <= 7), the per-component kernel above that.
template <int N>
constexpr bool vjp_onepass() {
  return N <= 8;
}

template <int N, int Q, typename T>
static hipError_t launch_vjp_nq(const ConvPlan& P, const void* u, const void* w, void* g, hipStream_t s) {
  constexpr int DER = vjp_der<N, Q, (int)sizeof(T)>(), FXL = vjp_fxl<N, Q, (int)sizeof(T)>();
  using ShC = VjpShapeC<N, Q, (int)sizeof(T), DER, FXL>;
  using Sh1 = VjpShape1<N, Q, (int)sizeof(T)>;
  constexpr bool ONE = vjp_onepass<N>();
  if constexpr (ONE ? !Sh1::FITS : !ShC::FITS) {
    return hipErrorInvalidConfiguration;
  } else {
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
    hipError_t err;
    const ConvTab<N, Q, T>* dt = nullptr;   // FP32 kernels use the compile-time tables
    if (sizeof(T) == 8) {
      const ConvTab<N, Q, T> t = make_conv_tab<N, Q, T>(P.S.data(), P.G.data(), P.w.data());
      dt = device_table_of("convective", t, &err);
      if (!dt) return err;
    }
    // every pencil of n contiguous values starts at a multiple of n values from
    // u (resp. w): 16-byte loads apply when both are 16-byte aligned.  Used in
    // FP32 (k=7, 11: 5-6 % faster); FP64 measured 0-4 % slower with them
    const bool a16 = sizeof(T) == 4 && (reinterpret_cast<uintptr_t>(u) % 16) == 0 &&
                     (reinterpret_cast<uintptr_t>(w) % 16) == 0;
    if constexpr (ONE) {
      const int grid = (P.mesh.n_el + Sh1::E - 1) / Sh1::E;
      hipLaunchKernelGGL((vjp_onepass_kernel<N, Q, T, Sh1::E, Sh1::TH>), dim3(grid), dim3(Sh1::TH), 0, s,
                         (const T*)u, (const T*)w, (T*)g, P.mesh, dt, sc, a16);
    } else {
      const GaussDeriv<Q, T>* dd = nullptr;
      if (DER) {
        dd = device_table_of("vjp_gauss_deriv", make_gauss_deriv<N, Q, T>(), &err);
        if (!dd) return err;
      }
      const int grid = (P.mesh.n_el + ShC::E - 1) / ShC::E;
      hipLaunchKernelGGL((vjp_percomp_kernel<N, Q, T, ShC::E, ShC::TH, DER, FXL>), dim3(grid), dim3(ShC::TH), 0, s,
                         (const T*)u, (const T*)w, (T*)g, P.mesh, dt, dd, sc, a16);
    }
    return hipGetLastError();
  }
}

template <typename T>
static hipError_t launch_vjp_t(const ConvPlan& P, const void* u, const void* w, void* g, hipStream_t s) {
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
    case 10: return launch_vjp_nq<11, 16, T>(P, u, w, g, s);
    case 11: return launch_vjp_nq<12, 17, T>(P, u, w, g, s);
    default: return hipErrorInvalidConfiguration;
  }
}

int vjp_max_degree(bool) { return 11; }

hipError_t launch_convective_vjp(const ConvPlan& P, bool f32, const void* u, const void* w, void* g,
                                 hipStream_t s) {
  return f32 ? launch_vjp_t<float>(P, u, w, g, s) : launch_vjp_t<double>(P, u, w, g, s);
}

}  // namespace dgmf
