// C ABI of libdgmf: argument validation, 1D tables, dispatch to the kernels.
#include "dgmf.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "api_internal.h"
#include "basis1d.h"
#include "ops.h"

namespace dgmf {

namespace {
thread_local std::string g_last_error;
std::mutex g_basis_mutex;
std::map<std::pair<int, int>, Basis1D> g_basis;
std::mutex g_table_mutex;
std::map<std::pair<int, std::string>, void*> g_tables;
std::mutex g_child_mutex;
std::map<int, std::vector<double>> g_child;   // key 2k + c: child_interp(k, c)
}  // namespace

const void* device_table(const std::string& key, const void* host, size_t bytes, hipError_t* err) {
  *err = hipSuccess;
  int dev = 0;
  if ((*err = hipGetDevice(&dev)) != hipSuccess) return nullptr;
  std::string full = key + "/" + std::to_string(bytes);
  std::lock_guard<std::mutex> lock(g_table_mutex);
  auto k = std::make_pair(dev, full);
  auto it = g_tables.find(k);
  if (it != g_tables.end()) return it->second;
  void* d = nullptr;
  if ((*err = hipMalloc(&d, bytes)) != hipSuccess) return nullptr;
  if ((*err = hipMemcpy(d, host, bytes, hipMemcpyHostToDevice)) != hipSuccess) {
    (void)hipFree(d);
    return nullptr;
  }
  g_tables[k] = d;
  return d;
}

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int ok() {
  g_last_error.clear();
  return DG_OK;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(DG_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

const Basis1D& basis(int k, int m) {
  std::lock_guard<std::mutex> lock(g_basis_mutex);
  auto key = std::make_pair(k, m);
  auto it = g_basis.find(key);
  if (it == g_basis.end()) it = g_basis.emplace(key, make_basis(k, m)).first;
  return it->second;
}

int validate_desc(const dg_op_desc* d) {
  if (!d) return fail(DG_ERR_INVALID_ARG, "descriptor is NULL");
  if (d->degree < 1 || d->degree > kMaxDegree)
    return fail(DG_ERR_UNSUPPORTED, "degree " + std::to_string(d->degree) + " outside 1.." +
                                        std::to_string(kMaxDegree));
  long long nel = 1;
  for (int i = 0; i < 3; ++i) {
    if (d->n_el[i] < 1) return fail(DG_ERR_INVALID_ARG, "n_el must be >= 1 in every direction");
    if (!(std::isfinite(d->length[i]) && d->length[i] > 0))
      return fail(DG_ERR_INVALID_ARG, "length must be finite and > 0");
    nel *= d->n_el[i];
  }
  const long long n3 = (long long)(d->degree + 1) * (d->degree + 1) * (d->degree + 1);
  if (nel * 3 > (1LL << 31) - 1 || nel * 3 * n3 > (1LL << 40))
    return fail(DG_ERR_INVALID_ARG, "mesh too large");
  if (d->n_q < 0 || d->n_q > kMaxNq) return fail(DG_ERR_UNSUPPORTED, "n_q outside 0..32");
  if (!std::isfinite(d->penalty_factor) || !std::isfinite(d->scale) || !std::isfinite(d->lf_factor))
    return fail(DG_ERR_INVALID_ARG, "penalty_factor, scale and lf_factor must be finite");
  return DG_OK;
}

long long num_elements(const dg_op_desc* d) {
  return (long long)d->n_el[0] * d->n_el[1] * d->n_el[2];
}

long long dofs_per_element(const dg_op_desc* d) {
  const long long n = d->degree + 1;
  return n * n * n;
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  return pa < pb + nb && pb < pa + na;
}

MeshArgs mesh_args(const dg_op_desc* d) {
  MeshArgs m;
  m.nx = d->n_el[0];
  m.ny = d->n_el[1];
  m.nz = d->n_el[2];
  m.n_el = m.nx * m.ny * m.nz;
  return m;
}

// X = A^-1 R for a small SPD matrix A (n x n, row major) and m right-hand
// sides R (n x m, row major), by Cholesky factorisation.
std::vector<double> solve_spd(const std::vector<double>& A, int n, const std::vector<double>& R, int m) {
  std::vector<double> Lc(n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double s = A[j * n + j];
    for (int k = 0; k < j; ++k) s -= Lc[j * n + k] * Lc[j * n + k];
    Lc[j * n + j] = std::sqrt(s);
    for (int i = j + 1; i < n; ++i) {
      double t = A[i * n + j];
      for (int k = 0; k < j; ++k) t -= Lc[i * n + k] * Lc[j * n + k];
      Lc[i * n + j] = t / Lc[j * n + j];
    }
  }
  std::vector<double> X(R);
  for (int c = 0; c < m; ++c) {
    for (int i = 0; i < n; ++i) {   // forward: Lc y = r
      double t = X[i * m + c];
      for (int k = 0; k < i; ++k) t -= Lc[i * n + k] * X[k * m + c];
      X[i * m + c] = t / Lc[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {   // backward: Lc^T x = y
      double t = X[i * m + c];
      for (int k = i + 1; k < n; ++k) t -= Lc[k * n + i] * X[k * m + c];
      X[i * m + c] = t / Lc[i * n + i];
    }
  }
  return X;
}

double cell_volume(const dg_op_desc* d) {
  double vol = 1.0;
  for (int i = 0; i < 3; ++i) vol *= d->length[i] / d->n_el[i];
  return vol;
}

std::vector<double> inverse_mass_1d(int k) {
  const int n = k + 1;
  const Basis1D& B = basis(k, n);
  std::vector<double> I(n * n, 0.0);
  for (int i = 0; i < n; ++i) I[i * n + i] = 1.0;
  return solve_spd(B.Mref, n, I, n);
}

ProjPlan make_proj_plan(const dg_op_desc* desc) {
  const int k = desc->degree, n = k + 1;
  const Basis1D& B = basis(k, n);
  ProjPlan P;
  P.k = k;
  P.mesh = mesh_args(desc);
  P.S = B.S;
  P.Dg = B.Dg;
  P.M1 = B.Mref;
  P.w = B.wq;
  P.vol = cell_volume(desc);
  for (int i = 0; i < 3; ++i) {
    const double h = desc->length[i] / desc->n_el[i];
    P.ih[i] = 1.0 / h;
    P.area[i] = P.vol / h;
  }
  return P;
}

LaplacePlan make_laplace_plan(const dg_op_desc* d, int n_comp) {
  const int k = d->degree;
  const int m = d->n_q ? d->n_q : k + 1;
  const Basis1D& B = basis(k, m);
  const double sigma = d->penalty_factor * (k + 1.0) * (k + 1.0);
  Sipg1D S = make_sipg_1d(B, sigma);
  LaplacePlan P;
  P.k = k;
  P.n_comp = n_comp;
  P.mesh = mesh_args(d);
  P.Mref = B.Mref;
  P.Kown = S.Kown;
  P.D = B.D;
  double h[3], vol = 1.0;
  for (int i = 0; i < 3; ++i) {
    h[i] = d->length[i] / d->n_el[i];
    vol *= h[i];
  }
  for (int i = 0; i < 3; ++i) P.c[i] = d->scale * vol / (h[i] * h[i]);
  P.sigma = sigma;
  // mass-factored form: L = M^-1 Kown and M^-1 times the coupling columns
  // (right end value hd1 - sigma e_{n-1}, left end value -hd0 - sigma e_0,
  // right half slope -e_{n-1}, left half slope e_0)
  const int n = k + 1;
  std::vector<double> rhs(n * (n + 4), 0.0);   // columns: Kown (n), cR, cL, gR, gL
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) rhs[i * (n + 4) + j] = S.Kown[i * n + j];
    const double hd0 = 0.5 * B.D[i], hd1 = 0.5 * B.D[(n - 1) * n + i];
    rhs[i * (n + 4) + n + 0] = hd1 - (i == n - 1 ? sigma : 0.0);
    rhs[i * (n + 4) + n + 1] = -hd0 - (i == 0 ? sigma : 0.0);
    rhs[i * (n + 4) + n + 2] = (i == n - 1) ? -1.0 : 0.0;
    rhs[i * (n + 4) + n + 3] = (i == 0) ? 1.0 : 0.0;
  }
  std::vector<double> sol = solve_spd(B.Mref, n, rhs, n + 4);
  P.Lown.assign(n * n, 0.0);
  P.cR.assign(n, 0.0);
  P.cL.assign(n, 0.0);
  P.gR.assign(n, 0.0);
  P.gL.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) P.Lown[i * n + j] = sol[i * (n + 4) + j];
    P.cR[i] = sol[i * (n + 4) + n + 0];
    P.cL[i] = sol[i * (n + 4) + n + 1];
    P.gR[i] = sol[i * (n + 4) + n + 2];
    P.gL[i] = sol[i * (n + 4) + n + 3];
  }
  return P;
}

int default_conv_nq(int k) { return (3 * k) / 2 + 1; }

int make_conv_plan(const dg_op_desc* d, ConvPlan& P) {
  const int k = d->degree;
  const int m = default_conv_nq(k);
  if (d->n_q != 0 && d->n_q != m)
    return fail(DG_ERR_UNSUPPORTED, "convective form is built for n_q = floor(3k/2)+1 = " + std::to_string(m));
  const Basis1D& B = basis(k, m);
  P.k = k;
  P.m = m;
  P.mesh = mesh_args(d);
  P.S = B.S;
  P.G = B.G;
  P.w = B.wq;
  double h[3], vol = 1.0;
  for (int i = 0; i < 3; ++i) {
    h[i] = d->length[i] / d->n_el[i];
    vol *= h[i];
  }
  for (int i = 0; i < 3; ++i) {
    P.cell[i] = -vol / h[i];
    P.area[i] = vol / h[i];
  }
  P.lf = d->lf_factor;
  return DG_OK;
}

DivPlan make_div_plan(const dg_op_desc* d) {
  const int k = d->degree, n = k + 1;
  const int m = d->n_q ? d->n_q : k + 1;
  const Basis1D& B = basis(k, m);
  DivPlan P;
  P.k = k;
  P.mesh = mesh_args(d);
  P.Mref = B.Mref;
  P.Bown.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0;
      for (int q = 0; q < m; ++q) s += B.wq[q] * B.G[q * n + i] * B.S[q * n + j];
      P.Bown[i * n + j] = -s;
    }
  P.Bown[(n - 1) * n + (n - 1)] += 0.5;
  P.Bown[0] -= 0.5;
  double h[3], vol = 1.0;
  for (int i = 0; i < 3; ++i) {
    h[i] = d->length[i] / d->n_el[i];
    vol *= h[i];
  }
  for (int i = 0; i < 3; ++i) P.c[i] = vol / h[i];
  return P;
}

}  // namespace dgmf

using namespace dgmf;

extern "C" {

const char* dg_error_string(int code) {
  switch (code) {
    case DG_OK: return "success";
    case DG_ERR_INVALID_ARG: return "invalid argument";
    case DG_ERR_UNSUPPORTED: return "unsupported degree or quadrature";
    case DG_ERR_ALIAS: return "output overlaps an input";
    case DG_ERR_HIP: return "HIP runtime error";
    case DG_NOT_CONVERGED: return "solver did not converge";
    case DG_ERR_BREAKDOWN: return "solver breakdown";
    default: return "unknown error code";
  }
}

const char* dg_last_error(void) { return g_last_error.c_str(); }

int dg_lgl_nodes(int32_t degree, double* nodes_host) {
  if (!nodes_host) return fail(DG_ERR_INVALID_ARG, "nodes_host is NULL");
  if (degree < 1 || degree > 64) return fail(DG_ERR_UNSUPPORTED, "degree outside 1..64");
  lgl_nodes(degree, nodes_host);
  return ok();
}

int dg_laplace_diagonal(const dg_op_desc* desc, double* diag_host) {
  int rc = validate_desc(desc);
  if (rc) return rc;
  if (!diag_host) return fail(DG_ERR_INVALID_ARG, "diag_host is NULL");
  if (desc->n_q != 0 && desc->n_q < desc->degree + 1)
    return fail(DG_ERR_UNSUPPORTED, "the Laplace form needs n_q >= k+1 (exact Gauss integration)");
  const int k = desc->degree, n = k + 1;
  const int m = desc->n_q ? desc->n_q : k + 1;
  const Basis1D& B = basis(k, m);
  const double sigma = desc->penalty_factor * (k + 1.0) * (k + 1.0);
  Sipg1D S = make_sipg_1d(B, sigma);
  LaplacePlan P = make_laplace_plan(desc, 1);
  // 1D diagonals per direction; with a single element in a direction the
  // element is its own neighbour and the couplings land on the diagonal.
  std::vector<double> kd(3 * n), md(n);
  for (int i = 0; i < n; ++i) md[i] = B.Mref[i * n + i];
  for (int d = 0; d < 3; ++d)
    for (int i = 0; i < n; ++i) {
      double v = S.Kown[i * n + i];
      if (desc->n_el[d] == 1) v += S.Kl[i * n + i] + S.Kr[i * n + i];
      kd[d * n + i] = v;
    }
  for (int c = 0; c < n; ++c)
    for (int b = 0; b < n; ++b)
      for (int a = 0; a < n; ++a)
        diag_host[a + n * (b + n * c)] = P.c[0] * kd[0 * n + a] * md[b] * md[c] +
                                         P.c[1] * md[a] * kd[1 * n + b] * md[c] +
                                         P.c[2] * md[a] * md[b] * kd[2 * n + c];
  return ok();
}

int dg_apply_laplace(const dg_op_desc* desc, dg_dtype dtype, const void* src, void* dst,
                     void* hip_stream) {
  int rc = validate_desc(desc);
  if (rc) return rc;
  if (dtype != DG_F64 && dtype != DG_F32) return fail(DG_ERR_INVALID_ARG, "dtype must be DG_F64 or DG_F32");
  if (desc->n_comp != 1 && desc->n_comp != 3) return fail(DG_ERR_INVALID_ARG, "n_comp must be 1 or 3");
  if (!src || !dst) return fail(DG_ERR_INVALID_ARG, "src/dst is NULL");
  if (desc->n_q != 0 && desc->n_q < desc->degree + 1)
    return fail(DG_ERR_UNSUPPORTED, "the Laplace form needs n_q >= k+1 (exact Gauss integration)");
  const size_t bytes = (size_t)desc->n_comp * num_elements(desc) * dofs_per_element(desc) *
                       (dtype == DG_F64 ? 8 : 4);
  if (overlaps(src, bytes, dst, bytes)) return fail(DG_ERR_ALIAS, "dst overlaps src");
  LaplacePlan P = make_laplace_plan(desc, desc->n_comp);
  hipError_t e = launch_laplace(P, dtype == DG_F32, src, dst, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "laplace kernel launch");
  return ok();
}

int dg_apply_helmholtz(const dg_op_desc* desc, dg_dtype dtype, double mass_factor, const void* src, void* dst,
                       void* hip_stream) {
  int rc = validate_desc(desc);
  if (rc) return rc;
  if (dtype != DG_F64 && dtype != DG_F32) return fail(DG_ERR_INVALID_ARG, "dtype must be DG_F64 or DG_F32");
  if (desc->n_comp != 1 && desc->n_comp != 3) return fail(DG_ERR_INVALID_ARG, "n_comp must be 1 or 3");
  if (!src || !dst) return fail(DG_ERR_INVALID_ARG, "src/dst is NULL");
  if (!(mass_factor >= 0.0) || !std::isfinite(mass_factor))
    return fail(DG_ERR_INVALID_ARG, "mass_factor must be finite and >= 0");
  if (desc->n_q != 0 && desc->n_q < desc->degree + 1)
    return fail(DG_ERR_UNSUPPORTED, "the Helmholtz form needs n_q >= k+1 (exact Gauss integration)");
  const size_t bytes = (size_t)desc->n_comp * num_elements(desc) * dofs_per_element(desc) *
                       (dtype == DG_F64 ? 8 : 4);
  if (overlaps(src, bytes, dst, bytes)) return fail(DG_ERR_ALIAS, "dst overlaps src");
  LaplacePlan P = make_laplace_plan(desc, desc->n_comp);
  P.shift = mass_factor * cell_volume(desc);
  hipError_t e = launch_laplace(P, dtype == DG_F32, src, dst, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "helmholtz kernel launch");
  return ok();
}

int dg_apply_projection(const dg_op_desc* desc, dg_dtype dtype, const void* u, const void* tau_d,
                        const void* tau_c, void* y, void* hip_stream) {
  int rc = validate_desc(desc);
  if (rc) return rc;
  if (dtype != DG_F64 && dtype != DG_F32) return fail(DG_ERR_INVALID_ARG, "dtype must be DG_F64 or DG_F32");
  if (desc->n_comp != 3) return fail(DG_ERR_INVALID_ARG, "the projection operator needs n_comp = 3");
  if (!u || !tau_d || !tau_c || !y) return fail(DG_ERR_INVALID_ARG, "u/tau_d/tau_c/y is NULL");
  if (desc->n_q != 0 && desc->n_q != desc->degree + 1)
    return fail(DG_ERR_UNSUPPORTED, "the projection operator is built for n_q = k+1");
  const size_t es = dtype == DG_F64 ? 8 : 4;
  const size_t bytes = (size_t)3 * num_elements(desc) * dofs_per_element(desc) * es;
  const size_t tb = (size_t)num_elements(desc) * es;
  if (overlaps(u, bytes, y, bytes) || overlaps(tau_d, tb, y, bytes) || overlaps(tau_c, tb, y, bytes))
    return fail(DG_ERR_ALIAS, "y overlaps an input");
  const ProjPlan P = make_proj_plan(desc);
  hipError_t e = launch_projection(P, dtype == DG_F32, u, y, tau_d, tau_c, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "projection kernel launch");
  return ok();
}

int dg_apply_convective(const dg_op_desc* desc, dg_dtype dtype, const void* u, void* r,
                        void* hip_stream) {
  int rc = validate_desc(desc);
  if (rc) return rc;
  if (dtype != DG_F64 && dtype != DG_F32) return fail(DG_ERR_INVALID_ARG, "dtype must be DG_F64 or DG_F32");
  if (!u || !r) return fail(DG_ERR_INVALID_ARG, "u/r is NULL");
  const size_t bytes = (size_t)3 * num_elements(desc) * dofs_per_element(desc) * (dtype == DG_F64 ? 8 : 4);
  if (overlaps(u, bytes, r, bytes)) return fail(DG_ERR_ALIAS, "r overlaps u");
  ConvPlan P;
  rc = make_conv_plan(desc, P);
  if (rc) return rc;
  hipError_t e = launch_convective(P, dtype == DG_F32, u, r, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "convective kernel launch");
  return ok();
}

int dg_vjp_convective(const dg_op_desc* desc, dg_dtype dtype, const void* u, const void* w,
                      void* grad_u, void* hip_stream) {
  int rc = validate_desc(desc);
  if (rc) return rc;
  if (dtype != DG_F64 && dtype != DG_F32) return fail(DG_ERR_INVALID_ARG, "dtype must be DG_F64 or DG_F32");
  if (!u || !w || !grad_u) return fail(DG_ERR_INVALID_ARG, "u/w/grad_u is NULL");
  const int kmax = vjp_max_degree(dtype == DG_F32);
  if (desc->degree > kmax)
    return fail(DG_ERR_UNSUPPORTED, "convective VJP is built for degree <= " + std::to_string(kmax) +
                                        (dtype == DG_F32 ? " in FP32" : " in FP64"));
  const size_t bytes = (size_t)3 * num_elements(desc) * dofs_per_element(desc) * (dtype == DG_F64 ? 8 : 4);
  if (overlaps(u, bytes, grad_u, bytes) || overlaps(w, bytes, grad_u, bytes))
    return fail(DG_ERR_ALIAS, "grad_u overlaps u or w");
  ConvPlan P;
  rc = make_conv_plan(desc, P);
  if (rc) return rc;
  hipError_t e = launch_convective_vjp(P, dtype == DG_F32, u, w, grad_u, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "convective VJP kernel launch");
  return ok();
}

int dg_apply_divergence(const dg_op_desc* desc, dg_dtype dtype, const void* u, void* b,
                        void* hip_stream) {
  int rc = validate_desc(desc);
  if (rc) return rc;
  if (dtype != DG_F64 && dtype != DG_F32) return fail(DG_ERR_INVALID_ARG, "dtype must be DG_F64 or DG_F32");
  if (!u || !b) return fail(DG_ERR_INVALID_ARG, "u/b is NULL");
  const size_t es = dtype == DG_F64 ? 8 : 4;
  const size_t nb = (size_t)num_elements(desc) * dofs_per_element(desc) * es;
  if (overlaps(u, 3 * nb, b, nb)) return fail(DG_ERR_ALIAS, "b overlaps u");
  DivPlan P = make_div_plan(desc);
  hipError_t e = launch_divergence(P, dtype == DG_F32, u, b, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "divergence kernel launch");
  return ok();
}

int dg_apply_gradient(const dg_op_desc* desc, dg_dtype dtype, const void* p, void* y, void* hip_stream) {
  int rc = validate_desc(desc);
  if (rc) return rc;
  if (dtype != DG_F64 && dtype != DG_F32) return fail(DG_ERR_INVALID_ARG, "dtype must be DG_F64 or DG_F32");
  if (!p || !y) return fail(DG_ERR_INVALID_ARG, "p/y is NULL");
  const size_t es = dtype == DG_F64 ? 8 : 4;
  const size_t np = (size_t)num_elements(desc) * dofs_per_element(desc) * es;
  if (overlaps(p, np, y, 3 * np)) return fail(DG_ERR_ALIAS, "y overlaps p");
  DivPlan P = make_div_plan(desc);
  hipError_t e = launch_gradient(P, dtype == DG_F32, p, y, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "gradient kernel launch");
  return ok();
}

static int transfer(const dg_op_desc* coarse, dg_dtype dtype, bool prolong, const void* src, void* dst,
                    void* hip_stream) {
  int rc = validate_desc(coarse);
  if (rc) return rc;
  if (dtype != DG_F64 && dtype != DG_F32) return fail(DG_ERR_INVALID_ARG, "dtype must be DG_F64 or DG_F32");
  if (coarse->n_comp != 1 && coarse->n_comp != 3) return fail(DG_ERR_INVALID_ARG, "n_comp must be 1 or 3");
  if (!src || !dst) return fail(DG_ERR_INVALID_ARG, "src/dst is NULL");
  for (int d = 0; d < 3; ++d)
    if (coarse->n_el[d] > (1 << 29)) return fail(DG_ERR_INVALID_ARG, "fine mesh too large");
  const long long nc = num_elements(coarse);
  if (8 * nc > (1LL << 31) - 1) return fail(DG_ERR_INVALID_ARG, "fine mesh too large");
  const size_t es = dtype == DG_F64 ? 8 : 4;
  const size_t cb = (size_t)coarse->n_comp * nc * dofs_per_element(coarse) * es;
  if (overlaps(src, prolong ? cb : 8 * cb, dst, prolong ? 8 * cb : cb)) return fail(DG_ERR_ALIAS, "dst overlaps src");
  TransferPlan P;
  P.k = coarse->degree;
  P.nxc = coarse->n_el[0];
  P.nyc = coarse->n_el[1];
  P.nzc = coarse->n_el[2];
  P.n_comp = coarse->n_comp;
  {
    std::lock_guard<std::mutex> lock(g_child_mutex);
    for (int c = 0; c < 2; ++c) {
      auto it = g_child.find(2 * P.k + c);
      if (it == g_child.end()) it = g_child.emplace(2 * P.k + c, child_interp(P.k, c)).first;
      P.P[c] = it->second;
    }
  }
  hipError_t e = launch_transfer(P, prolong, dtype == DG_F32, src, dst, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, prolong ? "prolongation kernel launch" : "restriction kernel launch");
  return ok();
}

int dg_prolongate(const dg_op_desc* coarse, dg_dtype dtype, const void* uc, void* uf, void* hip_stream) {
  return transfer(coarse, dtype, true, uc, uf, hip_stream);
}

int dg_restrict(const dg_op_desc* coarse, dg_dtype dtype, const void* rf, void* rc, void* hip_stream) {
  return transfer(coarse, dtype, false, rf, rc, hip_stream);
}

int dg_apply_inverse_mass(const dg_op_desc* desc, dg_dtype dtype, const void* src, void* dst,
                          void* hip_stream) {
  int rc = validate_desc(desc);
  if (rc) return rc;
  if (dtype != DG_F64 && dtype != DG_F32) return fail(DG_ERR_INVALID_ARG, "dtype must be DG_F64 or DG_F32");
  if (desc->n_comp != 1 && desc->n_comp != 3) return fail(DG_ERR_INVALID_ARG, "n_comp must be 1 or 3");
  if (!src || !dst) return fail(DG_ERR_INVALID_ARG, "src/dst is NULL");
  if (desc->n_q != 0 && desc->n_q < desc->degree + 1)
    return fail(DG_ERR_UNSUPPORTED, "the inverse mass needs n_q >= k+1 (exact Gauss integration)");
  const long long nblocks = (long long)desc->n_comp * num_elements(desc);
  const size_t bytes = (size_t)nblocks * dofs_per_element(desc) * (dtype == DG_F64 ? 8 : 4);
  if (src != dst && overlaps(src, bytes, dst, bytes)) return fail(DG_ERR_ALIAS, "dst overlaps src (not in place)");
  hipError_t e = launch_inverse_mass(desc->degree, inverse_mass_1d(desc->degree), 1.0 / cell_volume(desc), nblocks,
                                     dtype == DG_F32, src, dst, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "inverse mass kernel launch");
  return ok();
}

}  // extern "C"
