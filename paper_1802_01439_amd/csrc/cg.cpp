// Preconditioned CG for the SIPG pressure Poisson problem (Sec. 3.3), host
// driver.  Everything of size N_DoFs lives on the GPU: the FP64 operator
// applies, residuals, dot products and the x, r, p updates; with the
// Chebyshev preconditioner the smoother runs FP32 operator applies.  The
// iteration scalars stay on the device; the host reads them once per batch
// of iterations.  Vector work is fused into the operator applies where that
// measured faster: the FP64 apply sums p.Ap in its epilogue, each FP32 apply
// performs its Chebyshev step in the epilogue (the first one forms its
// operand from the FP64 residual, the last one sums what the flexible beta
// needs).  Per iteration: FP64 apply with the p.Ap
// sums, x/r update, the FP32 applies, p update, and one-workgroup kernels
// finishing the sums.
//
// Variant: flexible (Polak-Ribiere) CG, beta = r+.(z+ - z)/(r.z), so that a
// single-precision preconditioner that is symmetric only up to rounding keeps
// convergence.  On periodic meshes (project_mean) the residual and the
// preconditioned residual are kept at zero coefficient mean, the subspace on
// which the SIPG operator is invertible.
//
// Preconditioners: Jacobi (D^-1 in FP64), and the Chebyshev iteration of
// Adams et al. (2003) on D^-1 A (Sec. 3.3: degree 5, smoothing range 20)
// started from zero in FP32: theta = (lmax+lmin)/2, delta = (lmax-lmin)/2,
// x1 = D^-1 r / theta, rho_0 = delta/theta, then for each further step
// rho_k = 1/(2 theta/delta - rho_{k-1}),
// d_k = rho_k rho_{k-1} d_{k-1} + (2 rho_k/delta) D^-1 (r - A x_k), x += d_k,
// evaluated in the equivalent three-term form x_{k+1} = x_k + rho_k rho_{k-1}
// (x_k - x_{k-1}) + (2 rho_k/delta) D^-1 (r - A x_k) with x_0 = 0, so that
// no step vector is stored.
// lmax is 1.1x the largest Ritz value of 25 Lanczos steps (plain Jacobi-PCG
// on a hashed random zero-mean vector), computed once per operator and kept;
// lmin = lmax / range.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "api_internal.h"
#include "cg_kernels.h"
#include "cg_laplace.h"
#include "dgmf.h"
#include "ops.h"

namespace dgmf {

namespace {

struct Workspace {
  long long n = 0;
  double *r = nullptr, *p = nullptr, *q = nullptr, *z = nullptr, *zold = nullptr, *tmp = nullptr;
  float *r32 = nullptr, *x32 = nullptr, *t32 = nullptr, *za32 = nullptr, *zb32 = nullptr;
  double* partial = nullptr;   // npartial doubles
  long npartial = 0;
  double* res = nullptr;       // 8 results (device)
  double* host = nullptr;      // 8 results (pinned host)
  double* st = nullptr;        // main-loop state (device), kStateSize
  double* host_st = nullptr;   // its pinned host copy
  double* dinv = nullptr;      // n3
  float* dinv32 = nullptr;     // n3
};

std::mutex g_ws_mutex;
std::map<int, Workspace> g_ws;

// lambda_max estimates by operator (degree, mesh, box, n_q, penalty, scale,
// projection): the Lanczos start vector is a fixed hash, so a repeated solve
// on the same operator would compute the same value
std::mutex g_lmax_mutex;
std::map<std::vector<double>, double> g_lmax;

std::vector<double> lmax_key(const dg_op_desc* d, bool project) {
  return {(double)d->degree, (double)d->n_el[0], (double)d->n_el[1], (double)d->n_el[2], d->length[0],
          d->length[1], d->length[2], (double)d->n_q, d->penalty_factor, d->scale, project ? 1.0 : 0.0};
}

hipError_t ensure(Workspace& w, long long n, long npartial) {
  hipError_t e;
  npartial = std::max<long>(npartial, 8L * kCgBlocks);
  if (w.npartial < npartial) {
    if (w.partial) (void)hipFree(w.partial);
    w.partial = nullptr;
    w.npartial = 0;
    if ((e = hipMalloc((void**)&w.partial, npartial * sizeof(double))) != hipSuccess) return e;
    w.npartial = npartial;
  }
  if (!w.res && (e = hipMalloc((void**)&w.res, 8 * sizeof(double))) != hipSuccess) return e;
  if (!w.host && (e = hipHostMalloc((void**)&w.host, 8 * sizeof(double), 0)) != hipSuccess) return e;
  if (!w.st && (e = hipMalloc((void**)&w.st, kStateSize * sizeof(double))) != hipSuccess) return e;
  if (!w.host_st && (e = hipHostMalloc((void**)&w.host_st, kStateSize * sizeof(double), 0)) != hipSuccess) return e;
  if (!w.dinv && (e = hipMalloc((void**)&w.dinv, 1728 * sizeof(double))) != hipSuccess) return e;
  if (!w.dinv32 && (e = hipMalloc((void**)&w.dinv32, 1728 * sizeof(float))) != hipSuccess) return e;
  if (w.n >= n) return hipSuccess;
  double** d8[] = {&w.r, &w.p, &w.q, &w.z, &w.zold, &w.tmp};
  float** d4[] = {&w.r32, &w.x32, &w.t32, &w.za32, &w.zb32};
  for (double** pp : d8) {
    if (*pp) (void)hipFree(*pp);
    *pp = nullptr;
  }
  for (float** pp : d4) {
    if (*pp) (void)hipFree(*pp);
    *pp = nullptr;
  }
  w.n = 0;
  for (double** pp : d8)
    if ((e = hipMalloc((void**)pp, (size_t)n * 8)) != hipSuccess) return e;
  for (float** pp : d4)
    if ((e = hipMalloc((void**)pp, (size_t)n * 4)) != hipSuccess) return e;
  w.n = n;
  return hipSuccess;
}

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// largest eigenvalue of the symmetric tridiagonal (a diag, b off-diag) by bisection
double tridiag_max_eig(const std::vector<double>& a, const std::vector<double>& b) {
  const int m = (int)a.size();
  double lo = 0, hi = 0;
  for (int i = 0; i < m; ++i) {
    double rad = (i > 0 ? std::fabs(b[i - 1]) : 0) + (i + 1 < m ? std::fabs(b[i]) : 0);
    hi = std::fmax(hi, a[i] + rad);
    lo = std::fmin(lo, a[i] - rad);
  }
  auto count_below = [&](double x) {   // eigenvalues < x (Sturm sequence)
    int c = 0;
    double d = 1.0;
    for (int i = 0; i < m; ++i) {
      d = a[i] - x - (i > 0 ? b[i - 1] * b[i - 1] / d : 0.0);
      if (d == 0.0) d = -1e-300;
      if (d < 0) ++c;
    }
    return c;
  };
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (count_below(mid) == m) hi = mid; else lo = mid;
  }
  return hi;
}

// Device tables of the FP64 and FP32 Laplace kernels (nullptr: the library's
// table cache).
struct Tables {
  const void* f64 = nullptr;
  const void* f32 = nullptr;
};

struct Solver {
  const dg_op_desc* desc;
  LaplacePlan P;
  Tables tab;
  Workspace* w;
  hipStream_t s;
  long long n;
  int n3;
  bool project;
  int matvec64 = 0, matvec32 = 0;
  hipError_t err = hipSuccess;

  bool ok(hipError_t e) {
    if (e != hipSuccess && err == hipSuccess) err = e;
    return e == hipSuccess;
  }
  // reduce nq partials and read them on the host
  bool fetch(int nq) {
    if (!ok(cg_finalize(w->partial, nq, w->res, s))) return false;
    if (!ok(hipMemcpyAsync(w->host, w->res, nq * sizeof(double), hipMemcpyDeviceToHost, s))) return false;
    return ok(hipStreamSynchronize(s));
  }
  bool apply64(const double* in, double* out) {
    ++matvec64;
    return ok(launch_laplace(P, false, in, out, s, tab.f64));
  }
  bool apply32(const float* in, float* out) {
    ++matvec32;
    return ok(launch_laplace(P, true, in, out, s, tab.f32));
  }
};

// 1.1 x the largest Ritz value of 25 Lanczos steps of plain Jacobi-PCG on D^-1 A
// (the Lanczos tridiagonal from the PCG coefficients), started from a hashed
// zero-mean (with projection) vector; W.dinv must hold D^-1 of one element.
// Stored in the per-operator cache.
int lanczos_lmax(Solver& S, const dg_op_desc* desc, double* lmax_out) {
  Workspace& W = *S.w;
  double* H = W.host;
  const long long n = S.n;
  const double dn = (double)n;
  const int L = 25;
  S.ok(cg_hash_fill(W.tmp, 12345ULL, n, W.partial, S.s));
  if (!S.fetch(1)) return hip_fail(S.err, "Lanczos start");
  const double mu0 = S.project ? H[0] / dn : 0.0;
  S.ok(cg_axpb(W.r, W.tmp, 1.0, -mu0, n, S.s));
  S.ok(cg_fill(W.zold, 0.0, n, S.s));
  S.ok(cg_jacobi(W.r, W.z, W.zold, W.dinv, S.n3, 0.0, n, W.partial, S.s));
  if (!S.fetch(4)) return hip_fail(S.err, "Lanczos start");
  double muz = S.project ? H[0] / dn : 0.0, rz = H[1];
  S.ok(cg_update_p(W.z, W.p, W.zold, muz, 0.0, n, S.s));
  std::vector<double> al, be;
  for (int it = 0; it < L; ++it) {
    S.apply64(W.p, W.q);
    S.ok(cg_dot(W.p, W.q, n, W.partial, S.s));
    if (!S.fetch(1)) return hip_fail(S.err, "Lanczos");
    const double pq = H[0];
    if (!(pq > 0) || !(rz > 0)) break;
    const double alpha = rz / pq;
    S.ok(cg_update_xr(W.tmp, W.r, W.p, W.q, alpha, n, W.partial, S.s));
    if (!S.fetch(1)) return hip_fail(S.err, "Lanczos");
    const double mur = S.project ? H[0] / dn : 0.0;
    S.ok(cg_jacobi(W.r, W.z, W.zold, W.dinv, S.n3, mur, n, W.partial, S.s));
    if (!S.fetch(4)) return hip_fail(S.err, "Lanczos");
    muz = S.project ? H[0] / dn : 0.0;
    const double rz_new = H[1];
    const double beta = rz_new / rz;
    al.push_back(alpha);
    be.push_back(beta);
    S.ok(cg_update_p(W.z, W.p, W.zold, muz, beta, n, S.s));
    rz = rz_new;
    if (!(rz > 0)) break;
  }
  const int m = (int)al.size();
  if (m == 0) return fail(DG_ERR_BREAKDOWN, "eigenvalue estimate failed (operator not positive definite?)");
  std::vector<double> ta(m), tb(m > 1 ? m - 1 : 0);
  for (int i = 0; i < m; ++i) {
    ta[i] = 1.0 / al[i] + (i > 0 ? be[i - 1] / al[i - 1] : 0.0);
    if (i + 1 < m) tb[i] = std::sqrt(be[i]) / al[i];
  }
  *lmax_out = 1.1 * tridiag_max_eig(ta, tb);
  std::lock_guard<std::mutex> lk(g_lmax_mutex);
  g_lmax[lmax_key(desc, S.project)] = *lmax_out;
  return DG_OK;
}

// D^-1 of one element of the operator of desc, in W.dinv / W.dinv32
int upload_dinv(const dg_op_desc* desc, Workspace& W, hipStream_t s, std::vector<double>& dinv) {
  const long long n3 = dofs_per_element(desc);
  std::vector<double> diag(n3);
  std::vector<float> dinv32(n3);
  dinv.assign(n3, 0.0);
  int rc = dg_laplace_diagonal(desc, diag.data());
  if (rc) return rc;
  for (long long i = 0; i < n3; ++i) {
    if (!(diag[i] > 0)) return fail(DG_ERR_BREAKDOWN, "operator diagonal is not positive");
    dinv[i] = 1.0 / diag[i];
    dinv32[i] = (float)dinv[i];
  }
  hipError_t e;
  if ((e = hipMemcpyAsync(W.dinv, dinv.data(), n3 * 8, hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(W.dinv32, dinv32.data(), n3 * 4, hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return hip_fail(e, "diagonal upload");
  return DG_OK;
}

// Arguments of dg_cg_solve and its allocation-free variant; sets the DoF
// counts.
int cg_validate(const dg_op_desc* desc, const dg_cg_opts* opts, const double* b, const double* x, long long* n_out,
                long long* n3_out) {
  int rc = validate_desc(desc);
  if (rc) return rc;
  if (!opts) return fail(DG_ERR_INVALID_ARG, "opts is NULL");
  if (!b || !x) return fail(DG_ERR_INVALID_ARG, "b/x is NULL");
  if (desc->n_comp != 1) return fail(DG_ERR_INVALID_ARG, "dg_cg_solve needs n_comp = 1");
  if (opts->precond != DG_PC_JACOBI_F64 && opts->precond != DG_PC_CHEB_F32)
    return fail(DG_ERR_INVALID_ARG, "unknown preconditioner");
  const bool cheb = opts->precond == DG_PC_CHEB_F32;
  if (cheb && (opts->cheb_degree < 1 || opts->cheb_degree > 64 || !(opts->cheb_range > 1.0) ||
               !std::isfinite(opts->cheb_range)))
    return fail(DG_ERR_INVALID_ARG, "cheb_degree must be 1..64 and cheb_range finite > 1");
  if (!(opts->rtol >= 0) || !(opts->atol >= 0) || !std::isfinite(opts->rtol) || !std::isfinite(opts->atol))
    return fail(DG_ERR_INVALID_ARG, "rtol/atol must be finite and >= 0");
  if (opts->max_iter < 1) return fail(DG_ERR_INVALID_ARG, "max_iter must be >= 1");
  const long long n3 = dofs_per_element(desc);
  const long long n = num_elements(desc) * n3;
  if (overlaps(b, (size_t)n * 8, x, (size_t)n * 8)) return fail(DG_ERR_ALIAS, "x overlaps b");
  *n_out = n;
  *n3_out = n3;
  return DG_OK;
}

// The solve on a workspace W whose vectors hold n values and whose partial
// buffer holds max(grid64, 3 grid32, 8 kCgBlocks) doubles.
int cg_run(const dg_op_desc* desc, const dg_cg_opts* opts, const double* b, double* x, dg_cg_report* report,
           void* hip_stream, Workspace& W, const LaplacePlan& LP, Tables tabs, long long n, long long n3,
           double t_start) {
  const bool cheb = opts->precond == DG_PC_CHEB_F32;
  const long grid64 = cg_apply_grid(LP, false), grid32 = cg_apply_grid(LP, true);
  int rc;
  Solver S;
  S.desc = desc;
  S.P = LP;
  S.tab = tabs;
  S.w = &W;
  S.s = (hipStream_t)hip_stream;
  S.n = n;
  S.n3 = (int)n3;
  S.project = opts->project_mean != 0;

  // ---- setup: diagonal, eigenvalue estimate ----
  std::vector<double> dinv;
  if ((rc = upload_dinv(desc, W, S.s, dinv)) != DG_OK) return rc;
  double* H = W.host;
  const double dn = (double)n;
  double lmax = 0, theta = 0, delta = 0;
  bool have_lmax = false;
  if (cheb) {
    std::lock_guard<std::mutex> lk(g_lmax_mutex);
    auto it = g_lmax.find(lmax_key(desc, S.project));
    if (it != g_lmax.end()) {
      lmax = it->second;
      have_lmax = true;
    }
  }
  if (cheb && !have_lmax) {
    if ((rc = lanczos_lmax(S, desc, &lmax)) != DG_OK) return rc;
    S.matvec64 = 0;
  }
  if (cheb) {
    const double lmin = lmax / opts->cheb_range;
    theta = 0.5 * (lmax + lmin);
    delta = 0.5 * (lmax - lmin);
  }
  if (!S.ok(hipStreamSynchronize(S.s))) return hip_fail(S.err, "setup");
  const double t_setup = now();

  // ---- main loop ----
  // The iteration scalars (alpha, beta, means, |r|, convergence) are computed
  // on the device and stay there; the host enqueues a batch of iterations and
  // reads the state once per batch.  Iterations queued after convergence are
  // no-ops (alpha = 0), so the result does not depend on the batch size.
  // Jacobi (a fixed symmetric preconditioner) uses the standard PCG beta,
  // Chebyshev in FP32 the flexible one.
  int status = DG_OK;
  int it = 0;
  double rel = 0, bnorm = 0;
  S.apply64(x, W.q);
  S.ok(cg_residual(b, W.q, W.r, n, W.partial, S.s));
  if (!S.fetch(4)) return hip_fail(S.err, "initial residual");
  const double sum_b = H[2], sum_bb = H[3];
  bnorm = std::sqrt(std::fmax(0.0, S.project ? sum_bb - sum_b * sum_b / dn : sum_bb));
  const double tol = std::fmax(opts->rtol * bnorm, opts->atol);
  double sum_d = 0;
  for (long long i = 0; i < n3; ++i) sum_d += dinv[i];
  sum_d *= (double)num_elements(desc);
  S.ok(cg_state_init(W.st, tol * tol, opts->max_iter, sum_d, n, S.project, S.s));
  // FP32 double buffers, rotated by the host in enqueue order (iterations
  // queued after convergence rotate them too; they no longer touch x):
  //   Xb: intermediate Chebyshev iterates x_2, x_3, ...: step j reads x_j from
  //       Xb[j % 2] and x_{j-1} from Xb[(j + 1) % 2], which x_{j+1} overwrites
  //   Zb: smoother outputs, the current one and the one before (flexible beta)
  float* Xb[2] = {W.x32, W.t32};
  float* Zb[2] = {W.za32, W.zb32};
  int zn = 0;     // Zb[zn]: next smoother output; Zb[1 - zn]: the latest one
  S.ok(cg_fill(W.p, 0.0, n, S.s));
  if (cheb) S.ok(cg_fill32(Zb[1], 0.0f, n, S.s));
  const int napp = cheb ? opts->cheb_degree - 1 : 0;
  // scalars of the current residual (sums of r from the x/r update), then
  // z = M^-1 r' with the sums of the flexible beta
  auto precondition = [&](bool start) {
    if (!cheb) {
      S.ok(cg_fin_jacobi(W.partial, W.st, start, S.s));
      S.ok(cg_update_p_jacobi(W.r, W.p, W.dinv, S.n3, W.st, n, S.s));
      return;
    }
    S.ok(cg_fin_resid(W.partial, W.st, start, S.s));
    if (napp == 0) {
      S.ok(cg_cheb1(W.r, Zb[zn], Zb[1 - zn], W.dinv32, S.n3, W.st, (float)(1.0 / theta), n, W.partial, S.s));
    }
    double rho_prev = delta / theta;
    for (int j = 1; j <= napp; ++j) {
      const double rho = 1.0 / (2.0 * theta / delta - rho_prev);
      ChebStepArgs a{};
      a.r = W.r;
      a.xin = j >= 2 ? Xb[j % 2] : nullptr;
      a.xprev = j >= 3 ? Xb[(j + 1) % 2] : nullptr;
      a.xout = j == napp ? Zb[zn] : Xb[(j + 1) % 2];
      a.r32 = W.r32;
      a.dinv = W.dinv32;
      a.zprev = Zb[1 - zn];
      a.st = W.st;
      a.partial = W.partial;
      a.c1 = (float)(rho * rho_prev);
      a.c2 = (float)(2.0 * rho / delta);
      a.inv_theta = (float)(1.0 / theta);
      ++S.matvec32;
      S.ok(cg_apply_cheb(LP, j, j == napp, a, S.s, tabs.f32));
      rho_prev = rho;
    }
    S.ok(cg_fin_cheb(W.partial, napp == 0 ? kCgBlocks : (int)grid32, W.st, start, S.s));
    S.ok(cg_update_p_cheb(Zb[zn], W.p, W.st, n, S.s));
    zn = 1 - zn;
  };
  // start: alpha is 0 in the fresh state, so this only forms the sums of r0
  S.ok(cg_update_xr_st(x, W.r, W.p, W.q, W.dinv, S.n3, W.st, !cheb, n, W.partial, S.s));
  precondition(true);
  // batch size: up to max_batch, fewer when the observed contraction rate
  // says the tolerance is that close (keeps queued no-op iterations rare)
  const int max_batch = cheb ? 4 : 8;
  int batch = max_batch;
  long long queued = 0;
  double* HS = W.host_st;
  double rn2_prev = -1, it_prev = 0;
  for (;;) {
    if (!S.ok(hipMemcpyAsync(HS, W.st, kStateSize * sizeof(double), hipMemcpyDeviceToHost, S.s)) ||
        !S.ok(hipStreamSynchronize(S.s)))
      return hip_fail(S.err, "CG state");
    if (HS[kDone] != 0.0 || queued > (long long)opts->max_iter + max_batch) break;
    batch = max_batch;
    if (rn2_prev > 0 && HS[kRN2] > 0 && HS[kRN2] < rn2_prev && HS[kIter] > it_prev) {
      const double rate = std::log(HS[kRN2] / rn2_prev) / (HS[kIter] - it_prev);   // per iteration, < 0
      const double left = std::log(HS[kTol2] / HS[kRN2]) / rate;
      if (std::isfinite(left)) batch = (int)std::max(1.0, std::min((double)max_batch, std::ceil(left)));
    }
    rn2_prev = HS[kRN2];
    it_prev = HS[kIter];
    for (int b2 = 0; b2 < batch; ++b2) {
      // q = A p with the p.q partials
      ++S.matvec64;
      S.ok(cg_apply_dot(LP, W.p, W.q, W.partial, S.s, tabs.f64));
      S.ok(cg_fin_alpha(W.partial, (int)grid64, W.st, S.s));
      S.ok(cg_update_xr_st(x, W.r, W.p, W.q, W.dinv, S.n3, W.st, !cheb, n, W.partial, S.s));
      precondition(false);
    }
    queued += batch;
    if (S.err != hipSuccess) return hip_fail(S.err, "CG iteration");
  }
  it = (int)HS[kIter];
  rel = std::sqrt(std::fmax(0.0, HS[kRN2])) / (bnorm > 0 ? bnorm : 1.0);
  if (HS[kStatus] == 2.0) status = DG_ERR_BREAKDOWN;
  else if (HS[kStatus] == 1.0 || HS[kDone] == 0.0) status = DG_NOT_CONVERGED;
  if (!S.ok(hipStreamSynchronize(S.s))) return hip_fail(S.err, "solve");
  const double t_solve = now();
  // true residual in FP64
  S.apply64(x, W.q);
  S.ok(cg_residual(b, W.q, W.tmp, n, W.partial, S.s));
  if (!S.fetch(4)) return hip_fail(S.err, "true residual");
  const double tr2 = S.project ? H[1] - H[0] * H[0] / dn : H[1];
  const double true_rel = std::sqrt(std::fmax(0.0, tr2)) / (bnorm > 0 ? bnorm : 1.0);
  if (report) {
    report->iterations = it;
    report->matvec_f64 = S.matvec64;
    report->matvec_f32 = S.matvec32;
    report->rel_res = rel;
    report->true_rel_res = true_rel;
    report->lambda_max = lmax;
    report->seconds_setup = t_setup - t_start;
    report->seconds_solve = t_solve - t_setup;
  }
  if (status == DG_ERR_BREAKDOWN) return fail(status, "CG breakdown (p.Ap <= 0 or non-finite residual)");
  if (status == DG_NOT_CONVERGED) return fail(status, "CG reached max_iter");
  return ok();
}

}  // namespace

int laplace_lambda_max(const dg_op_desc* desc, bool project, void* hip_stream, double* lmax) {
  int rc = validate_desc(desc);
  if (rc) return rc;
  if (desc->n_comp != 1) return fail(DG_ERR_INVALID_ARG, "the eigenvalue estimate needs n_comp = 1");
  {
    std::lock_guard<std::mutex> lk(g_lmax_mutex);
    auto it = g_lmax.find(lmax_key(desc, project));
    if (it != g_lmax.end()) {
      *lmax = it->second;
      return DG_OK;
    }
  }
  std::lock_guard<std::mutex> lock(g_ws_mutex);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  Workspace& W = g_ws[dev];
  const LaplacePlan LP = make_laplace_plan(desc, 1);
  const long long n = num_elements(desc) * dofs_per_element(desc);
  if ((e = ensure(W, n, std::max(cg_apply_grid(LP, false), 3 * cg_apply_grid(LP, true)))) != hipSuccess)
    return hip_fail(e, "CG workspace allocation");
  Solver S;
  S.desc = desc;
  S.P = LP;
  S.w = &W;
  S.s = (hipStream_t)hip_stream;
  S.n = n;
  S.n3 = (int)dofs_per_element(desc);
  S.project = project;
  std::vector<double> dinv;
  if ((rc = upload_dinv(desc, W, S.s, dinv)) != DG_OK) return rc;
  return lanczos_lmax(S, desc, lmax);
}

}  // namespace dgmf

using namespace dgmf;

extern "C" int dg_cg_solve(const dg_op_desc* desc, const dg_cg_opts* opts, const double* b, double* x,
                           dg_cg_report* report, void* hip_stream) {
  const double t_start = now();
  long long n = 0, n3 = 0;
  int rc = cg_validate(desc, opts, b, x, &n, &n3);
  if (rc) return rc;
  if (report) *report = dg_cg_report{};
  std::lock_guard<std::mutex> lock(g_ws_mutex);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  Workspace& W = g_ws[dev];
  const LaplacePlan LP = make_laplace_plan(desc, 1);
  const long grid64 = cg_apply_grid(LP, false), grid32 = cg_apply_grid(LP, true);
  if ((e = ensure(W, n, std::max(grid64, 3 * grid32))) != hipSuccess) return hip_fail(e, "CG workspace allocation");
  return cg_run(desc, opts, b, x, report, hip_stream, W, LP, Tables{}, n, n3, t_start);
}

// ---- allocation-free variant ----
//
// dg_cg_solve_noalloc runs the same solve with every piece of device memory
// beyond b and x (work vectors, partial sums, iteration state, diagonal,
// operator tables) carved from one file-scope device array of fixed size,
// and host reads through stack buffers, so that it calls no hipMalloc,
// hipHostMalloc or hipFree.  In host code `scratch` names a host-side
// stand-in: its device address is taken once per device with
// hipGetSymbolAddress and only that address is used.
namespace dgmf {

namespace {

constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mutex;
void* g_scratch_dev[kMaxDevices] = {};

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Byte offsets of the pieces in the scratch array.
struct ScratchLayout {
  size_t st, res, dinv, dinv32, tab64, tab32, partial, vec64[6], vec32[5], total;
  size_t tab64_bytes, tab32_bytes;
  long npartial;
};

ScratchLayout scratch_layout(const LaplacePlan& LP, long long n) {
  ScratchLayout L{};
  L.tab64_bytes = lap_table_fill(LP, false, nullptr);
  L.tab32_bytes = lap_table_fill(LP, true, nullptr);
  L.npartial = std::max<long>(std::max(cg_apply_grid(LP, false), 3 * cg_apply_grid(LP, true)), 8L * kCgBlocks);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  L.st = take(kStateSize * sizeof(double));
  L.res = take(8 * sizeof(double));
  L.dinv = take(1728 * sizeof(double));
  L.dinv32 = take(1728 * sizeof(float));
  L.tab64 = take(L.tab64_bytes);
  L.tab32 = take(L.tab32_bytes);
  L.partial = take((size_t)L.npartial * sizeof(double));
  for (size_t& v : L.vec64) v = take((size_t)n * sizeof(double));
  for (size_t& v : L.vec32) v = take((size_t)n * sizeof(float));
  L.total = o;
  return L;
}

}  // namespace

}  // namespace dgmf

extern "C" int dg_cg_solve_noalloc(const dg_op_desc* desc, const dg_cg_opts* opts, const double* b, double* x,
                                   dg_cg_report* report, void* hip_stream) {
  const double t_start = now();
  long long n = 0, n3 = 0;
  int rc = cg_validate(desc, opts, b, x, &n, &n3);
  if (rc) return rc;
  const LaplacePlan LP = make_laplace_plan(desc, 1);
  const ScratchLayout L = scratch_layout(LP, n);
  if (L.total > kNoAllocScratchBytes)
    return fail(DG_ERR_INVALID_ARG, "dg_cg_solve_noalloc: " + std::to_string(n) + " DoFs need " +
                                        std::to_string(L.total) + " bytes of scratch; the static array holds " +
                                        std::to_string(kNoAllocScratchBytes) + " (68 bytes per DoF)");
  if (report) *report = dg_cg_report{};
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(DG_ERR_INVALID_ARG, "device index beyond the scratch table");
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess)
      return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_dev[dev] = p;
  }
  unsigned char* base = static_cast<unsigned char*>(g_scratch_dev[dev]);
  Workspace W;
  W.n = n;
  W.st = reinterpret_cast<double*>(base + L.st);
  W.res = reinterpret_cast<double*>(base + L.res);
  W.dinv = reinterpret_cast<double*>(base + L.dinv);
  W.dinv32 = reinterpret_cast<float*>(base + L.dinv32);
  W.partial = reinterpret_cast<double*>(base + L.partial);
  W.npartial = L.npartial;
  double** d8[] = {&W.r, &W.p, &W.q, &W.z, &W.zold, &W.tmp};
  float** d4[] = {&W.r32, &W.x32, &W.t32, &W.za32, &W.zb32};
  for (int i = 0; i < 6; ++i) *d8[i] = reinterpret_cast<double*>(base + L.vec64[i]);
  for (int i = 0; i < 5; ++i) *d4[i] = reinterpret_cast<float*>(base + L.vec32[i]);
  // host ends of the state reads: ordinary (pageable) memory, read after a
  // stream synchronisation
  double host_res[8], host_st[kStateSize];
  W.host = host_res;
  W.host_st = host_st;
  // the operator tables, built on the host and copied into the scratch array
  // (the host copies live until the solve has returned)
  std::vector<unsigned char> t64(L.tab64_bytes), t32(L.tab32_bytes);
  lap_table_fill(LP, false, t64.data());
  lap_table_fill(LP, true, t32.data());
  const hipStream_t s = (hipStream_t)hip_stream;
  if ((e = hipMemcpyAsync(base + L.tab64, t64.data(), L.tab64_bytes, hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(base + L.tab32, t32.data(), L.tab32_bytes, hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_fail(e, "operator table upload");
  Tables tabs;
  tabs.f64 = base + L.tab64;
  tabs.f32 = base + L.tab32;
  rc = cg_run(desc, opts, b, x, report, hip_stream, W, LP, tabs, n, n3, t_start);
  const hipError_t se = hipStreamSynchronize(s);
  if (rc == DG_OK && se != hipSuccess) return hip_fail(se, "dg_cg_solve_noalloc");
  return rc;
}
