// CG for the projection and Helmholtz equations, preconditioned with the
// inverse mass matrix (Sec. 3.3: the mass is block diagonal and its inverse is
// applied matrix-free at the cost of a diagonal scaling, which makes it the
// preconditioner of both steps).  FP64 throughout.
//
// Per iteration: q = A p (projection or Helmholtz kernel, with the partial
// sums of p.q in its epilogue) and alpha;
// one fused kernel for x += alpha p, r -= alpha q, z = M^-1 r and the sums
// r.r, r.z (56 B/DoF instead of 80 for the three separate passes); the
// convergence test and beta; p = z + beta p.
// The scalars stay on the device; the host reads the state once per batch of
// iterations, sized from the observed contraction rate.  Once converged, the
// remaining iterations of a batch change nothing (alpha = 0).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>
#include <mutex>

#include "api_internal.h"
#include "cg_kernels.h"
#include "cg_laplace.h"
#include "dgmf.h"
#include "ops.h"

namespace dgmf {

namespace {

struct MassPcgWs {
  long long n = 0;
  double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
  double* partial = nullptr;   // npartial doubles
  long long npartial = 0;
  double* res = nullptr;       // 4 results (device)
  double* host = nullptr;      // 4 results (pinned host)
  double* st = nullptr;        // iteration state (device), kStateSize
  double* host_st = nullptr;   // its pinned host copy
};

std::mutex g_mpcg_mutex;
std::map<int, MassPcgWs> g_mpcg;

hipError_t ensure(MassPcgWs& w, long long n, long long npartial) {
  hipError_t e;
  npartial = std::max<long long>(npartial, 4LL * kCgBlocks);
  if (w.npartial < npartial) {
    if (w.partial) (void)hipFree(w.partial);
    w.partial = nullptr;
    w.npartial = 0;
    if ((e = hipMalloc((void**)&w.partial, (size_t)npartial * sizeof(double))) != hipSuccess) return e;
    w.npartial = npartial;
  }
  if (!w.res && (e = hipMalloc((void**)&w.res, 4 * sizeof(double))) != hipSuccess) return e;
  if (!w.host && (e = hipHostMalloc((void**)&w.host, 4 * sizeof(double), 0)) != hipSuccess) return e;
  if (!w.st && (e = hipMalloc((void**)&w.st, kStateSize * sizeof(double))) != hipSuccess) return e;
  if (!w.host_st && (e = hipHostMalloc((void**)&w.host_st, kStateSize * sizeof(double), 0)) != hipSuccess) return e;
  if (w.n < n) {
    double** v[4] = {&w.r, &w.z, &w.p, &w.q};
    for (double** pp : v) {
      if (*pp) (void)hipFree(*pp);
      *pp = nullptr;
    }
    w.n = 0;
    for (double** pp : v)
      if ((e = hipMalloc((void**)pp, (size_t)n * sizeof(double))) != hipSuccess) return e;
    w.n = n;
  }
  return hipSuccess;
}

// the nq finalized sums, read on the host
hipError_t read_sums(MassPcgWs& w, int nq, hipStream_t s) {
  hipError_t e;
  if ((e = cg_finalize(w.partial, nq, w.res, s)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(w.host, w.res, nq * sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

}  // namespace

}  // namespace dgmf

using namespace dgmf;

int dgmf::mass_pcg_solve(const dg_op_desc* desc, int32_t op, double mass_factor, const double* tau_d,
                         const double* tau_c, const double* b, double* x, double rtol, int32_t max_iter,
                         dg_cg_report* report, void* hip_stream, bool true_residual) {
  const auto t0 = std::chrono::steady_clock::now();
  int rc = validate_desc(desc);
  if (rc) return rc;
  if (!b || !x) return fail(DG_ERR_INVALID_ARG, "b/x is NULL");
  if (!(rtol > 0.0) || !std::isfinite(rtol)) return fail(DG_ERR_INVALID_ARG, "rtol must be finite and > 0");
  if (max_iter < 0) return fail(DG_ERR_INVALID_ARG, "max_iter must be >= 0");
  if (desc->n_q != 0 && desc->n_q != desc->degree + 1)
    return fail(DG_ERR_UNSUPPORTED, "the mass-preconditioned solves are built for n_q = k+1");
  const long long nel = num_elements(desc);
  const long long nblocks = (long long)desc->n_comp * nel;
  const long long n = nblocks * dofs_per_element(desc);
  const size_t bytes = (size_t)n * sizeof(double);
  ProjPlan PP;
  LaplacePlan LP;
  if (op == DG_OP_PROJECTION) {
    if (desc->n_comp != 3) return fail(DG_ERR_INVALID_ARG, "the projection equation needs n_comp = 3");
    if (!tau_d || !tau_c) return fail(DG_ERR_INVALID_ARG, "tau_d/tau_c is NULL");
    const size_t tb = (size_t)nel * sizeof(double);
    if (overlaps(tau_d, tb, x, bytes) || overlaps(tau_c, tb, x, bytes))
      return fail(DG_ERR_ALIAS, "x overlaps tau_d or tau_c");
    PP = make_proj_plan(desc);
  } else if (op == DG_OP_HELMHOLTZ) {
    if (desc->n_comp != 1 && desc->n_comp != 3) return fail(DG_ERR_INVALID_ARG, "n_comp must be 1 or 3");
    if (!(mass_factor > 0.0) || !std::isfinite(mass_factor))
      return fail(DG_ERR_INVALID_ARG, "mass_factor must be finite and > 0");
    LP = make_laplace_plan(desc, desc->n_comp);
    LP.shift = mass_factor * cell_volume(desc);
  } else {
    return fail(DG_ERR_INVALID_ARG, "op must be DG_OP_HELMHOLTZ or DG_OP_PROJECTION");
  }
  if (overlaps(b, bytes, x, bytes)) return fail(DG_ERR_ALIAS, "x overlaps b");
  hipStream_t s = (hipStream_t)hip_stream;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lock(g_mpcg_mutex);
  MassPcgWs& w = g_mpcg[dev];
  const long long pgrid = pcg_precond_grid(desc->degree, nblocks);
  // workgroups of the operator launch, each writing one partial sum of p.q
  const long long qgrid = op == DG_OP_PROJECTION ? projection_grid(PP) : cg_apply_grid(LP, false);
  if (pgrid <= 0 || pgrid > (1LL << 30) || qgrid <= 0 || qgrid > (1LL << 30))
    return fail(DG_ERR_INVALID_ARG, "mesh too large for the fused steps");
  if ((e = ensure(w, n, std::max(2 * pgrid, qgrid))) != hipSuccess) return hip_fail(e, "work vectors");
  const std::vector<double> Minv = inverse_mass_1d(desc->degree);
  const double ivol = 1.0 / cell_volume(desc);
  auto apply = [&](const double* src, double* dst) {
    return op == DG_OP_PROJECTION ? launch_projection(PP, false, src, dst, tau_d, tau_c, s)
                                  : launch_laplace(LP, false, src, dst, s);
  };
  // q = A p with the partial sums of p.q
  auto apply_dot = [&](const double* src, double* dst, double* partial) {
    return op == DG_OP_PROJECTION ? launch_projection(PP, false, src, dst, tau_d, tau_c, s, partial)
                                  : cg_apply_dot(LP, src, dst, partial, s);
  };
  auto precond = [&](const double* src, double* dst) {
    return launch_inverse_mass(desc->degree, Minv, ivol, nblocks, false, src, dst, s);
  };
#define MPCG_CHECK(call, what)                     \
  do {                                             \
    if ((e = (call)) != hipSuccess) return hip_fail(e, what); \
  } while (0)
  const auto t1 = std::chrono::steady_clock::now();
  int matvec = 0, it = 0;
  // r = b - A x; sums r.r and b.b
  MPCG_CHECK(apply(x, w.q), "operator launch");
  ++matvec;
  MPCG_CHECK(cg_residual(b, w.q, w.r, n, w.partial, s), "residual");
  MPCG_CHECK(read_sums(w, 4, s), "sums");
  const double bb = w.host[3];
  double rr = w.host[1];
  int status = DG_OK;
  if (bb == 0.0) {   // A x = 0 has the solution 0
    MPCG_CHECK(cg_fill(x, 0.0, n, s), "fill");
    rr = 0.0;
  } else if (rr > rtol * rtol * bb) {
    const double tol2 = rtol * rtol * bb;
    MPCG_CHECK(cg_state_init(w.st, tol2, max_iter, 0.0, n, false, s), "state");
    MPCG_CHECK(precond(w.r, w.z), "inverse mass launch");
    MPCG_CHECK(cg_dot(w.r, w.z, n, w.partial, s), "dot");
    MPCG_CHECK(mpcg_start(w.partial, w.st, s), "start");
    MPCG_CHECK(cg_axpb(w.p, w.z, 1.0, 0.0, n, s), "copy");
    int batch = std::max(1, std::min(4, (int)max_iter)), launched = 0;
    double rr_prev = rr;
    for (;;) {
      if (max_iter == 0) {
        status = DG_NOT_CONVERGED;
        break;
      }
      for (int i = 0; i < batch; ++i) {
        MPCG_CHECK(apply_dot(w.p, w.q, w.partial), "operator launch");
        MPCG_CHECK(cg_fin_alpha(w.partial, (int)qgrid, w.st, s), "alpha");
        MPCG_CHECK(launch_pcg_precond(desc->degree, Minv, ivol, nblocks, x, w.r, w.p, w.q, w.z, w.st, w.partial, s),
                   "update and inverse mass");
        MPCG_CHECK(mpcg_beta(w.partial, w.partial + pgrid, (int)pgrid, w.st, s), "beta");
        MPCG_CHECK(mpcg_xpby(w.p, w.z, w.st, n, s), "direction update");
      }
      matvec += batch;
      launched += batch;
      MPCG_CHECK(hipMemcpyAsync(w.host_st, w.st, kStateSize * sizeof(double), hipMemcpyDeviceToHost, s), "state copy");
      MPCG_CHECK(hipStreamSynchronize(s), "state sync");
      it = (int)w.host_st[kIter];
      rr = w.host_st[kRN2];
      if (w.host_st[kDone] != 0.0) {
        const int st_code = (int)w.host_st[kStatus];
        status = st_code == 2 ? DG_ERR_BREAKDOWN : st_code == 1 ? DG_NOT_CONVERGED : DG_OK;
        break;
      }
      // next batch: the iterations the observed contraction rate still needs (1..8)
      const double rho = std::pow(rr / rr_prev, 1.0 / batch);
      int need = 8;
      if (rho > 0.0 && rho < 1.0) need = (int)std::ceil(std::log(tol2 / rr) / std::log(rho));
      batch = std::max(1, std::min(8, std::min(need, max_iter - launched)));
      rr_prev = rr;
    }
  }
  const auto t2 = std::chrono::steady_clock::now();
  if (report) {
    double true_rr = std::nan("");
    if (true_residual) {
      MPCG_CHECK(apply(x, w.q), "operator launch");
      ++matvec;
      MPCG_CHECK(cg_residual(b, w.q, w.z, n, w.partial, s), "residual");
      MPCG_CHECK(read_sums(w, 4, s), "sums");
      true_rr = w.host[1];
    }
    const double bn = std::sqrt(bb);
    report->iterations = it;
    report->matvec_f64 = matvec;
    report->matvec_f32 = 0;
    report->rel_res = bn > 0 ? std::sqrt(rr) / bn : 0.0;
    report->true_rel_res = bn > 0 ? std::sqrt(true_rr) / bn : 0.0;
    report->lambda_max = 0.0;
    report->seconds_solve = std::chrono::duration<double>(t2 - t1).count();
    report->seconds_setup = std::chrono::duration<double>(t1 - t0).count();
  }
#undef MPCG_CHECK
  if (status == DG_ERR_BREAKDOWN) return fail(DG_ERR_BREAKDOWN, "p.Ap <= 0 (operator not SPD?)");
  if (status == DG_NOT_CONVERGED) return fail(DG_NOT_CONVERGED, "max_iter reached");
  return ok();
}

extern "C" int dg_mass_pcg_solve(const dg_op_desc* desc, int32_t op, double mass_factor, const double* tau_d,
                                 const double* tau_c, const double* b, double* x, double rtol, int32_t max_iter,
                                 dg_cg_report* report, void* hip_stream) {
  return dgmf::mass_pcg_solve(desc, op, mass_factor, tau_d, tau_c, b, x, rtol, max_iter, report, hip_stream, true);
}
