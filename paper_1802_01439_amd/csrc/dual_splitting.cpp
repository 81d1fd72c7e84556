// One time step of the dual splitting scheme (Sec. 3.1, matrix form of
// Sec. 3.3) for the incompressible Navier-Stokes equations on a periodic
// Cartesian mesh, in double precision on the GPU, host orchestration of the
// library's operators and solvers:
//
//   1. convective step   U^ = (sum_i alpha_i U^{n-i} - dt M^-1 sum_i beta_i C(U^{n-i})) / gamma_0
//   2. pressure step     L P = -(gamma_0/dt) D U^   (degree k-1: FP64 CG with the FP32 V-cycle
//                                                    or FP32 Chebyshev preconditioner, zero-mean
//                                                    iterates)
//   3. projection step   (M + A_D + A_C) U^^ = M U^ - (dt/gamma_0) G P   (inverse-mass PCG)
//   4. viscous step      (gamma_0/dt M + nu L) U^{n+1} = (gamma_0/dt) M U^^   (inverse-mass PCG)
//
// with BDF1 (gamma_0 = 1, alpha = 1, beta = 1; the start-up step) or BDF2
// (gamma_0 = 3/2, alpha = (2, -1/2), extrapolation beta = (2, -1)), the
// penalty parameters tau_D, tau_C of A_D, A_C from the extrapolated velocity
// sum_i beta_i U^{n-i} (Sec. 3.2), D and G the mixed-order divergence and
// gradient (velocity degree k, pressure k-1), and the diagnostics e_k, eps of
// U^{n+1} (Sec. 4.2).  Also the C entry points of the mixed-order operators
// and of the diagnostics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>
#include <mutex>

#include "api_internal.h"
#include "dgmf.h"
#include "ops.h"

namespace dgmf {

namespace {

struct StepWs {
  long long nu3 = 0, np = 0, nel = 0;
  double* v[5] = {};        // velocity-sized work vectors
  double* bp = nullptr;     // pressure right-hand side
  double* tau = nullptr;    // tau_D (nel), tau_C (nel)
  double* partial = nullptr;   // 2 nel
  double* out2 = nullptr;      // 2
};

std::mutex g_step_mutex;
std::map<int, StepWs> g_step;

hipError_t step_ensure(StepWs& w, long long nu3, long long np, long long nel) {
  hipError_t e;
  if (w.nu3 < nu3) {
    for (double*& p : w.v) {
      if (p) (void)hipFree(p);
      p = nullptr;
    }
    w.nu3 = 0;
    for (double*& p : w.v)
      if ((e = hipMalloc((void**)&p, (size_t)nu3 * 8)) != hipSuccess) return e;
    w.nu3 = nu3;
  }
  if (w.np < np) {
    if (w.bp) (void)hipFree(w.bp);
    w.bp = nullptr;
    w.np = 0;
    if ((e = hipMalloc((void**)&w.bp, (size_t)np * 8)) != hipSuccess) return e;
    w.np = np;
  }
  if (w.nel < nel) {
    double** pp[] = {&w.tau, &w.partial};
    for (double** p : pp) {
      if (*p) (void)hipFree(*p);
      *p = nullptr;
    }
    w.nel = 0;
    for (double** p : pp)
      if ((e = hipMalloc((void**)p, (size_t)(2 * nel) * 8)) != hipSuccess) return e;
    w.nel = nel;
  }
  if (!w.out2 && (e = hipMalloc((void**)&w.out2, 2 * 8)) != hipSuccess) return e;
  return hipSuccess;
}

int validate_mixed(const dg_op_desc* d) {
  int rc = validate_desc(d);
  if (rc) return rc;
  if (d->degree < 2) return fail(DG_ERR_UNSUPPORTED, "the mixed-order pair needs velocity degree k >= 2");
  if (d->n_q != 0 && d->n_q != d->degree + 1)
    return fail(DG_ERR_UNSUPPORTED, "the mixed-order operators are built for n_q = k+1");
  return DG_OK;
}

// (e_k, eps) of u on the host (synchronises the stream)
int diagnostics(const dg_op_desc* d, const double* u, double nu, StepWs& W, hipStream_t s, double* out) {
  double h[3], ih[3], vol = 1.0;
  for (int i = 0; i < 3; ++i) {
    h[i] = d->length[i] / d->n_el[i];
    ih[i] = 1.0 / h[i];
    vol *= h[i];
  }
  hipError_t e = launch_diagnostics(d->degree, mesh_args(d), u, W.partial, W.out2, vol, ih, s);
  if (e != hipSuccess) return hip_fail(e, "diagnostics kernel launch");
  double r[2];
  if ((e = hipMemcpyAsync(r, W.out2, sizeof(r), hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return hip_fail(e, "diagnostics read-back");
  const double V = vol * (double)num_elements(d);
  out[0] = 0.5 * r[0] / V;
  out[1] = nu * r[1] / V;
  return DG_OK;
}

}  // namespace

}  // namespace dgmf

using namespace dgmf;

extern "C" int dg_apply_divergence_mixed(const dg_op_desc* desc, dg_dtype dtype, const void* u, void* b,
                                         void* hip_stream) {
  int rc = validate_mixed(desc);
  if (rc) return rc;
  if (dtype != DG_F64 && dtype != DG_F32) return fail(DG_ERR_INVALID_ARG, "dtype must be DG_F64 or DG_F32");
  if (!u || !b) return fail(DG_ERR_INVALID_ARG, "u/b is NULL");
  const size_t es = dtype == DG_F64 ? 8 : 4;
  const long long nel = num_elements(desc), k = desc->degree;
  if (overlaps(u, (size_t)(3 * nel * (k + 1) * (k + 1) * (k + 1)) * es, b, (size_t)(nel * k * k * k) * es))
    return fail(DG_ERR_ALIAS, "b overlaps u");
  const DivPlan P = make_div_plan(desc);
  hipError_t e = launch_mixed(P, false, dtype == DG_F32, u, b, 1.0, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "mixed divergence kernel launch");
  return ok();
}

extern "C" int dg_apply_gradient_mixed(const dg_op_desc* desc, dg_dtype dtype, const void* p, void* y,
                                       void* hip_stream) {
  int rc = validate_mixed(desc);
  if (rc) return rc;
  if (dtype != DG_F64 && dtype != DG_F32) return fail(DG_ERR_INVALID_ARG, "dtype must be DG_F64 or DG_F32");
  if (!p || !y) return fail(DG_ERR_INVALID_ARG, "p/y is NULL");
  const size_t es = dtype == DG_F64 ? 8 : 4;
  const long long nel = num_elements(desc), k = desc->degree;
  if (overlaps(p, (size_t)(nel * k * k * k) * es, y, (size_t)(3 * nel * (k + 1) * (k + 1) * (k + 1)) * es))
    return fail(DG_ERR_ALIAS, "y overlaps p");
  const DivPlan P = make_div_plan(desc);
  hipError_t e = launch_mixed(P, true, dtype == DG_F32, p, y, 1.0, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "mixed gradient kernel launch");
  return ok();
}

extern "C" int dg_tgv_diagnostics(const dg_op_desc* desc, const double* u, double nu, double* out,
                                  void* hip_stream) {
  int rc = validate_desc(desc);
  if (rc) return rc;
  if (!u || !out) return fail(DG_ERR_INVALID_ARG, "u/out is NULL");
  if (!std::isfinite(nu)) return fail(DG_ERR_INVALID_ARG, "nu must be finite");
  std::lock_guard<std::mutex> lock(g_step_mutex);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  StepWs& W = g_step[dev];
  const long long nel = num_elements(desc);
  if ((e = step_ensure(W, 0, 0, nel)) != hipSuccess) return hip_fail(e, "diagnostics workspace");
  rc = diagnostics(desc, u, nu, W, (hipStream_t)hip_stream, out);
  return rc ? rc : ok();
}

namespace {

// The step of dg_dual_splitting_step; conv_nm1 (order 2, optional): C(u_nm1)
// kept from the previous step, conv_n (optional): C(u_n) for the next one.
int dual_splitting_step(const dg_op_desc* desc, const dg_step_opts* opts, const double* u_n, const double* u_nm1,
                        const double* conv_nm1, double* conv_n, double* u_np1, double* p, dg_step_report* report,
                        void* hip_stream) {
  const auto t0 = std::chrono::steady_clock::now();
  int rc = validate_mixed(desc);
  if (rc) return rc;
  if (!opts) return fail(DG_ERR_INVALID_ARG, "opts is NULL");
  if (opts->order != 1 && opts->order != 2) return fail(DG_ERR_INVALID_ARG, "order must be 1 or 2");
  if (!(opts->dt > 0) || !std::isfinite(opts->dt) || !(opts->nu >= 0) || !std::isfinite(opts->nu))
    return fail(DG_ERR_INVALID_ARG, "dt must be finite and > 0, nu finite and >= 0");
  if (!(opts->zeta_d >= 0) || !(opts->zeta_c >= 0) || !std::isfinite(opts->zeta_d) || !std::isfinite(opts->zeta_c))
    return fail(DG_ERR_INVALID_ARG, "zeta_d and zeta_c must be finite and >= 0");
  for (double r : {opts->rtol_pressure, opts->rtol_projection, opts->rtol_viscous})
    if (!(r > 0) || !std::isfinite(r)) return fail(DG_ERR_INVALID_ARG, "tolerances must be finite and > 0");
  if (!(opts->atol_pressure >= 0) || !std::isfinite(opts->atol_pressure))
    return fail(DG_ERR_INVALID_ARG, "atol_pressure must be finite and >= 0");
  if (opts->max_iter < 1) return fail(DG_ERR_INVALID_ARG, "max_iter must be >= 1");
  if (opts->pressure_precond != DG_STEP_PC_CHEB_F32 && opts->pressure_precond != DG_STEP_PC_GMG_F32)
    return fail(DG_ERR_INVALID_ARG, "pressure_precond must be DG_STEP_PC_CHEB_F32 or DG_STEP_PC_GMG_F32");
  if (!u_n || !u_np1 || !p || (opts->order == 2 && !u_nm1))
    return fail(DG_ERR_INVALID_ARG, "u_n, u_np1, p (and u_nm1 for order 2) must not be NULL");
  const int k = desc->degree;
  const long long nel = num_elements(desc);
  const long long nu3 = 3 * nel * (long long)(k + 1) * (k + 1) * (k + 1);
  const long long np = nel * (long long)k * k * k;
  const size_t ub = (size_t)nu3 * 8, pb = (size_t)np * 8;
  if (overlaps(u_np1, ub, u_n, ub) || (u_nm1 && overlaps(u_np1, ub, u_nm1, ub)) || overlaps(p, pb, u_np1, ub) ||
      overlaps(p, pb, u_n, ub) || (u_nm1 && overlaps(p, pb, u_nm1, ub)))
    return fail(DG_ERR_ALIAS, "u_np1 and p must not overlap each other or the inputs");
  if (opts->order == 1) conv_nm1 = nullptr;
  for (const double* c : {(const double*)conv_n, conv_nm1}) {
    if (!c) continue;
    if (overlaps(c, ub, u_n, ub) || (u_nm1 && overlaps(c, ub, u_nm1, ub)) || overlaps(c, ub, u_np1, ub) ||
        overlaps(c, ub, p, pb))
      return fail(DG_ERR_ALIAS, "conv_n and conv_nm1 must not overlap the velocities or p");
  }
  if (conv_n && conv_nm1 && overlaps(conv_n, ub, conv_nm1, ub))
    return fail(DG_ERR_ALIAS, "conv_n must not overlap conv_nm1");
  if (report) *report = dg_step_report{};

  const double dt = opts->dt, nu = opts->nu;
  const bool bdf2 = opts->order == 2;
  const double g0 = bdf2 ? 1.5 : 1.0, a0 = bdf2 ? 2.0 : 1.0, a1 = bdf2 ? -0.5 : 0.0;
  const double b0 = bdf2 ? 2.0 : 1.0, b1 = bdf2 ? -1.0 : 0.0;
  hipStream_t s = (hipStream_t)hip_stream;

  std::lock_guard<std::mutex> lock(g_step_mutex);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  StepWs& W = g_step[dev];
  if ((e = step_ensure(W, nu3, np, nel)) != hipSuccess) return hip_fail(e, "step workspace allocation");
  double *C = W.v[0], *C2 = W.v[1], *gp = W.v[2], *rhs3 = W.v[3], *rhs4 = W.v[4];
  // U^, U^^ and U^{n+1} are formed in u_np1 itself: each solve starts in
  // place from the previous substep's velocity, its initial guess
  double* const uhat = u_np1;

  // descriptors: velocity (3 components), pressure (degree k-1)
  dg_op_desc dv = *desc;
  dv.n_comp = 3;
  dv.scale = 1.0;
  dv.n_q = 0;
  dg_op_desc dc = dv;   // convective: its own 3/2-rule quadrature
  dc.n_q = 0;
  dg_op_desc dp = *desc;
  dp.degree = k - 1;
  dp.n_comp = 1;
  dp.scale = 1.0;
  dp.n_q = 0;
  auto step_fail = [&](int code, const char* what) {
    return code < 0 ? code : fail(code, std::string(what) + " did not converge");
  };

  // 1. convective step: C(u_n) into conv_n where the caller keeps it, C(u_nm1)
  // from conv_nm1 where the caller kept it; the BDF combination, the inverse
  // mass and U^ in one pass
  double* const cn = conv_n ? conv_n : C;
  if ((rc = dg_apply_convective(&dc, DG_F64, u_n, cn, s))) return rc;
  if (bdf2) {
    const double* cm = conv_nm1;
    if (!cm) {
      if ((rc = dg_apply_convective(&dc, DG_F64, u_nm1, C2, s))) return rc;
      cm = C2;
    }
    if ((e = launch_convective_substep(k, inverse_mass_1d(k), 1.0 / cell_volume(&dv), 3 * nel, cn, cm, b0, b1, u_n,
                                       u_nm1, a0 / g0, a1 / g0, -dt / g0, uhat, s)) != hipSuccess)
      return hip_fail(e, "convective substep");
  } else {
    if ((e = launch_convective_substep(k, inverse_mass_1d(k), 1.0 / cell_volume(&dv), 3 * nel, cn, nullptr, b0, b1,
                                       u_n, nullptr, a0 / g0, a1 / g0, -dt / g0, uhat, s)) != hipSuccess)
      return hip_fail(e, "convective substep");
  }
  // 2. pressure step: L P = -(gamma_0/dt) D U^
  const DivPlan DP = make_div_plan(&dv);
  if ((e = launch_mixed(DP, false, false, uhat, W.bp, -g0 / dt, s)) != hipSuccess)
    return hip_fail(e, "mixed divergence kernel launch");
  dg_cg_report cr{};
  if (opts->pressure_precond == DG_STEP_PC_GMG_F32) {
    // as many levels as the element counts allow: all halved while even with
    // halves of at least 2, at most 5 levels
    int levels = 1;
    while (levels < 5) {
      bool ok = true;
      for (int d = 0; d < 3; ++d) {
        const int m = dp.n_el[d] >> (levels - 1);
        ok = ok && m % 2 == 0 && m / 2 >= 2;
      }
      if (!ok) break;
      ++levels;
    }
    rc = gmg_cg_solve(&dp, levels, 5, 20.0, 10, nullptr, DG_F32, W.bp, p, opts->rtol_pressure, opts->atol_pressure,
                      opts->max_iter, &cr, hip_stream, false);
  } else {
    dg_cg_opts co{};
    co.precond = DG_PC_CHEB_F32;
    co.cheb_degree = 5;
    co.cheb_range = 20.0;
    co.rtol = opts->rtol_pressure;
    co.atol = opts->atol_pressure;
    co.max_iter = opts->max_iter;
    co.project_mean = 1;
    rc = dg_cg_solve(&dp, &co, W.bp, p, &cr, hip_stream);
  }
  if (rc) return step_fail(rc, "pressure CG");
  // 3. projection step: penalties from the extrapolated velocity
  const double* uex = u_n;
  if (bdf2) {
    if ((e = launch_lincomb(C2, u_n, u_nm1, nullptr, b0, b1, 0.0, nu3, s)) != hipSuccess)
      return hip_fail(e, "lincomb");
    uex = C2;
  }
  double vol = 1.0;
  for (int i = 0; i < 3; ++i) vol *= desc->length[i] / desc->n_el[i];
  const double hh = std::cbrt(vol);
  if ((e = launch_penalty(k, mesh_args(desc), uex, W.tau, W.tau + nel, opts->zeta_d * hh / (k + 1) * dt,
                          opts->zeta_c * dt, s)) != hipSuccess)
    return hip_fail(e, "penalty kernel launch");
  // mass applies: vol (M1 (x) M1 (x) M1) per element, the structure of the
  // inverse mass with the 1D mass matrix (a third of the time of the
  // Helmholtz kernel with a zero Laplace part)
  const std::vector<double>& M1 = basis(k, k + 1).Mref;
  if ((e = launch_inverse_mass(k, M1, vol, 3 * nel, false, uhat, rhs3, s)) != hipSuccess)   // M U^
    return hip_fail(e, "mass apply");
  if ((e = launch_mixed(DP, true, false, p, gp, 1.0, s)) != hipSuccess)
    return hip_fail(e, "mixed gradient kernel launch");
  if ((e = launch_lincomb(rhs3, rhs3, gp, nullptr, 1.0, -dt / g0, 0.0, nu3, s)) != hipSuccess)
    return hip_fail(e, "lincomb");
  dg_cg_report pr{};
  rc = mass_pcg_solve(&dv, DG_OP_PROJECTION, 0.0, W.tau, W.tau + nel, rhs3, u_np1, opts->rtol_projection,
                      opts->max_iter, &pr, hip_stream, false);
  if (rc) return step_fail(rc, "projection CG");
  // 4. viscous step
  if ((e = launch_inverse_mass(k, M1, vol * (g0 / dt), 3 * nel, false, u_np1, rhs4, s)) != hipSuccess)
    return hip_fail(e, "mass apply");
  dg_op_desc dvv = dv;
  dvv.scale = nu;
  dg_cg_report vr{};
  rc = mass_pcg_solve(&dvv, DG_OP_HELMHOLTZ, g0 / dt, nullptr, nullptr, rhs4, u_np1, opts->rtol_viscous,
                      opts->max_iter, &vr, hip_stream, false);
  if (rc) return step_fail(rc, "viscous CG");
  if (report) {
    double d2[2] = {0, 0};
    if ((rc = diagnostics(desc, u_np1, nu, W, s, d2))) return rc;
    report->it_pressure = cr.iterations;
    report->it_projection = pr.iterations;
    report->it_viscous = vr.iterations;
    report->kinetic_energy = d2[0];
    report->dissipation = d2[1];
  }
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "step");
  if (report) report->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return ok();
}

}  // namespace

extern "C" int dg_dual_splitting_step(const dg_op_desc* desc, const dg_step_opts* opts, const double* u_n,
                                      const double* u_nm1, double* u_np1, double* p, dg_step_report* report,
                                      void* hip_stream) {
  return dual_splitting_step(desc, opts, u_n, u_nm1, nullptr, nullptr, u_np1, p, report, hip_stream);
}

extern "C" int dg_dual_splitting_step_conv(const dg_op_desc* desc, const dg_step_opts* opts, const double* u_n,
                                           const double* u_nm1, const double* conv_nm1, double* conv_n,
                                           double* u_np1, double* p, dg_step_report* report, void* hip_stream) {
  return dual_splitting_step(desc, opts, u_n, u_nm1, conv_nm1, conv_n, u_np1, p, report, hip_stream);
}
