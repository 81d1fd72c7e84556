// One V-cycle of geometric multigrid for the SIPG Laplacian (Sec. 3.3: the
// pressure Poisson preconditioner, Chebyshev smoothing of D^-1 A with
// smoothing range 20, a Chebyshev method with a fixed number of steps on the
// coarsest level, matrix-free level transfers), in FP64 or FP32.
//
// Level l is the periodic mesh coarsened l times by two per direction, with
// its own SIPG operator (the Laplace kernels with the level's plan) and
// diagonal.  cycle(l, b):
//   x = Cheb_l(b)                                   pre-smoothing from zero
//   x += P cycle(l+1, R (b - A_l x))                coarse-grid correction
//   x += Cheb_l(b - A_l x)                          post-smoothing
// and on the coarsest level x = Cheb(b) of the coarse degree.  Cheb is the
// zero-start Chebyshev iteration of D^-1 A on [lambda_max/range, lambda_max]
// in its three-term form; its scalars are formed on the host, and its steps
// after the first, like the residuals b - A_l x, run in the epilogue of the
// Laplace apply.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "api_internal.h"
#include "cg_kernels.h"
#include "cg_laplace.h"
#include "dgmf.h"
#include "ops.h"

namespace dgmf {

namespace {

// Device and pinned host buffers of the multigrid calls, kept for reuse: a
// cycle or solve borrows them and hands them back when it returns (both
// calls block until their work is done), so repeated calls on the same
// hierarchy (the pressure solve of every time step) allocate nothing.
struct MgPool {
  std::mutex m;
  std::multimap<std::tuple<int, bool, size_t>, void*> free;   // (device, pinned host, bytes)
};
MgPool& mg_pool() {
  static MgPool pool;
  return pool;
}
hipError_t pool_get(bool host, size_t bytes, void** p, int* dev) {
  hipError_t e = hipGetDevice(dev);
  if (e != hipSuccess) return e;
  {
    MgPool& P = mg_pool();
    std::lock_guard<std::mutex> lk(P.m);
    auto it = P.free.find(std::make_tuple(*dev, host, bytes));
    if (it != P.free.end()) {
      *p = it->second;
      P.free.erase(it);
      return hipSuccess;
    }
  }
  return host ? hipHostMalloc(p, bytes, 0) : hipMalloc(p, bytes);
}
void pool_put(int dev, bool host, size_t bytes, void* p) {
  MgPool& P = mg_pool();
  std::lock_guard<std::mutex> lk(P.m);
  P.free.emplace(std::make_tuple(dev, host, bytes), p);
}

template <typename T>
struct MgLevel {
  dg_op_desc desc{};
  LaplacePlan plan;
  long long n = 0;
  double lmax = 0;
  T *dinv = nullptr, *b = nullptr, *x = nullptr, *t = nullptr, *d = nullptr, *res = nullptr, *e = nullptr;
};

// the cycle's vectors and arithmetic in T (double or float)
template <typename T>
struct MgRun {
  static constexpr bool F32 = sizeof(T) == 4;
  std::vector<MgLevel<T>> lv;
  struct Owned {
    void* p;
    size_t bytes;
    int dev;
    bool host;
  };
  std::vector<Owned> owned;   // borrowed from the pool, handed back at destruction
  int degree = 5, coarse_degree = 10, n3 = 0, k = 0;
  double range = 20.0;
  hipStream_t s = nullptr;
  std::vector<double> P0, P1;
  long long applies = 0;   // level operator applications launched (all levels)

  ~MgRun() {
    for (const Owned& o : owned) pool_put(o.dev, o.host, o.bytes, o.p);
  }
  template <typename U>
  hipError_t alloc(U** p, long long n, bool host = false) {
    int dev = 0;
    const size_t bytes = (size_t)n * sizeof(U);
    hipError_t e = pool_get(host, bytes, (void**)p, &dev);
    if (e == hipSuccess) owned.push_back({(void*)*p, bytes, dev, host});
    return e;
  }

  // 1 / theta of level l's Chebyshev interval [lmax / range, lmax]
  double cheb_scale(const MgLevel<T>& L) const { return 1.0 / (0.5 * (L.lmax + L.lmax / range)); }

  // x = Cheb(b) on level l (deg steps, deg - 1 operator applications);
  // first_done: the first step (d = x = D^-1 b / theta) was taken by the
  // kernel that produced b.  add_to: the last step, where it is a fused
  // step, adds its iterate to add_to instead of storing it (then *added)
  hipError_t cheb(MgLevel<T>& L, const T* b, T* x, int deg, bool first_done = false, T* add_to = nullptr,
                  bool* added = nullptr) {
    if (added) *added = false;
    const double lmin = L.lmax / range;
    const double theta = 0.5 * (L.lmax + lmin), delta = 0.5 * (L.lmax - lmin);
    hipError_t e;
    if (!first_done && (e = mg_cheb_first(b, L.dinv, n3, (T)cheb_scale(L), L.d, x, L.n, s)) != hipSuccess) return e;
    double rho_prev = delta / theta;
    int step = 1;
    if ((deg - 1) % 2 == 1) {
      // an odd number of steps: the first one apart (apply, then the update
      // in place), so that the fused steps, which alternate between x and
      // L.t, end in x
      if ((e = launch_laplace(L.plan, F32, x, L.t, s)) != hipSuccess) return e;
      ++applies;
      const double rho = 1.0 / (2.0 * theta / delta - rho_prev);
      if ((e = mg_cheb_next(b, L.t, L.dinv, n3, (T)(rho * rho_prev), (T)(2.0 * rho / delta), L.d, x, L.n, s)) !=
          hipSuccess)
        return e;
      rho_prev = rho;
      step = 2;
    }
    T *cur = x, *nxt = L.t;
    for (; step < deg; ++step) {
      const double rho = 1.0 / (2.0 * theta / delta - rho_prev);
      if (add_to && step == deg - 1) {
        if ((e = mg_apply_cheb_add<T>(L.plan, cur, b, L.dinv, (T)(rho * rho_prev), (T)(2.0 * rho / delta), L.d, add_to,
                                      s)) != hipSuccess)
          return e;
        ++applies;
        if (added) *added = true;
        return hipSuccess;
      }
      if ((e = mg_apply_cheb<T>(L.plan, cur, b, L.dinv, (T)(rho * rho_prev), (T)(2.0 * rho / delta), L.d, nxt, s)) !=
          hipSuccess)
        return e;
      ++applies;
      std::swap(cur, nxt);
      rho_prev = rho;
    }
    return hipSuccess;
  }

  TransferPlan transfer_plan(int coarse) const {
    TransferPlan TP;
    TP.k = k;
    TP.nxc = lv[coarse].desc.n_el[0];
    TP.nyc = lv[coarse].desc.n_el[1];
    TP.nzc = lv[coarse].desc.n_el[2];
    TP.n_comp = 1;
    TP.P[0] = P0;
    TP.P[1] = P1;
    return TP;
  }

  // lv[l].x = cycle(l, lv[l].b); first_done: see cheb
  hipError_t cycle(int l, bool first_done = false) {
    MgLevel<T>& L = lv[l];
    hipError_t e;
    const bool last = l + 1 == (int)lv.size();
    if ((e = cheb(L, L.b, L.x, last ? coarse_degree : degree, first_done)) != hipSuccess) return e;
    if (last) return hipSuccess;
    if ((e = mg_apply_residual<T>(L.plan, L.x, L.b, L.res, s)) != hipSuccess) return e;
    ++applies;
    const TransferPlan TP = transfer_plan(l + 1);
    MgLevel<T>& Lc = lv[l + 1];
    if ((e = launch_restrict_cheb_first(TP, F32, L.res, Lc.b, Lc.dinv, (double)(T)cheb_scale(Lc), Lc.d, Lc.x, s)) !=
        hipSuccess)
      return e;
    if ((e = cycle(l + 1, true)) != hipSuccess) return e;
    if ((e = launch_prolongate_add(TP, F32, lv[l + 1].x, L.x, s)) != hipSuccess) return e;
    if ((e = mg_apply_residual_cheb_first<T>(L.plan, L.x, L.b, L.dinv, (T)cheb_scale(L), L.res, L.d, L.e, s)) !=
        hipSuccess)
      return e;
    ++applies;
    bool added = false;
    if ((e = cheb(L, L.res, L.e, degree, true, L.x, &added)) != hipSuccess) return e;
    return added ? hipSuccess : mg_add(L.x, L.e, L.n, s);
  }
};

}  // namespace

}  // namespace dgmf

using namespace dgmf;

namespace dgmf {
namespace {

// validation and level set-up shared by the cycle and the solver
// in, out: the caller's finest-level input and output, which must not
// overlap; own_top: the cycle allocates its own finest-level b and x (the
// FP32 cycle inside the FP64 solver, whose in and out are then FP64)
template <typename T>
int mg_setup(MgRun<T>& M, const dg_op_desc* desc, int levels, int degree, double smoothing_range, int coarse_degree,
             const double* lambda_max, hipStream_t s, const void* in, const void* out, bool own_top) {
  int rc = validate_desc(desc);
  if (rc) return rc;
  if (desc->n_comp != 1) return fail(DG_ERR_INVALID_ARG, "the V-cycle needs n_comp = 1");
  if (levels < 1 || levels > 10) return fail(DG_ERR_INVALID_ARG, "levels must be 1..10");
  if (degree < 1 || coarse_degree < 1) return fail(DG_ERR_INVALID_ARG, "smoother degrees must be >= 1");
  if (!(smoothing_range > 1.0) || !std::isfinite(smoothing_range))
    return fail(DG_ERR_INVALID_ARG, "smoothing_range must be finite and > 1");
  if (desc->n_q != 0 && desc->n_q < desc->degree + 1)
    return fail(DG_ERR_UNSUPPORTED, "the Laplace form needs n_q >= k+1 (exact Gauss integration)");
  if (lambda_max)
    for (int l = 0; l < levels; ++l)
      if (!(lambda_max[l] > 0.0) || !std::isfinite(lambda_max[l]))
        return fail(DG_ERR_INVALID_ARG, "lambda_max must be finite and > 0 on every level");
  for (int d = 0; d < 3; ++d)
    if (desc->n_el[d] % (1 << (levels - 1)) != 0)
      return fail(DG_ERR_INVALID_ARG, "element counts must be divisible by 2^(levels-1)");
  const size_t bytes = (size_t)num_elements(desc) * dofs_per_element(desc) * (own_top ? sizeof(double) : sizeof(T));
  if (overlaps(in, bytes, out, bytes)) return fail(DG_ERR_ALIAS, "the output overlaps the input");
  M.k = desc->degree;
  M.n3 = (int)dofs_per_element(desc);
  M.degree = degree;
  M.coarse_degree = coarse_degree;
  M.range = smoothing_range;
  M.s = s;
  M.P0 = child_interp(M.k, 0);
  M.P1 = child_interp(M.k, 1);
  M.lv.resize(levels);
  hipError_t e;
  std::vector<double> diag(M.n3);
  std::vector<T> dinv(M.n3);
  for (int l = 0; l < levels; ++l) {
    MgLevel<T>& L = M.lv[l];
    L.desc = *desc;
    for (int d = 0; d < 3; ++d) L.desc.n_el[d] = desc->n_el[d] >> l;
    L.plan = make_laplace_plan(&L.desc, 1);
    L.n = num_elements(&L.desc) * M.n3;
    if (lambda_max) {
      L.lmax = lambda_max[l];
    } else if ((rc = laplace_lambda_max(&L.desc, true, M.s, &L.lmax)) != DG_OK) {
      return rc;   // the level's bound: the estimate of the Chebyshev-preconditioned CG
    }
    if ((rc = dg_laplace_diagonal(&L.desc, diag.data())) != DG_OK) return rc;
    for (int i = 0; i < M.n3; ++i) dinv[i] = (T)(1.0 / diag[i]);
    if ((e = M.alloc(&L.dinv, M.n3)) != hipSuccess) return hip_fail(e, "V-cycle tables");
    if ((e = hipMemcpyAsync(L.dinv, dinv.data(), M.n3 * sizeof(T), hipMemcpyHostToDevice, M.s)) != hipSuccess)
      return hip_fail(e, "V-cycle tables");
    if ((e = hipStreamSynchronize(M.s)) != hipSuccess) return hip_fail(e, "V-cycle tables");
    T** bufs[5] = {&L.t, &L.d, &L.res, &L.e, &L.b};
    const bool top = l > 0 || own_top;
    for (int i = 0; i < (top ? 5 : 4); ++i)
      if ((e = M.alloc(bufs[i], L.n)) != hipSuccess) return hip_fail(e, "V-cycle work vectors");
    if (top && (e = M.alloc(&L.x, L.n)) != hipSuccess) return hip_fail(e, "V-cycle work vectors");
  }
  return DG_OK;
}

}  // namespace
}  // namespace dgmf

namespace {

template <typename T>
int vcycle_once(const dg_op_desc* desc, int levels, int degree, double smoothing_range, int coarse_degree,
                const double* lambda_max, const void* r, void* z, void* hip_stream) {
  // every argument is checked before the set-up allocates anything
  MgRun<T> M;
  int rc = mg_setup(M, desc, levels, degree, smoothing_range, coarse_degree, lambda_max, (hipStream_t)hip_stream, r,
                    z, false);
  if (rc) return rc;
  M.lv[0].b = const_cast<T*>(static_cast<const T*>(r));   // read only
  M.lv[0].x = static_cast<T*>(z);
  hipError_t e;
  if ((e = M.cycle(0)) != hipSuccess) return hip_fail(e, "V-cycle launch");
  if ((e = hipStreamSynchronize(M.s)) != hipSuccess) return hip_fail(e, "V-cycle");
  return ok();
}

}  // namespace

extern "C" int dg_gmg_vcycle(const dg_op_desc* desc, int32_t levels, int32_t degree, double smoothing_range,
                             int32_t coarse_degree, const double* lambda_max, int32_t dtype, const void* r, void* z,
                             void* hip_stream) {
  if (!r || !z) return fail(DG_ERR_INVALID_ARG, "r/z is NULL");
  int rc = validate_desc(desc);
  if (rc) return rc;
  if (dtype == DG_F64)
    return vcycle_once<double>(desc, levels, degree, smoothing_range, coarse_degree, lambda_max, r, z, hip_stream);
  if (dtype == DG_F32)
    return vcycle_once<float>(desc, levels, degree, smoothing_range, coarse_degree, lambda_max, r, z, hip_stream);
  return fail(DG_ERR_INVALID_ARG, "dtype must be DG_F64 or DG_F32");
}

namespace dgmf {
namespace {

// FP64 CG preconditioned by one V-cycle per iteration, for the periodic
// pressure Poisson equation (Sec. 3.3): residual and preconditioned residual
// kept at zero coefficient mean, flexible (Polak-Ribiere) beta as in the
// Chebyshev-preconditioned CG.  The cycle runs in T: with T = float the
// residual r' = r - mean is rounded to FP32 on the way in and the cycle's
// output enters the FP64 direction update directly, the outer iteration
// staying FP64 (the mixed-precision split of Sec. 3.3).  The iteration
// scalars stay on the device (the state array and kernels of the CG loop):
// the host enqueues a batch of iterations and reads the state once per
// batch; iterations queued after convergence leave x and r unchanged.  The
// level vectors are set up once per solve.
template <typename T>
int gmg_cg(const dg_op_desc* desc, int32_t levels, int degree, double smoothing_range, int coarse_degree,
           const double* lambda_max, const double* b, double* x, double rtol, double atol, int32_t max_iter,
           dg_cg_report* report, void* hip_stream, bool true_residual) {
  const auto t0 = std::chrono::steady_clock::now();
  MgRun<T> M;
  int rc = mg_setup(M, desc, levels, degree, smoothing_range, coarse_degree, lambda_max, (hipStream_t)hip_stream, b,
                    x, MgRun<T>::F32);
  if (rc) return rc;
  const long long n = M.lv[0].n;
  hipStream_t s = M.s;
  hipError_t e;
  const LaplacePlan& A = M.lv[0].plan;
  const long grid64 = cg_apply_grid(A, false);
  double *r, *p, *q, *partial, *res, *st, *host;
  T *rin, *zb[2];
#define GMG_CHECK(call, what)                                 \
  do {                                                        \
    if ((e = (call)) != hipSuccess) return hip_fail(e, what); \
  } while (0)
  GMG_CHECK(M.alloc(&r, n), "work vectors");
  GMG_CHECK(M.alloc(&p, n), "work vectors");
  GMG_CHECK(M.alloc(&q, n), "work vectors");
  GMG_CHECK(M.alloc(&zb[0], n), "work vectors");
  GMG_CHECK(M.alloc(&zb[1], n), "work vectors");
  if constexpr (MgRun<T>::F32) {
    rin = M.lv[0].b;   // the level's own FP32 input vector
  } else {
    GMG_CHECK(M.alloc(&rin, n), "work vectors");
  }
  GMG_CHECK(M.alloc(&partial, std::max<long long>(4LL * kCgBlocks, (long long)grid64)), "work vectors");
  GMG_CHECK(M.alloc(&res, 4), "work vectors");
  GMG_CHECK(M.alloc(&st, kStateSize), "work vectors");
  GMG_CHECK(M.alloc(&host, kStateSize, true), "pinned results");
  auto sums = [&](int nq) -> hipError_t {
    hipError_t er;
    if ((er = cg_finalize(partial, nq, res, s)) != hipSuccess) return er;
    if ((er = hipMemcpyAsync(host, res, nq * sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess) return er;
    return hipStreamSynchronize(s);
  };
  const double dn = (double)n;
  const auto t1 = std::chrono::steady_clock::now();
  long long matvec = 0;
  int it = 0, status = DG_OK;
  double rr = 0.0;
  GMG_CHECK(launch_laplace(A, false, x, q, s), "operator launch");
  ++matvec;
  GMG_CHECK(cg_residual(b, q, r, n, partial, s), "residual");
  GMG_CHECK(sums(4), "sums");
  const double bb = host[3] - host[2] * host[2] / dn;   // |b - mean(b)|^2
  const double tol = std::max(rtol * std::sqrt(std::max(bb, 0.0)), atol);
  const double tol2 = tol * tol;
  // z = V r' with the sums of the flexible beta, then the direction update;
  // zb[zn] receives the new output, zb[1 - zn] holds the previous one
  int zn = 0;
  auto precondition = [&](bool start) -> hipError_t {
    hipError_t er;
    if ((er = cg_fin_resid(partial, st, start, s)) != hipSuccess) return er;
    if ((er = cg_rprime(r, st, rin, n, s)) != hipSuccess) return er;
    M.lv[0].b = rin;
    M.lv[0].x = zb[zn];
    if ((er = M.cycle(0)) != hipSuccess) return er;
    if ((er = cg_zsums(r, zb[zn], zb[1 - zn], st, n, partial, s)) != hipSuccess) return er;
    if ((er = cg_fin_cheb(partial, kCgBlocks, st, start, s)) != hipSuccess) return er;
    if ((er = cg_update_p_z(zb[zn], p, st, n, s)) != hipSuccess) return er;
    zn = 1 - zn;
    return hipSuccess;
  };
  if (bb > 0.0) {
    GMG_CHECK(cg_state_init(st, tol2, max_iter, 0.0, n, true, s), "state");
    GMG_CHECK(cg_fill(p, 0.0, n, s), "fill");
    if constexpr (MgRun<T>::F32) {
      GMG_CHECK(mg_convert(p, zb[1], n, s), "fill");   // zeros
    } else {
      GMG_CHECK(cg_fill(zb[1], 0.0, n, s), "fill");
    }
    // start: alpha is 0 in the fresh state, so this only forms the sums of r0
    GMG_CHECK(cg_update_xr_st(x, r, p, q, nullptr, M.n3, st, false, n, partial, s), "update");
    GMG_CHECK(precondition(true), "V-cycle");
    // batch size: up to 4, fewer when the observed contraction rate says the
    // tolerance is that close (keeps queued no-op iterations rare)
    constexpr int max_batch = 4;
    long long queued = 0;
    double rn2_prev = -1, it_prev = 0;
    for (;;) {
      GMG_CHECK(hipMemcpyAsync(host, st, kStateSize * sizeof(double), hipMemcpyDeviceToHost, s), "CG state");
      GMG_CHECK(hipStreamSynchronize(s), "CG state");
      if (host[kDone] != 0.0 || queued > (long long)max_iter + max_batch) break;
      int batch = max_batch;
      if (rn2_prev > 0 && host[kRN2] > 0 && host[kRN2] < rn2_prev && host[kIter] > it_prev) {
        const double rate = std::log(host[kRN2] / rn2_prev) / (host[kIter] - it_prev);   // per iteration, < 0
        const double left = std::log(host[kTol2] / host[kRN2]) / rate;
        if (std::isfinite(left)) batch = (int)std::max(1.0, std::min((double)max_batch, std::ceil(left)));
      }
      rn2_prev = host[kRN2];
      it_prev = host[kIter];
      for (int b2 = 0; b2 < batch; ++b2) {
        // q = A p with the p.q partials, alpha, x/r update with the sums of r
        ++matvec;
        GMG_CHECK(cg_apply_dot(A, p, q, partial, s), "operator launch");
        GMG_CHECK(cg_fin_alpha(partial, (int)grid64, st, s), "alpha");
        GMG_CHECK(cg_update_xr_st(x, r, p, q, nullptr, M.n3, st, false, n, partial, s), "update");
        GMG_CHECK(precondition(false), "V-cycle");
      }
      queued += batch;
    }
    it = (int)host[kIter];
    rr = host[kRN2];
    if (host[kStatus] == 2.0) status = DG_ERR_BREAKDOWN;
    else if (host[kStatus] == 1.0 || host[kDone] == 0.0) status = DG_NOT_CONVERGED;
  } else if (bb == 0.0) {
    GMG_CHECK(cg_fill(x, 0.0, n, s), "fill");
  }
  GMG_CHECK(hipStreamSynchronize(s), "solve");
  const auto t2 = std::chrono::steady_clock::now();
  if (report) {
    double true_rr = std::nan("");
    if (true_residual) {
      GMG_CHECK(launch_laplace(A, false, x, q, s), "operator launch");
      ++matvec;
      GMG_CHECK(cg_residual(b, q, r, n, partial, s), "residual");
      GMG_CHECK(sums(4), "sums");
      true_rr = host[1] - host[0] * host[0] / dn;
    }
    const double bn = std::sqrt(bb);
    report->iterations = it;
    // outer FP64 applies (queued no-op iterations included) plus every level
    // apply of the cycles, by precision
    report->matvec_f64 = (int)matvec + (MgRun<T>::F32 ? 0 : (int)M.applies);
    report->matvec_f32 = MgRun<T>::F32 ? (int)M.applies : 0;
    report->rel_res = bn > 0 ? std::sqrt(std::max(rr, 0.0)) / bn : 0.0;
    report->true_rel_res = !true_residual ? std::nan("") : bn > 0 ? std::sqrt(std::max(true_rr, 0.0)) / bn : 0.0;
    report->lambda_max = M.lv[0].lmax;
    report->seconds_solve = std::chrono::duration<double>(t2 - t1).count();
    report->seconds_setup = std::chrono::duration<double>(t1 - t0).count();
  }
#undef GMG_CHECK
  if (status == DG_ERR_BREAKDOWN) return fail(DG_ERR_BREAKDOWN, "p.Ap <= 0 or a non-finite residual");
  if (status == DG_NOT_CONVERGED) return fail(DG_NOT_CONVERGED, "max_iter reached");
  return ok();
}

}  // namespace

int gmg_cg_solve(const dg_op_desc* desc, int levels, int degree, double smoothing_range, int coarse_degree,
                 const double* lambda_max, int cycle_dtype, const double* b, double* x, double rtol, double atol,
                 int max_iter, dg_cg_report* report, void* hip_stream, bool true_residual) {
  if (!b || !x) return fail(DG_ERR_INVALID_ARG, "b/x is NULL");
  if (!(rtol > 0.0) || !std::isfinite(rtol)) return fail(DG_ERR_INVALID_ARG, "rtol must be finite and > 0");
  if (!(atol >= 0.0) || !std::isfinite(atol)) return fail(DG_ERR_INVALID_ARG, "atol must be finite and >= 0");
  if (max_iter < 0) return fail(DG_ERR_INVALID_ARG, "max_iter must be >= 0");
  if (cycle_dtype == DG_F64)
    return gmg_cg<double>(desc, levels, degree, smoothing_range, coarse_degree, lambda_max, b, x, rtol, atol,
                          max_iter, report, hip_stream, true_residual);
  if (cycle_dtype == DG_F32)
    return gmg_cg<float>(desc, levels, degree, smoothing_range, coarse_degree, lambda_max, b, x, rtol, atol,
                         max_iter, report, hip_stream, true_residual);
  return fail(DG_ERR_INVALID_ARG, "cycle_dtype must be DG_F64 or DG_F32");
}

}  // namespace dgmf

extern "C" int dg_gmg_cg_solve(const dg_op_desc* desc, int32_t levels, int32_t degree, double smoothing_range,
                               int32_t coarse_degree, const double* lambda_max, int32_t cycle_dtype, const double* b,
                               double* x, double rtol, int32_t max_iter, dg_cg_report* report, void* hip_stream) {
  return dgmf::gmg_cg_solve(desc, levels, degree, smoothing_range, coarse_degree, lambda_max, cycle_dtype, b, x, rtol,
                            0.0, max_iter, report, hip_stream);
}
