// Vector kernels of the CG solver (launch wrappers).  Reductions write
// kCgBlocks partials per quantity; cg_finalize sums them in a fixed order.
#pragma once

#include <hip/hip_runtime.h>

namespace dgmf {

constexpr int kCgThreads = 256;
constexpr int kCgBlocks = 1024;

// Device-side state of the main CG loop (doubles).
enum : int {
  kRZ = 0,      // r'.z' of the current residual
  kAlpha,       // step length of the current iteration
  kBeta,        // direction update coefficient
  kMuR,         // mean of r (0 without projection)
  kMuZ,         // mean of D^-1 r' or of the Chebyshev output
  kRN2,         // |r'|^2
  kDone,        // 1: converged, broken down or out of iterations
  kStatus,      // 0 ok, 1 max_iter reached, 2 breakdown
  kIter,        // iterations done
  kTol2,        // stopping threshold on |r'|^2
  kMaxIt,       // iteration limit
  kSumD,        // sum of D^-1 over all DoFs
  kN,           // number of DoFs
  kProj,        // 1: project on zero coefficient mean
  kPQ,          // p.Ap of the current iteration
  kSumRp,       // sum r' (0 with projection)
  kStateSize
};

hipError_t cg_finalize(const double* partial, int nq, double* out, hipStream_t s);
hipError_t cg_residual(const double* b, const double* q, double* r, long long n, double* partial, hipStream_t s);
hipError_t cg_dot(const double* x, const double* y, long long n, double* partial, hipStream_t s);
hipError_t cg_update_xr(double* x, double* r, const double* p, const double* q, double alpha, long long n,
                        double* partial, hipStream_t s);
hipError_t cg_jacobi(double* r, double* z, const double* zold, const double* dinv, int n3, double mu_r, long long n,
                     double* partial, hipStream_t s);
hipError_t cg_update_p(double* z, double* p, double* zold, double mu_z, double beta, long long n, hipStream_t s);
hipError_t cg_hash_fill(double* v, unsigned long long seed, long long n, double* partial, hipStream_t s);
hipError_t cg_axpb(double* y, const double* x, double a, double c, long long n, hipStream_t s);
hipError_t cg_fill(double* y, double c, long long n, hipStream_t s);
hipError_t cg_xpby(double* y, const double* x, double b, long long n, hipStream_t s);   // y = x + b y

// main loop with device-side scalars
hipError_t cg_state_init(double* st, double tol2, int max_it, double sum_d, long long n, bool proj, hipStream_t s);
hipError_t cg_fin_alpha(const double* partial, int nblocks, double* st, hipStream_t s);
hipError_t cg_update_xr_st(double* x, double* r, const double* p, const double* q, const double* dinv, int n3,
                           const double* st, bool jacobi, long long n, double* partial, hipStream_t s);
hipError_t cg_fin_jacobi(const double* partial, double* st, bool start, hipStream_t s);
hipError_t cg_fin_resid(const double* partial, double* st, bool start, hipStream_t s);
hipError_t cg_fin_cheb(const double* partial, int nblocks, double* st, bool start, hipStream_t s);
hipError_t cg_cheb1(const double* r, float* z, const float* zprev, const float* dinv32, int n3, const double* st,
                    float inv_theta, long long n, double* partial, hipStream_t s);
hipError_t cg_fill32(float* y, float c, long long n, hipStream_t s);
hipError_t cg_update_p_jacobi(const double* r, double* p, const double* dinv, int n3, const double* st, long long n,
                              hipStream_t s);
hipError_t cg_update_p_cheb(const float* z, double* p, const double* st, long long n, hipStream_t s);

// a preconditioner that is a separate call (the V-cycle), in FP64 or FP32:
// its input r' = r - mu_r, the partials of the flexible beta (for
// cg_fin_cheb with kCgBlocks), and p = (z - mu_z) + beta p
hipError_t cg_rprime(const double* r, const double* st, double* out, long long n, hipStream_t s);
hipError_t cg_rprime(const double* r, const double* st, float* out, long long n, hipStream_t s);
hipError_t cg_zsums(const double* r, const double* z, const double* zprev, const double* st, long long n,
                    double* partial, hipStream_t s);
hipError_t cg_zsums(const double* r, const float* z, const float* zprev, const double* st, long long n,
                    double* partial, hipStream_t s);
hipError_t cg_update_p_z(const double* z, double* p, const double* st, long long n, hipStream_t s);
hipError_t cg_update_p_z(const float* z, double* p, const double* st, long long n, hipStream_t s);

// inverse-mass-preconditioned CG with device-side scalars (same state layout)
hipError_t mpcg_start(const double* partial, double* st, hipStream_t s);
hipError_t mpcg_beta(const double* rr_partial, const double* rz_partial, int nblocks, double* st, hipStream_t s);
hipError_t mpcg_xpby(double* p, const double* z, const double* st, long long n, hipStream_t s);

// multigrid V-cycle: Chebyshev smoother steps and vector updates (FP64, FP32)
hipError_t mg_cheb_first(const double* b, const double* dinv, int n3, double s, double* d, double* x, long long n,
                         hipStream_t st);
hipError_t mg_cheb_next(const double* b, const double* t, const double* dinv, int n3, double c1, double c2, double* d, double* x,
                        long long n, hipStream_t st);
hipError_t mg_add(double* x, const double* t, long long n, hipStream_t st);
hipError_t mg_cheb_first(const float* b, const float* dinv, int n3, float s, float* d, float* x, long long n,
                         hipStream_t st);
hipError_t mg_cheb_next(const float* b, const float* t, const float* dinv, int n3, float c1, float c2, float* d, float* x,
                        long long n, hipStream_t st);
hipError_t mg_add(float* x, const float* t, long long n, hipStream_t st);
hipError_t mg_convert(const double* a, float* b, long long n, hipStream_t st);
hipError_t mg_convert(const float* a, double* b, long long n, hipStream_t st);

}  // namespace dgmf
