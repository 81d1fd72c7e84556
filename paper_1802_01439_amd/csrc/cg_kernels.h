// Vector kernels of the CG solver (launch wrappers).  Reductions write
// kCgBlocks partials per quantity; cg_finalize sums them in a fixed order.
#pragma once

#include <hip/hip_runtime.h>

namespace dgmf {

constexpr int kCgThreads = 256;
constexpr int kCgBlocks = 1024;

hipError_t cg_finalize(const double* partial, int nq, double* out, hipStream_t s);
hipError_t cg_residual(const double* b, const double* q, double* r, long long n, double* partial, hipStream_t s);
hipError_t cg_dot(const double* x, const double* y, long long n, double* partial, hipStream_t s);
hipError_t cg_update_xr(double* x, double* r, const double* p, const double* q, double alpha, long long n,
                        double* partial, hipStream_t s);
hipError_t cg_jacobi(double* r, double* z, const double* zold, const double* dinv, int n3, double mu_r, long long n,
                     double* partial, hipStream_t s);
hipError_t cg_update_p(double* z, double* p, double* zold, double mu_z, double beta, long long n, hipStream_t s);
hipError_t cg_cheb_init(double* r, float* r32, float* x32, float* d32, const float* dinv32, int n3, double mu_r,
                        float inv_theta, long long n, hipStream_t s);
hipError_t cg_cheb_step(float* x32, float* d32, const float* r32, const float* t32, const float* dinv32, int n3,
                        float c1, float c2, long long n, hipStream_t s);
hipError_t cg_cheb_final(const double* r, double* z, const double* zold, const float* x32, long long n,
                         double* partial, hipStream_t s);
hipError_t cg_hash_fill(double* v, unsigned long long seed, long long n, double* partial, hipStream_t s);
hipError_t cg_axpb(double* y, const double* x, double a, double c, long long n, hipStream_t s);
hipError_t cg_fill(double* y, double c, long long n, hipStream_t s);

}  // namespace dgmf
