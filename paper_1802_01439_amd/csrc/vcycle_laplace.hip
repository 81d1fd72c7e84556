// Multigrid smoother work fused into the epilogue of the Laplace apply
// (Sec. 3.3, the V-cycle's Chebyshev smoother), FP64 and FP32:
//   Chebyshev step  d <- c1 d + c2 D^-1 (b - A x),  x' = x + d
//   residual        res = b - A x
//   residual and the first step of a zero-start Chebyshev smoother on it
//                   res = b - A x,  d = e = s D^-1 res
//   last Chebyshev step of the post-smoothing, added to the level's iterate
//                   y += x + (c1 d + c2 D^-1 (b - A x))
// The operand x is read for neighbour DoFs by other workgroups, so the new
// iterate goes to a second buffer x'; d is read and written only by the
// thread that owns each DoF, in place.  D^-1 is one element's diagonal
// inverse, indexed by the local node.
#include "laplace_kernels.h"
#include "ops.h"

namespace dgmf {

namespace {

template <typename T>
struct MgChebIO {
  const T* __restrict__ x;
  const T* __restrict__ b;
  const T* __restrict__ dinv;
  T* __restrict__ d;
  T* __restrict__ xout;
  T c1, c2;
  __device__ __forceinline__ void begin() {}
  __device__ __forceinline__ T load(size_t i, int) const { return x[i]; }
  __device__ __forceinline__ void store(size_t i, int loc, T in, T out) {
    const T v = c1 * d[i] + c2 * dinv[loc] * (b[i] - out);
    d[i] = v;
    xout[i] = in + v;
  }
  template <int THREADS, size_t BYTES>
  __device__ __forceinline__ void finish(void*) {}
};

template <typename T>
struct MgResIO {
  const T* __restrict__ x;
  const T* __restrict__ b;
  T* __restrict__ res;
  __device__ __forceinline__ void begin() {}
  __device__ __forceinline__ T load(size_t i, int) const { return x[i]; }
  __device__ __forceinline__ void store(size_t i, int, T, T out) { res[i] = b[i] - out; }
  template <int THREADS, size_t BYTES>
  __device__ __forceinline__ void finish(void*) {}
};

template <typename T>
struct MgChebAddIO {
  const T* __restrict__ x;
  const T* __restrict__ b;
  const T* __restrict__ dinv;
  const T* __restrict__ d;
  T* __restrict__ y;
  T c1, c2;
  __device__ __forceinline__ void begin() {}
  __device__ __forceinline__ T load(size_t i, int) const { return x[i]; }
  __device__ __forceinline__ void store(size_t i, int loc, T in, T out) {
    const T v = c1 * d[i] + c2 * dinv[loc] * (b[i] - out);
    const T xn = in + v;
    y[i] = y[i] + xn;
  }
  template <int THREADS, size_t BYTES>
  __device__ __forceinline__ void finish(void*) {}
};

template <typename T>
struct MgResChebIO {
  const T* __restrict__ x;
  const T* __restrict__ b;
  const T* __restrict__ dinv;
  T* __restrict__ res;
  T* __restrict__ d;
  T* __restrict__ e;
  T s;
  __device__ __forceinline__ void begin() {}
  __device__ __forceinline__ T load(size_t i, int) const { return x[i]; }
  __device__ __forceinline__ void store(size_t i, int loc, T, T out) {
    const T r = b[i] - out;
    res[i] = r;
    const T v = s * dinv[loc] * r;
    d[i] = v;
    e[i] = v;
  }
  template <int THREADS, size_t BYTES>
  __device__ __forceinline__ void finish(void*) {}
};

template <typename T, typename IO>
hipError_t dispatch(const LaplacePlan& P, const IO& io, hipStream_t s) {
  switch (P.k) {
    case 1: return launch_laplace_io<2, T>(P, io, nullptr, s);
    case 2: return launch_laplace_io<3, T>(P, io, nullptr, s);
    case 3: return launch_laplace_io<4, T>(P, io, nullptr, s);
    case 4: return launch_laplace_io<5, T>(P, io, nullptr, s);
    case 5: return launch_laplace_io<6, T>(P, io, nullptr, s);
    case 6: return launch_laplace_io<7, T>(P, io, nullptr, s);
    case 7: return launch_laplace_io<8, T>(P, io, nullptr, s);
    case 8: return launch_laplace_io<9, T>(P, io, nullptr, s);
    case 9: return launch_laplace_io<10, T>(P, io, nullptr, s);
    case 10: return launch_laplace_io<11, T>(P, io, nullptr, s);
    case 11: return launch_laplace_io<12, T>(P, io, nullptr, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

template <typename T>
hipError_t mg_apply_cheb(const LaplacePlan& P, const T* x, const T* b, const T* dinv, T c1, T c2, T* d, T* xout,
                         hipStream_t s) {
  MgChebIO<T> io{x, b, dinv, d, xout, c1, c2};
  return dispatch<T>(P, io, s);
}

template <typename T>
hipError_t mg_apply_residual(const LaplacePlan& P, const T* x, const T* b, T* res, hipStream_t s) {
  MgResIO<T> io{x, b, res};
  return dispatch<T>(P, io, s);
}

template <typename T>
hipError_t mg_apply_cheb_add(const LaplacePlan& P, const T* x, const T* b, const T* dinv, T c1, T c2, const T* d, T* y,
                             hipStream_t s) {
  MgChebAddIO<T> io{x, b, dinv, d, y, c1, c2};
  return dispatch<T>(P, io, s);
}

template <typename T>
hipError_t mg_apply_residual_cheb_first(const LaplacePlan& P, const T* x, const T* b, const T* dinv, T scale, T* res,
                                        T* d, T* e, hipStream_t s) {
  MgResChebIO<T> io{x, b, dinv, res, d, e, scale};
  return dispatch<T>(P, io, s);
}

template hipError_t mg_apply_cheb<double>(const LaplacePlan&, const double*, const double*, const double*, double,
                                          double, double*, double*, hipStream_t);
template hipError_t mg_apply_cheb<float>(const LaplacePlan&, const float*, const float*, const float*, float, float,
                                         float*, float*, hipStream_t);
template hipError_t mg_apply_residual<double>(const LaplacePlan&, const double*, const double*, double*, hipStream_t);
template hipError_t mg_apply_residual<float>(const LaplacePlan&, const float*, const float*, float*, hipStream_t);
template hipError_t mg_apply_cheb_add<double>(const LaplacePlan&, const double*, const double*, const double*, double,
                                              double, const double*, double*, hipStream_t);
template hipError_t mg_apply_cheb_add<float>(const LaplacePlan&, const float*, const float*, const float*, float, float,
                                             const float*, float*, hipStream_t);
template hipError_t mg_apply_residual_cheb_first<double>(const LaplacePlan&, const double*, const double*,
                                                         const double*, double, double*, double*, double*,
                                                         hipStream_t);
template hipError_t mg_apply_residual_cheb_first<float>(const LaplacePlan&, const float*, const float*, const float*,
                                                        float, float*, float*, float*, hipStream_t);

}  // namespace dgmf
