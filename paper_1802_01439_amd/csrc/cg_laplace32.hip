// FP32 Chebyshev steps of the CG preconditioner with the step recurrence
// (and, for the last step, the partial sums the flexible CG needs) fused
// into the epilogue of the Laplace apply.
#include "cg_kernels.h"
#include "cg_laplace.h"
#include "laplace_kernels.h"

namespace dgmf {

namespace {

template <bool FIRST, bool LAST>
struct ChebIO {
  ChebStepArgs a;
  double mu, muz_prev;
  double acc[3];

  __device__ __forceinline__ void begin() {
    mu = a.st[kMuR];
    muz_prev = a.st[kMuZ];
    acc[0] = acc[1] = acc[2] = 0.0;
  }
  // operand x: FIRST forms x1 = D^-1 r' / theta from r
  __device__ __forceinline__ float load(size_t i, int loc) const {
    if constexpr (FIRST) {
      const float rf = (float)(a.r[i] - mu);
      return a.dinv[loc] * rf * a.inv_theta;
    } else {
      return a.xin[i];
    }
  }
  __device__ __forceinline__ void store(size_t i, int loc, float x, float t) {
    double rp = 0.0;
    float rf;
    if constexpr (FIRST || LAST) {
      rp = a.r[i] - mu;
      rf = (float)rp;
    } else {
      rf = a.r32[i];
    }
    if constexpr (FIRST && !LAST) a.r32[i] = rf;
    float dold;
    if constexpr (FIRST) dold = x;
    else dold = a.d[i];
    const float dn = a.c1 * dold + a.c2 * a.dinv[loc] * (rf - t);
    if constexpr (!LAST) a.d[i] = dn;
    const float xn = x + dn;
    a.xout[i] = xn;
    if constexpr (LAST) {
      const double z = (double)xn;
      acc[0] += z;
      acc[1] = fma(rp, z, acc[1]);
      acc[2] = fma(rp, (double)a.zprev[i] - muz_prev, acc[2]);
    }
  }
  template <int THREADS, size_t BYTES>
  __device__ __forceinline__ void finish(void* lds) {
    if constexpr (LAST) wg_partials<THREADS, BYTES, 3>(acc, a.partial, lds);
  }
};

template <int N, bool FIRST, bool LAST>
hipError_t step_n(const LaplacePlan& P, const ChebStepArgs& a, hipStream_t s) {
  ChebIO<FIRST, LAST> io{};
  io.a = a;
  return launch_laplace_io<N, float>(P, io, nullptr, s);
}

template <int N>
hipError_t step_fl(const LaplacePlan& P, bool first, bool last, const ChebStepArgs& a, hipStream_t s) {
  if (first) return last ? step_n<N, true, true>(P, a, s) : step_n<N, true, false>(P, a, s);
  return last ? step_n<N, false, true>(P, a, s) : step_n<N, false, false>(P, a, s);
}

}  // namespace

hipError_t cg_apply_cheb(const LaplacePlan& P, bool first, bool last, const ChebStepArgs& a, hipStream_t s) {
  switch (P.k) {
    case 1: return step_fl<2>(P, first, last, a, s);
    case 2: return step_fl<3>(P, first, last, a, s);
    case 3: return step_fl<4>(P, first, last, a, s);
    case 4: return step_fl<5>(P, first, last, a, s);
    case 5: return step_fl<6>(P, first, last, a, s);
    case 6: return step_fl<7>(P, first, last, a, s);
    case 7: return step_fl<8>(P, first, last, a, s);
    case 8: return step_fl<9>(P, first, last, a, s);
    case 9: return step_fl<10>(P, first, last, a, s);
    case 10: return step_fl<11>(P, first, last, a, s);
    case 11: return step_fl<12>(P, first, last, a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dgmf
