// FP32 Chebyshev steps of the CG preconditioner with the three-term
// recurrence (and, for the last step, the partial sums the flexible CG needs)
// fused into the epilogue of the Laplace apply.
#include "cg_kernels.h"
#include "cg_laplace.h"
#include "laplace_kernels.h"

namespace dgmf {

namespace {

// KIND 0: first step (x_{k-1} = x_0 = 0, operand x_1 = D^-1 r' / theta formed
// from r); 1: second step (x_{k-1} = x_1, recomputed from r'); 2: later steps
// (x_{k-1} read from its buffer, which x_{k+1} then overwrites in place: each
// thread reads and writes only its own DoFs there).
template <int KIND, bool LAST>
struct ChebIO {
  ChebStepArgs a;
  double mu, muz_prev;
  double acc[3];

  __device__ __forceinline__ void begin() {
    mu = a.st[kMuR];
    muz_prev = a.st[kMuZ];
    acc[0] = acc[1] = acc[2] = 0.0;
  }
  __device__ __forceinline__ float load(size_t i, int loc) const {
    if constexpr (KIND == 0) {
      const float rf = (float)(a.r[i] - mu);
      return a.dinv[loc] * rf * a.inv_theta;
    } else {
      return a.xin[i];
    }
  }
  __device__ __forceinline__ void store(size_t i, int loc, float x, float t) {
    double rp = 0.0;
    float rf;
    if constexpr (KIND == 0 || LAST) {
      rp = a.r[i] - mu;
      rf = (float)rp;
    } else {
      rf = a.r32[i];
    }
    if constexpr (KIND == 0 && !LAST) a.r32[i] = rf;
    const float di = a.dinv[loc];
    float xm1 = 0.0f;
    if constexpr (KIND == 1) xm1 = di * rf * a.inv_theta;
    if constexpr (KIND == 2) xm1 = a.xprev[i];
    const float xn = x + (a.c1 * (x - xm1) + a.c2 * di * (rf - t));
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

template <int N, int KIND, bool LAST>
hipError_t step_n(const LaplacePlan& P, const ChebStepArgs& a, hipStream_t s, const void* tab) {
  ChebIO<KIND, LAST> io{};
  io.a = a;
  return launch_laplace_io<N, float>(P, io, static_cast<const LapTab<N, float>*>(tab), s);
}

template <int N>
hipError_t step_fl(const LaplacePlan& P, int step, bool last, const ChebStepArgs& a, hipStream_t s,
                   const void* t) {
  if (step == 1) return last ? step_n<N, 0, true>(P, a, s, t) : step_n<N, 0, false>(P, a, s, t);
  if (step == 2) return last ? step_n<N, 1, true>(P, a, s, t) : step_n<N, 1, false>(P, a, s, t);
  return last ? step_n<N, 2, true>(P, a, s, t) : step_n<N, 2, false>(P, a, s, t);
}

}  // namespace

hipError_t cg_apply_cheb(const LaplacePlan& P, int step, bool last, const ChebStepArgs& a, hipStream_t s,
                         const void* tab) {
  switch (P.k) {
    case 1: return step_fl<2>(P, step, last, a, s, tab);
    case 2: return step_fl<3>(P, step, last, a, s, tab);
    case 3: return step_fl<4>(P, step, last, a, s, tab);
    case 4: return step_fl<5>(P, step, last, a, s, tab);
    case 5: return step_fl<6>(P, step, last, a, s, tab);
    case 6: return step_fl<7>(P, step, last, a, s, tab);
    case 7: return step_fl<8>(P, step, last, a, s, tab);
    case 8: return step_fl<9>(P, step, last, a, s, tab);
    case 9: return step_fl<10>(P, step, last, a, s, tab);
    case 10: return step_fl<11>(P, step, last, a, s, tab);
    case 11: return step_fl<12>(P, step, last, a, s, tab);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dgmf
