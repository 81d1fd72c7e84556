// FP64 operator application of the CG loop with the p.Ap partial sums fused
// into the Laplace kernel.
#include "cg_kernels.h"
#include "cg_laplace.h"
#include "laplace_kernels.h"

namespace dgmf {

namespace {

// q = A p with the partial sums of p.q in the epilogue.  (Forming p = z +
// beta p_old inside the apply as well was measured slower: three loads per
// operand value where the plain kernel has one, at half the occupancy.)
struct CgDotIO {
  const double* __restrict__ p;
  double* __restrict__ q;
  double* __restrict__ partial;
  double acc[1];

  __device__ __forceinline__ void begin() { acc[0] = 0.0; }
  __device__ __forceinline__ double load(size_t i, int) const { return p[i]; }
  __device__ __forceinline__ void store(size_t i, int, double in, double out) {
    q[i] = out;
    acc[0] = fma(in, out, acc[0]);
  }
  template <int THREADS, size_t BYTES>
  __device__ __forceinline__ void finish(void* lds) {
    wg_partials<THREADS, BYTES, 1>(acc, partial, lds);
  }
};

template <int N>
const LapTab<N, double>* tab_of(const void* tab) {
  return static_cast<const LapTab<N, double>*>(tab);
}

template <typename IO>
hipError_t dispatch64(const LaplacePlan& P, const IO& io, hipStream_t s, const void* tab) {
  switch (P.k) {
    case 1: return launch_laplace_io<2, double>(P, io, tab_of<2>(tab), s);
    case 2: return launch_laplace_io<3, double>(P, io, tab_of<3>(tab), s);
    case 3: return launch_laplace_io<4, double>(P, io, tab_of<4>(tab), s);
    case 4: return launch_laplace_io<5, double>(P, io, tab_of<5>(tab), s);
    case 5: return launch_laplace_io<6, double>(P, io, tab_of<6>(tab), s);
    case 6: return launch_laplace_io<7, double>(P, io, tab_of<7>(tab), s);
    case 7: return launch_laplace_io<8, double>(P, io, tab_of<8>(tab), s);
    case 8: return launch_laplace_io<9, double>(P, io, tab_of<9>(tab), s);
    case 9: return launch_laplace_io<10, double>(P, io, tab_of<10>(tab), s);
    case 10: return launch_laplace_io<11, double>(P, io, tab_of<11>(tab), s);
    case 11: return launch_laplace_io<12, double>(P, io, tab_of<12>(tab), s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
long grid_t(const LaplacePlan& P) {
  switch (P.k) {
    case 1: return lap_grid<2, T>(P);
    case 2: return lap_grid<3, T>(P);
    case 3: return lap_grid<4, T>(P);
    case 4: return lap_grid<5, T>(P);
    case 5: return lap_grid<6, T>(P);
    case 6: return lap_grid<7, T>(P);
    case 7: return lap_grid<8, T>(P);
    case 8: return lap_grid<9, T>(P);
    case 9: return lap_grid<10, T>(P);
    case 10: return lap_grid<11, T>(P);
    case 11: return lap_grid<12, T>(P);
    default: return 0;
  }
}

}  // namespace

long cg_apply_grid(const LaplacePlan& P, bool f32) { return f32 ? grid_t<float>(P) : grid_t<double>(P); }

hipError_t cg_apply_dot(const LaplacePlan& P, const double* p, double* q, double* partial, hipStream_t s,
                        const void* tab) {
  CgDotIO io{};
  io.p = p;
  io.q = q;
  io.partial = partial;
  return dispatch64(P, io, s, tab);
}

}  // namespace dgmf
