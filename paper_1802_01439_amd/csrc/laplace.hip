// SIPG Laplace apply y = A x (plain IO policy of the kernels in
// laplace_kernels.h), FP64 and FP32, degrees 1..11.
#include "laplace_kernels.h"

namespace dgmf {

template <int N, typename T>
static hipError_t launch_laplace_n(const LaplacePlan& P, const void* src, void* dst, hipStream_t stream) {
  LapPlainIO<T> io{(const T*)src, (T*)dst};
  return launch_laplace_io<N, T>(P, io, nullptr, stream);
}

template <typename T>
static hipError_t launch_laplace_t(const LaplacePlan& P, const void* src, void* dst,
                                   hipStream_t s) {
  switch (P.k) {
    case 1: return launch_laplace_n<2, T>(P, src, dst, s);
    case 2: return launch_laplace_n<3, T>(P, src, dst, s);
    case 3: return launch_laplace_n<4, T>(P, src, dst, s);
    case 4: return launch_laplace_n<5, T>(P, src, dst, s);
    case 5: return launch_laplace_n<6, T>(P, src, dst, s);
    case 6: return launch_laplace_n<7, T>(P, src, dst, s);
    case 7: return launch_laplace_n<8, T>(P, src, dst, s);
    case 8: return launch_laplace_n<9, T>(P, src, dst, s);
    case 9: return launch_laplace_n<10, T>(P, src, dst, s);
    case 10: return launch_laplace_n<11, T>(P, src, dst, s);
    case 11: return launch_laplace_n<12, T>(P, src, dst, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_laplace(const LaplacePlan& P, bool f32, const void* src, void* dst,
                          hipStream_t stream) {
  return f32 ? launch_laplace_t<float>(P, src, dst, stream)
             : launch_laplace_t<double>(P, src, dst, stream);
}

}  // namespace dgmf
