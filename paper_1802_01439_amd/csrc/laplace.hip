// SIPG Laplace apply y = A x (plain IO policy of the kernels in
// laplace_kernels.h), FP64 and FP32, degrees 1..11.
#include <cstring>

#include "laplace_kernels.h"

namespace dgmf {

template <int N, typename T>
static hipError_t launch_laplace_n(const LaplacePlan& P, const void* src, void* dst, hipStream_t stream,
                                   const void* tab) {
  LapPlainIO<T> io{(const T*)src, (T*)dst};
  return launch_laplace_io<N, T>(P, io, static_cast<const LapTab<N, T>*>(tab), stream);
}

template <typename T>
static hipError_t launch_laplace_t(const LaplacePlan& P, const void* src, void* dst, hipStream_t s,
                                   const void* tab) {
  switch (P.k) {
    case 1: return launch_laplace_n<2, T>(P, src, dst, s, tab);
    case 2: return launch_laplace_n<3, T>(P, src, dst, s, tab);
    case 3: return launch_laplace_n<4, T>(P, src, dst, s, tab);
    case 4: return launch_laplace_n<5, T>(P, src, dst, s, tab);
    case 5: return launch_laplace_n<6, T>(P, src, dst, s, tab);
    case 6: return launch_laplace_n<7, T>(P, src, dst, s, tab);
    case 7: return launch_laplace_n<8, T>(P, src, dst, s, tab);
    case 8: return launch_laplace_n<9, T>(P, src, dst, s, tab);
    case 9: return launch_laplace_n<10, T>(P, src, dst, s, tab);
    case 10: return launch_laplace_n<11, T>(P, src, dst, s, tab);
    case 11: return launch_laplace_n<12, T>(P, src, dst, s, tab);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_laplace(const LaplacePlan& P, bool f32, const void* src, void* dst, hipStream_t stream,
                          const void* tab) {
  return f32 ? launch_laplace_t<float>(P, src, dst, stream, tab)
             : launch_laplace_t<double>(P, src, dst, stream, tab);
}

template <int N, typename T>
static size_t tab_fill(const LaplacePlan& P, void* out) {
  if (out) {
    const LapTab<N, T> t = make_lap_tab<N, T>(P);
    std::memcpy(out, &t, sizeof(t));
  }
  return sizeof(LapTab<N, T>);
}

template <typename T>
static size_t tab_fill_t(const LaplacePlan& P, void* out) {
  switch (P.k) {
    case 1: return tab_fill<2, T>(P, out);
    case 2: return tab_fill<3, T>(P, out);
    case 3: return tab_fill<4, T>(P, out);
    case 4: return tab_fill<5, T>(P, out);
    case 5: return tab_fill<6, T>(P, out);
    case 6: return tab_fill<7, T>(P, out);
    case 7: return tab_fill<8, T>(P, out);
    case 8: return tab_fill<9, T>(P, out);
    case 9: return tab_fill<10, T>(P, out);
    case 10: return tab_fill<11, T>(P, out);
    case 11: return tab_fill<12, T>(P, out);
    default: return 0;
  }
}

size_t lap_table_fill(const LaplacePlan& P, bool f32, void* host_out) {
  return f32 ? tab_fill_t<float>(P, host_out) : tab_fill_t<double>(P, host_out);
}

}  // namespace dgmf
