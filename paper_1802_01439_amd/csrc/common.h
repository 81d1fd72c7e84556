// Shared definitions of the HIP operator library (host and device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dgmf {

// Mesh geometry handed to every kernel by value.
struct MeshArgs {
  int nx, ny, nz;   // elements per direction
  int n_el;         // nx*ny*nz
};

__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Neighbour of element (ex,ey,ez) across the face of direction d at side s
// (s = 0: reference coordinate 0, s = 1: coordinate 1), periodic wrap.
__device__ __forceinline__ int neighbor(const MeshArgs& m, int ex, int ey, int ez, int d, int s) {
  if (d == 0) ex = s ? (ex + 1 == m.nx ? 0 : ex + 1) : (ex == 0 ? m.nx - 1 : ex - 1);
  else if (d == 1) ey = s ? (ey + 1 == m.ny ? 0 : ey + 1) : (ey == 0 ? m.ny - 1 : ey - 1);
  else ez = s ? (ez + 1 == m.nz ? 0 : ez + 1) : (ez == 0 ? m.nz - 1 : ez - 1);
  return ex + m.nx * (ey + m.ny * ez);
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  This bijection on [0, G) gives every XCD one contiguous range of
// logical batches, so neighbouring elements (and the face data they share)
// are processed by the same XCD and found in its L2.
__device__ __forceinline__ int xcd_remap(int b, int G) {
  const int q = G >> 3, r = G & 7, x = b & 7;
  return x * q + (x < r ? x : r) + (b >> 3);
}

// A table pointer passed through an empty asm and returned in the constant
// address space (loads through it are scalar loads).  Loads issued after it
// cannot be merged with loads of the same entries elsewhere in the kernel, so
// a kernel that calls it at the start of each phase or loop step loads the
// table rows it uses when it uses them, instead of having the compiler hoist
// the whole (loop-invariant) table into scalar registers and spill it.
template <typename P>
using const_ptr = const __attribute__((address_space(4))) P*;

template <typename P>
__device__ __forceinline__ const_ptr<P> fresh(const P* p) {
  uint64_t x = (uint64_t)p;
  asm volatile("" : "+v"(x));
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
  return (const_ptr<P>)(((uint64_t)hi << 32) | lo);
}

// Host-side launch status: 0 or a hipError_t from the launch.
struct LaunchStatus {
  hipError_t err = hipSuccess;
};

}  // namespace dgmf
