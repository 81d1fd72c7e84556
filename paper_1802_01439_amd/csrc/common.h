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

// Traversal of the element batches.  A batch is a run of E consecutive
// elements inside one z-plane (plane-linear index j*E .. j*E+E-1, so only the
// last batch of a plane can be short); planes are numbered pz = comp*Nz + ez.
// Batches are grouped into strips of S consecutive runs (a few element rows)
// and a strip is walked plane by plane: logical id L -> (strip, pz, run in
// strip).  Consecutive ids are x-neighbours, ids S apart are z-neighbours and
// y-neighbours sit within the same strip, so the neighbour data an element
// needs was loaded a few dozen workgroups earlier and is still in L2.
struct Traversal {
  int PB;   // batches per plane
  int PZ;   // planes (n_comp * Nz)
  int S;    // runs per strip
};

__device__ __forceinline__ void strip_order(int L, const Traversal& t, int& j, int& pz) {
  const int F = t.PB / t.S, R = t.PB - F * t.S;
  const int full = F * t.S * t.PZ;
  if (L < full) {
    const int s = L / (t.S * t.PZ), rem = L - s * t.S * t.PZ;
    pz = rem / t.S;
    j = s * t.S + (rem - pz * t.S);
  } else {
    const int rem = L - full;
    pz = rem / R;
    j = F * t.S + (rem - pz * R);
  }
}

// Host-side launch status: 0 or a hipError_t from the launch.
struct LaunchStatus {
  hipError_t err = hipSuccess;
};

}  // namespace dgmf
