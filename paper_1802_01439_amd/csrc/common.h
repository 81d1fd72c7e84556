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

// Host-side launch status: 0 or a hipError_t from the launch.
struct LaunchStatus {
  hipError_t err = hipSuccess;
};

}  // namespace dgmf
