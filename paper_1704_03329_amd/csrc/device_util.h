// Device helpers shared by the kernels of libmdpl.
#pragma once

#include <hip/hip_runtime.h>

namespace mdpl {

// Fold a coordinate into [0, L): x - L floor(x / L), each operation rounded
// (no contraction), then one correction step against rounding to L.
__device__ __forceinline__ double fold(double x, double L) {
#pragma clang fp contract(off)
  double w = x - L * floor(x / L);
  if (w >= L) w -= L;
  if (w < 0.0) w += L;
  return w;
}

// Exact FP64 minimum-image squared distance, contraction off:
//   d = a - b; d > L/2 ? d - L : (d < -L/2 ? d + L : d);  (dx*dx + dy*dy) + dz*dz
__device__ __forceinline__ double exact_d2(double xi, double yi, double zi, double xj, double yj,
                                           double zj, double Lx, double Ly, double Lz, double hx,
                                           double hy, double hz) {
#pragma clang fp contract(off)
  // both wraps are formed and selected, so no lane branches
  double dx = xi - xj;
  dx = dx > hx ? dx - Lx : (dx < -hx ? dx + Lx : dx);
  double dy = yi - yj;
  dy = dy > hy ? dy - Ly : (dy < -hy ? dy + Ly : dy);
  double dz = zi - zj;
  dz = dz > hz ? dz - Lz : (dz < -hz ? dz + Lz : dz);
  return (dx * dx + dy * dy) + dz * dz;
}

// Same, also returning the separation vector.
__device__ __forceinline__ double exact_sep(double xi, double yi, double zi, double xj, double yj,
                                            double zj, double Lx, double Ly, double Lz, double hx,
                                            double hy, double hz, double& dx, double& dy,
                                            double& dz) {
#pragma clang fp contract(off)
  dx = xi - xj;
  if (dx > hx) dx = dx - Lx;
  else if (dx < -hx) dx = dx + Lx;
  dy = yi - yj;
  if (dy > hy) dy = dy - Ly;
  else if (dy < -hy) dy = dy + Ly;
  dz = zi - zj;
  if (dz > hz) dz = dz - Lz;
  else if (dz < -hz) dz = dz + Lz;
  return (dx * dx + dy * dy) + dz * dz;
}

// (dx*dx + dy*dy) + dz*dz with each operation rounded (no contraction)
__device__ __forceinline__ double sq_sum(double dx, double dy, double dz) {
#pragma clang fp contract(off)
  return (dx * dx + dy * dy) + dz * dz;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over a 256-thread block; the result is valid in thread 0.  Fixed
// order (wave butterflies, then the four wave sums pairwise).
__device__ __forceinline__ double block_sum256(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return r;
}

__device__ __forceinline__ double block_max256(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    r = sh[0];
    for (int w = 1; w < 4; ++w) r = sh[w] > r ? sh[w] : r;
  }
  __syncthreads();
  return r;
}

}  // namespace mdpl
