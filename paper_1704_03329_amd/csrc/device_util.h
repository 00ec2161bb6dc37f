// Device helpers shared by the kernels of libmdpl.
#pragma once

#include <hip/hip_runtime.h>

namespace mdpl {

// LDS reaction accumulators in 64-bit fixed point, units of 2^-32: FP32
// atomic adds in LDS run one lane at a time on this chip (about 3 cycles per
// active lane, some 40 times the cost of an integer add), while integer sums
// are also exact and independent of their order.  A value must satisfy
// fix_fits (|v| < 2^19, false for inf and NaN) to go through them; then
// v 2^32 lies within 2^51 of zero, and adding 1.5 2^52 to it in FP64 rounds
// it to an integer in the low bits of the sum (one FMA and a 64-bit
// subtraction instead of a conversion to a 64-bit integer).
constexpr double kFixUnit = 4294967296.0;    // 2^32 per unit
constexpr double kFixMax = 524288.0;         // 2^19
constexpr double kFixMagic = 6755399441055744.0;  // 1.5 2^52
__device__ __forceinline__ bool fix_fits(double v) { return __builtin_fabs(v) < kFixMax; }
__device__ __forceinline__ unsigned long long fix_of(double v) {
  const double t = __builtin_fma(v, kFixUnit, kFixMagic);
  return (unsigned long long)__double_as_longlong(t) -
         (unsigned long long)__double_as_longlong(kFixMagic);
}
__device__ __forceinline__ double fix_value(unsigned long long a) {
  return (double)(long long)a * (1.0 / kFixUnit);
}

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

// Cross-lane moves on DPP (data-parallel primitives: a lane reads another
// lane's register within the same instruction, no LDS round trip as with
// __shfl).  CTRL: 0xB1 = quad_perm [1,0,3,2] (lane ^ 1), 0x4E = quad_perm
// [2,3,0,1] (lane ^ 2), 0x110 + n = row_shr:n, 0x142 / 0x143 =
// row_bcast:15 / row_bcast:31 (ROWS selects the rows written; a lane with
// no source keeps 0).
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ int dpp_i32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(dpp_i32<CTRL, ROWS>(__float_as_int(v)));
}
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ double dpp_move(double v) {
  return __hiloint2double(dpp_i32<CTRL, ROWS>(__double2hiint(v)),
                          dpp_i32<CTRL, ROWS>(__double2loint(v)));
}

__device__ __forceinline__ float readlane63(float v) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
__device__ __forceinline__ double readlane63(double v) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                          __builtin_amdgcn_readlane(__double2loint(v), 63));
}

// Largest value over the 64 lanes of a wave (all active), for values >= 0:
// a running maximum within each row of 16 lanes, then across rows; lane 63
// ends with the wave's maximum, which is returned to every lane.
__device__ __forceinline__ int wave_max_nonneg(int v) {
  int o;
  o = dpp_i32<0x111>(v); v = o > v ? o : v;
  o = dpp_i32<0x112>(v); v = o > v ? o : v;
  o = dpp_i32<0x114>(v); v = o > v ? o : v;
  o = dpp_i32<0x118>(v); v = o > v ? o : v;
  o = dpp_i32<0x142, 0xa>(v); v = o > v ? o : v;
  o = dpp_i32<0x143, 0xc>(v); v = o > v ? o : v;
  return __builtin_amdgcn_readlane(v, 63);
}
__device__ __forceinline__ double wave_max_nonneg(double v) {
  double o;
  o = dpp_move<0x111>(v); v = o > v ? o : v;
  o = dpp_move<0x112>(v); v = o > v ? o : v;
  o = dpp_move<0x114>(v); v = o > v ? o : v;
  o = dpp_move<0x118>(v); v = o > v ? o : v;
  o = dpp_move<0x142, 0xa>(v); v = o > v ? o : v;
  o = dpp_move<0x143, 0xc>(v); v = o > v ? o : v;
  return readlane63(v);
}

// Sum over the 64 lanes of a wave (all active) in a fixed order, on DPP:
// the quads by lane ^ 1 and lane ^ 2, the rows of 16 by rotations of 4 and
// 8 lanes, then the rows into lane 63 by the two row broadcasts; the total
// is returned to every lane.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  v += dpp_move<0xB1>(v);        // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);        // quad_perm [2,3,0,1]
  v += dpp_move<0x124>(v);       // row_ror:4
  v += dpp_move<0x128>(v);       // row_ror:8
  v += dpp_move<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_move<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  return readlane63(v);
}

// Sum over a 256-thread block; the result is valid in thread 0.  Fixed
// order (the wave sums above, then the four wave sums pairwise).
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
  v = wave_max_nonneg(v);  // callers pass values >= 0
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
