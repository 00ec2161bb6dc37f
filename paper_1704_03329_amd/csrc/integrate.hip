// Particle loops of the time integration: velocity Verlet (Alg.
// VelocityVerlet), the Andersen thermostat of the crystallisation run
// (Sec. 5.2), fixed-order reductions of per-block partials, and the skin
// check of the list reuse (Sec. 3.5).
#include "device_util.h"
#include "internal.h"

namespace mdpl {

// ------------------------------------------------------------ random numbers
// Philox4x64 with 10 rounds (Salmon, Moraes, Dror and Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC'11): each round forms the 128-bit
// products of counter words 0 and 2 with two fixed odd multipliers and
// recombines the halves with words 1 and 3 and the key; the key advances by
// two Weyl increments between rounds.
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
  constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull, kM1 = 0xCA5A826395121157ull;
  constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull, kW1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += kW0;
      k1 += kW1;
    }
    const uint64_t hi0 = __umul64hi(kM0, c[0]), lo0 = kM0 * c[0];
    const uint64_t hi1 = __umul64hi(kM1, c[2]), lo1 = kM1 * c[2];
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// [0, 1) from the top 53 bits
__device__ __forceinline__ double uniform53(uint64_t b) { return (double)(b >> 11) * 0x1.0p-53; }

// The Andersen collision of one particle (see struct Andersen): Box-Muller
// normals sqrt(-2 ln(1 - U1)) (cos, sin)(2 pi U2) and sqrt(-2 ln(1 - U3))
// cos(2 pi U4) from the words after the collision test.
__device__ __forceinline__ void andersen_collide(const Andersen& th, int64_t s, double& a, double& b,
                                                 double& cc) {
#pragma clang fp contract(off)
  const uint64_t pid = (uint64_t)(int64_t)th.ids[s];
  uint64_t c[4] = {(uint64_t)th.step, pid, 0, 0};
  philox4x64_10(c, th.seed, 0);
  if (!(uniform53(c[0]) < th.p)) return;
  uint64_t d[4] = {(uint64_t)th.step, pid, 1, 0};
  philox4x64_10(d, th.seed, 0);
  const double two_pi = 2.0 * 3.141592653589793;
  const double r1 = sqrt(-2.0 * log(1.0 - uniform53(c[1])));
  const double t1 = two_pi * uniform53(c[2]);
  const double r2 = sqrt(-2.0 * log(1.0 - uniform53(c[3])));
  const double t2 = two_pi * uniform53(d[0]);
  a = th.sd * (r1 * cos(t1));
  b = th.sd * (r1 * sin(t1));
  cc = th.sd * (r2 * cos(t2));
}

// ------------------------------------------------------------ velocity Verlet
// Listing position_update / velocity_update: v += F dt/(2m); r += dt v.
template <typename FT>
__global__ __launch_bounds__(256) void k_vv(const double* __restrict__ x,
                                            const double* __restrict__ y,
                                            const double* __restrict__ z, double* __restrict__ nx,
                                            double* __restrict__ ny, double* __restrict__ nz,
                                            double* __restrict__ vx, double* __restrict__ vy,
                                            double* __restrict__ vz, const FT* __restrict__ fx,
                                            const FT* __restrict__ fy, const FT* __restrict__ fz,
                                            int64_t n, double h, double dt, int mode, int ke,
                                            double* ke_part, uint32_t* flags, Andersen th,
                                            KickTrack kt) {
#pragma clang fp contract(off)
  __shared__ double sh[4];
  if (mode == 0 || mode == 1) kick_publish(kt, sh);
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double k = 0.0, m2 = 0.0;
  if (s < n) {
    double a = vx[s], b = vy[s], cc = vz[s];
    if (mode != 3) {
      const double gx = h * (double)fx[s], gy = h * (double)fy[s], gz = h * (double)fz[s];
      a = a + gx;
      b = b + gy;
      cc = cc + gz;
      if (mode == 1 || mode == 2) k = (a * a + b * b) + cc * cc;
      if ((mode == 1 || mode == 2) && th.p > 0.0) andersen_collide(th, s, a, b, cc);
      if (mode == 1) {
        a = a + gx;
        b = b + gy;
        cc = cc + gz;
      }
      if (mode != 2) {
        nx[s] = x[s] + dt * a;
        ny[s] = y[s] + dt * b;
        nz[s] = z[s] + dt * cc;
      }
      vx[s] = a;
      vy[s] = b;
      vz[s] = cc;
      m2 = (a * a + b * b) + cc * cc;
      if (!(m2 < 1e300)) atomicOr(flags, MDPL_FLAG_NONFINITE);
    } else {
      k = (a * a + b * b) + cc * cc;
    }
  }
  if (ke) {
    const double t = block_sum256(k, sh);
    if (threadIdx.x == 0) ke_part[blockIdx.x] = t;
  }
  if (mode == 0 || mode == 1) {
    const double mb = block_max256(m2, sh);  // a NaN speed is caught by the non-finite flag
    if (threadIdx.x == 0) kick_store(kt, mb);
  }
}

// The pending record of the rebuild rule, one workgroup (the host needs it now).
__global__ __launch_bounds__(256) void k_publish(KickTrack kt) {
  __shared__ double sh[4];
  kick_publish(kt, sh);
}

hipError_t publish_record(const KickTrack& kt, hipStream_t st) {
  hipLaunchKernelGGL(k_publish, dim3(1), dim3(256), 0, st, kt);
  return hipGetLastError();
}

hipError_t vv_step(const double* x, const double* y, const double* z, double* nx, double* ny,
                   double* nz, double* vx, double* vy, double* vz, const void* fx, const void* fy,
                   const void* fz, int precision, int64_t n, double h, double dt, int mode, bool ke,
                   double* ke_partials, uint32_t* flags, hipStream_t st, int* nblocks_out,
                   const Andersen* th, const KickTrack* track) {
  const unsigned nb = (unsigned)div_up(n, 256);
  if (nblocks_out) *nblocks_out = (int)nb;
  const Andersen none{nullptr, 0.0, 0.0, 0, 0};
  const Andersen& a = th ? *th : none;
  KickTrack kt{};
  if (track) kt = *track;
  if (precision == 1)
    hipLaunchKernelGGL(k_vv<float>, dim3(nb), dim3(256), 0, st, x, y, z, nx, ny, nz, vx, vy, vz,
                       (const float*)fx, (const float*)fy, (const float*)fz, n, h, dt, mode,
                       ke ? 1 : 0, ke_partials, flags, a, kt);
  else
    hipLaunchKernelGGL(k_vv<double>, dim3(nb), dim3(256), 0, st, x, y, z, nx, ny, nz, vx, vy, vz,
                       (const double*)fx, (const double*)fy, (const double*)fz, n, h, dt, mode,
                       ke ? 1 : 0, ke_partials, flags, a, kt);
  return hipGetLastError();
}

// ------------------------------------------------------------ reductions
// out[c] = scale * sum_k partials[k*stride + c], fixed order, one block.
__global__ __launch_bounds__(256) void k_reduce_partials(const double* __restrict__ p, int nb,
                                                         int stride, int ncomp, double* out,
                                                         double scale) {
  __shared__ double sh[4];
  for (int comp = 0; comp < ncomp; ++comp) {
    double v = 0.0;
    for (int k = threadIdx.x; k < nb; k += 256) v += p[(int64_t)k * stride + comp];
    const double t = block_sum256(v, sh);
    if (threadIdx.x == 0) out[comp] = scale * t;
  }
}

hipError_t reduce_partials(const double* partials, int nblocks, int stride, int ncomp,
                           double* out, double scale, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(256), 0, st, partials, nblocks, stride,
                     ncomp, out, scale);
  return hipGetLastError();
}

// A thermo row in one launch: component c of the partials (the same fixed
// order as k_reduce_partials) times o.scale[c] to o.dst[c] (skipped if
// null), then the optional 8-byte copy and zero.
__global__ __launch_bounds__(256) void k_reduce_row(const double* __restrict__ p, int nb,
                                                    int stride, int ncomp, RowOut o) {
  __shared__ double sh[4];
  for (int comp = 0; comp < ncomp; ++comp) {
    double v = 0.0;
    for (int k = threadIdx.x; k < nb; k += 256) v += p[(int64_t)k * stride + comp];
    const double t = block_sum256(v, sh);
    if (threadIdx.x == 0 && o.dst[comp]) *o.dst[comp] = o.scale[comp] * t;
  }
  if (threadIdx.x == 0) {
    if (o.cdst) *o.cdst = *o.csrc;
    if (o.zdst) *o.zdst = 0.0;
  }
}

hipError_t reduce_row(const double* partials, int nblocks, int stride, int ncomp, const RowOut& o,
                      hipStream_t st) {
  if (ncomp < 0 || ncomp > 3) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_reduce_row, dim3(1), dim3(256), 0, st, partials, nblocks, stride, ncomp, o);
  return hipGetLastError();
}

}  // namespace mdpl

namespace mdpl {

// ------------------------------------------------------------ skin check
// Largest squared displacement since the last list build, per block.
__global__ __launch_bounds__(256) void k_disp_partials(
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
    const double* __restrict__ xb, const double* __restrict__ yb, const double* __restrict__ zb,
    int64_t n, double* __restrict__ part) {
  __shared__ double sh[4];
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double d = 0.0;
  if (s < n) {
    const double a = x[s] - xb[s], b = y[s] - yb[s], c = z[s] - zb[s];
    d = a * a + b * b + c * c;
    if (!(d < 1e300)) d = 1e300;
  }
  const double m = block_max256(d, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = m;
}

hipError_t disp_partials(const double* x, const double* y, const double* z, const double* xb,
                         const double* yb, const double* zb, int64_t n, double* partials,
                         hipStream_t st, int* nblocks_out) {
  const unsigned nb = (unsigned)div_up(n, 256);
  *nblocks_out = (int)nb;
  hipLaunchKernelGGL(k_disp_partials, dim3(nb), dim3(256), 0, st, x, y, z, xb, yb, zb, n, partials);
  return hipGetLastError();
}

// max over the partials -> displacement; record the largest; flag when it
// reaches half the skin (a pair inside rc could then be missing from the list).
__global__ __launch_bounds__(256) void k_skin_check(const double* __restrict__ part, int nb,
                                                    double half_skin, double* max_disp,
                                                    uint32_t* flags) {
  __shared__ double sh[4];
  double v = 0.0;
  for (int k = threadIdx.x; k < nb; k += 256) v = part[k] > v ? part[k] : v;
  const double m2 = block_max256(v, sh);
  if (threadIdx.x == 0) {
    const double d = sqrt(m2);
    if (d > *max_disp) *max_disp = d;
    if (d >= half_skin) atomicOr(flags, MDPL_FLAG_SKIN);
  }
}

hipError_t skin_check(const double* partials, int nblocks, double half_skin, double* max_disp,
                      uint32_t* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_skin_check, dim3(1), dim3(256), 0, st, partials, nblocks, half_skin,
                     max_disp, flags);
  return hipGetLastError();
}

}  // namespace mdpl

namespace mdpl {

__global__ void k_scale_v(double* __restrict__ vx, double* __restrict__ vy, double* __restrict__ vz,
                          int64_t n, double f) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  vx[i] *= f;
  vy[i] *= f;
  vz[i] *= f;
}

hipError_t scale_velocities(double* vx, double* vy, double* vz, int64_t n, double factor,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_scale_v, dim3((unsigned)div_up(n, 256)), dim3(256), 0, st, vx, vy, vz, n,
                     factor);
  return hipGetLastError();
}

}  // namespace mdpl
