// Lennard-Jones pair loop with full neighbour lists (the default pair loop).
//
// Force (Eq. LJforce): f_ij = 48 eps [(s^2/d2)^7 - 1/2 (s^2/d2)^4] / s^2 * dr_ij,
// dr_ij = r_i - r_j (min image), summed over the neighbour list of i and
// written once per particle (gather only, no atomics: the paper's choice of
// looping over all ordered pairs and writing to the first particle, Sec. 2).
// Each workgroup handles one brick of cells and stages the image positions of
// its neighbourhood in LDS (tile.h): the plain pass keeps x and y of a slot
// side by side and z apart, the energy pass three arrays.  A list entry is 16
// times the partner's slot, the byte offset of its x-y pair; half of it
// indexes the 8-byte arrays.  The cutoff test d2 < rc^2 uses the FP64 separation; the periodic
// image is added to a tile position once, and the plain pass forms d2 with
// fused multiply-adds, so a pair can be classified differently from the
// definition only within a few units in the last place of rc^2.  The
// energy pass uses the definition's uncontracted d2.
//
// Precision (FP32 mode): the separation and the test in FP64, the pair force
// factor in FP32 from the rounded squared distance, per-particle sums in
// FP64 (cheaper than converting the three separations), stored as FP32.  Energy and
// virial (sampled steps) are formed per pair in FP64 and reduced per block
// with wavefront shuffles into FP64 partials; a single-block pass sums the
// partials in a fixed order, so results are reproducible run to run.
//
// Potential energy: PE = 1/2 sum over ordered pairs (each unordered pair
// once), e_i = 1/2 sum_j V(r_ij); virial W = 1/2 sum over ordered pairs of
// dr . f.
#include <type_traits>

#include "device_util.h"
#include "internal.h"
#include "tile.h"

namespace mdpl {

// The kick-kick-drift of k_vv mode 1 for one particle, same operations in
// the same order; returns |v|^2 after the first kick (the sampled KE) and
// sets m2 = |v|^2 of the velocity of the drift.
__device__ __forceinline__ double fused_kick(const ForceOut& out, int64_t s, double xi, double yi,
                                             double zi, double a, double b, double cc, double fx,
                                             double fy, double fz, double& m2) {
#pragma clang fp contract(off)
  const double gx = out.h * fx, gy = out.h * fy, gz = out.h * fz;
  a = a + gx;
  b = b + gy;
  cc = cc + gz;
  const double k = (a * a + b * b) + cc * cc;
  a = a + gx;
  b = b + gy;
  cc = cc + gz;
  out.nx[s] = xi + out.dt * a;
  out.ny[s] = yi + out.dt * b;
  out.nz[s] = zi + out.dt * cc;
  out.vx[s] = a;
  out.vy[s] = b;
  out.vz[s] = cc;
  m2 = (a * a + b * b) + cc * cc;
  if (!(m2 < 1e300)) atomicOr(out.flags, MDPL_FLAG_NONFINITE);
  return k;
}

// Largest |v|^2 of the workgroup (v2 per thread, 0 where none) to the rule's
// tracking; one barrier.
__device__ __forceinline__ void block_track(const KickTrack& kt, double v2, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(v2, off, 64);
    v2 = o > v2 ? o : v2;
  }
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v2;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    double m = sh[0];
    for (int k = 1; k < nw; ++k) m = sh[k] > m ? sh[k] : m;
    kick_track(kt, m);
  }
}

// One workgroup per brick: the tile holds the image positions of the brick's
// neighbourhood, so a pair needs one LDS gather and plain FP64 differences.
// MT: arithmetic type of the pair force; OT: stored force type.  The pair
// force is accumulated in FP64 (one conversion of the scalar factor per pair
// instead of three of the separation).
// Both passes ask for 8 waves per SIMD (<= 64 VGPRs), so that two
// 1024-thread workgroups (LDS: two tiles) share a CU.
template <typename MT, typename OT, bool ENERGY>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8)))
void k_lj_force(const double* __restrict__ x, const double* __restrict__ y,
                const double* __restrict__ z, const int32_t* __restrict__ cs, Grid g, TileList tl,
                LJConst c, ForceOut out) {
  // plain pass: x and y side by side (one 16-byte gather per entry, measured
  // faster); energy pass: three arrays (measured faster there)
  using Tile = std::conditional_t<ENERGY, TileShared, TileXY>;
  __shared__ Tile t;
  __shared__ double red[48];  // up to 16 waves: e, w, ke
  __shared__ double vred[16];
  const int brick = brick_of_block(g);
  if (brick >= g.nbricks) {  // padding workgroup: still counted by the rule's tracking
    if (out.fuse && threadIdx.x == 0) kick_track(out.track, 0.0);
    return;
  }
  const int total = tile_cells(g, brick, cs, t);
  if constexpr (ENERGY) tile_load<true>(g, x, y, z, total, t);
  else tile_load_xy(g, x, y, z, total, t);
  const int s0 = cs[brick * g.V], s1 = cs[(brick + 1) * g.V];
  // plain pass: f_ij / dr_ij = x^4 (A x^3 - B) with x = 1 / d2, A = 48 eps s^12, B = 24 eps s^6
  const double sig6 = c.sigma2 * c.sigma2 * c.sigma2;
  const MT fa = (MT)(48.0 * c.eps * sig6 * sig6), fb = (MT)(24.0 * c.eps * sig6);
  double scale = out.scale;
  if (out.scale_dev) scale *= *out.scale_dev;
  double e = 0.0, w = 0.0, ke = 0.0, vmax2 = 0.0;
  // two lanes per particle, each taking every other list word (more waves in flight)
  constexpr int LPP = 2;
  const int part = (int)threadIdx.x % LPP;
  for (int s = s0 + (int)threadIdx.x / LPP; s < s1; s += (int)blockDim.x / LPP) {
    const double xi = x[s], yi = y[s], zi = z[s];
    // velocities for the fused kick: the plain pass loads them early so that
    // the pair loop hides the latency; the energy pass, short of registers,
    // after the loop
    double vxi = 0.0, vyi = 0.0, vzi = 0.0;
    if (!ENERGY && out.fuse && part == 0) {
      vxi = out.vx[s];
      vyi = out.vy[s];
      vzi = out.vz[s];
    }
    const int ngroups = (tl.cnt[s] + 3) >> 2;
    const uint64_t* __restrict__ col = tl.nbr + s;
    double ax = 0.0, ay = 0.0, az = 0.0, ei = 0.0;
    uint64_t next = part < ngroups ? col[(int64_t)part * tl.stride] : 0;
    for (int gi = part; gi < ngroups; gi += LPP) {
      const uint64_t word = next;
      if (gi + LPP < ngroups) next = col[(int64_t)(gi + LPP) * tl.stride];
      // FP32 plain pass: entry k + 1's tile position is read while entry k is
      // computed (the other variants have no registers to spare for it)
      constexpr bool kAhead = !ENERGY && sizeof(MT) == 4;
      double qx, qy, qz;
      auto tile_pos = [&](int k) {
        // entry: the slot's byte offset in the 16-byte x-y pairs; half of it
        // in the 8-byte arrays
        const unsigned off = (unsigned)(word >> (16 * k)) & 0xffffu;
        const unsigned off8 = (unsigned)(word >> (16 * k + 1)) & 0x7fffu;
        if constexpr (ENERGY) {
          qx = *(const double*)((const char*)t.x + off8);
          qy = *(const double*)((const char*)t.y + off8);
        } else {
          const double2 q = *(const double2*)((const char*)t.xy + off);
          qx = q.x;
          qy = q.y;
        }
        qz = *(const double*)((const char*)t.z + off8);
      };
      tile_pos(0);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (!kAhead && k > 0) tile_pos(k);
        const double dx = xi - qx, dy = yi - qy, dz = zi - qz;
        if (kAhead && k < 3) tile_pos(k + 1);
        double g;
        if (ENERGY) {
          // pair energy and virial in FP64 on the sampled steps
          const double d2 = sq_sum(dx, dy, dz);
          const bool in = d2 < c.rc2;
          // reciprocal: hardware estimate and two Newton steps (a few ulp)
          double inv = __builtin_amdgcn_rcp(d2);
          inv = __builtin_fma(inv, __builtin_fma(-d2, inv, 1.0), inv);
          inv = __builtin_fma(inv, __builtin_fma(-d2, inv, 1.0), inv);
          const double s2 = c.sigma2 * inv;
          const double s6 = s2 * s2 * s2;
          const double gg = 48.0 * c.eps * inv * s6 * (s6 - 0.5);
          const double v = 4.0 * c.eps * (s6 * s6 - s6) + c.shift_v;
          g = in ? gg : 0.0;
          ei += in ? 0.5 * v : 0.0;
          w += 0.5 * g * d2;
        } else {
          const double d2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
          const bool in = d2 < c.rc2;
          MT inv;
          if constexpr (sizeof(MT) == 4) {
            // outside the cutoff the reciprocal of FLT_MAX drives the factor to zero
            inv = __builtin_amdgcn_rcpf(in ? (float)d2 : 3.0e38f);
          } else {
            inv = 1.0 / d2;
          }
          const MT x2 = inv * inv;
          MT gg = (x2 * x2) * (fa * (x2 * inv) - fb);
          if constexpr (sizeof(MT) != 4) gg = in ? gg : (MT)0;
          g = (double)gg;
        }
        ax = __builtin_fma(g, dx, ax);
        ay = __builtin_fma(g, dy, ay);
        az = __builtin_fma(g, dz, az);
      }
    }
    if (LPP == 2) {
      ax += __shfl_xor(ax, 1, 64);
      ay += __shfl_xor(ay, 1, 64);
      az += __shfl_xor(az, 1, 64);
      if (ENERGY) ei += __shfl_xor(ei, 1, 64);
      if (part) continue;
    }
    if (out.fuse) {
      if (ENERGY) {
        vxi = out.vx[s];
        vyi = out.vy[s];
        vzi = out.vz[s];
      }
      // the kicks use the force as stored (rounded to OT), like k_vv
      double m2;
      ke += fused_kick(out, s, xi, yi, zi, vxi, vyi, vzi, (double)(OT)(ax * scale),
                       (double)(OT)(ay * scale), (double)(OT)(az * scale), m2);
      vmax2 = m2 > vmax2 ? m2 : vmax2;
      if (ENERGY) e += ei;
      continue;
    }
    const int64_t o = out.scatter ? (int64_t)out.scatter[s] : (int64_t)s;
    ((OT*)out.fx)[o] = (OT)(ax * scale);
    ((OT*)out.fy)[o] = (OT)(ay * scale);
    ((OT*)out.fz)[o] = (OT)(az * scale);
    if (ENERGY) {
      if (out.e_atom) out.e_atom[o] = ei;
      e += ei;
    }
  }
  if (out.fuse && out.track.ring) block_track(out.track, vmax2, vred);
  if (ENERGY) {
    // brick sums: wave butterflies, then the wave sums in order
    e = wave_sum(e);
    w = wave_sum(w);
    ke = wave_sum(ke);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
      red[wave] = e;
      red[16 + wave] = w;
      red[32 + wave] = ke;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const int nw = (blockDim.x + 63) >> 6;
      double pe = 0.0, ww = 0.0, kk = 0.0;
      for (int k = 0; k < nw; ++k) {
        pe += red[k];
        ww += red[16 + k];
        kk += red[32 + k];
      }
      if (out.fuse) {
        out.partials[3 * brick] = pe;
        out.partials[3 * brick + 1] = ww;
        out.partials[3 * brick + 2] = kk;
      } else {
        out.partials[2 * brick] = pe;
        out.partials[2 * brick + 1] = ww;
      }
    }
  }
}

template <typename MT, typename OT>
static void launch_force(bool energy, hipStream_t st, const double* x, const double* y,
                         const double* z, const int32_t* cs, const Grid& g, const TileList& tl,
                         const LJConst& c, const ForceOut& out) {
  const dim3 grid(tile_grid(g));
  const unsigned two = 2 * tl.threads < 1024 ? 2 * tl.threads : 1024;
  if (energy)
    hipLaunchKernelGGL((k_lj_force<MT, OT, true>), grid, dim3(two), 0, st, x, y, z, cs, g, tl, c, out);
  else
    hipLaunchKernelGGL((k_lj_force<MT, OT, false>), grid, dim3(two), 0, st, x, y, z, cs, g, tl, c,
                       out);
}

hipError_t lj_force(const double* x, const double* y, const double* z, const int32_t* cell_start,
                    const Grid& g, const TileList& tl, const LJConst& c, int precision, bool energy,
                    const ForceOut& out, int64_t n, hipStream_t st, int* nblocks_out) {
  if (nblocks_out) *nblocks_out = g.nbricks;
  if (tl.cells) return lj_force_cells(x, y, z, cell_start, g, c, precision, energy, out, st);
  if (tl.half) return lj_force_half(x, y, z, cell_start, g, tl, c, precision, energy, out, n, st);
  // precision: 0 FP64 math/double out, 1 FP32 math/float out,
  //            2 FP64 math/double out (backward), 3 FP32 math/double out (backward)
  switch (precision) {
    case 0:
    case 2:
      launch_force<double, double>(energy, st, x, y, z, cell_start, g, tl, c, out);
      break;
    case 1:
      launch_force<float, float>(energy, st, x, y, z, cell_start, g, tl, c, out);
      break;
    default:
      launch_force<float, double>(energy, st, x, y, z, cell_start, g, tl, c, out);
      break;
  }
  return hipGetLastError();
}

}  // namespace mdpl
