// Lennard-Jones pair loop with full neighbour lists (the default pair loop).
//
// Force (Eq. LJforce): f_ij = 48 eps [(s^2/d2)^7 - 1/2 (s^2/d2)^4] / s^2 * dr_ij,
// dr_ij = r_i - r_j (min image), summed over the neighbour list of i and
// written once per particle (gather only, no atomics: the paper's choice of
// looping over all ordered pairs and writing to the first particle, Sec. 2).
// Each workgroup handles one brick of cells and stages its neighbourhood (the
// tile, tile.h) in LDS; a list entry is 16 times the partner's tile slot.
//
// FP32 mode (k_lj_force32): the tile holds FP32 coordinates relative to the
// tile centre (one 16-byte gather per entry) and the whole pair loop is
// FP32; pairs whose FP32 squared distance falls in a narrow band around rc^2
// are classified by the FP64 test instead (see the derivation there).
// Forces are stored as FP32.  Energy and virial (sampled steps) are formed
// per pair in FP64 from the FP64 image positions and reduced per block with
// wavefront shuffles into FP64 partials; a single-block pass sums the
// partials in a fixed order, so results are reproducible run to run.  The
// energy pass computes its forces with the plain pass's FP32 arithmetic, so
// sampling a step leaves the trajectory unchanged.
//
// FP64 mode (k_lj_force<double, ...>): FP64 image positions in the tile, the
// uncontracted squared distance of the definition, the reciprocal by
// estimate and Newton steps; the plain and the energy pass share the pair
// arithmetic.  The cutoff test uses the FP64 separation of the image
// positions, so a pair can be classified differently from the definition
// only within a few units in the last place of rc^2.
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

// FP64 pair arithmetic of the FP64 passes (one definition, so that their
// plain and energy passes give the same forces): the reciprocal of d2 by the hardware
// estimate and two Newton steps (a few ulp), s6 = (s^2/d2)^3 and the force
// factor f/dr = 48 eps s6 (s6 - 1/2) / d2.
__device__ __forceinline__ double lj_inv64(double d2) {
#pragma clang fp contract(off)
  double inv = __builtin_amdgcn_rcp(d2);
  inv = __builtin_fma(inv, __builtin_fma(-d2, inv, 1.0), inv);
  inv = __builtin_fma(inv, __builtin_fma(-d2, inv, 1.0), inv);
  return inv;
}
__device__ __forceinline__ double lj_g64(double inv, const LJConst& c, double& s6) {
#pragma clang fp contract(off)
  const double s2 = c.sigma2 * inv;
  s6 = s2 * s2 * s2;
  return 48.0 * c.eps * inv * s6 * (s6 - 0.5);
}
__device__ __forceinline__ double lj_v64(double s6, const LJConst& c) {
#pragma clang fp contract(off)
  return 4.0 * c.eps * (s6 * s6 - s6) + c.shift_v;
}

// Largest |v|^2 of the workgroup (v2 per thread, 0 where none) to the rule's
// tracking; one barrier.
__device__ __forceinline__ void block_track(const KickTrack& kt, double v2, double* sh) {
  v2 = wave_max_nonneg(v2);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v2;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    double m = sh[0];
    for (int k = 1; k < nw; ++k) m = sh[k] > m ? sh[k] : m;
    kick_store(kt, m);
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
  if (out.fuse) kick_publish(out.track, vred);
  const int brick = brick_of_block(g);
  if (brick >= g.nbricks) {  // padding workgroup: its (empty) maximum still goes to the rule
    if (out.fuse && threadIdx.x == 0) kick_store(out.track, 0.0);
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
        // entry: 4 x the slot; the byte offset in the 16-byte x-y pairs is
        // four times it, in the 8-byte arrays twice
        const unsigned e = (unsigned)(word >> (16 * k)) & 0xffffu;
        const unsigned off = e << 2, off8 = e << 1;
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
          double s6;
          const double gg = lj_g64(lj_inv64(d2), c, s6);
          g = in ? gg : 0.0;
          ei += in ? 0.5 * lj_v64(s6, c) : 0.0;
          w += 0.5 * g * d2;
        } else if constexpr (sizeof(MT) == 8) {
          // the energy pass's force factor (same operations)
          const double d2 = sq_sum(dx, dy, dz);
          double s6;
          const double gg = lj_g64(lj_inv64(d2), c, s6);
          g = d2 < c.rc2 ? gg : 0.0;
        } else {
          const double d2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
          const bool in = d2 < c.rc2;
          // outside the cutoff the reciprocal of FLT_MAX drives the factor to zero
          const MT inv = __builtin_amdgcn_rcpf(in ? (float)d2 : 3.0e38f);
          const MT x2 = inv * inv;
          g = (double)((x2 * x2) * (fa * (x2 * inv) - fb));
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

// ------------------------------------------------------------ FP32 path
// Pair forces of the FP32 precision mode from FP32 coordinates relative to
// the centre of the brick's tile: X = fl32((x + k L) - o), |X| below
// (B/2 + 1) cell sides.  A pair's separation is the FP32 difference of two
// such values, so the pair loop needs no FP64 arithmetic: one 16-byte LDS
// gather, three FP32 differences, the squared distance, the reciprocal and
// the force factor x^4 (A x^3 - B), x = 1/d2, accumulated in FP32.
//
// Cutoff classification.  The FP32 squared distance d2f of a pair is within
// e of the FP64 one formed from the image positions (bound derived in
// lj_force32_band), so d2f < rc^2 - band and d2f >= rc^2 + band decide the
// pair as the FP64 test would.  A particle with an entry between the two
// (about one in a thousand) walks its list again with the exact rule: for
// such entries the FP64 test on the image separation, the same as in the
// energy pass.  Both passes therefore include the same pairs and, sharing
// the FP32 force arithmetic and the order of the sums, give bit-identical
// forces: a sampled step does not perturb the trajectory.
struct F32Const {
  float fa, fb;      // 48 eps s^12, 24 eps s^6
  float r2lo, r2hi;  // rc^2 -/+ band, rounded outward
};

// FP32 force factor f/dr of a pair: in selects the pair (the reciprocal of
// FLT_MAX drives the factor of an excluded pair to zero).
__device__ __forceinline__ float lj_g32(float d2f, bool in, float fa, float nfb) {
#pragma clang fp contract(off)
  const float inv = __builtin_amdgcn_rcpf(in ? d2f : 3.0e38f);
  const float x2 = inv * inv;
  return (x2 * x2) * __builtin_fmaf(fa, x2 * inv, nfb);
}
__device__ __forceinline__ float lj_g32(float d2f, bool in, const F32Const& k) {
  return lj_g32(d2f, in, k.fa, -k.fb);
}

__device__ __forceinline__ float d2_32(float dx, float dy, float dz) {
  return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
}

// FP64 squared distance of the exact rule: the particle's stored position
// minus the image position of the partner (the energy pass forms it from
// the same values).
__device__ __forceinline__ double d2_image(double xs, double ys, double zs, double qx, double qy,
                                           double qz) {
  return sq_sum(xs - qx, ys - qy, zs - qz);
}

// FP64 image position of tile slot u (its cell found by a search over the
// tile's prefix).
template <typename TS>
__device__ __forceinline__ void slot_image(const TS& t, const Grid& g, const double* __restrict__ x,
                                           const double* __restrict__ y,
                                           const double* __restrict__ z, int u, double& qx,
                                           double& qy, double& qz) {
  const int lo = tile_cell_of(t, (g.B[0] + 2) * (g.B[1] + 2) * (g.B[2] + 2), u);
  const int src = t.src[lo] + (u - t.prefix[lo]);
  const int code = t.code[lo];
  qx = image_coord(x[src], code & 3, g.box[0]);
  qy = image_coord(y[src], (code >> 2) & 3, g.box[1]);
  qz = image_coord(z[src], (code >> 4) & 3, g.box[2]);
}

// Lane groups of the FP32 pair loops, shared by the plain and the energy
// pass so that both sum a particle's pairs in the same order.  The brick's
// particles are taken in passes of kGroupWidth/2 with two lanes each; a
// last, partial pass of m particles gives each T lanes, T the largest power
// of two up to 16 with m T <= kGroupWidth, so that a few leftover particles
// do not hold the workgroup for a whole pass.  Lane p of a group takes the
// list words p, p + T, p + 2T, ...; the group's sums are combined by
// butterflies.  A pass has kGroupWidth lane slots, which a workgroup of
// fewer threads runs in turns (slot t on thread t mod blockDim, the same
// lane of a wave, since blockDim is a multiple of 64).
constexpr int kGroupWidth = 1024;
struct LaneGroup {
  int la;    // particle index from the brick's first slot
  int part;  // lane within the group
  int T;     // lanes per particle
};
__device__ __forceinline__ int lane_group_T(int m) {
  int T = 16;
  while (T > 2 && m * T > kGroupWidth) T >>= 1;
  return T;
}
// Lanes per particle of the pass starting at particle p0 (m of its particles).
__device__ __forceinline__ int lane_pass_T(int p0, int npart, int& m) {
  constexpr int half = kGroupWidth >> 1;
  m = npart - p0 < half ? npart - p0 : half;
  return m == half ? 2 : lane_group_T(m);
}
// Group of lane slot t in the pass starting at particle p0; false if none.
__device__ __forceinline__ bool lane_group(int p0, int npart, int t, LaneGroup& lg) {
  int m;
  const int T = lane_pass_T(p0, npart, m);
  if (t >= m * T) return false;
  lg.la = p0 + t / T;
  lg.part = t % T;
  lg.T = T;
  return true;
}
template <typename V>
__device__ __forceinline__ V group_sum(V v, int T) {
  // butterflies: lane ^ 1 and lane ^ 2 on DPP, wider ones through LDS
  if (T > 1) v += dpp_move<0xB1>(v);
  if (T > 2) v += dpp_move<0x4E>(v);
  for (int off = 4; off < T; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Workgroup size of the plain FP32 pass (its LDS fits three workgroups per CU).
#ifndef MDPL_PLAIN_THREADS
#define MDPL_PLAIN_THREADS 512
#endif
constexpr int kPlainThreads = MDPL_PLAIN_THREADS;

// Plain FP32 pass: the pair loop of every particle of the brick (its own
// coordinates from its tile slot); the lanes of a wave take the same number
// of trips, so the band test of an entry costs one comparison and the flags
// of the wave are one scalar mask; a group with an entry in the band walks
// its list again with the exact rule.  The group's first lane then stores
// the force or applies the fused kick-kick-drift at once, so the kick's
// memory traffic overlaps the pair loops of the other waves instead of
// following them after a workgroup barrier (none of the FP64 state of the
// kick is live in the pair loop).
template <typename OT>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8)))
void k_lj_force32_plain(const double* __restrict__ x, const double* __restrict__ y,
                        const double* __restrict__ z, const int32_t* __restrict__ cs, Grid g,
                        TileList tl, LJConst c, F32Const k, ForceOut out) {
  __shared__ TileF32 t;
  __shared__ uint16_t home[kBrickMax];
  __shared__ double vred[16];
  if (out.fuse) kick_publish(out.track, vred);
  const int brick = brick_of_block(g);
  if (brick >= g.nbricks) {  // padding workgroup: its (empty) maximum still goes to the rule
    if (out.fuse && threadIdx.x == 0) kick_store(out.track, 0.0);
    return;
  }
  // the tile tables as the list build left them
  const int total = tile_tables_load(g, tl.tab + (int64_t)brick * kTabInts, t);
  const int s0 = cs[brick * g.V], s1 = cs[(brick + 1) * g.V];
  const int npart = s1 - s0 < kBrickMax ? s1 - s0 : kBrickMax;  // more: flagged by the build
  double ox, oy, oz;
  tile_centre(g, brick, ox, oy, oz);
  // The wave's pass and its lanes per particle are the same for all its lanes
  // (blockDim and kGroupWidth are multiples of 64), so they live in scalar
  // registers; every lane of the wave takes the same number of trips (the
  // wave's longest list part, lanes past their own part read the dummy
  // word), so that the band flags of a trip are one wave mask.
  const int lane = (int)threadIdx.x & 63;
  const int wbase = __builtin_amdgcn_readfirstlane((int)threadIdx.x & ~63);
  constexpr uint64_t kDummyWord = 0x0001000100010001ull * (uint64_t)(4 * TileF32::kDummy);
  // the count and first list word of the wave's first pass, loaded before
  // the tile so that their latency overlaps the tile's
  int cnt0 = 0;
  uint64_t word0 = 0;
  {
    const int p0 = (wbase / kGroupWidth) * (kGroupWidth >> 1);
    if (p0 < npart) {
      int m;
      const int T = lane_pass_T(p0, npart, m);
      const int tt = wbase % kGroupWidth + lane;
      const int part = tt & (T - 1);
      if (tt < m * T) {
        const int s = s0 + p0 + tt / T;
        cnt0 = tl.cnt[s];
        if (4 * part < tl.max_nb) word0 = tl.nbr[s + (int64_t)part * tl.stride];
      }
    }
  }
  tile_load_f32(g, x, y, z, total, ox, oy, oz, s0, t, home);
  double scale = out.scale;
  if (out.scale_dev) scale *= *out.scale_dev;
  double vmax2 = 0.0;
  for (int base = wbase;; base += blockDim.x) {
    const int p0 = (base / kGroupWidth) * (kGroupWidth >> 1);
    if (p0 >= npart) break;
    int m;
    const int T = lane_pass_T(p0, npart, m);
    const int sh = __builtin_ctz(T);
    const int tt = base % kGroupWidth + lane;
    const bool has = tt < m * T;
    const int la = has ? p0 + (tt >> sh) : 0;
    const int part = tt & (T - 1);
    const int s = s0 + la;
    const int hu = home[la];
    const float xi = t.px[hu], yi = t.py[hu], zi = t.pz[hu];
    const bool first = base == wbase;
    const int ngroups = has ? ((first ? cnt0 : tl.cnt[s]) + 3) >> 2 : 0;
    const int trips = ngroups > part ? (ngroups - part + T - 1) >> sh : 0;
    const int wtrips = wave_max_nonneg(trips);
    const uint64_t* __restrict__ col = tl.nbr + s;
    const int64_t step = (int64_t)T * tl.stride;
    float ax = 0.0f, ay = 0.0f, az = 0.0f;
    uint64_t bandm = 0;  // lanes with an entry in the band
    // -fb in a vector register for the whole loop (an FMA takes one scalar
    // operand, fa); the zero product keeps the compiler from folding it back
    const float nfb = __builtin_fmaf(0.0f, xi, -k.fb);
    auto pair = [&](unsigned e) {
      // e: 4 x the partner's slot, its byte offset in the three arrays
      const float dx = xi - *(const float*)((const char*)t.px + e);
      const float dy = yi - *(const float*)((const char*)t.py + e);
      const float dz = zi - *(const float*)((const char*)t.pz + e);
      const float d2f = d2_32(dx, dy, dz);
      const bool lo = d2f < k.r2lo, hi = d2f < k.r2hi;
      // the band (r2lo <= d2f < r2hi) as wave masks of the two comparisons
      bandm |= __builtin_amdgcn_ballot_w64(hi) & ~__builtin_amdgcn_ballot_w64(lo);
      const float gf = lj_g32(d2f, lo, k.fa, nfb);
      ax = __builtin_fmaf(gf, dx, ax);
      ay = __builtin_fmaf(gf, dy, ay);
      az = __builtin_fmaf(gf, dz, az);
    };
    // one word (four entries) per trip; the next trip's word is loaded
    // while this one's entries are computed
    const uint64_t* __restrict__ p = col + (int64_t)part * tl.stride;
    uint64_t next = 0;
    if (trips > 0) next = first ? word0 : *p;
    for (int q = 0; q < wtrips; ++q) {
      // a lane past its own part reads the dummy slot (no force, no band)
      const uint64_t word = q < trips ? next : kDummyWord;
      p += step;
      if (q + 1 < trips) next = *p;
#pragma unroll
      for (int j = 0; j < 4; ++j) pair((unsigned)(word >> (16 * j)) & 0xffffu);
    }
    // an entry in the band: the group walks again with the exact rule
    if ((bandm >> (lane & ~(T - 1))) & ((1ull << T) - 1)) {
      const double xr = x[s], yr = y[s], zr = z[s];
      ax = ay = az = 0.0f;
      for (int gi = part; gi < ngroups; gi += T) {
        const uint64_t word = col[(int64_t)gi * tl.stride];
        for (int j = 0; j < 4; ++j) {
          const unsigned u = (unsigned)(word >> (16 * j + kFullShift)) & 0x3fffu;
          const float dx = xi - t.px[u], dy = yi - t.py[u], dz = zi - t.pz[u];
          const float d2f = d2_32(dx, dy, dz);
          const bool lo = d2f < k.r2lo, hi = d2f < k.r2hi;
          bool in = lo;
          if (lo != hi && u != (unsigned)TileF32::kDummy) {
            double qx, qy, qz;
            slot_image(t, g, x, y, z, (int)u, qx, qy, qz);
            in = d2_image(xr, yr, zr, qx, qy, qz) < c.rc2;
          }
          const float gf = lj_g32(d2f, in, k);
          ax = __builtin_fmaf(gf, dx, ax);
          ay = __builtin_fmaf(gf, dy, ay);
          az = __builtin_fmaf(gf, dz, az);
        }
      }
    }
    ax = group_sum(ax, T);
    ay = group_sum(ay, T);
    az = group_sum(az, T);
    if (has && part == 0) {
      // the kicks use the force as stored (rounded to OT), like k_vv
      const OT fx = (OT)((double)ax * scale);
      const OT fy = (OT)((double)ay * scale);
      const OT fz = (OT)((double)az * scale);
      if (out.fuse) {
        double m2;
        (void)fused_kick(out, s, x[s], y[s], z[s], out.vx[s], out.vy[s], out.vz[s], (double)fx,
                         (double)fy, (double)fz, m2);
        vmax2 = m2 > vmax2 ? m2 : vmax2;
      } else {
        const int64_t o = out.scatter ? (int64_t)out.scatter[s] : (int64_t)s;
        ((OT*)out.fx)[o] = fx;
        ((OT*)out.fy)[o] = fy;
        ((OT*)out.fz)[o] = fz;
      }
    }
  }
  if (out.fuse && out.track.ring) block_track(out.track, vmax2, vred);
}

// s6 = (sigma^2 / d2)^3 in FP64, the reciprocal of d2 by two Newton steps
// from the FP32 reciprocal of d2f that the pair's force factor takes anyway
// (d2f: the FP32 square distance of the same pair).  Each step squares the
// relative error of the seed, about 2^-18 sigma / r from the rounding of the
// tile coordinates, so that the result is as accurate as the hardware FP64
// reciprocal's two steps down to r of about 0.05 sigma (a pair energy of
// 10^16 eps) and still within 2e-14 at 0.01 sigma.  This takes the FP64
// reciprocal, a quarter-rate instruction, out of the energy pass's loop.
__device__ __forceinline__ double lj_s6_seeded(double d2, float seed, const LJConst& c) {
#pragma clang fp contract(off)
  double inv = (double)seed;
  inv = __builtin_fma(inv, __builtin_fma(-d2, inv, 1.0), inv);
  inv = __builtin_fma(inv, __builtin_fma(-d2, inv, 1.0), inv);
  const double s2 = c.sigma2 * inv;
  return s2 * s2 * s2;
}

// Energy FP32 pass: the FP64 image positions in the tile (energy and virial
// are FP64 per pair); the FP32 coordinates of each partner are formed from
// them with the plain tile's conversion, the pairs summed by the same lane
// groups, and every entry classified by the exact rule.  Workgroups of
// kEnergyThreads: two share a CU (LDS: two FP64 tiles) at six waves per SIMD,
// which leaves 80 VGPRs, enough for the pair loop without spills (the
// 1024-thread shape, at 64 VGPRs, spilled ten and ran 5 % slower).
constexpr int kEnergyThreads = 768;
template <typename OT>
__global__ __launch_bounds__(kEnergyThreads) __attribute__((amdgpu_waves_per_eu(6)))
void k_lj_force32_energy(const double* __restrict__ x, const double* __restrict__ y,
                         const double* __restrict__ z, const int32_t* __restrict__ cs, Grid g,
                         TileList tl, LJConst c, F32Const k, ForceOut out) {
  __shared__ TileShared t;
  __shared__ double red[48];  // up to 16 waves: e, w, ke
  __shared__ double vred[16];
  if (out.fuse) kick_publish(out.track, vred);
  const int brick = brick_of_block(g);
  if (brick >= g.nbricks) {
    if (out.fuse && threadIdx.x == 0) kick_store(out.track, 0.0);
    return;
  }
  // the tile tables as the list build left them
  const int total = tile_tables_load(g, tl.tab + (int64_t)brick * kTabInts, t);
  double ox, oy, oz;
  tile_centre(g, brick, ox, oy, oz);
  tile_load_f64_cells(g, x, y, z, total, t);
  const int s0 = cs[brick * g.V], s1 = cs[(brick + 1) * g.V];
  const int npart = s1 - s0 < kBrickMax ? s1 - s0 : kBrickMax;
  double scale = out.scale;
  if (out.scale_dev) scale *= *out.scale_dev;
  double e = 0.0, w = 0.0, ke = 0.0, vmax2 = 0.0;
  const double w24 = 24.0 * c.eps, e2 = 2.0 * c.eps, hshift = 0.5 * c.shift_v;
  for (int slot = threadIdx.x; slot < npart * 2 + kGroupWidth; slot += blockDim.x) {
    const int p0 = (slot / kGroupWidth) * (kGroupWidth >> 1);
    if (p0 >= npart) break;
    LaneGroup lg;
    if (!lane_group(p0, npart, slot % kGroupWidth, lg)) continue;
    const int s = s0 + lg.la;
    const double xs = x[s], ys = y[s], zs = z[s];
    const float xi = rel32(xs, ox), yi = rel32(ys, oy), zi = rel32(zs, oz);
    const int ngroups = (tl.cnt[s] + 3) >> 2;
    const uint64_t* __restrict__ col = tl.nbr + s;
    float ax = 0.0f, ay = 0.0f, az = 0.0f;
    double s12 = 0.0, s6s = 0.0;  // sums of s6^2 and s6 over the pairs in range
    int nin = 0;                  // and their number
    for (int gi = lg.part; gi < ngroups; gi += lg.T) {
      const uint64_t word = col[(int64_t)gi * tl.stride];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        // entry: 4 x the partner's slot; twice it in the 8-byte arrays
        const unsigned off8 = ((unsigned)(word >> (16 * m)) & 0xffffu) << 1;
        const double qx = *(const double*)((const char*)t.x + off8);
        const double qy = *(const double*)((const char*)t.y + off8);
        const double qz = *(const double*)((const char*)t.z + off8);
        const float dx = xi - rel32(qx, ox);
        const float dy = yi - rel32(qy, oy);
        const float dz = zi - rel32(qz, oz);
        const float d2f = d2_32(dx, dy, dz);
        const double d2 = d2_image(xs, ys, zs, qx, qy, qz);
        const bool lo = d2f < k.r2lo, hi = d2f < k.r2hi;
        const bool in = lo != hi ? d2 < c.rc2 : lo;
        // the FP32 force factor, then s6 in FP64 from the same reciprocal
        // (zero for an entry out of range); the pair energies and virial
        // terms follow from the sums of s6^2 and s6 after the loop
        const float gf = lj_g32(d2f, in, k);
        const double s6r = lj_s6_seeded(d2, __builtin_amdgcn_rcpf(in ? d2f : 3.0e38f), c);
        const double s6 = in ? s6r : 0.0;
        s12 = __builtin_fma(s6, s6, s12);
        s6s += s6;
        nin += in ? 1 : 0;
        ax = __builtin_fmaf(gf, dx, ax);
        ay = __builtin_fmaf(gf, dy, ay);
        az = __builtin_fmaf(gf, dz, az);
      }
    }
    // the lane's pair energies, half of each pair's 4 eps (s6^2 - s6) + shift,
    // and its virial terms, half of each pair's r f(r) = 48 eps (s6^2 - s6/2)
    w = __builtin_fma(w24, __builtin_fma(-0.5, s6s, s12), w);
    double ei = __builtin_fma(e2, s12 - s6s, hshift * (double)nin);
    ax = group_sum(ax, lg.T);
    ay = group_sum(ay, lg.T);
    az = group_sum(az, lg.T);
    ei = group_sum(ei, lg.T);
    if (lg.part != 0) continue;
    const OT fx = (OT)((double)ax * scale);
    const OT fy = (OT)((double)ay * scale);
    const OT fz = (OT)((double)az * scale);
    e += ei;
    if (out.fuse) {
      double m2;
      ke += fused_kick(out, s, xs, ys, zs, out.vx[s], out.vy[s], out.vz[s], (double)fx, (double)fy,
                       (double)fz, m2);
      vmax2 = m2 > vmax2 ? m2 : vmax2;
      continue;
    }
    const int64_t o = out.scatter ? (int64_t)out.scatter[s] : (int64_t)s;
    ((OT*)out.fx)[o] = fx;
    ((OT*)out.fy)[o] = fy;
    ((OT*)out.fz)[o] = fz;
    if (out.e_atom) out.e_atom[o] = ei;
  }
  if (out.fuse && out.track.ring) block_track(out.track, vmax2, vred);
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
    for (int q = 0; q < nw; ++q) {
      pe += red[q];
      ww += red[16 + q];
      kk += red[32 + q];
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

// The band of the FP32 classification.  A tile coordinate |X| < M = 2^p
// (M above (B/2 + 1) cell sides) is within 2^(p-25) of its FP64 value
// (whose own rounding, ~1e-14, is covered by the factor below); an FP32
// difference of a pair near the cutoff, below rc (1 + e) <= 2^q, is rounded
// within 2^(q-25).  So
// each separation component is within D = 2^(p-24) + 2^(q-25) of the FP64
// one, and the FP32 squared distance of a pair near the cutoff within
// e = 2 sqrt(3) rc D + 3 D^2 + 3 2^-24 rc^2 (three rounded operations).  The
// band is 4 e.
static F32Const f32_const(const Grid& g, const LJConst& c) {
  F32Const k;
  const double sig6 = c.sigma2 * c.sigma2 * c.sigma2;
  k.fa = (float)(48.0 * c.eps * sig6 * sig6);
  k.fb = (float)(24.0 * c.eps * sig6);
  double m = 0.0;
  for (int a = 0; a < 3; ++a) {
    const double h = (0.5 * g.B[a] + 1.0) * (g.box[a] / g.nc[a]);
    m = h > m ? h : m;
  }
  const double ulp = 1.0 / 16777216.0;  // 2^-24
  const double pm = exp2(ceil(log2(m * (1.0 + 1e-9))));
  const double rc = sqrt(c.rc2);
  const double pr = exp2(ceil(log2(rc * (1.0 + 1e-6))));
  const double d = pm * ulp + 0.5 * pr * ulp;
  const double err = 2.0 * sqrt(3.0) * rc * d + 3.0 * d * d + 3.0 * ulp * c.rc2;
  const double band = 4.0 * err;
  k.r2lo = nextafterf((float)(c.rc2 - band), 0.0f);
  k.r2hi = nextafterf((float)(c.rc2 + band), 3.0e38f);
  return k;
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
    case 1: {
      const F32Const k = f32_const(g, c);
      const dim3 grid(tile_grid(g));
      if (energy)
        hipLaunchKernelGGL((k_lj_force32_energy<float>), grid, dim3(kEnergyThreads), 0, st, x, y, z,
                           cell_start, g, tl, c, k, out);
      else
        hipLaunchKernelGGL((k_lj_force32_plain<float>), grid, dim3(kPlainThreads), 0, st, x, y, z,
                           cell_start, g, tl, c, k, out);
      break;
    }
    default:
      launch_force<float, double>(energy, st, x, y, z, cell_start, g, tl, c, out);
      break;
  }
  return hipGetLastError();
}

}  // namespace mdpl
