// The two other pair loops of the LJ path (the default, full lists, is in
// lj.hip): half lists with Newton's third law and the list-free loop over
// the cell stencil.  Both compute the pair force of Eq. LJforce exactly as
// the full-list pass does; they differ in how pairs are found and summed.
#include "device_util.h"
#include "internal.h"
#include "tile.h"

namespace mdpl {

// ------------------------------------------------------------ half lists
// Newton's third law: each pair is listed once (see the list builder), its
// force is added to the listing particle i in registers and subtracted from
// j in an LDS accumulator of j's tile slot.  When the brick is done, every
// brick particle's own sum and every tile slot's accumulator (periodic
// images map to their particle) are added to the outputs with device-scope
// atomics, so the outputs must be zero beforehand and a force is complete
// only when the pass has ended; the order of the additions, hence the last
// bits of the result, varies from run to run.  PE and the virial count each
// pair once; e_atom gives half of V to each particle (EATOM).
//
// Accumulators: FP32 atomic adds in LDS are several times slower on this
// chip than integer ones, so the FP32 pass sums the reactions as 64-bit
// integers in units of 2^-32 (exact integer sums, finer than FP32); a pair
// force component of 2^19 or more bypasses them and goes to the output
// directly.  The FP64 pass sums in double.
template <typename MT>
struct HalfAcc {  // LDS accumulator of the reactions (see above)
  using T = unsigned long long;
  static __device__ __forceinline__ bool fits(double v) { return fix_fits(v); }
  static __device__ __forceinline__ void add(T* a, double v) { atomicAdd(a, fix_of(v)); }
  static __device__ __forceinline__ double get(T a) { return fix_value(a); }
};
template <>
struct HalfAcc<double> {
  using T = double;
  static __device__ __forceinline__ bool fits(double) { return true; }
  static __device__ __forceinline__ void add(T* a, double v) { atomicAdd(a, v); }
  static __device__ __forceinline__ double get(T a) { return a; }
};

template <typename MT, typename OT, bool ENERGY, bool EATOM>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8)))
void k_lj_force_half(const double* __restrict__ x, const double* __restrict__ y,
                     const double* __restrict__ z, const int32_t* __restrict__ cs, Grid g,
                     TileList tl, LJConst c, ForceOut out) {
  using A = HalfAcc<MT>;
  __shared__ TileHalf t;
  __shared__ typename A::T acc[3][kTileMaxHalf];
  __shared__ double acce[EATOM ? kTileMaxHalf : 1];
  __shared__ double red[32];  // up to 16 waves: e, w
  const int brick = brick_of_block(g);
  if (brick >= g.nbricks) return;
  const int total = tile_cells(g, brick, cs, t, true);
  const int nt = total < TileHalf::kCap ? total : TileHalf::kCap;
  for (int u = threadIdx.x; u < kTileMaxHalf; u += blockDim.x) {
    acc[0][u] = 0;
    acc[1][u] = 0;
    acc[2][u] = 0;
    if (EATOM) acce[u] = 0.0;
  }
  tile_load<true>(g, x, y, z, total, t);  // ends with a barrier
  const int s0 = cs[brick * g.V], s1 = cs[(brick + 1) * g.V];
  const double sig6 = c.sigma2 * c.sigma2 * c.sigma2;
  const MT fa = (MT)(48.0 * c.eps * sig6 * sig6), fb = (MT)(24.0 * c.eps * sig6);
  double scale = out.scale;
  if (out.scale_dev) scale *= *out.scale_dev;
  OT* const fx = (OT*)out.fx;
  OT* const fy = (OT*)out.fy;
  OT* const fz = (OT*)out.fz;
  double e = 0.0, w = 0.0;
  constexpr int LPP = 2;
  const int part = (int)threadIdx.x % LPP;
  for (int s = s0 + (int)threadIdx.x / LPP; s < s1; s += (int)blockDim.x / LPP) {
    const double xi = x[s], yi = y[s], zi = z[s];
    const int ngroups = (tl.cnt[s] + 3) >> 2;
    const uint64_t* __restrict__ col = tl.nbr + s;
    double ax = 0.0, ay = 0.0, az = 0.0, ei = 0.0;
    uint64_t next = part < ngroups ? col[(int64_t)part * tl.stride] : 0;
    for (int gi = part; gi < ngroups; gi += LPP) {
      const uint64_t word = next;
      if (gi + LPP < ngroups) next = col[(int64_t)(gi + LPP) * tl.stride];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int u = (int)((word >> (16 * k)) & 0xffffu) >> kHalfShift;  // tile slot of j
        const double dx = xi - t.x[u], dy = yi - t.y[u], dz = zi - t.z[u];
        double gd;
        bool in;
        double v = 0.0;
        if (ENERGY) {
          const double d2 = sq_sum(dx, dy, dz);
          in = d2 < c.rc2;
          double inv = __builtin_amdgcn_rcp(d2);
          inv = __builtin_fma(inv, __builtin_fma(-d2, inv, 1.0), inv);
          inv = __builtin_fma(inv, __builtin_fma(-d2, inv, 1.0), inv);
          const double s2 = c.sigma2 * inv;
          const double s6 = s2 * s2 * s2;
          const double gg = 48.0 * c.eps * inv * s6 * (s6 - 0.5);
          v = 4.0 * c.eps * (s6 * s6 - s6) + c.shift_v;
          gd = in ? gg : 0.0;
          v = in ? v : 0.0;
          ei += 0.5 * v;
          e += v;
          w += gd * d2;
        } else {
          const double d2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
          in = d2 < c.rc2;
          MT inv;
          if constexpr (sizeof(MT) == 4) {
            inv = __builtin_amdgcn_rcpf(in ? (float)d2 : 3.0e38f);
          } else {
            inv = 1.0 / d2;
          }
          const MT x2 = inv * inv;
          MT gg = (x2 * x2) * (fa * (x2 * inv) - fb);
          if constexpr (sizeof(MT) != 4) gg = in ? gg : (MT)0;
          gd = (double)gg;
        }
        const double px = gd * dx, py = gd * dy, pz = gd * dz;
        ax += px;
        ay += py;
        az += pz;
        if (in) {  // the reaction on j
          if (A::fits(px) && A::fits(py) && A::fits(pz)) {
            A::add(&acc[0][u], -px);
            A::add(&acc[1][u], -py);
            A::add(&acc[2][u], -pz);
          } else {  // too large for the accumulator: straight to the output
            const int cell = t.cell[u];
            const int slot = t.src[cell] + (u - t.prefix[cell]);
            const int64_t o = out.scatter ? (int64_t)out.scatter[slot] : (int64_t)slot;
            unsafeAtomicAdd(&fx[o], (OT)(-px * scale));
            unsafeAtomicAdd(&fy[o], (OT)(-py * scale));
            unsafeAtomicAdd(&fz[o], (OT)(-pz * scale));
          }
          if (EATOM) atomicAdd(&acce[u], 0.5 * v);
        }
      }
    }
    ax += __shfl_xor(ax, 1, 64);
    ay += __shfl_xor(ay, 1, 64);
    az += __shfl_xor(az, 1, 64);
    if (EATOM) ei += __shfl_xor(ei, 1, 64);
    if (part) continue;
    const int64_t o = out.scatter ? (int64_t)out.scatter[s] : (int64_t)s;
    unsafeAtomicAdd(&fx[o], (OT)(ax * scale));
    unsafeAtomicAdd(&fy[o], (OT)(ay * scale));
    unsafeAtomicAdd(&fz[o], (OT)(az * scale));
    if (EATOM) unsafeAtomicAdd(&out.e_atom[o], ei);
  }
  __syncthreads();
  for (int u = threadIdx.x; u < nt; u += blockDim.x) {
    const double ux = A::get(acc[0][u]), uy = A::get(acc[1][u]), uz = A::get(acc[2][u]);
    const double ue = EATOM ? acce[u] : 0.0;
    if (ux == 0.0 && uy == 0.0 && uz == 0.0 && ue == 0.0) continue;  // never a partner here
    const int cell = t.cell[u];
    const int slot = t.src[cell] + (u - t.prefix[cell]);
    const int64_t o = out.scatter ? (int64_t)out.scatter[slot] : (int64_t)slot;
    unsafeAtomicAdd(&fx[o], (OT)(ux * scale));
    unsafeAtomicAdd(&fy[o], (OT)(uy * scale));
    unsafeAtomicAdd(&fz[o], (OT)(uz * scale));
    if (EATOM) unsafeAtomicAdd(&out.e_atom[o], ue);
  }
  if (ENERGY) {
    e = wave_sum(e);
    w = wave_sum(w);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
      red[wave] = e;
      red[16 + wave] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const int nw = (blockDim.x + 63) >> 6;
      double pe = 0.0, ww = 0.0;
      for (int k = 0; k < nw; ++k) {
        pe += red[k];
        ww += red[16 + k];
      }
      out.partials[2 * brick] = pe;
      out.partials[2 * brick + 1] = ww;
    }
  }
}

// ------------------------------------------------------------ no list
// The pair loop straight from the cell list (Sec. 3.5 without the neighbour
// list): one wave per home cell of the brick; its na particles are spread
// over the 64 lanes as na x K (K = 64 / na) and lane (a, k) visits
// candidates k, k+K, ... of each of the 9 stencil rows (three consecutive
// tile cells, one contiguous range of the tile of FP64 image positions).
// Separations, the cutoff test and the pair force are those of k_lj_force;
// each lane sums its candidates in FP64 and the K partial sums of a
// particle are added in a fixed order with cross-lane reads, so the result
// is reproducible.  A tile over its capacity raises the overflow flag.
template <typename MT, typename OT, bool ENERGY>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8)))
void k_lj_force_cells(const double* __restrict__ x, const double* __restrict__ y,
                      const double* __restrict__ z, const int32_t* __restrict__ cs, Grid g,
                      LJConst c, ForceOut out) {
  __shared__ TileShared t;
  __shared__ double red[32];  // up to 16 waves: e, w
  const int brick = brick_of_block(g);
  if (brick >= g.nbricks) return;
  const int total = tile_cells(g, brick, cs, t);
  if (threadIdx.x == 0 && total > kTileCap) atomicOr(out.flags, MDPL_FLAG_NL_OVERFLOW);
  tile_load<true>(g, x, y, z, total, t);  // ends with a barrier
  const double sig6 = c.sigma2 * c.sigma2 * c.sigma2;
  const MT fa = (MT)(48.0 * c.eps * sig6 * sig6), fb = (MT)(24.0 * c.eps * sig6);
  double scale = out.scale;
  if (out.scale_dev) scale *= *out.scale_dev;
  const int TX = g.B[0] + 2, TXY = TX * (g.B[1] + 2);
  int bx, by, bz;
  brick_coords(g, brick, bx, by, bz);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  double e = 0.0, w = 0.0;
  for (int lc = wave; lc < g.V; lc += nwaves) {
    const int lx = lc % g.B[0], ly = (lc / g.B[0]) % g.B[1], lz = lc / (g.B[0] * g.B[1]);
    // the last brick along an axis may be partial: its missing cells would
    // alias periodic images of another brick's cells
    if (bx * g.B[0] + lx >= g.nc[0] || by * g.B[1] + ly >= g.nc[1] || bz * g.B[2] + lz >= g.nc[2])
      continue;
    const int tc0 = ((lz + 1) * (g.B[1] + 2) + (ly + 1)) * TX + (lx + 1);
    const int ncell = t.prefix[tc0 + 1] - t.prefix[tc0];
    for (int a0 = 0; a0 < ncell; a0 += 64) {
      const int na = ncell - a0 < 64 ? ncell - a0 : 64;
      const int K = 64 / na;
      const int a = a0 + lane % na, k = lane / na;
      const int self = t.prefix[tc0] + a;
      const bool ok = k < K && self < kTileCap;
      const double xi = ok ? t.x[self] : 0.0, yi = ok ? t.y[self] : 0.0, zi = ok ? t.z[self] : 0.0;
      double ax = 0.0, ay = 0.0, az = 0.0, ei = 0.0;
      for (int oz = -1; oz <= 1; ++oz) {
        for (int oy = -1; oy <= 1; ++oy) {
          const int tcl = tc0 + oz * TXY + oy * TX - 1;
          int ue = t.prefix[tcl + 3];
          ue = ue < kTileCap ? ue : kTileCap;
          if (!ok) ue = 0;
#pragma unroll 4
          for (int u = t.prefix[tcl] + k; u < ue; u += K) {
            const double dx = xi - t.x[u], dy = yi - t.y[u], dz = zi - t.z[u];
            double gd;
            if (ENERGY) {
              const double d2 = sq_sum(dx, dy, dz);
              const bool in = d2 < c.rc2 && u != self;
              double inv = __builtin_amdgcn_rcp(d2);
              inv = __builtin_fma(inv, __builtin_fma(-d2, inv, 1.0), inv);
              inv = __builtin_fma(inv, __builtin_fma(-d2, inv, 1.0), inv);
              const double s2 = c.sigma2 * inv;
              const double s6 = s2 * s2 * s2;
              const double gg = 48.0 * c.eps * inv * s6 * (s6 - 0.5);
              const double v = 4.0 * c.eps * (s6 * s6 - s6) + c.shift_v;
              gd = in ? gg : 0.0;
              ei += in ? 0.5 * v : 0.0;
              w += 0.5 * gd * d2;
            } else {
              const double d2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
              const bool in = d2 < c.rc2 && u != self;
              MT inv;
              if constexpr (sizeof(MT) == 4) {
                inv = __builtin_amdgcn_rcpf(in ? (float)d2 : 3.0e38f);
              } else {
                inv = 1.0 / d2;
              }
              const MT x2 = inv * inv;
              MT gg = (x2 * x2) * (fa * (x2 * inv) - fb);
              if constexpr (sizeof(MT) != 4) gg = in ? gg : (MT)0;
              gd = (double)gg;
            }
            ax = __builtin_fma(gd, dx, ax);
            ay = __builtin_fma(gd, dy, ay);
            az = __builtin_fma(gd, dz, az);
          }
        }
      }
      // the K partial sums of particle a, in the order k = 0, 1, ..., K - 1
      const int base = lane % na;
      double sx = ax, sy = ay, sz = az, se = ei;
      for (int kk = 1; kk < K; ++kk) {
        const int src = base + na * kk;
        sx += __shfl(ax, src, 64);
        sy += __shfl(ay, src, 64);
        sz += __shfl(az, src, 64);
        if (ENERGY) se += __shfl(ei, src, 64);
      }
      if (!ok || k != 0) continue;
      const int s = t.src[tc0] + a;
      const int64_t o = out.scatter ? (int64_t)out.scatter[s] : (int64_t)s;
      ((OT*)out.fx)[o] = (OT)(sx * scale);
      ((OT*)out.fy)[o] = (OT)(sy * scale);
      ((OT*)out.fz)[o] = (OT)(sz * scale);
      if (ENERGY) {
        if (out.e_atom) out.e_atom[o] = se;
        e += se;
      }
    }
  }
  if (ENERGY) {
    e = wave_sum(e);
    w = wave_sum(w);
    if (lane == 0) {
      red[wave] = e;
      red[16 + wave] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double pe = 0.0, ww = 0.0;
      for (int q = 0; q < nwaves; ++q) {
        pe += red[q];
        ww += red[16 + q];
      }
      out.partials[2 * brick] = pe;
      out.partials[2 * brick + 1] = ww;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_fill0(T* __restrict__ a, T* __restrict__ b,
                                               T* __restrict__ c, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    a[i] = (T)0;
    b[i] = (T)0;
    c[i] = (T)0;
  }
}

template <typename MT, typename OT>
static void launch_half(bool energy, hipStream_t st, const double* x, const double* y,
                        const double* z, const int32_t* cs, const Grid& g, const TileList& tl,
                        const LJConst& c, const ForceOut& out, int64_t n) {
  const dim3 grid(tile_grid(g));
  const unsigned two = 2 * tl.threads < 1024 ? 2 * tl.threads : 1024;
  // outputs accumulate with atomics: clear them first (caller order, n entries)
  const dim3 zb((unsigned)div_up(n, 256));
  hipLaunchKernelGGL(k_fill0<OT>, zb, dim3(256), 0, st, (OT*)out.fx, (OT*)out.fy, (OT*)out.fz, n);
  if (out.e_atom)
    hipLaunchKernelGGL(k_fill0<double>, zb, dim3(256), 0, st, out.e_atom, out.e_atom, out.e_atom, n);
  if (energy && out.e_atom)
    hipLaunchKernelGGL((k_lj_force_half<MT, OT, true, true>), grid, dim3(two), 0, st, x, y, z, cs,
                       g, tl, c, out);
  else if (energy)
    hipLaunchKernelGGL((k_lj_force_half<MT, OT, true, false>), grid, dim3(two), 0, st, x, y, z, cs,
                       g, tl, c, out);
  else
    hipLaunchKernelGGL((k_lj_force_half<MT, OT, false, false>), grid, dim3(two), 0, st, x, y, z,
                       cs, g, tl, c, out);
}

template <typename MT, typename OT>
static void launch_cells(bool energy, hipStream_t st, const double* x, const double* y,
                         const double* z, const int32_t* cs, const Grid& g, const LJConst& c,
                         const ForceOut& out) {
  const dim3 grid(tile_grid(g));
  const unsigned waves = g.V * 64 < 1024 ? (unsigned)g.V * 64 : 1024u;  // one wave per home cell
  if (energy)
    hipLaunchKernelGGL((k_lj_force_cells<MT, OT, true>), grid, dim3(waves), 0, st, x, y, z, cs, g,
                       c, out);
  else
    hipLaunchKernelGGL((k_lj_force_cells<MT, OT, false>), grid, dim3(waves), 0, st, x, y, z, cs, g,
                       c, out);
}

// precision as in lj_force
hipError_t lj_force_half(const double* x, const double* y, const double* z,
                         const int32_t* cell_start, const Grid& g, const TileList& tl,
                         const LJConst& c, int precision, bool energy, const ForceOut& out,
                         int64_t n, hipStream_t st) {
  switch (precision) {
    case 0:
    case 2:
      launch_half<double, double>(energy, st, x, y, z, cell_start, g, tl, c, out, n);
      break;
    case 1:
      launch_half<float, float>(energy, st, x, y, z, cell_start, g, tl, c, out, n);
      break;
    default:
      launch_half<float, double>(energy, st, x, y, z, cell_start, g, tl, c, out, n);
      break;
  }
  return hipGetLastError();
}

hipError_t lj_force_cells(const double* x, const double* y, const double* z,
                          const int32_t* cell_start, const Grid& g, const LJConst& c,
                          int precision, bool energy, const ForceOut& out, hipStream_t st) {
  switch (precision) {
    case 0:
    case 2:
      launch_cells<double, double>(energy, st, x, y, z, cell_start, g, c, out);
      break;
    case 1:
      launch_cells<float, float>(energy, st, x, y, z, cell_start, g, c, out);
      break;
    default:
      launch_cells<float, double>(energy, st, x, y, z, cell_start, g, c, out);
      break;
  }
  return hipGetLastError();
}

}  // namespace mdpl
