// Neighbour-list construction from the cell list (Sec. 3.5: visit the cell
// of i and its 26 neighbours, keep the pairs closer than the list radius;
// GPU neighbour matrix W_{m,i} = m-th neighbour of i).
//
// The pair test is the exact FP64 minimum-image predicate
//   dx = xi - xj; dx > L/2 ? dx - L : (dx < -L/2 ? dx + L : dx)
//   d2 = (dx*dx + dy*dy) + dz*dz < r2
// with floating-point contraction off, on the caller's FP64 values, so the
// list is bit-identical to the all-pairs definition.
//
// Two builders:
//  * the LJ list: one workgroup per brick stages its tile (stored positions,
//    no images) in LDS, one wave per home cell tests the 27 tile cells of its
//    stencil (a full list: each cell's particles of the lower half along x
//    first, so that a particle skips the half of the next or previous cell
//    along x that lies beyond the list radius, 5/6 of each stencil row); entries are 16-bit tile byte offsets (16 x slot), column-major, so the force
//    pass reads one coalesced word per four neighbours.  A half list (each
//    pair once, Newton's third law) keeps j in the list of i only if j's tile
//    index is larger (tile.h): four of the nine stencil rows whole, and the
//    row of i's cell from i on;
//  * the analysis list (bond order / CNA): one thread per particle walks the
//    9 rows of 3 consecutive cells in global memory, entries are sorted-slot
//    indices, row-major so a whole list is one contiguous read.
#include <math.h>

#include "device_util.h"
#include "internal.h"
#include "tile.h"

namespace mdpl {

// ------------------------------------------------------------------ LJ list
// One wave per home cell at a time.  The cell's particles (na <= 64 per
// pass) are spread over the 64 lanes as na x K (K = 64 / na): lane
// (a, k) tests particle a against candidates k, k+K, k+2K, ... of each
// stencil row (three consecutive tile cells, one contiguous index range),
// so all lanes walk the same 9 rows together and lanes with equal k read
// the same tile slot.  Accepted neighbours get their rank from a
// per-particle LDS counter and are stored as 16-bit halves of the list
// words; a final pass pads the last word and writes the counts.
//
// Exactness with an FP32 screen.  The tile holds FP32 positions relative to
// its corner with the periodic image already applied, X = fl32((x + s L) - o).
// Each coordinate is then within 2^-24 span of the exact image (span = tile
// extent), a difference within 2^-24 (2 span + 2 r_ext) of the exact one,
// and the FP32 squared distance d2f of any pair near the list radius
// within e = 2 sqrt(3) r_ext 2^-24 (2 span + 2 r_ext) + 3 2^-24 r^2 of the
// definition's d2 (whose own rounding is ~1e-14).  With the guard band
// g = 8 e, d2f < r^2 - g proves d2 < r^2 and d2f > r^2 + g proves d2 >= r^2;
// the rare pairs in between are decided by the definition itself (the
// conditional minimum image on the stored FP64 positions).  The list is
// therefore bit-identical to the all-pairs definition.
constexpr float kFarF = 1e30f;  // dummy slot: its d2f overflows to +inf

struct RowScan {
  float xi, yi, zi;            // FP32 tile coordinates of the particle
  float r2lo, r2hi;            // r^2 -/+ g
  double xs, ys, zs;           // its stored FP64 position (exact test)
  const double *x, *y, *z;     // stored FP64 positions, sorted slots
  double r2, Lx, Ly, Lz, hx, hy, hz;
  int self, K, max_nb;
  int* cnt;                    // the particle's LDS counter
  uint16_t* base;              // its list: entry m at base[(m >> 2) * stride4 + (m & 3)]
  uint32_t stride4;
  uint32_t pitch;              // bytes per word row, 2 * stride4
};

// Candidates u = ub, ub + K, ... < ue (one contiguous range of tile
// indices), UNROLL at a time so that their LDS loads overlap; slots past the
// end read the far-away dummy.  One LDS atomic reserves the ranks of all
// accepted candidates of a step; each candidate's offset among them is
// known before it, so a store needs one comparison with the capacity.
// A24: the word-row pitch is below 2^24 bytes, so the byte offset of rank m
// (below 2^32, as m >> 2 < 2^8) comes from a 24-bit product.
// Candidate indices are carried as byte offsets into the 4-byte tile
// arrays (4 u), which saves a shift per candidate.
template <int UNROLL, int SHIFT, bool A24, typename TS>
__device__ __forceinline__ void scan_range(const TS& t, int ub, int ue, const RowScan& q) {
  const int ue4 = 4 * ue, step4 = 4 * UNROLL * q.K, k4 = 4 * q.K, self4 = 4 * q.self;
  for (int u04 = 4 * ub; u04 < ue4; u04 += step4) {
    constexpr uint32_t kNone = 1u << 20;  // offset of a rejected candidate: past any list
    int uu4[UNROLL];
    uint32_t rank[UNROLL];  // offset among this step's accepted candidates, or kNone
    uint32_t na = 0;
#pragma unroll
    for (int j = 0; j < UNROLL; ++j) {
      const int u4 = u04 + j * k4;
      uu4[j] = u4 < ue4 ? u4 : 4 * TS::kDummy;
    }
#pragma unroll
    for (int j = 0; j < UNROLL; ++j) {
      const float dx = q.xi - *(const float*)((const char*)t.x + uu4[j]);
      const float dy = q.yi - *(const float*)((const char*)t.y + uu4[j]);
      const float dz = q.zi - *(const float*)((const char*)t.z + uu4[j]);
      const float d2f = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
      const bool other = uu4[j] != self4;
      bool acc = other && d2f < q.r2lo;
      if (other && !(d2f < q.r2lo) && d2f <= q.r2hi) {
        // inside the guard band: the definition decides
        const int u = uu4[j] >> 2;
        const int c = t.cell[u];
        const int sj = t.src[c] + (u - t.prefix[c]);
        acc = exact_d2(q.xs, q.ys, q.zs, q.x[sj], q.y[sj], q.z[sj], q.Lx, q.Ly, q.Lz, q.hx, q.hy,
                       q.hz) < q.r2;
      }
      rank[j] = acc ? na : kNone;
      na += acc ? 1u : 0u;
    }
    if (na) {
      const uint32_t m = (uint32_t)atomicAdd(q.cnt, (int)na);
#pragma unroll
      for (int j = 0; j < UNROLL; ++j) {
        const uint32_t mj = m + rank[j];
        if (mj < (uint32_t)q.max_nb) {
          if constexpr (A24)
            *(uint16_t*)((char*)q.base + (__umul24(mj >> 2, q.pitch) + ((mj & 3u) << 1))) =
                (uint16_t)(uu4[j] << (SHIFT - 2));
          else
            q.base[(uint64_t)(mj >> 2) * q.stride4 + (mj & 3u)] = (uint16_t)(uu4[j] << (SHIFT - 2));
        }
      }
    }
  }
}

// One wave per home cell (up to 16 per workgroup); at most 64 VGPRs so that
// two 1024-thread workgroups share a CU.  TS: the tile (full or half list).
template <typename TS, bool HALF, bool A24>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) void k_build_tile_nlist(
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
    const int32_t* __restrict__ skeys, const int32_t* __restrict__ cs, Grid g, double r2,
    float guard, TileList tl, uint32_t* __restrict__ flags, int32_t* __restrict__ maxcount) {
  __shared__ TS t;
  __shared__ int acnt[kBrickMax];
  __shared__ int tlow[kTileCells];  // per tile cell, its particles in the lower x half
  const int brick = brick_of_block(g);
  if (brick >= g.nbricks) return;
  const bool xh = !HALF && tl.xlow != nullptr;
  const int total = tile_cells(g, brick, cs, t, HALF, tl.xlow, xh ? tlow : nullptr);
  if (!HALF && tl.tab) tile_tables_store(g, t, tl.tab + (int64_t)brick * kTabInts);
  const int s0 = cs[brick * g.V], s1 = cs[(brick + 1) * g.V];
  const int nbrick = s1 - s0;
  if (threadIdx.x == 0 && (total > TS::kCap || nbrick > kBrickMax))
    atomicOr(flags, MDPL_FLAG_NL_OVERFLOW);
  for (int a = threadIdx.x; a < kBrickMax; a += blockDim.x) acnt[a] = 0;
  const double Lx = g.box[0], Ly = g.box[1], Lz = g.box[2];
  const int TX = g.B[0] + 2, TXY = TX * (g.B[1] + 2);
  const int ntc = TXY * (g.B[2] + 2);
  int bx, by, bz;
  brick_coords(g, brick, bx, by, bz);
  // the tile corner (one cell below the brick) and FP32 relative image positions
  const double ox = (double)(bx * g.B[0] - 1) * (Lx / g.nc[0]);
  const double oy = (double)(by * g.B[1] - 1) * (Ly / g.nc[1]);
  const double oz = (double)(bz * g.B[2] - 1) * (Lz / g.nc[2]);
  tile_slot_cells(ntc, total, t);
  {
    const int nt = total < TS::kCap ? total : TS::kCap;
    if (threadIdx.x == 0) {
      t.x[TS::kDummy] = kFarF;
      t.y[TS::kDummy] = kFarF;
      t.z[TS::kDummy] = kFarF;
    }
    for (int u = threadIdx.x; u < nt; u += blockDim.x) {
      const int c = t.cell[u];
      const int src = t.src[c] + (u - t.prefix[c]);
      const int code = t.code[c];
      t.x[u] = (float)((x[src] + (double)((code & 3) - 1) * Lx) - ox);
      t.y[u] = (float)((y[src] + (double)(((code >> 2) & 3) - 1) * Ly) - oy);
      t.z[u] = (float)((z[src] + (double)(((code >> 4) & 3) - 1) * Lz) - oz);
    }
    __syncthreads();
  }
  const int max_nb = tl.max_nb;
  uint16_t* __restrict__ half = (uint16_t*)tl.nbr;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const float r2lo = (float)(r2 - (double)guard), r2hi = (float)(r2 + (double)guard);
  for (int lc = wave; lc < g.V; lc += nwaves) {
    const int lx = lc % g.B[0], ly = (lc / g.B[0]) % g.B[1], lz = lc / (g.B[0] * g.B[1]);
    // the last brick along an axis may be partial: its missing cells would
    // alias periodic images of another brick's cells
    if (bx * g.B[0] + lx >= g.nc[0] || by * g.B[1] + ly >= g.nc[1] || bz * g.B[2] + lz >= g.nc[2])
      continue;
    const int tc0 = ((lz + 1) * (g.B[1] + 2) + (ly + 1)) * TX + (lx + 1);
    const int ncell = t.prefix[tc0 + 1] - t.prefix[tc0];
    const int slot0 = t.src[tc0];
    for (int a0 = 0; a0 < ncell; a0 += 64) {
      const int na = ncell - a0 < 64 ? ncell - a0 : 64;
      const int K = 64 / na;
      const int a = a0 + lane % na, k = lane / na;
      const bool active = k < K;
      const int self = t.prefix[tc0] + a;
      const int s = slot0 + a;          // sorted slot of particle a
      const int la = s - s0;            // its index within the brick
      const bool ok = active && self < TS::kCap && la >= 0 && la < kBrickMax && s < s1;
      RowScan q;
      q.xi = ok ? t.x[self] : 0.0f;
      q.yi = ok ? t.y[self] : 0.0f;
      q.zi = ok ? t.z[self] : 0.0f;
      q.r2lo = r2lo;
      q.r2hi = r2hi;
      q.xs = ok ? x[s] : 0.0;
      q.ys = ok ? y[s] : 0.0;
      q.zs = ok ? z[s] : 0.0;
      q.x = x;
      q.y = y;
      q.z = z;
      q.r2 = r2;
      q.Lx = Lx;
      q.Ly = Ly;
      q.Lz = Lz;
      q.hx = 0.5 * Lx;
      q.hy = 0.5 * Ly;
      q.hz = 0.5 * Lz;
      q.self = self;
      q.K = K;
      q.max_nb = max_nb;
      q.cnt = &acnt[ok ? la : 0];
      q.base = half + (int64_t)(ok ? s : 0) * 4;
      q.stride4 = (uint32_t)(tl.stride * 4);
      q.pitch = (uint32_t)(tl.stride * 8);
      // a particle in the lower x half of its cell skips the upper half of
      // the next cell along x, one in the upper half the lower half of the
      // previous cell: more than a cell width, which exceeds the list
      // radius, away along x alone
      const bool lower = xh && a < tlow[tc0];
      const bool upper = xh && !lower;
      for (int oz = -1; oz <= 1; ++oz) {
        for (int oy2 = -1; oy2 <= 1; ++oy2) {
          // a stencil row: three consecutive tile cells, one contiguous index range
          const int tcl = tc0 + oz * TXY + oy2 * TX - 1;
          if (!ok) continue;
          // half list: only tile indices past the particle's own (rows below it are empty)
          if (HALF && (oz < 0 || (oz == 0 && oy2 < 0))) continue;
          int ub = t.prefix[tcl] + (upper ? tlow[tcl] : 0);
          if (HALF && ub <= self) ub = self + 1;
          int ue = lower ? t.prefix[tcl + 2] + tlow[tcl + 2] : t.prefix[tcl + 3];
          ue = ue < TS::kCap ? ue : TS::kCap;
          scan_range<4, HALF ? kHalfShift : kFullShift, A24>(t, ub + k, ue, q);
        }
      }
    }
  }
  __syncthreads();
  // every slot of the brick gets its count (zero past kBrickMax, flagged above)
  int most = 0;
  for (int la = threadIdx.x; la < nbrick; la += blockDim.x) {
    const int s = s0 + la;
    const int count = la < kBrickMax ? acnt[la] : 0;
    const int kept = count < max_nb ? count : max_nb;
    for (int m = kept; m < ((kept + 3) & ~3); ++m)  // pad the last word
      half[((int64_t)(m >> 2) * tl.stride + s) * 4 + (m & 3)] =
          (uint16_t)(TS::kDummy << (HALF ? kHalfShift : kFullShift));
    tl.cnt[s] = kept;
    if (count > max_nb) atomicOr(flags, MDPL_FLAG_NL_OVERFLOW);
    most = count > most ? count : most;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const int o = __shfl_xor(most, off, 64);
    most = o > most ? o : most;
  }
  if ((threadIdx.x & 63) == 0 && most > 0) atomicMax(maxcount, most);
}

hipError_t build_tile_nlist(const double* x, const double* y, const double* z,
                            const int32_t* skeys, const int32_t* cell_start, const Grid& g,
                            double r2, TileList tl, uint32_t* flags, int32_t* maxcount,
                            hipStream_t st) {
  const unsigned threads = g.V * 64 < 1024 ? (unsigned)g.V * 64 : 1024u;
  // guard band of the FP32 screen (see the derivation above k_build_tile_nlist)
  double span = 0.0;
  for (int k = 0; k < 3; ++k) {
    const double e = (double)(g.B[k] + 2) * (g.box[k] / g.nc[k]);
    span = e > span ? e : span;
  }
  const double u32 = 1.0 / 16777216.0;  // 2^-24
  const double rext = sqrt(r2);
  const double err = 2.0 * sqrt(3.0) * rext * u32 * (2.0 * span + 2.0 * rext) + 3.0 * u32 * r2;
  const float guard = (float)(8.0 * err);
  const dim3 grid(tile_grid(g));
  if (tl.half)
    hipLaunchKernelGGL((k_build_tile_nlist<TileHalf32, true, false>), grid, dim3(threads), 0, st,
                       x, y, z, skeys, cell_start, g, r2, guard, tl, flags, maxcount);
  else if (tl.stride * 8 < (int64_t)(1 << 24))
    hipLaunchKernelGGL((k_build_tile_nlist<TileShared32, false, true>), grid, dim3(threads), 0, st,
                       x, y, z, skeys, cell_start, g, r2, guard, tl, flags, maxcount);
  else
    hipLaunchKernelGGL((k_build_tile_nlist<TileShared32, false, false>), grid, dim3(threads), 0,
                       st, x, y, z, skeys, cell_start, g, r2, guard, tl, flags, maxcount);
  return hipGetLastError();
}

// Directed pairs in the caller's indices: entry m of slot s goes to
// offsets[s] + m; the tile index is mapped back to its sorted slot.
__global__ __launch_bounds__(1024) void k_export_tile_pairs(
    TileList tl, const int32_t* __restrict__ cs, Grid g, const int32_t* __restrict__ perm,
    const int32_t* __restrict__ offsets, int32_t* __restrict__ i_out, int32_t* __restrict__ j_out,
    int64_t cap) {
  __shared__ TileCells t;
  const int brick = brick_of_block(g);
  if (brick >= g.nbricks) return;
  tile_cells(g, brick, cs, t, tl.half != 0);
  const int ntc = (g.B[0] + 2) * (g.B[1] + 2) * (g.B[2] + 2);
  const int s0 = cs[brick * g.V], s1 = cs[(brick + 1) * g.V];
  for (int s = s0 + (int)threadIdx.x; s < s1; s += blockDim.x) {
    const int c = tl.cnt[s];
    const int64_t o = offsets[s];
    const int32_t pi = perm[s];
    for (int m = 0; m < c; ++m) {
      if (o + m >= cap) break;
      const int u = (int)((tl.nbr[(int64_t)(m >> 2) * tl.stride + s] >> (16 * (m & 3))) & 0xffff) >>
                    (tl.half ? kHalfShift : kFullShift);
      const int lo = tile_cell_of(t, ntc, u);
      i_out[o + m] = pi;
      j_out[o + m] = perm[t.src[lo] + (u - t.prefix[lo])];
    }
  }
}

hipError_t export_tile_pairs(const TileList& tl, const int32_t* cell_start, const Grid& g,
                             const int32_t* perm, const int32_t* offsets, int32_t* i_out,
                             int32_t* j_out, int64_t cap, hipStream_t st) {
  hipLaunchKernelGGL(k_export_tile_pairs, dim3(tile_grid(g)), dim3(tl.threads), 0,
                     st, tl, cell_start, g, perm, offsets, i_out, j_out, cap);
  return hipGetLastError();
}

// ------------------------------------------------------------ analysis list
__global__ __launch_bounds__(256) void k_build_nlist(
    const double* __restrict__ sx, const double* __restrict__ sy, const double* __restrict__ sz,
    const int32_t* __restrict__ skeys, const int32_t* __restrict__ cs, int64_t n, Grid g, double r2,
    NList nl, uint32_t* __restrict__ flags, int32_t* __restrict__ maxcount) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int count = 0;
  if (s < n) {
    const double xi = sx[s], yi = sy[s], zi = sz[s];
    const double Lx = g.box[0], Ly = g.box[1], Lz = g.box[2];
    const double hx = 0.5 * Lx, hy = 0.5 * Ly, hz = 0.5 * Lz;
    const int n0 = g.nc[0], n1 = g.nc[1], n2 = g.nc[2];
    const int key = skeys[s];  // B = (1,1,1): x-fastest cell index
    const int cx = key % n0;
    const int cy = (key / n0) % n1;
    const int cz = key / (n0 * n1);
    const int max_nb = nl.max_nb;
    for (int oz = -1; oz <= 1; ++oz) {
      int z2 = cz + oz;
      z2 += (z2 < 0) ? n2 : 0;
      z2 -= (z2 >= n2) ? n2 : 0;
      for (int oy = -1; oy <= 1; ++oy) {
        int y2 = cy + oy;
        y2 += (y2 < 0) ? n1 : 0;
        y2 -= (y2 >= n1) ? n1 : 0;
        const int row = (z2 * n1 + y2) * n0;
        int b[3], e[3], nr;
        if (cx >= 1 && cx <= n0 - 2) {
          b[0] = cs[row + cx - 1];
          e[0] = cs[row + cx + 2];
          nr = 1;
        } else {
          const int xm = (cx == 0) ? n0 - 1 : cx - 1;
          const int xp = (cx == n0 - 1) ? 0 : cx + 1;
          b[0] = cs[row + xm];
          e[0] = cs[row + xm + 1];
          b[1] = cs[row + cx];
          e[1] = cs[row + cx + 1];
          b[2] = cs[row + xp];
          e[2] = cs[row + xp + 1];
          nr = 3;
        }
        for (int r = 0; r < nr; ++r) {
          for (int t = b[r]; t < e[r]; ++t) {
            if (t == s) continue;
            const double d2 = exact_d2(xi, yi, zi, sx[t], sy[t], sz[t], Lx, Ly, Lz, hx, hy, hz);
            if (d2 < r2) {
              if (count < max_nb) nl.nbr[s * (int64_t)max_nb + count] = t;
              ++count;
            }
          }
        }
      }
    }
    nl.cnt[s] = count;  // true count: callers see an overflow per particle
    if (count > max_nb) atomicOr(flags, MDPL_FLAG_NL_OVERFLOW);
  }
  int m = count;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const int o = __shfl_xor(m, off, 64);
    m = o > m ? o : m;
  }
  if ((threadIdx.x & 63) == 0 && m > 0) atomicMax(maxcount, m);
}

hipError_t build_nlist(const double* sx, const double* sy, const double* sz,
                       const int32_t* skeys, const int32_t* cell_start, int64_t n, const Grid& g,
                       double r2, NList nl, uint32_t* flags, int32_t* maxcount, hipStream_t st) {
  if (g.V != 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_build_nlist, dim3((unsigned)div_up(n, 256)), dim3(256), 0, st, sx, sy, sz,
                     skeys, cell_start, n, g, r2, nl, flags, maxcount);
  return hipGetLastError();
}

}  // namespace mdpl
