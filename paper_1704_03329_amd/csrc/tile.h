// LDS tiles of the LJ path.
//
// A workgroup owns one brick of cells.  Its tile is the brick grown by one
// cell on every side, (B+2)^3 cells, listed x-fastest; cell tc holds
// particles [prefix[tc], prefix[tc+1]) of the tile, copied from the sorted
// slots starting at src[tc].  Every particle of the brick finds all its
// 27-cell stencil inside the tile, and the three x-neighbour cells of a
// stencil row are consecutive tile cells, i.e. one contiguous index range.
//
// Tile cells outside the box are periodic images; code[tc] records the
// image (-1, 0, +1 per axis) so that a tile may be filled either with the
// stored positions (exact minimum-image tests) or with the image positions
// (plain differences, no per-pair image arithmetic).
//
// Half lists (each pair once) list j for i when j's tile index is larger:
// tile indices run z, y, x lexicographically, so that is the case when j's
// cell is one of the 13 "upper" neighbours of i's cell (offset (ox, oy, oz)
// with oz > 0, or oz = 0 and oy > 0, or oz = oy = 0 and ox > 0) or the same
// cell at a later slot.  The rule depends on the offset only, so the pair
// (i, j) is listed by exactly one of its particles whatever bricks and
// periodic images hold them.  Such a tile needs only the cells from the
// brick's first cell on (94 of 125 for 3^3 bricks); the others are left
// empty.
#pragma once

#include "device_util.h"
#include "internal.h"

namespace mdpl {

constexpr int kHomeBit = 64;  // in a tile cell's code: the cell belongs to the brick

template <typename T, int CAP>
struct TileOf {
  static constexpr int kSlots = CAP;
  static constexpr int kDummy = CAP - 1;  // padding slot
  static constexpr int kCap = CAP - 1;    // particles a tile can hold
  T x[CAP];
  T y[CAP];
  T z[CAP];
  int prefix[kTileCells + 1];
  int src[kTileCells];
  int code[kTileCells];
  uint8_t cell[CAP];  // tile cell of each filled slot (tile_slot_cells)
};
static_assert(kTileCells <= 256, "a tile cell index must fit the byte map");
// full-list force pass: x and y of a slot side by side (one 16-byte read),
// z apart; a full-list entry is the byte offset of the slot's x-y pair
template <int CAP>
struct TileXYOf {
  static constexpr int kSlots = CAP;
  static constexpr int kDummy = CAP - 1;
  static constexpr int kCap = CAP - 1;
  double2 xy[CAP];
  double z[CAP];
  int prefix[kTileCells + 1];
  int src[kTileCells];
  int code[kTileCells];
  uint8_t cell[CAP];
};
// FP32 force pass: x, y, z of a slot relative to the tile centre in three
// arrays (three 4-byte gathers per entry conflict less in the LDS banks than
// one 12-byte gather at a 16-byte stride); a full-list entry (4 x slot) is
// the byte offset in each
template <int CAP>
struct TileF32Of {
  static constexpr int kSlots = CAP;
  static constexpr int kDummy = CAP - 1;
  static constexpr int kCap = CAP - 1;
  float px[CAP];
  float py[CAP];
  float pz[CAP];
  int prefix[kTileCells + 1];
  int src[kTileCells];
  int code[kTileCells];
};
// the cell table alone (kernels that map tile indices to slots only)
struct TileCells {
  int prefix[kTileCells + 1];
  int src[kTileCells];
  int code[kTileCells];
};
// full lists: FP64 image positions (force and descriptor passes) and FP32
// positions relative to the tile origin (list build)
using TileShared = TileOf<double, kTileMax>;
using TileShared32 = TileOf<float, kTileMax>;
// half lists: the same with the capacity of a half tile
using TileHalf = TileOf<double, kTileMaxHalf>;
using TileHalf32 = TileOf<float, kTileMaxHalf>;
using TileXY = TileXYOf<kTileMax>;
using TileF32 = TileF32Of<kTileMax>;

// Workgroups are dealt round-robin to the 8 XCDs; give each XCD a contiguous
// run of bricks (a slab of the box) so that tile reloads hit its own L2.
// With a brick order (built on the host, see brick_order), the full bricks
// and then the thin ones (the last brick along an axis whose cell count is
// not a multiple of B) are each dealt to the XCDs in 8 contiguous pieces, so
// that every round of 8 workgroups carries equal work and light workgroups
// fill the final round.  Returns nbricks for padding workgroups.
__device__ __forceinline__ int brick_of_block(const Grid& g) {
  if (g.order) return g.order[blockIdx.x];
  const int per = (g.nbricks + 7) >> 3;
  return (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
}

// Workgroups of a tile kernel: the brick order's length, else one per brick
// rounded up to whole rounds of the 8 XCDs.
inline unsigned tile_grid(const Grid& g) {
  return g.order ? (unsigned)g.norder : (unsigned)(((g.nbricks + 7) >> 3) * 8);
}

__device__ __forceinline__ void brick_coords(const Grid& g, int brick, int& bx, int& by, int& bz) {
  bx = brick % g.nb[0];
  by = (brick / g.nb[0]) % g.nb[1];
  bz = brick / (g.nb[0] * g.nb[1]);
}

// Fills prefix/src/code for the tile of `brick`; returns the particle count
// (possibly above the tile's capacity).  half: the cells before the brick's
// first cell are left empty.  Ends with a barrier.
template <typename TS>
__device__ inline int tile_cells(const Grid& g, int brick, const int32_t* __restrict__ cs, TS& t,
                                 bool half = false, const int32_t* __restrict__ xlow = nullptr,
                                 int* tlow = nullptr) {
  const int TX = g.B[0] + 2, TY = g.B[1] + 2, TZ = g.B[2] + 2;
  const int ntc = TX * TY * TZ;
  int bx, by, bz;
  brick_coords(g, brick, bx, by, bz);
  const int ox = bx * g.B[0] - 1, oy = by * g.B[1] - 1, oz = bz * g.B[2] - 1;
  const int first = half ? (TY + 1) * TX + 1 : 0;  // tile index of the brick's first cell
  for (int tc = threadIdx.x; tc < ntc; tc += blockDim.x) {
    const int lx = tc % TX, ly = (tc / TX) % TY, lz = tc / (TX * TY);
    int cx = ox + lx, cy = oy + ly, cz = oz + lz;
    int sx = 0, sy = 0, sz = 0;
    if (cx < 0) { cx += g.nc[0]; sx = -1; } else if (cx >= g.nc[0]) { cx -= g.nc[0]; sx = 1; }
    if (cy < 0) { cy += g.nc[1]; sy = -1; } else if (cy >= g.nc[1]) { cy -= g.nc[1]; sy = 1; }
    if (cz < 0) { cz += g.nc[2]; sz = -1; } else if (cz >= g.nc[2]) { cz -= g.nc[2]; sz = 1; }
    const int key = cell_key(g, cx, cy, cz);
    const int b = cs[key];
    t.src[tc] = b;
    if (tlow) tlow[tc] = xlow[key];
    t.prefix[tc + 1] = tc < first ? 0 : cs[key + 1] - b;
    // bit 6: a cell of the brick itself (inside the box; a partial brick's
    // missing cells are images of other bricks' cells)
    const bool home = lx >= 1 && lx <= g.B[0] && ly >= 1 && ly <= g.B[1] && lz >= 1 &&
                      lz <= g.B[2] && (sx | sy | sz) == 0;
    t.code[tc] = (sx + 1) | ((sy + 1) << 2) | ((sz + 1) << 4) | (home ? kHomeBit : 0);
  }
  if (threadIdx.x == 0) t.prefix[0] = 0;
  __syncthreads();
  if (threadIdx.x < 64) {  // inclusive scan of the counts by wave 0
    const int lane = threadIdx.x;
    int carry = 0;
    for (int base = 1; base <= ntc; base += 64) {
      const int i = base + lane;
      int v = (i <= ntc) ? t.prefix[i] : 0;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(v, off, 64);
        if (lane >= off) v += o;
      }
      if (i <= ntc) t.prefix[i] = v + carry;
      carry += __shfl(v, 63, 64);
    }
  }
  __syncthreads();
  return t.prefix[ntc];
}

// The tables tile_cells filled, to global memory (kTabInts ints: prefix,
// then src, then code at fixed offsets), and back.  tile_tables_load ends
// with a barrier and returns the particle count.
template <typename TS>
__device__ inline void tile_tables_store(const Grid& g, const TS& t, int32_t* __restrict__ tab) {
  const int ntc = (g.B[0] + 2) * (g.B[1] + 2) * (g.B[2] + 2);
  for (int i = threadIdx.x; i <= ntc; i += blockDim.x) tab[i] = t.prefix[i];
  for (int i = threadIdx.x; i < ntc; i += blockDim.x) {
    tab[kTileCells + 1 + i] = t.src[i];
    tab[2 * kTileCells + 1 + i] = t.code[i];
  }
}
template <typename TS>
__device__ inline int tile_tables_load(const Grid& g, const int32_t* __restrict__ tab, TS& t) {
  const int ntc = (g.B[0] + 2) * (g.B[1] + 2) * (g.B[2] + 2);
  for (int i = threadIdx.x; i <= ntc; i += blockDim.x) t.prefix[i] = tab[i];
  for (int i = threadIdx.x; i < ntc; i += blockDim.x) {
    t.src[i] = tab[kTileCells + 1 + i];
    t.code[i] = tab[2 * kTileCells + 1 + i];
  }
  __syncthreads();
  return t.prefix[ntc];
}

// Fills the byte map t.cell[u] = tile cell of slot u for the first
// min(total, TS::kCap) slots, eight threads per cell, so that a slot finds
// its cell with one LDS read instead of a search over the prefix.  Ends
// with a barrier.
template <typename TS>
__device__ inline void tile_slot_cells(int ntc, int total, TS& t) {
  const int nt = total < TS::kCap ? total : TS::kCap;
  for (int tc = (int)threadIdx.x >> 3; tc < ntc; tc += (int)blockDim.x >> 3) {
    const int e = t.prefix[tc + 1] < nt ? t.prefix[tc + 1] : nt;
    for (int u = t.prefix[tc] + ((int)threadIdx.x & 7); u < e; u += 8) t.cell[u] = (uint8_t)tc;
  }
  __syncthreads();
}

// Copies the tile's positions (at most TS::kCap) into LDS; IMAGE adds the
// periodic image offsets.  Fills the slot map first.  Ends with a barrier.
template <bool IMAGE, typename TS>
__device__ inline void tile_load(const Grid& g, const double* __restrict__ x,
                                 const double* __restrict__ y, const double* __restrict__ z,
                                 int total, TS& t) {
  const int ntc = (g.B[0] + 2) * (g.B[1] + 2) * (g.B[2] + 2);
  const int nt = total < TS::kCap ? total : TS::kCap;
  tile_slot_cells(ntc, total, t);
  if (threadIdx.x == 0) {  // padding slot: no pair with it is ever inside the cutoff
    t.x[TS::kDummy] = 1e20;
    t.y[TS::kDummy] = 1e20;
    t.z[TS::kDummy] = 1e20;
  }
  for (int u = threadIdx.x; u < nt; u += blockDim.x) {
    const int lo = t.cell[u];
    const int src = t.src[lo] + (u - t.prefix[lo]);
    double a = x[src], b = y[src], c = z[src];
    if (IMAGE) {
      const int code = t.code[lo];
      a += (double)((code & 3) - 1) * g.box[0];
      b += (double)(((code >> 2) & 3) - 1) * g.box[1];
      c += (double)(((code >> 4) & 3) - 1) * g.box[2];
    }
    t.x[u] = a;
    t.y[u] = b;
    t.z[u] = c;
  }
  __syncthreads();
}

// tile_load for the x-y paired tile (image positions).  Ends with a barrier.
template <int CAP>
__device__ inline void tile_load_xy(const Grid& g, const double* __restrict__ x,
                                    const double* __restrict__ y, const double* __restrict__ z,
                                    int total, TileXYOf<CAP>& t) {
  const int ntc = (g.B[0] + 2) * (g.B[1] + 2) * (g.B[2] + 2);
  const int nt = total < TileXYOf<CAP>::kCap ? total : TileXYOf<CAP>::kCap;
  tile_slot_cells(ntc, total, t);
  if (threadIdx.x == 0) {  // padding slot: no pair with it is ever inside the cutoff
    t.xy[TileXYOf<CAP>::kDummy] = make_double2(1e20, 1e20);
    t.z[TileXYOf<CAP>::kDummy] = 1e20;
  }
  for (int u = threadIdx.x; u < nt; u += blockDim.x) {
    const int lo = t.cell[u];
    const int src = t.src[lo] + (u - t.prefix[lo]);
    const int code = t.code[lo];
    t.xy[u] = make_double2(x[src] + (double)((code & 3) - 1) * g.box[0],
                           y[src] + (double)(((code >> 2) & 3) - 1) * g.box[1]);
    t.z[u] = z[src] + (double)(((code >> 4) & 3) - 1) * g.box[2];
  }
  __syncthreads();
}

// Image position of a stored coordinate: x + k L with k = -1, 0, +1 from a
// tile cell's code (the product is exact, so contraction cannot change it).
__device__ __forceinline__ double image_coord(double x, int k, double L) {
  return x + (double)(k - 1) * L;
}

// Centre of a brick's tile (the middle of the brick's B cells per axis), the
// origin of the FP32 coordinates of the force pass.
__device__ __forceinline__ void tile_centre(const Grid& g, int brick, double& ox, double& oy,
                                            double& oz) {
  int bx, by, bz;
  brick_coords(g, brick, bx, by, bz);
  ox = ((double)(bx * g.B[0]) + 0.5 * (double)g.B[0]) * g.side[0];
  oy = ((double)(by * g.B[1]) + 0.5 * (double)g.B[1]) * g.side[1];
  oz = ((double)(bz * g.B[2]) + 0.5 * (double)g.B[2]) * g.side[2];
}

// FP32 coordinate of an image position relative to the tile centre.
__device__ __forceinline__ float rel32(double image, double o) { return (float)(image - o); }

// tile_load for the FP32 tile: rel32 of the image positions, eight threads
// per tile cell (a cell's particles are contiguous in memory; no slot map,
// which keeps the tile small enough for three workgroups per CU).  home
// (LDS, kBrickMax entries) receives the tile slot of each of the brick's own
// particles (by index from s0; the dummy slot for a particle the tile could
// not hold).  Up to four particles per thread and cell are loaded before
// any is used.  Ends with a barrier.
template <int CAP>
__device__ inline void tile_load_f32(const Grid& g, const double* __restrict__ x,
                                     const double* __restrict__ y, const double* __restrict__ z,
                                     int total, double ox, double oy, double oz, int s0,
                                     TileF32Of<CAP>& t, uint16_t* home) {
  using T = TileF32Of<CAP>;
  const int ntc = (g.B[0] + 2) * (g.B[1] + 2) * (g.B[2] + 2);
  const int nt = total < T::kCap ? total : T::kCap;
  for (int a = threadIdx.x; a < kBrickMax; a += blockDim.x) home[a] = T::kDummy;
  if (threadIdx.x == 0) {  // padding slot: no pair with it is ever inside the cutoff
    t.px[T::kDummy] = 1e18f;
    t.py[T::kDummy] = 1e18f;
    t.pz[T::kDummy] = 1e18f;
  }
  __syncthreads();
  constexpr int kPer = 4;
  const int sub = (int)threadIdx.x & 7;
  for (int tc = (int)threadIdx.x >> 3; tc < ntc; tc += (int)blockDim.x >> 3) {
    const int b = t.prefix[tc], e = t.prefix[tc + 1] < nt ? t.prefix[tc + 1] : nt;
    const int code = t.code[tc];
    const int off = t.src[tc] - b;  // sorted index of slot u: off + u
    const bool own = (code & kHomeBit) != 0;
    for (int u0 = b + sub; u0 < e; u0 += 8 * kPer) {
      double vx[kPer], vy[kPer], vz[kPer];
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        const int u = u0 + 8 * j;
        if (u < e) {
          vx[j] = x[off + u];
          vy[j] = y[off + u];
          vz[j] = z[off + u];
        }
      }
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        const int u = u0 + 8 * j;
        if (u < e) {
          t.px[u] = rel32(image_coord(vx[j], code & 3, g.box[0]), ox);
          t.py[u] = rel32(image_coord(vy[j], (code >> 2) & 3, g.box[1]), oy);
          t.pz[u] = rel32(image_coord(vz[j], (code >> 4) & 3, g.box[2]), oz);
          if (own && off + u - s0 < kBrickMax) home[off + u - s0] = (uint16_t)u;
        }
      }
    }
  }
  __syncthreads();
}

// FP64 image positions into a TileOf<double> cell by cell, eight threads per
// cell and up to four particles each loaded before use (no slot map is
// filled).  Ends with a barrier.
template <int CAP>
__device__ inline void tile_load_f64_cells(const Grid& g, const double* __restrict__ x,
                                           const double* __restrict__ y,
                                           const double* __restrict__ z, int total,
                                           TileOf<double, CAP>& t) {
  using T = TileOf<double, CAP>;
  const int ntc = (g.B[0] + 2) * (g.B[1] + 2) * (g.B[2] + 2);
  const int nt = total < T::kCap ? total : T::kCap;
  if (threadIdx.x == 0) {  // padding slot: no pair with it is ever inside the cutoff
    t.x[T::kDummy] = 1e20;
    t.y[T::kDummy] = 1e20;
    t.z[T::kDummy] = 1e20;
  }
  constexpr int kPer = 4;
  const int sub = (int)threadIdx.x & 7;
  for (int tc = (int)threadIdx.x >> 3; tc < ntc; tc += (int)blockDim.x >> 3) {
    const int b = t.prefix[tc], e = t.prefix[tc + 1] < nt ? t.prefix[tc + 1] : nt;
    const int code = t.code[tc];
    const int off = t.src[tc] - b;  // sorted index of slot u: off + u
    for (int u0 = b + sub; u0 < e; u0 += 8 * kPer) {
      double vx[kPer], vy[kPer], vz[kPer];
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        const int u = u0 + 8 * j;
        if (u < e) {
          vx[j] = x[off + u];
          vy[j] = y[off + u];
          vz[j] = z[off + u];
        }
      }
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        const int u = u0 + 8 * j;
        if (u < e) {
          t.x[u] = image_coord(vx[j], code & 3, g.box[0]);
          t.y[u] = image_coord(vy[j], (code >> 2) & 3, g.box[1]);
          t.z[u] = image_coord(vz[j], (code >> 4) & 3, g.box[2]);
        }
      }
    }
  }
  __syncthreads();
}

// Tile cell of tile particle u < total (binary search over the prefix;
// a tile has at least 27 cells, so the first halving always happens), for
// tables without the slot map.
template <typename TS>
__device__ __forceinline__ int tile_cell_of(const TS& t, int ntc, int u) {
  int lo = 0, hi = ntc;  // prefix[lo] <= u < prefix[hi]
  do {
    const int mid = (lo + hi) >> 1;
    if (t.prefix[mid] <= u) lo = mid;
    else hi = mid;
  } while (hi - lo > 1);
  return lo;
}

// Tile cell of a brick particle from its cell key.
__device__ __forceinline__ int home_tile_cell(const Grid& g, int brick, int key) {
  const int local = key - brick * g.V;
  const int lx = local % g.B[0], ly = (local / g.B[0]) % g.B[1], lz = local / (g.B[0] * g.B[1]);
  const int TX = g.B[0] + 2, TY = g.B[1] + 2;
  return ((lz + 1) * TY + (ly + 1)) * TX + (lx + 1);
}

}  // namespace mdpl
