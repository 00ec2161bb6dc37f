// Cell binning by counting sort (Sec. 3.5: every particle belongs to exactly
// one cell of side >= the list radius; the GPU cell-occupancy idea of the
// "Threading and GPU parallelisation" paragraph is realised here as a stable
// LSD radix sort of cell keys).
//
// Atomics stay in LDS: per-tile digit histograms use LDS atomics, ranks
// inside a tile come from wavefront ballots, tile offsets from a
// device-wide exclusive scan.  No global atomics, results are deterministic.
#include <math.h>

#include "device_util.h"
#include "internal.h"

namespace mdpl {

mdpl_status make_grid(const double box[3], double r, const int brick[3], Grid* g) {
  g->nbricks = 1;
  g->order = nullptr;
  g->norder = 0;
  for (int k = 0; k < 3; ++k) {
    double side_min = r * (1.0 + 1e-10);
    double q = floor(box[k] / side_min);
    if (!(q >= 3.0)) return MDPL_EBOX;
    if (q > 4096.0) q = 4096.0;
    g->nc[k] = (int)q;
    g->inv_side[k] = q / box[k];
    g->side[k] = box[k] / q;
    g->box[k] = box[k];
    int b = brick[k] < 1 ? 1 : brick[k];
    if (b > g->nc[k]) b = g->nc[k];
    g->B[k] = b;
    g->nb[k] = (g->nc[k] + b - 1) / b;
    g->nbricks *= g->nb[k];
  }
  g->V = g->B[0] * g->B[1] * g->B[2];
  const long long nk = (long long)g->nbricks * g->V;
  if (nk > (1ll << 30)) return MDPL_EBOX;
  g->nkeys = (int)nk;
  return MDPL_OK;
}

size_t sort_bytes(int64_t n) {
  int64_t ntiles = div_up(n, kSortTile);
  int64_t hist = (int64_t)kRadixBins * ntiles + 1;
  int64_t bs = div_up(hist > n ? hist : n, 1024) + 2;
  return 4 * align256(4 * (size_t)n) + align256(4 * (size_t)hist) + align256(4 * (size_t)bs);
}

void sort_carve(char*& p, int64_t n, SortBufs* s) {
  int64_t ntiles = div_up(n, kSortTile);
  int64_t hist = (int64_t)kRadixBins * ntiles + 1;
  int64_t bs = div_up(hist > n ? hist : n, 1024) + 2;
  for (int b = 0; b < 2; ++b) {
    s->keys[b] = (int32_t*)p;
    p += align256(4 * (size_t)n);
    s->vals[b] = (int32_t*)p;
    p += align256(4 * (size_t)n);
  }
  s->hist = (int32_t*)p;
  p += align256(4 * (size_t)hist);
  s->blocksums = (int32_t*)p;
  p += align256(4 * (size_t)bs);
  s->n = n;
  s->ntiles = (int)ntiles;
}

// Cell index along one axis; a non-finite coordinate lands in cell 0.
__device__ __forceinline__ int cell_coord(double x, double L, double inv_side, int nc) {
  const double q = fold(x, L) * inv_side;
  if (q >= 0.0 && q < (double)nc) return (int)q;
  return q >= (double)nc ? nc - 1 : 0;
}

// The particles of each cell in two runs, the lower half of the cell along x
// first (each run in sorted order, so the order stays deterministic), and
// the length of the first run.  The half comes with each sorted value (its
// top bit, set by k_cell_keys for the upper half).  A group of 16 lanes per
// cell, a particle per lane (16 at a time), four cells per wave.
constexpr int kPartLanes = 16;
__global__ __launch_bounds__(256) void k_xhalf_partition(const int32_t* __restrict__ cs, int nkeys,
                                                         const int32_t* __restrict__ vin,
                                                         int32_t* __restrict__ vout,
                                                         int32_t* __restrict__ xlow) {
  const int c = (int)((blockIdx.x * blockDim.x + threadIdx.x) / kPartLanes);
  if (c >= nkeys) return;
  const int lane = (int)threadIdx.x & 63, sub = lane % kPartLanes;
  const unsigned long long group = ((1ull << kPartLanes) - 1) << (lane - sub);
  const unsigned long long below = ((1ull << lane) - 1) & group;
  const int b = cs[c], e = cs[c + 1];
  int lo = 0;  // the cell's lower-half particles
  for (int s0 = b; s0 < e; s0 += kPartLanes) {
    const bool has = s0 + sub < e;
    lo += __popcll(__ballot(has && vin[has ? s0 + sub : b] >= 0) & group);
  }
  if (sub == 0) xlow[c] = lo;
  int nl = 0, nu = 0;  // placed so far
  for (int s0 = b; s0 < e; s0 += kPartLanes) {
    const bool has = s0 + sub < e;
    const int v = has ? vin[s0 + sub] : 0;
    const bool low = has && v >= 0;
    const unsigned long long ml = __ballot(low) & group, mu = __ballot(has && !low) & group;
    if (has)
      vout[low ? b + nl + __popcll(ml & below) : b + lo + nu + __popcll(mu & below)] =
          v & 0x7fffffff;
    nl += __popcll(ml);
    nu += __popcll(mu);
  }
}

__global__ void k_cell_keys(const double* __restrict__ x, const double* __restrict__ y,
                            const double* __restrict__ z, int64_t n, Grid g,
                            int32_t* __restrict__ keys, int32_t* __restrict__ vals, int xbit) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int cx = cell_coord(x[i], g.box[0], g.inv_side[0], g.nc[0]);
  // xbit: the top bit of the value marks the upper half of the cell along x
  // (decided on the quotient that gave the cell index)
  const bool upper = xbit && !(fold(x[i], g.box[0]) * g.inv_side[0] - (double)cx < 0.5);
  int cy = cell_coord(y[i], g.box[1], g.inv_side[1], g.nc[1]);
  int cz = cell_coord(z[i], g.box[2], g.inv_side[2], g.nc[2]);
  keys[i] = cell_key(g, cx, cy, cz);
  vals[i] = (int32_t)((uint32_t)i | (upper ? 0x80000000u : 0u));
}

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const int32_t* __restrict__ keys,
                                                             int64_t n, int shift, int ntiles,
                                                             int32_t* __restrict__ hist) {
  __shared__ int h[kRadixBins];
  const int tid = threadIdx.x;
  h[tid] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll
  for (int k = 0; k < kSortItems; ++k) {
    int64_t idx = base + k * kSortThreads + tid;
    if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & (kRadixBins - 1)], 1);
  }
  __syncthreads();
  hist[(int64_t)tid * ntiles + blockIdx.x] = h[tid];
}

// offs: the histogram scanned within blocks of 1024 counters, sums: the
// exclusive prefix of those blocks (the two halves of an exclusive scan).
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const int32_t* __restrict__ kin, const int32_t* __restrict__ vin, int64_t n, int shift,
    int ntiles, const int32_t* __restrict__ offs, const int32_t* __restrict__ sums,
    int32_t* __restrict__ kout, int32_t* __restrict__ vout) {
  constexpr int kWaves = kSortThreads / 64;
  __shared__ int run[kRadixBins];
  __shared__ int wc[kWaves][kRadixBins];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t hi = (int64_t)tid * ntiles + blockIdx.x;
  run[tid] = offs[hi] + sums[hi >> 10];
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int r = 0; r < kSortItems; ++r) {
#pragma unroll
    for (int w = 0; w < kWaves; ++w) wc[w][tid] = 0;
    __syncthreads();
    const int64_t idx = base + r * kSortThreads + tid;
    const bool valid = idx < n;
    const int key = valid ? kin[idx] : 0;
    const int d = (key >> shift) & (kRadixBins - 1);
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      const bool bit = (d >> b) & 1;
      const unsigned long long m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const int rank = __popcll(peers & below);
    if (valid && rank == 0) wc[wave][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int pos = run[d] + rank;
      for (int w = 0; w < wave; ++w) pos += wc[w][d];
      kout[pos] = key;
      vout[pos] = vin[idx];
    }
    __syncthreads();
    int add = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) add += wc[w][tid];
    run[tid] += add;
  }
}

__global__ void k_cell_start(const int32_t* __restrict__ skeys, int64_t n, int ncells,
                             int32_t* __restrict__ cs) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int k = skeys[s];
  const int prev = s > 0 ? skeys[s - 1] : -1;
  for (int c = prev + 1; c <= k; ++c) cs[c] = (int32_t)s;
  if (s == n - 1)
    for (int c = k + 1; c <= ncells; ++c) cs[c] = (int32_t)n;
}

// ----------------------------------------------------------------- scan
// Block of 256 threads scans 1024 consecutive values.
__global__ __launch_bounds__(256) void k_scan_blocks(const int32_t* in,
                                                     int32_t* out, int64_t n,
                                                     int32_t* __restrict__ sums) {
  __shared__ int wsum[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t base = (int64_t)blockIdx.x * 1024 + tid * 4;
  int v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = (base + k < n) ? in[base + k] : 0;
  int t = v[0] + v[1] + v[2] + v[3];
  // inclusive wave scan of t
  int incl = t;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int o = __shfl_up(incl, off, 64);
    if (lane >= off) incl += o;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  int wbase = 0;
  for (int w = 0; w < wave; ++w) wbase += wsum[w];
  int run = wbase + incl - t;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (tid == 255) sums[blockIdx.x] = wbase + incl;
}

// One block: exclusive scan of the block sums in place (any length), total
// to sums[nb].
__global__ __launch_bounds__(1024) void k_scan_sums(int32_t* __restrict__ sums, int64_t nb) {
  __shared__ int wsum[16];
  __shared__ int carry;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nb; base += 1024) {
    const int64_t i = base + tid;
    const int t = i < nb ? sums[i] : 0;
    int incl = t;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      int o = __shfl_up(incl, off, 64);
      if (lane >= off) incl += o;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int wbase = carry;
    for (int w = 0; w < wave; ++w) wbase += wsum[w];
    if (i < nb) sums[i] = wbase + incl - t;
    __syncthreads();
    if (tid == 1023) carry = wbase + incl;
    __syncthreads();
  }
  if (tid == 0) sums[nb] = carry;
}

__global__ __launch_bounds__(256) void k_scan_add(int32_t* __restrict__ out, int64_t n,
                                                  const int32_t* __restrict__ sums,
                                                  int write_total) {
  const int64_t base = (int64_t)blockIdx.x * 1024 + threadIdx.x * 4;
  const int add = sums[blockIdx.x];
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (base + k < n) out[base + k] += add;
  if (write_total && blockIdx.x == 0 && threadIdx.x == 0) {
    const int64_t nb = (n + 1023) / 1024;
    out[n] = sums[nb];
  }
}

hipError_t exclusive_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* blocksums,
                          bool write_total, hipStream_t st) {
  const int64_t nb = div_up(n, 1024);
  hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nb), dim3(256), 0, st, in, out, n, blocksums);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, st, blocksums, nb);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(256), 0, st, out, n, blocksums,
                     write_total ? 1 : 0);
  return hipGetLastError();
}

hipError_t bin_particles(const double* x, const double* y, const double* z, int64_t n,
                         const Grid& g, SortBufs& s, int32_t* cell_start, int32_t** keys_out,
                         int32_t** vals_out, hipStream_t st, int32_t* xlow) {
  const unsigned nb = (unsigned)div_up(n, 256);
  hipLaunchKernelGGL(k_cell_keys, dim3(nb), dim3(256), 0, st, x, y, z, n, g, s.keys[0], s.vals[0],
                     xlow ? 1 : 0);
  int bits = 1;
  while ((1ll << bits) < (long long)g.nkeys) ++bits;
  const int passes = (bits + kRadixBits - 1) / kRadixBits;
  int cur = 0;
  const int64_t hn = (int64_t)kRadixBins * s.ntiles;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * kRadixBits;
    hipLaunchKernelGGL(k_radix_hist, dim3(s.ntiles), dim3(kSortThreads), 0, st, s.keys[cur], n,
                       shift, s.ntiles, s.hist);
    // the scan's final add is left to the scatter (one launch fewer per pass)
    const int64_t nsb = div_up(hn, 1024);
    hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nsb), dim3(256), 0, st, s.hist, s.hist, hn,
                       s.blocksums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, st, s.blocksums, nsb);
    hipLaunchKernelGGL(k_radix_scatter, dim3(s.ntiles), dim3(kSortThreads), 0, st, s.keys[cur],
                       s.vals[cur], n, shift, s.ntiles, s.hist, s.blocksums, s.keys[cur ^ 1],
                       s.vals[cur ^ 1]);
    cur ^= 1;
  }
  hipLaunchKernelGGL(k_cell_start, dim3(nb), dim3(256), 0, st, s.keys[cur], n, g.nkeys,
                     cell_start);
  *keys_out = s.keys[cur];
  *vals_out = s.vals[cur];
  if (xlow) {
    hipLaunchKernelGGL(k_xhalf_partition, dim3((unsigned)div_up((int64_t)g.nkeys * kPartLanes, 256)), dim3(256), 0, st,
                       cell_start, g.nkeys, s.vals[cur], s.vals[cur ^ 1], xlow);
    *vals_out = s.vals[cur ^ 1];
  }
  return hipGetLastError();
}

// ----------------------------------------------------------------- gathers
__global__ void k_gather_pos(const double* __restrict__ x, const double* __restrict__ y,
                             const double* __restrict__ z, const int32_t* __restrict__ idx,
                             int64_t n, double* __restrict__ ox, double* __restrict__ oy,
                             double* __restrict__ oz, double Lx, double Ly, double Lz, int do_fold) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int32_t j = idx[s];
  double a = x[j], b = y[j], c = z[j];
  if (do_fold) {
    a = fold(a, Lx);
    b = fold(b, Ly);
    c = fold(c, Lz);
  }
  ox[s] = a;
  oy[s] = b;
  oz[s] = c;
}

hipError_t gather_positions(const double* x, const double* y, const double* z, const int32_t* idx,
                            int64_t n, double* ox, double* oy, double* oz, const double* box,
                            bool do_fold, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_pos, dim3((unsigned)div_up(n, 256)), dim3(256), 0, st, x, y, z, idx,
                     n, ox, oy, oz, box[0], box[1], box[2], do_fold ? 1 : 0);
  return hipGetLastError();
}

// Positions of the last build's slots, each moved to the periodic image
// nearest the centre of the cell it was binned in (the images the tiles
// assume), whatever image the caller passes.
__global__ void k_gather_canonical(const double* __restrict__ x, const double* __restrict__ y,
                                   const double* __restrict__ z, const int32_t* __restrict__ idx,
                                   const int32_t* __restrict__ skeys, int64_t n, Grid g,
                                   double* __restrict__ ox, double* __restrict__ oy,
                                   double* __restrict__ oz) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int key = skeys[s];
  const int brick = key / g.V, local = key - brick * g.V;
  const int bx = brick % g.nb[0], by = (brick / g.nb[0]) % g.nb[1], bz = brick / (g.nb[0] * g.nb[1]);
  const int cx = bx * g.B[0] + local % g.B[0];
  const int cy = by * g.B[1] + (local / g.B[0]) % g.B[1];
  const int cz = bz * g.B[2] + local / (g.B[0] * g.B[1]);
  const int32_t j = idx[s];
  const double p[3] = {x[j], y[j], z[j]};
  const int c[3] = {cx, cy, cz};
  double q[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double L = g.box[k];
    const double centre = ((double)c[k] + 0.5) / g.inv_side[k];
    q[k] = p[k] + L * rint((centre - p[k]) / L);
  }
  ox[s] = q[0];
  oy[s] = q[1];
  oz[s] = q[2];
}

hipError_t gather_canonical(const double* x, const double* y, const double* z, const int32_t* idx,
                            const int32_t* skeys, int64_t n, const Grid& g, double* ox, double* oy,
                            double* oz, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_canonical, dim3((unsigned)div_up(n, 256)), dim3(256), 0, st, x, y, z,
                     idx, skeys, n, g, ox, oy, oz);
  return hipGetLastError();
}

template <typename FT>
__global__ void k_reorder(StateArrays src, const int32_t* __restrict__ idx, int64_t n, double Lx,
                          double Ly, double Lz, StateArrays dst, double* xb, double* yb,
                          double* zb, double* bound) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (bound && s == 0) *bound = 0.0;
  if (s >= n) return;
  const int32_t j = idx[s];
  const double a = fold(src.x[j], Lx), b = fold(src.y[j], Ly), c = fold(src.z[j], Lz);
  dst.x[s] = a;
  dst.y[s] = b;
  dst.z[s] = c;
  if (xb) {
    xb[s] = a;
    yb[s] = b;
    zb[s] = c;
  }
  dst.vx[s] = src.vx[j];
  dst.vy[s] = src.vy[j];
  dst.vz[s] = src.vz[j];
  ((FT*)dst.fx)[s] = ((const FT*)src.fx)[j];
  ((FT*)dst.fy)[s] = ((const FT*)src.fy)[j];
  ((FT*)dst.fz)[s] = ((const FT*)src.fz)[j];
  dst.ids[s] = src.ids[j];
}

hipError_t reorder_state(const StateArrays& src, const int32_t* idx, int64_t n, int fbytes,
                         const double* box, StateArrays& dst, double* xb, double* yb, double* zb,
                         double* bound, hipStream_t st) {
  const unsigned nb = (unsigned)div_up(n, 256);
  if (fbytes == 4)
    hipLaunchKernelGGL(k_reorder<float>, dim3(nb), dim3(256), 0, st, src, idx, n, box[0], box[1],
                       box[2], dst, xb, yb, zb, bound);
  else
    hipLaunchKernelGGL(k_reorder<double>, dim3(nb), dim3(256), 0, st, src, idx, n, box[0], box[1],
                       box[2], dst, xb, yb, zb, bound);
  return hipGetLastError();
}

// dst[a][s] = src[a][s] for every array a whose two pointers differ, one
// launch for all of them (the end of a run hands the state back).
template <typename FT>
__global__ void k_copy_state(StateArrays src, StateArrays dst, int64_t n) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  if (src.x != dst.x) dst.x[s] = src.x[s];
  if (src.y != dst.y) dst.y[s] = src.y[s];
  if (src.z != dst.z) dst.z[s] = src.z[s];
  if (src.vx != dst.vx) dst.vx[s] = src.vx[s];
  if (src.vy != dst.vy) dst.vy[s] = src.vy[s];
  if (src.vz != dst.vz) dst.vz[s] = src.vz[s];
  if (src.fx != dst.fx) ((FT*)dst.fx)[s] = ((const FT*)src.fx)[s];
  if (src.fy != dst.fy) ((FT*)dst.fy)[s] = ((const FT*)src.fy)[s];
  if (src.fz != dst.fz) ((FT*)dst.fz)[s] = ((const FT*)src.fz)[s];
  if (src.ids != dst.ids) dst.ids[s] = src.ids[s];
}

hipError_t copy_state(const StateArrays& src, const StateArrays& dst, int64_t n, int fbytes,
                      hipStream_t st) {
  if (src.x == dst.x && src.y == dst.y && src.z == dst.z && src.vx == dst.vx && src.vy == dst.vy &&
      src.vz == dst.vz && src.fx == dst.fx && src.fy == dst.fy && src.fz == dst.fz &&
      src.ids == dst.ids)
    return hipSuccess;
  const unsigned nb = (unsigned)div_up(n, 256);
  if (fbytes == 4)
    hipLaunchKernelGGL(k_copy_state<float>, dim3(nb), dim3(256), 0, st, src, dst, n);
  else
    hipLaunchKernelGGL(k_copy_state<double>, dim3(nb), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

}  // namespace mdpl
