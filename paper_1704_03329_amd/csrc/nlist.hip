// Neighbour-list construction from the cell list (Sec. 3.1: visit the cell
// of i and its 26 neighbours, keep the pairs closer than the list radius;
// GPU neighbour matrix W_{m,i} = m-th neighbour of i).
//
// One thread per particle in cell order.  Candidate cells are walked as
// 9 rows of 3 consecutive cells (one contiguous range when the row does not
// wrap).  The pair test is the exact FP64 minimum-image predicate
//   dx = xi - xj; dx > L/2 ? dx - L : (dx < -L/2 ? dx + L : dx)
//   d2 = (dx*dx + dy*dy) + dz*dz < r2
// with floating-point contraction off, so the list is bit-identical to the
// all-pairs definition for the same FP64 inputs.
#include "device_util.h"
#include "internal.h"

namespace mdpl {

template <int LAYOUT>
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
    const int key = skeys[s];
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
        // up to three ranges along x
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
              if (count < max_nb) {
                if (LAYOUT == 0)
                  nl.nbr[(int64_t)count * nl.stride + s] = t;
                else
                  nl.nbr[s * (int64_t)max_nb + count] = t;
              }
              ++count;
            }
          }
        }
      }
    }
    // layout 0 (force lists) stores the clamped count, layout 1 (analysis)
    // the true count so callers can see an overflow per particle
    nl.cnt[s] = (LAYOUT == 0 && count > max_nb) ? max_nb : count;
    if (count > max_nb) atomicOr(flags, MDPL_FLAG_NL_OVERFLOW);
  }
  // one atomic per wave for the largest count
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
  const unsigned nb = (unsigned)div_up(n, 256);
  if (nl.layout == 0)
    hipLaunchKernelGGL(k_build_nlist<0>, dim3(nb), dim3(256), 0, st, sx, sy, sz, skeys, cell_start,
                       n, g, r2, nl, flags, maxcount);
  else
    hipLaunchKernelGGL(k_build_nlist<1>, dim3(nb), dim3(256), 0, st, sx, sy, sz, skeys, cell_start,
                       n, g, r2, nl, flags, maxcount);
  return hipGetLastError();
}

// Directed pairs in the caller's indices: for slot s, its entries go to
// [offsets[s], offsets[s] + cnt[s]).
__global__ void k_export_pairs(NList nl, const int32_t* __restrict__ perm,
                               const int32_t* __restrict__ offsets, int64_t n,
                               int32_t* __restrict__ i_out, int32_t* __restrict__ j_out,
                               int64_t cap) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int c = nl.cnt[s] > nl.max_nb ? nl.max_nb : nl.cnt[s];
  const int64_t o = offsets[s];
  const int32_t pi = perm[s];
  for (int m = 0; m < c; ++m) {
    if (o + m >= cap) break;
    const int32_t t = (nl.layout == 0) ? nl.nbr[(int64_t)m * nl.stride + s]
                                       : nl.nbr[s * (int64_t)nl.max_nb + m];
    i_out[o + m] = pi;
    j_out[o + m] = perm[t];
  }
}

hipError_t export_pairs(const NList& nl, const int32_t* perm, const int32_t* offsets, int64_t n,
                        int32_t* i_out, int32_t* j_out, int64_t cap, hipStream_t st) {
  hipLaunchKernelGGL(k_export_pairs, dim3((unsigned)div_up(n, 256)), dim3(256), 0, st, nl, perm,
                     offsets, n, i_out, j_out, cap);
  return hipGetLastError();
}

}  // namespace mdpl
