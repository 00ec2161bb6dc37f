// Structure analysis pair loops (Sec. 4).
//
// Bond order (Sec. 4.1, Eqs. Qell and qellm, Algs. sph_I and sph_II): one
// thread per particle walks the 27-cell stencil, tests bonds with the exact
// FP64 predicate and accumulates the moments of Y_l^m in registers; the
// particle loop of Alg. sph_II is fused at the end.  The harmonics are
// evaluated as Y_l^m = N_lm P~_l^m(z) (x + i y)^m with P~_l^m = d^m P_l/dz^m
// (recurrence in l at fixed m), so for l in {4,5,6}
//   Q_l = sqrt( sum_m w_lm (A_lm^2 + B_lm^2) ) / nu,
//   w_l0 = 1, w_lm = 2 (l-m)!/(l+m)! (m >= 1),
// where A + iB = sum_j P~_l^m(z_j) (x_j + i y_j)^m (the -m terms have the
// same modulus and are folded into the factor 2).  Unit vectors from the
// FP64 separation, harmonics in FP32.
//
// Common-neighbour analysis (Sec. 4.2, Algs. cna_I to cna_III and
// max_cluster_size): one thread per particle i.  The bonds among the
// neighbours of i are found once, by the exact bond test between every two
// members of N(i), and kept as adjacency bit masks over N(i) (bit b of
// adj[a] <=> neighbour a bonded to neighbour b).  For the bond
// (i, j = N(i)[b]): common neighbours C = adj[b] (members of N(i) bonded to
// j), n_cn = |C|, n_b = half the degree sum inside C, and n_lcb = largest
// number of edges in a connected component of C, by mask flood fill.  All
// integer work, bit-exact.
#include "device_util.h"
#include "internal.h"

namespace mdpl {

// 2 (l-m)!/(l+m)! for m >= 1 and 1 for m = 0.
__device__ __forceinline__ float qweight(int l, int m) {
  if (m == 0) return 1.0f;
  double r = 2.0;
  for (int k = l - m + 1; k <= l + m; ++k) r /= (double)k;
  return (float)r;
}

template <bool Q5>
__global__ __launch_bounds__(256) void k_boa(const double* __restrict__ sx,
                                             const double* __restrict__ sy,
                                             const double* __restrict__ sz,
                                             const int32_t* __restrict__ skeys,
                                             const int32_t* __restrict__ cs,
                                             const int32_t* __restrict__ perm, int64_t n, Grid g,
                                             double rc2, float* __restrict__ q4,
                                             float* __restrict__ q5, float* __restrict__ q6,
                                             int32_t* __restrict__ nnb) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  // moments: A[l][m] (m = 0..l), B[l][m] (m = 1..l) for l = 4, 5, 6
  float A4[5] = {0}, B4[5] = {0}, A5[6] = {0}, B5[6] = {0}, A6[7] = {0}, B6[7] = {0};
  int nu = 0;
  const double xi = sx[s], yi = sy[s], zi = sz[s];
  const double Lx = g.box[0], Ly = g.box[1], Lz = g.box[2];
  const double hx = 0.5 * Lx, hy = 0.5 * Ly, hz = 0.5 * Lz;
  const int n0 = g.nc[0], n1 = g.nc[1], n2 = g.nc[2];
  const int key = skeys[s];
  const int cx = key % n0, cy = (key / n0) % n1, cz = key / (n0 * n1);
  for (int oz = -1; oz <= 1; ++oz) {
    int z2 = cz + oz;
    z2 += (z2 < 0) ? n2 : 0;
    z2 -= (z2 >= n2) ? n2 : 0;
    for (int oy = -1; oy <= 1; ++oy) {
      int y2 = cy + oy;
      y2 += (y2 < 0) ? n1 : 0;
      y2 -= (y2 >= n1) ? n1 : 0;
      const int row = (z2 * n1 + y2) * n0;
      for (int ox = -1; ox <= 1; ++ox) {
        int x2 = cx + ox;
        x2 += (x2 < 0) ? n0 : 0;
        x2 -= (x2 >= n0) ? n0 : 0;
        const int c = row + x2;
        for (int t = cs[c]; t < cs[c + 1]; ++t) {
          if (t == s) continue;
          double dx, dy, dz;
          const double d2 =
              exact_sep(xi, yi, zi, sx[t], sy[t], sz[t], Lx, Ly, Lz, hx, hy, hz, dx, dy, dz);
          if (!(d2 < rc2)) continue;
          ++nu;
          const float ir = __builtin_amdgcn_rsqf((float)d2);  // the bond test above is FP64
          const float ux = (float)dx * ir, uy = (float)dy * ir, uz = (float)dz * ir;
          // (x + i y)^m, m = 0..6
          float cr[7], ci[7];
          cr[0] = 1.0f;
          ci[0] = 0.0f;
#pragma unroll
          for (int m = 1; m <= 6; ++m) {
            cr[m] = cr[m - 1] * ux - ci[m - 1] * uy;
            ci[m] = cr[m - 1] * uy + ci[m - 1] * ux;
          }
          // P~_l^m(z) for l = m..6 via (l-m) P_l = (2l-1) z P_{l-1} - (l+m-1) P_{l-2}
#pragma unroll
          for (int m = 0; m <= 6; ++m) {
            float dfact = 1.0f;  // (2m-1)!!
#pragma unroll
            for (int k = 1; k <= m; ++k) dfact *= (float)(2 * k - 1);
            float pm2 = 0.0f, pm1 = dfact;  // P_{m-1} (=0), P_m
#pragma unroll
            for (int l = m; l <= 6; ++l) {
              float p;
              if (l == m)
                p = dfact;
              else if (l == m + 1)
                p = (float)(2 * m + 1) * uz * dfact;
              else
                p = ((float)(2 * l - 1) * uz * pm1 - (float)(l + m - 1) * pm2) *
                    (1.0f / (float)(l - m));
              if (l > m) {
                pm2 = pm1;
                pm1 = p;
              }
              if (l == 4) {
                A4[m] += p * cr[m];
                B4[m] += p * ci[m];
              } else if (Q5 && l == 5) {
                A5[m] += p * cr[m];
                B5[m] += p * ci[m];
              } else if (l == 6) {
                A6[m] += p * cr[m];
                B6[m] += p * ci[m];
              }
            }
          }
        }
      }
    }
  }
  float s4 = 0.0f, s5 = 0.0f, s6 = 0.0f;
#pragma unroll
  for (int m = 0; m <= 4; ++m) s4 += qweight(4, m) * (A4[m] * A4[m] + B4[m] * B4[m]);
#pragma unroll
  for (int m = 0; m <= 5; ++m) s5 += qweight(5, m) * (A5[m] * A5[m] + B5[m] * B5[m]);
#pragma unroll
  for (int m = 0; m <= 6; ++m) s6 += qweight(6, m) * (A6[m] * A6[m] + B6[m] * B6[m]);
  const float inv = nu > 0 ? 1.0f / (float)nu : 0.0f;
  const int32_t o = perm[s];
  q4[o] = sqrtf(s4) * inv;
  if (q5) q5[o] = sqrtf(s5) * inv;
  q6[o] = sqrtf(s6) * inv;
  nnb[o] = nu;
}

hipError_t boa_q(const double* sx, const double* sy, const double* sz, const int32_t* skeys,
                 const int32_t* cell_start, const int32_t* perm, int64_t n, const Grid& g,
                 double rc2, float* q4, float* q5, float* q6, int32_t* nnb, hipStream_t st) {
  if (q5)
    hipLaunchKernelGGL(k_boa<true>, dim3((unsigned)div_up(n, 256)), dim3(256), 0, st, sx, sy, sz,
                       skeys, cell_start, perm, n, g, rc2, q4, q5, q6, nnb);
  else
    hipLaunchKernelGGL(k_boa<false>, dim3((unsigned)div_up(n, 256)), dim3(256), 0, st, sx, sy, sz,
                       skeys, cell_start, perm, n, g, rc2, q4, q5, q6, nnb);
  return hipGetLastError();
}

// ------------------------------------------------------------------- CNA
constexpr int kCnaThreads = 64;
constexpr int kCnaMax = 64;

__device__ __forceinline__ uint32_t pack_triplet(int ncn, int nb, int nlcb) {
  return ((uint32_t)ncn << 20) | ((uint32_t)nb << 10) | (uint32_t)nlcb;
}

template <typename M>
__device__ __forceinline__ int popc_mask(M m) {
  if constexpr (sizeof(M) == 8) return __popcll(m);
  else return __popc(m);
}
template <typename M>
__device__ __forceinline__ int lowest_bit(M m) {
  if constexpr (sizeof(M) == 8) return __ffsll((long long)m) - 1;
  else return __ffs(m) - 1;
}

// MAXNB: LDS columns per thread (16, 32 or 64); M: adjacency mask type with
// at least MAXNB bits.  Fewer columns, more waves per CU.
//
// The adjacency among N(i) (bonds with both ends in N(i), i.e. the part of
// Ebar(i) that any triplet of i can read) is formed from the exact FP64 bond
// test between every two members of N(i), on the stored positions.  It
// therefore needs only the complete list of i itself: an atom with at most
// max_nb bonds gets its exact triplets whatever the bond counts of its
// neighbours.  An atom with more than max_nb bonds gets no triplets and the
// label OTHER (every reference signature has 12 or 14 bonds, so the label
// is exact whenever max_nb >= 14).
template <int MAXNB, typename M>
__global__ __launch_bounds__(kCnaThreads) void k_cna(NList nl, const double* __restrict__ sx,
                                                     const double* __restrict__ sy,
                                                     const double* __restrict__ sz, Grid g,
                                                     double rc2, const int32_t* __restrict__ perm,
                                                     int64_t n, uint32_t* __restrict__ trip,
                                                     int32_t* __restrict__ nnb,
                                                     uint8_t* __restrict__ label, int max_out) {
  static_assert(8 * sizeof(M) >= MAXNB, "mask narrower than the list");
  // per-thread columns: L[k][tid] member k of N(i) (later the triplet codes);
  // adj[k][tid] the members bonded to member k
  __shared__ int32_t L[MAXNB][kCnaThreads];
  __shared__ M adj[MAXNB][kCnaThreads];
  const int tid = threadIdx.x;
  const int64_t s = (int64_t)blockIdx.x * kCnaThreads + tid;
  if (s >= n) return;
  const int max_nb = nl.max_nb;
  const int ni = nl.cnt[s];
  const int32_t o = perm[s];
  nnb[o] = ni;
  if (ni > max_nb) {  // list incomplete: no signature
    label[o] = 0;
    return;
  }
  const int32_t* row = nl.nbr + s * (int64_t)max_nb;
  for (int k = 0; k < ni; ++k) {
    L[k][tid] = row[k];
    adj[k][tid] = 0;
  }
  const double Lx = g.box[0], Ly = g.box[1], Lz = g.box[2];
  const double hx = 0.5 * Lx, hy = 0.5 * Ly, hz = 0.5 * Lz;
  for (int a = 0; a < ni; ++a) {
    const int32_t va = L[a][tid];
    const double xa = sx[va], ya = sy[va], za = sz[va];
    M ma = adj[a][tid];
    for (int b = a + 1; b < ni; ++b) {
      const int32_t vb = L[b][tid];
      if (exact_d2(xa, ya, za, sx[vb], sy[vb], sz[vb], Lx, Ly, Lz, hx, hy, hz) < rc2) {
        ma |= (M)1 << b;
        adj[b][tid] |= (M)1 << a;
      }
    }
    adj[a][tid] = ma;
  }
  // triplet of every bond (i, N(i)[b]); codes reuse the L column
  uint32_t* code = (uint32_t*)&L[0][0];
  for (int b = 0; b < ni; ++b) {
    const M cm = adj[b][tid];  // common neighbours of i and N(i)[b]
    const int ncn = popc_mask(cm);
    int deg = 0;
    for (M r = cm; r; r &= r - 1) deg += popc_mask(adj[lowest_bit(r)][tid] & cm);
    const int nbonds = deg >> 1;
    int best = 0;
    M rem = cm;
    while (rem) {
      M comp = rem & (~rem + (M)1);
      M front = comp;
      while (front) {
        M nxt = 0;
        for (M r = front; r; r &= r - 1) nxt |= adj[lowest_bit(r)][tid] & cm;
        nxt &= ~comp;
        comp |= nxt;
        front = nxt;
      }
      int e2 = 0;
      for (M r = comp; r; r &= r - 1) e2 += popc_mask(adj[lowest_bit(r)][tid] & comp);
      const int edges = e2 >> 1;
      best = edges > best ? edges : best;
      rem &= ~comp;
    }
    code[b * kCnaThreads + tid] = pack_triplet(ncn, nbonds, best);
  }
  // insertion sort of the codes (ascending)
  for (int a = 1; a < ni; ++a) {
    const uint32_t key = code[a * kCnaThreads + tid];
    int b = a - 1;
    while (b >= 0 && code[b * kCnaThreads + tid] > key) {
      code[(b + 1) * kCnaThreads + tid] = code[b * kCnaThreads + tid];
      --b;
    }
    code[(b + 1) * kCnaThreads + tid] = key;
  }
  const uint32_t t421 = pack_triplet(4, 2, 1), t422 = pack_triplet(4, 2, 2);
  const uint32_t t444 = pack_triplet(4, 4, 4), t666 = pack_triplet(6, 6, 6);
  int c421 = 0, c422 = 0, c444 = 0, c666 = 0;
  for (int a = 0; a < ni; ++a) {
    const uint32_t c = code[a * kCnaThreads + tid];
    c421 += c == t421;
    c422 += c == t422;
    c444 += c == t444;
    c666 += c == t666;
    if (a < max_out) trip[(int64_t)o * max_out + a] = c;
  }
  uint8_t lab = 0;
  if (ni == 12 && c421 == 12) lab = 1;
  else if (ni == 12 && c421 == 6 && c422 == 6) lab = 2;
  else if (ni == 14 && c666 == 8 && c444 == 6) lab = 3;
  label[o] = lab;
}

hipError_t cna_signatures(const NList& nl, const double* sx, const double* sy, const double* sz,
                          const Grid& g, double rc2, const int32_t* perm, int64_t n,
                          uint32_t* trip, int32_t* nnb, uint8_t* label, int max_out,
                          hipStream_t st) {
  const dim3 grid((unsigned)div_up(n, kCnaThreads)), block(kCnaThreads);
  if (nl.max_nb <= 16)
    hipLaunchKernelGGL((k_cna<16, uint32_t>), grid, block, 0, st, nl, sx, sy, sz, g, rc2, perm, n,
                       trip, nnb, label, max_out);
  else if (nl.max_nb <= 32)
    hipLaunchKernelGGL((k_cna<32, uint32_t>), grid, block, 0, st, nl, sx, sy, sz, g, rc2, perm, n,
                       trip, nnb, label, max_out);
  else
    hipLaunchKernelGGL((k_cna<kCnaMax, uint64_t>), grid, block, 0, st, nl, sx, sy, sz, g, rc2,
                       perm, n, trip, nnb, label, max_out);
  return hipGetLastError();
}

}  // namespace mdpl
