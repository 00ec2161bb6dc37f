// Atom-centred symmetry-function descriptors of the learned potential (not
// a construct of the paper; it runs on the paper's pair-loop machinery: the
// LJ tile list with a cutoff test at rc).
//
// Per atom i, neighbours j with r = |r_j - r_i| < rc, fc(r) = (cos(pi r/rc)+1)/2:
//   radial   G_k = sum_j exp(-eta_r (r - R_k)^2) fc,  R_k = 0.85 + 0.11 k, k < 16
//   angular  G_(zeta,lam,eta) = 2^(1-zeta) sum_{j != k} (1 + lam cos t_jik)^zeta w_j w_k,
//            w = exp(-eta r^2) fc, (zeta, lam, eta) in {1,4} x {+1,-1} x {0.5, 2}
// The angular double sum is formed from moments through the addition
// theorem: with P~_l^m = d^m P_l / dz^m and (x + i y)^m of the unit vector,
//   C_lm = sum_j w_j P~_l^m(z) Re (x+iy)^m,  S_lm = sum_j w_j P~_l^m(z) Im (x+iy)^m,
//   T_l  = sum_{j != k} P_l(cos t_jk) w_j w_k
//        = sum_m om_lm (C_lm^2 + S_lm^2) - sum_j w_j^2,
//   om_l0 = 1, om_lm = 2 (l-m)!/(l+m)!,
// and (1 + lam c)^zeta = sum_l a_l P_l(c):  zeta = 1: a = (1, lam);
//   zeta = 4: a = (16/5, 32 lam/5, 32/7, 8 lam/5, 8/35).
//
// Both passes take separations from the FP32 tile-centred coordinates of
// the LJ force pass (within about 4e-7 of the FP64 ones for these tiles);
// the features' error stays that of their FP32 arithmetic, about 5e-6 of
// the outermost radial feature, and a pair decided differently at rc adds
// nothing, as every term vanishes smoothly there.
//
// Moments are packed per eta as 25 floats, l = 0..4: C_l0 at l^2, C_lm at
// l^2 + 2m - 1, S_lm at l^2 + 2m.  The forward sums w z^k Re/Im (x+iy)^m
// (k <= 4 - m, also 25 per eta) over the pairs and forms the moments from
// them once per particle, with the coefficients of the P~_l^m.
//
// Backward (forces): with b_l = dE/dT_l, the adjoint coefficients
//   alpha_lm = 2 om_lm b_l C_lm, gamma_lm = 2 om_lm b_l S_lm, delta = -2 sum_l b_l
// make dE/du_ij = sum_eta [ w' Phi uh + w (grad Phi - (uh . grad Phi) uh) / r
//                          + delta w w' uh ] + sum_k dE/dG_k phi_k'(r) uh,
// Phi(x,y,z) = sum_lm P~_l^m(z) (alpha c_m + gamma s_m), u_ij = r_j - r_i,
// and F_a = sum_{j in N(a)} (dE_a/du_aj - dE_j/du_ja).  k_desc_bwd forms each
// term g_ij = dE_i/du_ij once, with centre i's coefficients only, and
// scatters it: + g_ij to particle i (a register sum) and - g_ij to
// neighbour j (a 64-bit fixed-point LDS atomic on the tile slot, then one
// global FP32 atomic per touched slot).  The order in which the global
// atomics land varies from run to run, so the last bits of the forces do too.
#include <math.h>

#include "device_util.h"
#include "internal.h"
#include "tile.h"

namespace mdpl {

constexpr int kNRad = 16;
constexpr int kNFeat = 24;
constexpr int kNMom = 25;
constexpr float kEtaR = 41.32231404958678f;  // 1 / (2 * 0.11^2)

// exp(x) on the hardware base-2 exponential
__device__ __forceinline__ float exp_hw(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }

// e_k = exp(-eta_r (r - R_k)^2), k < 16.  With eta_r = 1/(2 * 0.11^2) and
// R_{k+1} = R_k + 0.11 the ratio e_{k+1}/e_k = rho_k = exp((r - R_k)/0.11 - 1/2)
// and rho_{k+1} = rho_k / e, so three terms follow from every fourth by
// multiplication; the anchors are exact exponentials (a chain from k = 0
// would underflow for r far from R_0).
__device__ __forceinline__ void radial_basis(float r, float e[kNRad]) {
  const float inv_e = 0.36787944117144233f;
  float rho = exp_hw((r - 0.85f) * (1.0f / 0.11f) - 0.5f);  // rho_0
#pragma unroll
  for (int a = 0; a < kNRad; a += 4) {
    const float d = r - (0.85f + 0.11f * (float)a);
    e[a] = exp_hw(-kEtaR * d * d);
#pragma unroll
    for (int j = 1; j < 4; ++j) {
      e[a + j] = e[a + j - 1] * rho;
      rho *= inv_e;
    }
    rho *= inv_e;  // rho_{a+4}
  }
}

// 2 (l-m)!/(l+m)! (1 for m = 0), indexed l(l+1)/2 + m
__device__ __forceinline__ float omega(int idx) {
  const float t[15] = {1.0f,
                       1.0f, 1.0f,
                       1.0f, 1.0f / 3.0f, 1.0f / 12.0f,
                       1.0f, 1.0f / 6.0f, 1.0f / 60.0f, 1.0f / 360.0f,
                       1.0f, 1.0f / 10.0f, 1.0f / 180.0f, 1.0f / 2520.0f, 1.0f / 20160.0f};
  return t[idx];
}

// P~_l^m(z) = d^m P_l / dz^m for l <= 4, the polynomials behind the moment
// and adjoint coefficients below:
//   m = 0: 1, z, 1.5 z^2 - 0.5, 2.5 z^3 - 1.5 z, 4.375 z^4 - 3.75 z^2 + 0.375
//   m = 1: 1, 3 z, 7.5 z^2 - 1.5, 17.5 z^3 - 7.5 z          (l = 1 .. 4)
//   m = 2: 3, 15 z, 52.5 z^2 - 7.5                           (l = 2 .. 4)
//   m = 3: 15, 105 z                                         (l = 3, 4)
//   m = 4: 105                                               (l = 4)

// a_l of (1 + lam c)^zeta times 2^(1-zeta), for angular feature index a
// (a = zi*4 + li*2 + ei, zeta = (1,4)[zi], lam = (+1,-1)[li])
__device__ __forceinline__ float ang_coef(int a, int l) {
  const int zi = a >> 2, li = (a >> 1) & 1;
  const float lam = li ? -1.0f : 1.0f;
  if (zi == 0) return l == 0 ? 1.0f : (l == 1 ? lam : 0.0f);
  const float c4[5] = {3.2f, 6.4f, 32.0f / 7.0f, 1.6f, 8.0f / 35.0f};
  const float sgn = (l & 1) ? lam : 1.0f;
  return 0.125f * c4[l] * sgn;
}

struct DescIO {
  float* G;                // n x 24 (forward output)
  float* mom;              // n x 50 (forward output, nullable; backward input)
  const float* dEdG;       // n x 24 (backward input), caller order
  const int32_t* perm;     // slot -> caller index (nullable: identity)
  float* fx;               // forces (backward output; cleared by the forward if given), caller order
  float* fy;
  float* fz;
};

// The lowest set bit of the 128-bit mask (m0, m1), cleared; 128 when none is
// left.  Selects only, so that the masks stay in registers.
__device__ __forceinline__ int next_bit(uint64_t& m0, uint64_t& m1) {
  const bool lo = m0 != 0;
  const uint64_t mm = lo ? m0 : m1;
  const int b = mm ? __builtin_ctzll(mm) + (lo ? 0 : 64) : 128;
  const uint64_t cl = mm & (mm - 1);
  m0 = lo ? cl : m0;
  m1 = lo ? m1 : cl;
  return b;
}

// ------------------------------------------------------------- forward
__global__ __launch_bounds__(512) void k_desc_fwd(const double* __restrict__ x,
                                                   const double* __restrict__ y,
                                                   const double* __restrict__ z,
                                                   const int32_t* __restrict__ cs, Grid g,
                                                   TileList tl, float rc, DescIO io) {
  __shared__ TileF32 t;
  __shared__ uint16_t home[kBrickMax];
  const int brick = brick_of_block(g);
  if (brick >= g.nbricks) return;
  const int total = tile_cells(g, brick, cs, t);
  const int nt = total < TileF32::kCap ? total : TileF32::kCap;
  const int s0 = cs[brick * g.V], s1 = cs[(brick + 1) * g.V];
  double ox, oy, oz;
  tile_centre(g, brick, ox, oy, oz);
  tile_load_f32(g, x, y, z, total, ox, oy, oz, s0, t, home);  // ends with a barrier
  const float rc2 = rc * rc;
  const float half_rev = 0.5f / rc;  // revolutions per unit r of cos(pi r / rc)
  for (int s = s0 + (int)threadIdx.x; s < s1; s += blockDim.x) {
    const int hs = s - s0 < kBrickMax ? home[s - s0] : TileF32::kDummy;
    const float xi = t.px[hs], yi = t.py[hs], zi = t.pz[hs];
    float G[kNRad];
    float M[2][kNMom];
    float diag[2] = {0.0f, 0.0f};
#pragma unroll
    for (int k = 0; k < kNRad; ++k) G[k] = 0.0f;
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
      for (int k = 0; k < kNMom; ++k) M[e][k] = 0.0f;
    const int ng = (tl.cnt[s] + 3) >> 2;
    const uint64_t* __restrict__ col = tl.nbr + s;
    for (int c0 = 0; c0 < ng; c0 += 32) {
      // the in-range entries of up to 32 words as two bit masks (bit 4 w + q
      // of m[w / 16]: entry q of word c0 + w); the terms below then run on
      // the lanes' in-range entries only
      const int wn = ng - c0 < 32 ? ng - c0 : 32;
      uint64_t m0 = 0, m1 = 0;
      for (int wg = 0; wg < wn; wg += 4) {
        // four words in flight at once (rows past the lane's last word read
        // its last word again and are ignored)
        uint64_t wd[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
          wd[k] = col[(int64_t)(c0 + (wg + k < wn ? wg + k : wn - 1)) * tl.stride];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int w = wg + k;
          uint64_t bits = 0;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            int u = (int)((wd[k] >> (16 * q)) & 0xffff) >> kFullShift;
            u = u < nt ? u : TileF32::kDummy;  // padding: the far-away dummy slot
            const float dx = t.px[u] - xi, dy = t.py[u] - yi, dz = t.pz[u] - zi;
            const float d2 = dx * dx + dy * dy + dz * dz;
            if (d2 < rc2) bits |= 1ull << q;
          }
          if (w < wn) {
            if (w < 16) m0 |= bits << (4 * w);
            else m1 |= bits << (4 * (w - 16));
          }
        }
      }
      // one in-range entry per lane and trip; the word of the next one is
      // loaded a trip ahead
      // (the load goes to a valid row even when no bit is left)
      int b = next_bit(m0, m1);
      uint64_t word = col[(int64_t)(c0 + (b < 128 ? b >> 2 : 0)) * tl.stride];
      while (b < 128) {
        const int u = (int)((word >> (16 * (b & 3))) & 0xffff) >> kFullShift;
        b = next_bit(m0, m1);
        word = col[(int64_t)(c0 + (b < 128 ? b >> 2 : 0)) * tl.stride];
        // keep the load here, a trip ahead of its use (no memory operation
        // may move across this point)
        asm volatile("" ::: "memory");
        const float dx = t.px[u] - xi, dy = t.py[u] - yi, dz = t.pz[u] - zi;
        const float d2f = dx * dx + dy * dy + dz * dz;
        // 1/r from the hardware reciprocal square root (about 1 ulp), r = d2/r
        const float ir = __builtin_amdgcn_rsqf(d2f);
        const float r = d2f * ir;
        const float ux = dx * ir, uy = dy * ir, uz = dz * ir;
        const float fc = 0.5f * (__builtin_amdgcn_cosf(r * half_rev) + 1.0f);  // cos(pi r / rc)
        float eb[kNRad];
        radial_basis(r, eb);
#pragma unroll
        for (int k = 0; k < kNRad; ++k) G[k] += eb[k] * fc;
        // per eta the sums of w z^k Re/Im (x+iy)^m, k <= 4 - m (the moments
        // follow from them by the coefficients of P~_l^m, once per particle)
        const float z2 = uz * uz, z3 = z2 * uz, z4 = z2 * z2;
        const float c2 = ux * ux - uy * uy, s2 = 2.0f * ux * uy;
        const float c3 = c2 * ux - s2 * uy, s3 = c2 * uy + s2 * ux;
        const float c4 = c3 * ux - s3 * uy, s4 = c3 * uy + s3 * ux;
        const float q[kNMom] = {1.0f, uz,      z2,      z3, z4,      ux,      ux * uz, ux * z2, ux * z3,
                                uy,   uy * uz, uy * z2, uy * z3, c2, c2 * uz, c2 * z2, s2,      s2 * uz,
                                s2 * z2, c3, c3 * uz, s3, s3 * uz, c4, s4};
        const float g0 = exp_hw(-0.5f * r * r);
        const float g1 = (g0 * g0) * (g0 * g0);  // exp(-2 r^2)
        const float w0 = g0 * fc;
        const float w1 = g1 * fc;
        diag[0] += w0 * w0;
        diag[1] += w1 * w1;
#pragma unroll
        for (int k = 0; k < kNMom; ++k) {
          M[0][k] += w0 * q[k];
          M[1][k] += w1 * q[k];
        }
      }
    }
    // z-power sums (order of q above) -> C_lm, S_lm in the moment layout
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const float* N = M[e];
      float C[kNMom];
      C[0] = N[0];
      C[1] = N[1];
      C[4] = 1.5f * N[2] - 0.5f * N[0];
      C[9] = 2.5f * N[3] - 1.5f * N[1];
      C[16] = 4.375f * N[4] - 3.75f * N[2] + 0.375f * N[0];
      C[2] = N[5];                          // C_11
      C[3] = N[9];                          // S_11
      C[5] = 3.0f * N[6];                   // C_21
      C[6] = 3.0f * N[10];                  // S_21
      C[10] = 7.5f * N[7] - 1.5f * N[5];    // C_31
      C[11] = 7.5f * N[11] - 1.5f * N[9];   // S_31
      C[17] = 17.5f * N[8] - 7.5f * N[6];   // C_41
      C[18] = 17.5f * N[12] - 7.5f * N[10]; // S_41
      C[7] = 3.0f * N[13];                  // C_22
      C[8] = 3.0f * N[16];                  // S_22
      C[12] = 15.0f * N[14];                // C_32
      C[13] = 15.0f * N[17];                // S_32
      C[19] = 52.5f * N[15] - 7.5f * N[13]; // C_42
      C[20] = 52.5f * N[18] - 7.5f * N[16]; // S_42
      C[14] = 15.0f * N[19];                // C_33
      C[15] = 15.0f * N[21];                // S_33
      C[21] = 105.0f * N[20];               // C_43
      C[22] = 105.0f * N[22];               // S_43
      C[23] = 105.0f * N[23];               // C_44
      C[24] = 105.0f * N[24];               // S_44
#pragma unroll
      for (int k = 0; k < kNMom; ++k) M[e][k] = C[k];
    }
    float T[2][5];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
#pragma unroll
      for (int l = 0; l <= 4; ++l) {
        float acc = M[e][l * l] * M[e][l * l];
#pragma unroll
        for (int m = 1; m <= l; ++m) {
          const float a = M[e][l * l + 2 * m - 1], b = M[e][l * l + 2 * m];
          acc += omega(l * (l + 1) / 2 + m) * (a * a + b * b);
        }
        T[e][l] = acc - diag[e];
      }
    }
    const int64_t o = io.perm ? (int64_t)io.perm[s] : (int64_t)s;
    if (io.fx) {  // the backward's outputs, cleared for its atomics
      io.fx[o] = 0.0f;
      io.fy[o] = 0.0f;
      io.fz[o] = 0.0f;
    }
    float* __restrict__ Go = io.G + o * kNFeat;
#pragma unroll
    for (int k = 0; k < kNRad; ++k) Go[k] = G[k];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const int e = a & 1;
      float acc = 0.0f;
#pragma unroll
      for (int l = 0; l <= 4; ++l) acc += ang_coef(a, l) * T[e][l];
      Go[kNRad + a] = acc;
    }
    if (io.mom) {
      float* __restrict__ Mo = io.mom + o * (2 * kNMom);
#pragma unroll
      for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int k = 0; k < kNMom; ++k) Mo[e * kNMom + k] = M[e][k];
    }
  }
}

// ------------------------------------------------------------- adjoint
// Phi of one eta regrouped by m: Phi = sum_m A_m(z) Re (x+iy)^m + B_m(z) Im (x+iy)^m
// with A_m(z) = sum_{l>=m} alpha_lm P~_l^m(z) and B_m likewise with gamma.  The
// coefficients of A_m and B_m in powers of z (those of the P~_l^m in the
// table above, collected per m) are stored per eta, 25 floats, as
//   A_0[5] A_1[4] B_1[4] A_2[3] B_2[3] A_3[2] B_3[2] A_4 B_4   (constant term first).
// One pair then costs a Horner value and derivative per polynomial instead of
// the 15 (l, m) terms of each sum.
__device__ __forceinline__ void zpoly_of(const float* __restrict__ al, float* __restrict__ zc) {
  auto A = [&](int l, int m) { return al[m == 0 ? l * l : l * l + 2 * m - 1]; };
  auto B = [&](int l, int m) { return al[l * l + 2 * m]; };
  zc[0] = A(0, 0) - 0.5f * A(2, 0) + 0.375f * A(4, 0);
  zc[1] = A(1, 0) - 1.5f * A(3, 0);
  zc[2] = 1.5f * A(2, 0) - 3.75f * A(4, 0);
  zc[3] = 2.5f * A(3, 0);
  zc[4] = 4.375f * A(4, 0);
  zc[5] = A(1, 1) - 1.5f * A(3, 1);
  zc[6] = 3.0f * A(2, 1) - 7.5f * A(4, 1);
  zc[7] = 7.5f * A(3, 1);
  zc[8] = 17.5f * A(4, 1);
  zc[9] = B(1, 1) - 1.5f * B(3, 1);
  zc[10] = 3.0f * B(2, 1) - 7.5f * B(4, 1);
  zc[11] = 7.5f * B(3, 1);
  zc[12] = 17.5f * B(4, 1);
  zc[13] = 3.0f * A(2, 2) - 7.5f * A(4, 2);
  zc[14] = 15.0f * A(3, 2);
  zc[15] = 52.5f * A(4, 2);
  zc[16] = 3.0f * B(2, 2) - 7.5f * B(4, 2);
  zc[17] = 15.0f * B(3, 2);
  zc[18] = 52.5f * B(4, 2);
  zc[19] = 15.0f * A(3, 3);
  zc[20] = 105.0f * A(4, 3);
  zc[21] = 15.0f * B(3, 3);
  zc[22] = 105.0f * B(4, 3);
  zc[23] = 105.0f * A(4, 4);
  zc[24] = 105.0f * B(4, 4);
}

// K = (z-polynomials of Phi for eta 0.5 [25], for eta 2 [25], delta_0, delta_1,
//      dE/dG_k for the 16 radial features, k dE/dG_k) of one particle, from its
// dE/dG (24) and moments (50); formed where the backward needs them.
__device__ __forceinline__ void adjoint_coef(const float* __restrict__ d,
                                             const float* __restrict__ mm, float out[84]) {
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    float b[5];
    float bsum = 0.0f;
#pragma unroll
    for (int l = 0; l <= 4; ++l) {
      float acc = 0.0f;
#pragma unroll
      for (int a = e; a < 8; a += 2) acc += d[kNRad + a] * ang_coef(a, l);
      b[l] = acc;
      bsum += acc;
    }
    float al[kNMom];  // alpha_lm / gamma_lm in the moment layout
#pragma unroll
    for (int l = 0; l <= 4; ++l) {
      al[l * l] = 2.0f * b[l] * mm[e * kNMom + l * l];
#pragma unroll
      for (int m = 1; m <= l; ++m) {
        const float w = 2.0f * omega(l * (l + 1) / 2 + m) * b[l];
        al[l * l + 2 * m - 1] = w * mm[e * kNMom + l * l + 2 * m - 1];
        al[l * l + 2 * m] = w * mm[e * kNMom + l * l + 2 * m];
      }
    }
    zpoly_of(al, out + e * kNMom);
    out[50 + e] = -2.0f * bsum;
  }
#pragma unroll
  for (int k = 0; k < kNRad; ++k) {
    out[52 + k] = d[k];
    out[68 + k] = (float)k * d[k];
  }
}

// value v and derivative dv of c[0] + c[1] z + ... + c[D] z^D (Horner)
template <int D>
__device__ __forceinline__ void poly_vd(const float* __restrict__ c, float z, float& v, float& dv) {
  v = c[D];
  dv = 0.0f;
  if (D == 0) return;
  dv = v;
  v = v * z + c[D - 1];
#pragma unroll
  for (int i = D - 2; i >= 0; --i) {
    dv = dv * z + v;
    v = v * z + c[i];
  }
}

// dE/du for a centre with adjoint coefficients K and neighbour vector u
// (length r, 1/r = ir, unit vector uh), accumulated into (gx, gy, gz).
// With Phi in the z-polynomial form, grad Phi (of the polynomial in x, y, z) is
//   d/dz: sum_m A_m' Re (x+iy)^m + B_m' Im (x+iy)^m,
//   d/dx: sum_m m (A_m Re (x+iy)^(m-1) + B_m Im (x+iy)^(m-1)),
//   d/dy: sum_m m (-A_m Im (x+iy)^(m-1) + B_m Re (x+iy)^(m-1)).
__device__ __forceinline__ void pair_grad(const float* __restrict__ K, float r, float ir, float ux,
                                          float uy, float uz, float fc, float dfc, float& gx,
                                          float& gy, float& gz) {
  // (x + i y)^m, m = 1..4, and (m + 1) times them for the x and y derivatives
  const float c1 = ux, s1 = uy;
  const float c2 = ux * ux - uy * uy, s2 = 2.0f * ux * uy;
  const float c3 = c2 * ux - s2 * uy, s3 = c2 * uy + s2 * ux;
  const float c4 = c3 * ux - s3 * uy, s4 = c3 * uy + s3 * ux;
  const float h1 = 2.0f * c1, k1 = 2.0f * s1, h2 = 3.0f * c2, k2 = 3.0f * s2;
  const float h3 = 4.0f * c3, k3 = 4.0f * s3;
  // radial: sum_k dE/dG_k e_k (-2 eta_r (r - R_k) fc + dfc), R_k = 0.85 + 0.11 k,
  //       = (dfc - 2 eta_r (r - 0.85) fc) S0 + 0.22 eta_r fc S1,
  //   S0 = sum_k dE/dG_k e_k, S1 = sum_k k dE/dG_k e_k
  float eb[kNRad];
  radial_basis(r, eb);
  float S0 = 0.0f, S1 = 0.0f;
#pragma unroll
  for (int k = 0; k < kNRad; ++k) {
    S0 = __builtin_fmaf(K[52 + k], eb[k], S0);
    S1 = __builtin_fmaf(K[68 + k], eb[k], S1);
  }
  float S = (dfc - 2.0f * kEtaR * (r - 0.85f) * fc) * S0 + (0.22f * kEtaR) * fc * S1;
  float Gx = 0.0f, Gy = 0.0f, Gz = 0.0f;
  const float g0 = exp_hw(-0.5f * r * r);
  const float gsq = g0 * g0;
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const float eta = e ? 2.0f : 0.5f;
    const float ex = e ? gsq * gsq : g0;  // exp(-eta r^2)
    const float w = ex * fc;
    const float dw = ex * (-2.0f * eta * r * fc + dfc);
    const float* __restrict__ Z = K + e * kNMom;
    float a0, da0, a1, da1, b1, db1, a2, da2, b2, db2, a3, da3, b3, db3;
    poly_vd<4>(Z + 0, uz, a0, da0);
    poly_vd<3>(Z + 5, uz, a1, da1);
    poly_vd<3>(Z + 9, uz, b1, db1);
    poly_vd<2>(Z + 13, uz, a2, da2);
    poly_vd<2>(Z + 16, uz, b2, db2);
    poly_vd<1>(Z + 19, uz, a3, da3);
    poly_vd<1>(Z + 21, uz, b3, db3);
    const float a4 = Z[23], b4 = Z[24];
    const float phi = a0 + a1 * c1 + b1 * s1 + a2 * c2 + b2 * s2 + a3 * c3 + b3 * s3 + a4 * c4 + b4 * s4;
    const float pz = da0 + da1 * c1 + db1 * s1 + da2 * c2 + db2 * s2 + da3 * c3 + db3 * s3;
    const float px = a1 + a2 * h1 + b2 * k1 + a3 * h2 + b3 * k2 + a4 * h3 + b4 * k3;
    const float py = b1 - a2 * k1 + b2 * h1 - a3 * k2 + b3 * h2 - a4 * k3 + b4 * h3;
    // w' Phi uh + w (grad Phi - (uh . grad Phi) uh) / r + delta w w' uh
    const float dot = ux * px + uy * py + uz * pz;
    const float tw = w * ir;
    S += dw * (phi + K[50 + e] * w) - tw * dot;
    Gx += tw * px;
    Gy += tw * py;
    Gz += tw * pz;
  }
  gx += S * ux + Gx;
  gy += S * uy + Gy;
  gz += S * uz + Gz;
}

// ------------------------------------------------------------- backward
// The term of pair (i, j) that involves centre i's coefficients,
// g_ij = dE_i/du_ij, enters F_i with + and F_j with - (F_a = sum_j dE_a/du_aj
// - dE_j/du_ja), so each thread needs only its own K_i: it adds g_ij to its
// particle and subtracts it from the neighbour's LDS accumulator (64-bit
// fixed point, see fix_of; a term too large for it goes to the output
// directly); the block then adds its accumulators to the outputs with global
// atomics (the output is zeroed first).  Two lanes share a particle, each
// taking every other list word (512-thread workgroups: room for the 84
// coefficients in registers without spills).  Separations come
// from the FP32 tile-centred coordinates of the LJ force pass (about 1e-7 of
// a separation; the terms vanish smoothly at rc, so a pair that an FP32 test
// decides differently from an FP64 one changes nothing measurable).  A lane
// first marks its in-range entries in a bit mask and then walks the set bits
// only, so the wave's trips follow the in-range counts (the skin's entries
// and the ragged ends of the lists no longer idle lanes through whole pair
// terms).  The global FP32 atomics make the last bits of the forces depend on
// the order in which blocks and waves land.
__global__ void k_zero3(float* __restrict__ a, float* __restrict__ b, float* __restrict__ c,
                        int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    a[i] = 0.0f;
    b[i] = 0.0f;
    c[i] = 0.0f;
  }
}

// Workgroups of up to kBwdThreads: the fixed-point accumulators make the LDS
// of one workgroup fill most of a CU, so its own waves are all the latency
// hiding there is; at 161 VGPRs three waves per SIMD fit (768 threads: 197 ->
// 183 us against 512 at N = 262144).
constexpr int kBwdThreads = 768;
__global__ __launch_bounds__(kBwdThreads) void k_desc_bwd(const double* __restrict__ x,
                                                   const double* __restrict__ y,
                                                   const double* __restrict__ z,
                                                   const int32_t* __restrict__ cs, Grid g,
                                                   TileList tl, float rc, DescIO io) {
  __shared__ TileF32 t;
  __shared__ uint16_t home[kBrickMax];
  __shared__ unsigned long long acc[3][kTileMax];
  const int brick = brick_of_block(g);
  if (brick >= g.nbricks) return;
  const int total = tile_cells(g, brick, cs, t);
  const int ntc = (g.B[0] + 2) * (g.B[1] + 2) * (g.B[2] + 2);
  const int nt = total < TileF32::kCap ? total : TileF32::kCap;
  for (int u = threadIdx.x; u < nt; u += blockDim.x) {
    acc[0][u] = 0;
    acc[1][u] = 0;
    acc[2][u] = 0;
  }
  const int s0 = cs[brick * g.V], s1 = cs[(brick + 1) * g.V];
  double ox, oy, oz;
  tile_centre(g, brick, ox, oy, oz);
  tile_load_f32(g, x, y, z, total, ox, oy, oz, s0, t, home);  // ends with a barrier
  const float rc2 = rc * rc;
  const float pi_rc = 3.14159265358979f / rc;
  const float half_rev = 0.5f / rc;
  const int part = (int)threadIdx.x & 1;  // two lanes per particle, alternate list words
  for (int s = s0 + ((int)threadIdx.x >> 1); s < s1; s += (int)(blockDim.x >> 1)) {
    // FP32 coordinates relative to the tile centre (the force pass's), own
    // position from the particle's own slot
    const int hs = s - s0 < kBrickMax ? home[s - s0] : TileF32::kDummy;
    const float xi = t.px[hs], yi = t.py[hs], zi = t.pz[hs];
    const int64_t oi = io.perm ? (int64_t)io.perm[s] : (int64_t)s;
    float Ki[84];
    adjoint_coef(io.dEdG + oi * kNFeat, io.mom + oi * (2 * kNMom), Ki);
    float fx = 0.0f, fy = 0.0f, fz = 0.0f;
    const int ng = (tl.cnt[s] + 3) >> 2;
    const uint64_t* __restrict__ col = tl.nbr + s;
    const int nw = ng > part ? (ng - part + 1) >> 1 : 0;  // this lane's words: part + 2 w
    for (int w0 = 0; w0 < nw; w0 += 16) {
      // the in-range entries of up to 16 words as a bit mask (bit 4 w + q:
      // entry q of word w0 + w), so that the pair terms below run on the
      // lanes' in-range entries only, not on every entry of the list
      const int wn = nw - w0 < 16 ? nw - w0 : 16;
      uint64_t mask = 0;
      for (int wg = 0; wg < wn; wg += 4) {
        // four words in flight at once (rows past the lane's last word read
        // its last word again and are ignored)
        uint64_t wd[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
          wd[k] = col[(int64_t)(part + 2 * (w0 + (wg + k < wn ? wg + k : wn - 1))) * tl.stride];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int w = wg + k;
          uint64_t bits = 0;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            int u = (int)((wd[k] >> (16 * q)) & 0xffff) >> kFullShift;
            u = u < nt ? u : TileF32::kDummy;  // padding: the far-away dummy slot
            const float dx = t.px[u] - xi, dy = t.py[u] - yi, dz = t.pz[u] - zi;
            const float d2 = dx * dx + dy * dy + dz * dz;
            if (d2 < rc2) bits |= 1ull << q;
          }
          mask |= w < wn ? bits << (4 * w) : 0;
        }
      }
      // one in-range entry per lane and trip; the word of the next one is
      // loaded a trip ahead
      // (the load goes to a valid row even when no bit is left)
      int b = mask ? __builtin_ctzll(mask) : 64;
      uint64_t word = col[(int64_t)(part + 2 * (w0 + (b < 64 ? b >> 2 : 0))) * tl.stride];
      while (b < 64) {
        const int u = (int)((word >> (16 * (b & 3))) & 0xffff) >> kFullShift;
        mask &= mask - 1;
        b = mask ? __builtin_ctzll(mask) : 64;
        word = col[(int64_t)(part + 2 * (w0 + (b < 64 ? b >> 2 : 0))) * tl.stride];
        const float dx = t.px[u] - xi, dy = t.py[u] - yi, dz = t.pz[u] - zi;
        const float d2 = dx * dx + dy * dy + dz * dz;
        // 1/r from the hardware reciprocal square root (about 1 ulp), r = d2/r
        const float ir = __builtin_amdgcn_rsqf(d2);
        const float r = d2 * ir;
        const float ux = dx * ir, uy = dy * ir, uz = dz * ir;
        const float fc = 0.5f * (__builtin_amdgcn_cosf(r * half_rev) + 1.0f);
        const float dfc = -0.5f * pi_rc * __builtin_amdgcn_sinf(r * half_rev);
        float gx = 0.0f, gy = 0.0f, gz = 0.0f;
        pair_grad(Ki, r, ir, ux, uy, uz, fc, dfc, gx, gy, gz);
        fx += gx;
        fy += gy;
        fz += gz;
        if (fix_fits((double)(__builtin_fabsf(gx) + __builtin_fabsf(gy) + __builtin_fabsf(gz)))) {
          atomicAdd(&acc[0][u], fix_of(-(double)gx));
          atomicAdd(&acc[1][u], fix_of(-(double)gy));
          atomicAdd(&acc[2][u], fix_of(-(double)gz));
        } else {
          const int lo = tile_cell_of(t, ntc, u);
          const int sj = t.src[lo] + (u - t.prefix[lo]);
          const int64_t oj = io.perm ? (int64_t)io.perm[sj] : (int64_t)sj;
          unsafeAtomicAdd(&io.fx[oj], -gx);
          unsafeAtomicAdd(&io.fy[oj], -gy);
          unsafeAtomicAdd(&io.fz[oj], -gz);
        }
      }
    }
    unsafeAtomicAdd(&io.fx[oi], fx);
    unsafeAtomicAdd(&io.fy[oi], fy);
    unsafeAtomicAdd(&io.fz[oi], fz);
  }
  __syncthreads();
  for (int u = threadIdx.x; u < nt; u += blockDim.x) {
    const unsigned long long qx = acc[0][u], qy = acc[1][u], qz = acc[2][u];
    if (qx | qy | qz) {
      const int lo = tile_cell_of(t, ntc, u);
      const int sj = t.src[lo] + (u - t.prefix[lo]);
      const int64_t oj = io.perm ? (int64_t)io.perm[sj] : (int64_t)sj;
      const float ax = (float)fix_value(qx), ay = (float)fix_value(qy), az = (float)fix_value(qz);
      unsafeAtomicAdd(&io.fx[oj], ax);
      unsafeAtomicAdd(&io.fy[oj], ay);
      unsafeAtomicAdd(&io.fz[oj], az);
    }
  }
}

hipError_t desc_forward(const double* x, const double* y, const double* z,
                        const int32_t* cell_start, const Grid& g, const TileList& tl, float rc,
                        const int32_t* perm, float* G, float* mom, hipStream_t st, float* fx,
                        float* fy, float* fz) {
  DescIO io{G, mom, nullptr, perm, fx, fy, fz};
  const unsigned threads = tl.threads < 512 ? tl.threads : 512;
  hipLaunchKernelGGL(k_desc_fwd, dim3(tile_grid(g)), dim3(threads), 0, st, x, y,
                     z, cell_start, g, tl, rc, io);
  return hipGetLastError();
}

hipError_t desc_backward(const double* x, const double* y, const double* z,
                         const int32_t* cell_start, const Grid& g, const TileList& tl, float rc,
                         const int32_t* perm, const float* dEdG, const float* mom, int64_t n,
                         float* fx, float* fy, float* fz, hipStream_t st, bool zeroed) {
  DescIO io{nullptr, const_cast<float*>(mom), dEdG, perm, fx, fy, fz};
  if (!zeroed)
    hipLaunchKernelGGL(k_zero3, dim3((unsigned)div_up(n, 256)), dim3(256), 0, st, fx, fy, fz, n);
  const unsigned threads = 2 * tl.threads < kBwdThreads ? 2 * tl.threads : kBwdThreads;
  hipLaunchKernelGGL(k_desc_bwd, dim3(tile_grid(g)), dim3(threads), 0, st, x, y,
                     z, cell_start, g, tl, rc, io);
  return hipGetLastError();
}

}  // namespace mdpl
