// Dense layers of the learned potential on the matrix cores (BF16 inputs,
// FP32 accumulation): y = w3 . silu(W2 silu(W1 g + b1) + b2) + b3 with the
// standardised features g = (G - mu) / sd zero-padded to 32, silu(z) = z
// sigmoid(z), and E = e_mean + e_sd y.
//
// One wave handles 16 atoms at a time.  v_mfma_f32_16x16x32_bf16 takes lane
// l's A row l%16 and B column l%16 with K = 8(l/16)..+7 and returns rows
// 4(l/16)..+3 of column l%16.  Activations change layout through a 4 KB LDS
// scratch per wave.  The input gradient (EVAL) runs the transposed products
// dh1 = dz2 W2 and dg = dz1 W1.  TRAIN also forms the loss
// L = sum (y - t)^2 / B over a batch of B atoms and the weight gradients;
// their 16x16x16 MFMAs take the accumulator fragments of the forward tiles
// directly (rows = atoms are exactly the K index of those products).
// Partials are written per wave and reduced in a fixed order.
#include <math.h>

#include "device_util.h"
#include "internal.h"
#include "mlp_args.h"

namespace mdpl {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(short)))) short bf16x4;  // 16x16x16 operand bits
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef __attribute__((__vector_size__(4 * sizeof(unsigned)))) unsigned u32x4;
typedef __attribute__((__vector_size__(2 * sizeof(unsigned)))) unsigned u32x2;

constexpr int kMlpThreads = 256;
constexpr int kNIn = 24, kNPad = 32, kNH = 64;
// packed FP32 parameter vector: W1 [64][32] | b1 | W2 [64][64] | b2 | w3 | b3
constexpr int kOffW1 = 0, kOffB1 = 2048, kOffW2 = 2112, kOffB2 = 6208, kOffW3 = 6272, kOffB3 = 6336;
constexpr int kNParam = 6337;

__device__ __forceinline__ unsigned short f2bf(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even (finite inputs)
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

__device__ __forceinline__ bf16x8 pack8(const float v[8]) {
  u32x4 w;
#pragma unroll
  for (int i = 0; i < 4; ++i) w[i] = (unsigned)f2bf(v[2 * i]) | ((unsigned)f2bf(v[2 * i + 1]) << 16);
  return __builtin_bit_cast(bf16x8, w);
}
__device__ __forceinline__ bf16x4 pack4(const float v[4]) {
  bf16x4 w;
#pragma unroll
  for (int i = 0; i < 4; ++i) w[i] = (short)f2bf(v[i]);
  return w;
}
__device__ __forceinline__ bf16x8 load8(const unsigned short* p) {  // 8 consecutive bf16
  u32x4 w;
#pragma unroll
  for (int i = 0; i < 4; ++i) w[i] = (unsigned)p[2 * i] | ((unsigned)p[2 * i + 1] << 16);
  return __builtin_bit_cast(bf16x8, w);
}
__device__ __forceinline__ bf16x8 load8_strided(const unsigned short* p, int stride) {
  u32x4 w;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    w[i] = (unsigned)p[(2 * i) * stride] | ((unsigned)p[(2 * i + 1) * stride] << 16);
  return __builtin_bit_cast(bf16x8, w);
}

// sigmoid with the hardware reciprocal (about 1 ulp; the network's BF16
// operands dominate its error)
__device__ __forceinline__ float sigm(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

// Sum over the 16 lanes of a DPP row (the lanes 16 g .. 16 g + 15): the
// quads by lane ^ 1 and lane ^ 2, then the row's four quad sums by
// rotations of 4 and 8 lanes.  Every lane receives the row sum; lanes of
// quads 0 and 2 and of quads 1 and 3 pair the quad sums differently, so the
// two groups can differ in the last bit.
__device__ __forceinline__ float row16_sum(float v) {
  v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x124>(v);  // row_ror:4
  v += dpp_move<0x128>(v);  // row_ror:8
  return v;
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The raw features 8 grp .. 8 grp + 7 of row 16 tile + col (zero past the
// 24 features); ok: the row exists.
__device__ __forceinline__ void load_features(const MlpArgs& a, int64_t tile, int64_t ntiles,
                                              int col, int grp, float g[8], bool& ok) {
  const int64_t ra = tile * 16 + col;
  ok = tile < ntiles && ra < a.n;
  const int64_t ia = ok ? (a.index ? (int64_t)a.index[ra] : ra) : 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int f = 8 * grp + k;
    g[k] = (ok && f < kNIn) ? a.G[ia * kNIn + f] : 0.0f;
  }
}

template <bool TRAIN>
__global__ __launch_bounds__(kMlpThreads) void k_mlp(MlpArgs a) {
  __shared__ float scratch[kMlpThreads / 64][16][kNH + 1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  float(*S)[kNH + 1] = scratch[wv];
  const bool want_grad = TRAIN || a.dEdG != nullptr;

  // weight fragments, held for the whole kernel
  bf16x8 W1f[4], W2f[4][2], W2b[4][2], W1b[2][2];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    W1f[nt] = load8(a.w1 + (nt * 16 + col) * kNPad + 8 * grp);
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) W2f[nt][kc] = load8(a.w2 + (nt * 16 + col) * kNH + kc * 32 + 8 * grp);
  }
  if (want_grad) {
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int kc = 0; kc < 2; ++kc)
        W2b[nt][kc] = load8_strided(a.w2 + (kc * 32 + 8 * grp) * kNH + nt * 16 + col, kNH);
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int kc = 0; kc < 2; ++kc)
        W1b[nt][kc] = load8_strided(a.w1 + (kc * 32 + 8 * grp) * kNPad + nt * 16 + col, kNPad);
  }
  float b1c[4], b2c[4], w3c[4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    b1c[nt] = a.b1[nt * 16 + col];
    b2c[nt] = a.b2[nt * 16 + col];
    w3c[nt] = bf2f(a.w3[nt * 16 + col]);
  }
  const float b3 = a.b3[0];
  // reciprocals of the feature scales this lane uses: its eight layer-1
  // inputs (8 grp + k), and the features col and 16 + col of the gradients
  float isd8[8], isd2[2];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int f = 8 * grp + k;
    isd8[k] = f < kNIn ? 1.0f / a.sd[f] : 0.0f;
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int f = j * 16 + col;
    isd2[j] = f < kNIn ? 1.0f / a.sd[f] : 0.0f;
  }

  // TRAIN accumulators
  f32x4 gW2[4][4], gW1[4][2];
  float gb1[4] = {0, 0, 0, 0}, gb2[4] = {0, 0, 0, 0}, gw3[4] = {0, 0, 0, 0};
  float gb3 = 0.0f, loss = 0.0f;
  if (TRAIN) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int j = 0; j < 4; ++j) gW2[i][j] = f32x4{0, 0, 0, 0};
      gW1[i][0] = f32x4{0, 0, 0, 0};
      gW1[i][1] = f32x4{0, 0, 0, 0};
    }
  }

  const int64_t ntiles = (a.n + 15) >> 4;
  const int64_t wave_id = (int64_t)blockIdx.x * (kMlpThreads / 64) + wv;
  const int64_t nwaves = (int64_t)gridDim.x * (kMlpThreads / 64);
  // this lane's eight layer-1 features of a tile's row col, raw (the next
  // tile's are loaded while the current one is computed)
  float mu8[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int f = 8 * grp + k;
    mu8[k] = f < kNIn ? a.mu[f] : 0.0f;
  }
  float gnext[8];
  bool oknext = false;
  load_features(a, wave_id, ntiles, col, grp, gnext, oknext);
  for (int64_t tile = wave_id; tile < ntiles; tile += nwaves) {
    const int64_t r0 = tile * 16;
    // ---- layer 1: A fragment = standardised features of row r0 + col
    float gv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) gv[k] = oknext ? (gnext[k] - mu8[k]) * isd8[k] : 0.0f;
    load_features(a, tile + nwaves, ntiles, col, grp, gnext, oknext);
    // keep those loads here, a tile ahead of their use
    asm volatile("" ::: "memory");
    const bf16x8 A1 = pack8(gv);
    f32x4 z1[4], h1[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      z1[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1, W1f[nt], f32x4{0, 0, 0, 0}, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        z1[nt][r] += b1c[nt];
        h1[nt][r] = z1[nt][r] * sigm(z1[nt][r]);
        S[4 * grp + r][nt * 16 + col] = h1[nt][r];
      }
    }
    wave_lds_sync();
    bf16x8 A2[2];
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) {
      float v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] = S[col][kc * 32 + 8 * grp + k];
      A2[kc] = pack8(v);
    }
    // ---- layer 2 and the output
    f32x4 z2[4];
    float ypart[4] = {0, 0, 0, 0};
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A2[0], W2f[nt][0], f32x4{0, 0, 0, 0}, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A2[1], W2f[nt][1], acc, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        acc[r] += b2c[nt];
        ypart[r] += w3c[nt] * acc[r] * sigm(acc[r]);
      }
      z2[nt] = acc;
    }
    // sum over the 16 columns held by the lanes of this group
#pragma unroll
    for (int r = 0; r < 4; ++r) ypart[r] = row16_sum(ypart[r]) + b3;
    // ---- upstream gradient dL/dy (TRAIN) or dy/dy = 1 (EVAL)
    float dy[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = r0 + 4 * grp + r;
      const bool ok = row < a.n;
      if (TRAIN) {
        const int64_t ir = ok ? (a.index ? (int64_t)a.index[row] : row) : 0;
        // the target: the atom's energy standardised with the network's e_mean, e_sd
        const float t = ok ? (float)((a.target[ir] - (double)a.e_mean) / (double)a.e_sd) : 0.0f;
        const float diff = ok ? ypart[r] - t : 0.0f;
        dy[r] = 2.0f * diff * a.inv_batch;
        if (col == 0) loss += diff * diff * a.inv_batch;
      } else {
        dy[r] = ok ? 1.0f : 0.0f;
        if (ok && col == 0 && a.energy) a.energy[row] = a.e_mean + a.e_sd * ypart[r];
      }
    }
    if (!want_grad) {
      wave_lds_sync();
      continue;
    }
    // ---- dz2 = dy w3 silu'(z2)
    f32x4 dz2[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float zz = z2[nt][r];
        const float sg = sigm(zz);
        dz2[nt][r] = dy[r] * w3c[nt] * sg * (1.0f + zz * (1.0f - sg));
      }
    if (TRAIN) {
      // weight gradients: dW2 = dz2^T h1, dw3 = sum dy h2, db2 = sum dz2, db3 = sum dy
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float av[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) av[r] = dz2[i][r];
        const bf16x4 Ai = pack4(av);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          float bv[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) bv[r] = h1[j][r];
          gW2[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(Ai, pack4(bv), gW2[i][j], 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          gb2[i] += dz2[i][r];
          const float zz = z2[i][r];
          gw3[i] += dy[r] * zz * sigm(zz);
        }
      }
      if (col == 0) gb3 += dy[0] + dy[1] + dy[2] + dy[3];
    }
    // ---- dh1 = dz2 W2 (A = dz2 rows, through LDS)
    wave_lds_sync();
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) S[4 * grp + r][nt * 16 + col] = dz2[nt][r];
    wave_lds_sync();
    bf16x8 D2[2];
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) {
      float v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] = S[col][kc * 32 + 8 * grp + k];
      D2[kc] = pack8(v);
    }
    f32x4 dz1[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(D2[0], W2b[nt][0], f32x4{0, 0, 0, 0}, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(D2[1], W2b[nt][1], acc, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float zz = z1[nt][r];
        const float sg = sigm(zz);
        acc[r] *= sg * (1.0f + zz * (1.0f - sg));
      }
      dz1[nt] = acc;
    }
    if (TRAIN) {
      // dW1 = dz1^T g, db1 = sum dz1; g in accumulator layout: rows 4 grp + r, column f
      float gd[2][4];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int f = j * 16 + col;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = r0 + 4 * grp + r;
          const bool ok = row < a.n && f < kNIn;
          const int64_t ir = ok ? (a.index ? (int64_t)a.index[row] : row) : 0;
          gd[j][r] = ok ? (a.G[ir * kNIn + f] - a.mu[f]) * isd2[j] : 0.0f;
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float av[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          av[r] = dz1[i][r];
          gb1[i] += dz1[i][r];
        }
        const bf16x4 Ai = pack4(av);
#pragma unroll
        for (int j = 0; j < 2; ++j)
          gW1[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(Ai, pack4(gd[j]), gW1[i][j], 0, 0, 0);
      }
      wave_lds_sync();
      continue;
    }
    // ---- EVAL: dg = dz1 W1 (A = dz1 rows, through LDS)
    wave_lds_sync();
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) S[4 * grp + r][nt * 16 + col] = dz1[nt][r];
    wave_lds_sync();
    bf16x8 D1[2];
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) {
      float v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] = S[col][kc * 32 + 8 * grp + k];
      D1[kc] = pack8(v);
    }
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(D1[0], W1b[nt][0], f32x4{0, 0, 0, 0}, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(D1[1], W1b[nt][1], acc, 0, 0, 0);
      const int f = nt * 16 + col;
      if (f < kNIn) {
        const float sc = a.e_sd * isd2[nt];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = r0 + 4 * grp + r;
          if (row < a.n) a.dEdG[row * kNIn + f] = acc[r] * sc;
        }
      }
    }
    wave_lds_sync();
  }

  if (TRAIN) {
    float* __restrict__ P = a.partial + wave_id * (kNParam + 1);
    // accumulator tile (i, j): lane holds rows (n) 4 grp + r of tile i, column j*16 + col
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          P[kOffW2 + (i * 16 + 4 * grp + r) * kNH + j * 16 + col] = gW2[i][j][r];
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          P[kOffW1 + (i * 16 + 4 * grp + r) * kNPad + j * 16 + col] = gW1[i][j][r];
    }
    // column sums over the 4 lane groups
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float v1 = gb1[i], v2 = gb2[i], v3 = gw3[i];
      v1 += __shfl_xor(v1, 16, 64);
      v1 += __shfl_xor(v1, 32, 64);
      v2 += __shfl_xor(v2, 16, 64);
      v2 += __shfl_xor(v2, 32, 64);
      v3 += __shfl_xor(v3, 16, 64);
      v3 += __shfl_xor(v3, 32, 64);
      if (grp == 0) {
        P[kOffB1 + i * 16 + col] = v1;
        P[kOffB2 + i * 16 + col] = v2;
        P[kOffW3 + i * 16 + col] = v3;
      }
    }
    float t3 = gb3, tl = loss;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      t3 += __shfl_xor(t3, off, 64);
      tl += __shfl_xor(tl, off, 64);
    }
    if (lane == 0) {
      P[kOffB3] = t3;
      P[kNParam] = tl;
    }
  }
}

hipError_t mlp_eval(const MlpArgs& a, hipStream_t st) {
  // two waves per SIMD that each take many tiles: the weight fragments a
  // wave loads first are then reused over ~8 tiles at N = 262,144 (2048
  // blocks, two tiles per wave: 61 us; 1024: 48; 512: 43)
  int64_t tiles = (a.n + 15) >> 4;
  int64_t blocks = (tiles + 3) / 4;
  if (blocks > 512) blocks = 512;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_mlp<false>, dim3((unsigned)blocks), dim3(kMlpThreads), 0, st, a);
  return hipGetLastError();
}

int mlp_train_waves(int64_t n) {
  int64_t tiles = (n + 15) >> 4;
  int64_t blocks = (tiles + 3) / 4;
  if (blocks > 256) blocks = 256;
  if (blocks < 1) blocks = 1;
  return (int)(blocks * (kMlpThreads / 64));
}

hipError_t mlp_train_grad(const MlpArgs& a, hipStream_t st) {
  const int waves = mlp_train_waves(a.n);
  hipLaunchKernelGGL(k_mlp<true>, dim3((unsigned)(waves / 4)), dim3(kMlpThreads), 0, st, a);
  return hipGetLastError();
}

// out[k] = sum over waves of partial[w][k], k < kNParam + 1, fixed order
__global__ void k_sum_partials(const float* __restrict__ partial, int nwaves, float* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > kNParam) return;
  float s = 0.0f;
  for (int w = 0; w < nwaves; ++w) s += partial[(int64_t)w * (kNParam + 1) + k];
  out[k] = s;
}

hipError_t mlp_sum_partials(const float* partial, int nwaves, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_partials, dim3((kNParam + 1 + 255) / 256), dim3(256), 0, st, partial,
                     nwaves, out);
  return hipGetLastError();
}

// Adam (bias-corrected) on the FP32 master vector, then the bf16 copies of
// the three weight matrices.  W1 columns >= 24 stay zero.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1,
                       float c2, unsigned short* __restrict__ w1, unsigned short* __restrict__ w2,
                       unsigned short* __restrict__ w3) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= kNParam) return;
  float gk = g[k];
  if (k < kOffB1 && (k % kNPad) >= kNIn) gk = 0.0f;
  const float mk = b1 * m[k] + (1.0f - b1) * gk;
  const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  float pk = p[k] - lr * (mk / c1) / (sqrtf(vk / c2) + eps);
  if (k < kOffB1 && (k % kNPad) >= kNIn) pk = 0.0f;
  p[k] = pk;
  if (k < kOffB1) w1[k] = f2bf(pk);
  else if (k >= kOffW2 && k < kOffB2) w2[k - kOffW2] = f2bf(pk);
  else if (k >= kOffW3 && k < kOffB3) w3[k - kOffW3] = f2bf(pk);
}

hipError_t adam_step(float* p, const float* g, float* m, float* v, float lr, float b1, float b2,
                     float eps, int t, unsigned short* w1, unsigned short* w2, unsigned short* w3,
                     hipStream_t st) {
  const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_adam, dim3((kNParam + 255) / 256), dim3(256), 0, st, p, g, m, v, lr, b1, b2,
                     eps, c1, c2, w1, w2, w3);
  return hipGetLastError();
}

// BF16 copies of the weight matrices from the packed FP32 parameters
// (round to nearest even, as after every Adam step).
__global__ void k_bf16_weights(const float* __restrict__ p, unsigned short* __restrict__ w1,
                               unsigned short* __restrict__ w2, unsigned short* __restrict__ w3) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= kNParam) return;
  const float pk = p[k];
  if (k < kOffB1) w1[k] = f2bf(pk);
  else if (k >= kOffW2 && k < kOffB2) w2[k - kOffW2] = f2bf(pk);
  else if (k >= kOffW3 && k < kOffB3) w3[k - kOffW3] = f2bf(pk);
}

hipError_t bf16_weights(const float* p, unsigned short* w1, unsigned short* w2, unsigned short* w3,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_bf16_weights, dim3((kNParam + 255) / 256), dim3(256), 0, st, p, w1, w2, w3);
  return hipGetLastError();
}

// Standardisation statistics of the training set, FP64 in a fixed order:
// means, then the mean squared deviations from them (two passes, as the
// population standard deviation is defined).  Column c < 24 is feature c of
// G (n x 24 floats), column 24 the energy.  Pass 1 (ref null): per-block
// sums; pass 2 (ref = the means): per-block sums of squared deviations.
constexpr int kStdCols = kNIn + 1;
__global__ __launch_bounds__(256) void k_std_partials(const float* __restrict__ G,
                                                      const double* __restrict__ e, int64_t n,
                                                      const double* __restrict__ ref,
                                                      double* __restrict__ part) {
  __shared__ double sh[4];
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * per, r1 = r0 + per < n ? r0 + per : n;
  for (int c = 0; c < kStdCols; ++c) {
    const double m = ref ? ref[c] : 0.0;
    double acc = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
      const double v = c < kNIn ? (double)G[r * kNIn + c] : e[r];
      acc += ref ? (v - m) * (v - m) : v;
    }
    const double t = block_sum256(acc, sh);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * kStdCols + c] = t;
  }
}

// Sums the partials of every column in block order; out[c] = sum / n.  With
// fin: the feature spreads sqrt(.) + 1e-6 to sd (float), the means to mu,
// the energy's mean and spread sqrt(.) + 1e-12 to e_stats.
__global__ __launch_bounds__(64) void k_std_reduce(const double* __restrict__ part, int nb,
                                                   int64_t n, double* __restrict__ out, bool fin,
                                                   const double* __restrict__ mean, float* mu,
                                                   float* sd, double* e_stats) {
  const int c = threadIdx.x;
  if (c >= kStdCols) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[(int64_t)b * kStdCols + c];
  const double v = s / (double)n;
  out[c] = v;
  if (!fin) return;
  if (c < kNIn) {
    mu[c] = (float)mean[c];
    sd[c] = (float)(sqrt(v) + 1e-6);
  } else {
    e_stats[0] = mean[c];
    e_stats[1] = sqrt(v) + 1e-12;
  }
}

hipError_t mlp_standardise(const float* G, const double* e, int64_t n, float* mu, float* sd,
                           double* e_stats, double* scratch, hipStream_t st) {
  const int nb = kStdBlocks;
  double* part = scratch;
  double* mean = scratch + (int64_t)nb * kStdCols;
  double* var = mean + kStdCols;
  hipLaunchKernelGGL(k_std_partials, dim3(nb), dim3(256), 0, st, G, e, n, nullptr, part);
  hipLaunchKernelGGL(k_std_reduce, dim3(1), dim3(64), 0, st, part, nb, n, mean, false, nullptr,
                     nullptr, nullptr, nullptr);
  hipLaunchKernelGGL(k_std_partials, dim3(nb), dim3(256), 0, st, G, e, n, mean, part);
  hipLaunchKernelGGL(k_std_reduce, dim3(1), dim3(64), 0, st, part, nb, n, var, true, mean, mu, sd,
                     e_stats);
  return hipGetLastError();
}

// ------------------------------------------------------------ reductions
// partials[b] = sum of v over block b (FP64, fixed order).
__global__ __launch_bounds__(256) void k_sum_f32(const float* __restrict__ v, int64_t n,
                                                 double* __restrict__ partials) {
  __shared__ double sh[4];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double t = block_sum256(i < n ? (double)v[i] : 0.0, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

hipError_t sum_f32(const float* v, int64_t n, double* partials, hipStream_t st, int* nblocks_out) {
  const unsigned nb = (unsigned)div_up(n, 256);
  *nblocks_out = (int)nb;
  hipLaunchKernelGGL(k_sum_f32, dim3(nb), dim3(256), 0, st, v, n, partials);
  return hipGetLastError();
}

// partials[2b] = sum |f - g|^2, partials[2b+1] = sum |g|^2 over block b.
__global__ __launch_bounds__(256) void k_force_diff(const float* __restrict__ fx,
                                                    const float* __restrict__ fy,
                                                    const float* __restrict__ fz,
                                                    const double* __restrict__ gx,
                                                    const double* __restrict__ gy,
                                                    const double* __restrict__ gz, int64_t n,
                                                    double* __restrict__ partials) {
  __shared__ double sh[4];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double d = 0.0, r = 0.0;
  if (i < n) {
    const double a = (double)fx[i] - gx[i], b = (double)fy[i] - gy[i], c = (double)fz[i] - gz[i];
    d = a * a + b * b + c * c;
    r = gx[i] * gx[i] + gy[i] * gy[i] + gz[i] * gz[i];
  }
  const double td = block_sum256(d, sh);
  __syncthreads();
  const double tr = block_sum256(r, sh);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = td;
    partials[2 * blockIdx.x + 1] = tr;
  }
}

hipError_t force_diff(const float* fx, const float* fy, const float* fz, const double* gx,
                      const double* gy, const double* gz, int64_t n, double* partials,
                      hipStream_t st, int* nblocks_out) {
  const unsigned nb = (unsigned)div_up(n, 256);
  *nblocks_out = (int)nb;
  hipLaunchKernelGGL(k_force_diff, dim3(nb), dim3(256), 0, st, fx, fy, fz, gx, gy, gz, n,
                     partials);
  return hipGetLastError();
}

}  // namespace mdpl
