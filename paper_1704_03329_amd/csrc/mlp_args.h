// Arguments of the dense-layer kernels (shared by mlp.hip and api.hip).
#pragma once

#include <stdint.h>

namespace mdpl {

constexpr int kMlpParams = 6337;  // W1 [64][32] | b1 [64] | W2 [64][64] | b2 [64] | w3 [64] | b3
// floats per particle of the learned-potential MD workspace:
// G 24 | moments 50 | energy 1 | dE/dG 24
constexpr int kMlpRunFloats = 99;

struct MlpArgs {
  const unsigned short* w1;  // bf16 [64][32]
  const float* b1;
  const unsigned short* w2;  // bf16 [64][64]
  const float* b2;
  const unsigned short* w3;  // bf16 [64]
  const float* b3;
  const float* mu;           // 24
  const float* sd;           // 24
  float e_mean, e_sd;
  const float* G;            // features, row-major [atom][24]
  const int32_t* index;      // nullable: row a reads atom index[a]
  int64_t n;                 // rows
  float* energy;             // EVAL: E per row (nullable)
  float* dEdG;               // EVAL: [row][24] (nullable)
  const double* target;      // TRAIN: per-atom energies (indexed like G), standardised in the kernel
  float* partial;            // TRAIN: per-wave [kNParam + 1] (gradient, loss)
  float inv_batch;           // TRAIN: 1 / B
};


}  // namespace mdpl
