// Transport surrogate network 5 -> 64 -> 64 -> 4 (ReLU hidden units, linear
// output) on gfx950 matrix cores: bf16 operands, FP32 accumulation
// (v_mfma_f32_16x16x32_bf16).
//
// Operand layout of v_mfma_f32_16x16x32_bf16 for lane l (g = l / 16, c = l % 16):
//   A (16 x 32): row c, k = 8 g .. 8 g + 7;  B (32 x 16): column c, same k;
//   C (16 x 16): rows 4 g .. 4 g + 3, column c.
//
// Inference computes every layer transposed, Z^T = W^T H^T, with 16 photons per
// N-tile: a lane's accumulator then holds four hidden units of one photon,
// which is exactly the lane's share of the next layer's B operand once the K
// index inside each 32-wide K-tile is permuted as
//   slot 8 g + i  <->  unit 16 (2 kt + i / 4) + 4 g + i % 4.
// The A operands (weights) are stored pre-permuted, so activations never leave
// registers between layers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cphot {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMlpIn = 5;
constexpr int kMlpHidden = 64;
constexpr int kMlpOut = 4;
// canonical parameter vector: W1 [5][64], b1, W2 [64][64], b2, W3 [64][4], b3 (W[in][out])
constexpr int kOffW1 = 0;
constexpr int kOffB1 = 320;
constexpr int kOffW2 = 384;
constexpr int kOffB2 = 4480;
constexpr int kOffW3 = 4544;
constexpr int kOffB3 = 4800;
constexpr int kMlpParams = 4804;
constexpr int kMlpNorm = 24;  // in_lo[5], in_hi[5], in_scale[5], pad, out_mean[4], out_std[4]

// Everything inference needs, one contiguous image (copied into LDS per block).
struct MlpImage {
  bf16x8 a1[4][64];     // layer 1 A operand per M-tile (hidden units) and lane
  bf16x8 a2[4][2][64];  // layer 2 A operand per (M-tile, K-tile) and lane
  bf16x8 a3[2][64];     // layer 3 A operand per K-tile and lane (rows 0..3 used)
  float b1[64], b2[64], b3[4];
  float in_lo[5], in_hi[5], in_scale[5], pad0;
  float out_mean[4], out_std[4];
};
static_assert(sizeof(MlpImage) % 16 == 0, "image copied as 16-byte words");

// Canonical index of the hidden unit behind K slot (kt, g, i).
__host__ __device__ constexpr int mlp_unit_of_slot(int kt, int g, int i) {
  return 16 * (2 * kt + i / 4) + 4 * g + (i % 4);
}

__device__ __forceinline__ f32x4 mfma16(const bf16x8& a, const bf16x8& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Forward pass for the 64 photons of a wave (one per lane). Must be called by
// all 64 lanes together. x = raw inputs (h_e, cos zenith, azimuth, wavelength,
// h_obs); y = de-standardised outputs (dx, dy, optical path excess, log T).
__device__ __forceinline__ void mlp_forward_wave(const MlpImage* __restrict__ im, const float x[kMlpIn],
                                                 float y[kMlpOut]) {
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, c = lane & 15;
  float xs[kMlpIn];
#pragma unroll
  for (int j = 0; j < kMlpIn; ++j) xs[j] = fmaf(x[j] - im->in_lo[j], im->in_scale[j], -1.0f);
  // layer 1: B operand = scaled inputs of photon 16 nt + c in lanes g == 0
  bf16x8 bx[4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
#pragma unroll
    for (int j = 0; j < kMlpIn; ++j) {
      const float v = __shfl(xs[j], 16 * nt + c, 64);
      bx[nt][j] = (__bf16)(g == 0 ? v : 0.0f);
    }
#pragma unroll
    for (int j = kMlpIn; j < 8; ++j) bx[nt][j] = (__bf16)0.0f;
  }
  bf16x8 h1[2][4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const bf16x8 a = im->a1[m][lane];
    f32x4 bias;
#pragma unroll
    for (int r = 0; r < 4; ++r) bias[r] = im->b1[16 * m + 4 * g + r];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const f32x4 z = mfma16(a, bx[nt], bias);
#pragma unroll
      for (int r = 0; r < 4; ++r) h1[m >> 1][nt][4 * (m & 1) + r] = (__bf16)fmaxf(z[r], 0.0f);
    }
  }
  // layer 2
  bf16x8 h2[2][4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    f32x4 acc[4];
    f32x4 bias;
#pragma unroll
    for (int r = 0; r < 4; ++r) bias[r] = im->b2[16 * m + 4 * g + r];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = bias;
#pragma unroll
    for (int kt = 0; kt < 2; ++kt) {
      const bf16x8 a = im->a2[m][kt][lane];
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) acc[nt] = mfma16(a, h1[kt][nt], acc[nt]);
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) h2[m >> 1][nt][4 * (m & 1) + r] = (__bf16)fmaxf(acc[nt][r], 0.0f);
  }
  // layer 3: rows 0..3 of the output tile live in lanes g == 0
  f32x4 out[4];
  f32x4 bias3;
#pragma unroll
  for (int r = 0; r < 4; ++r) bias3[r] = (g == 0) ? im->b3[r] : 0.0f;
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) out[nt] = bias3;
#pragma unroll
  for (int kt = 0; kt < 2; ++kt) {
    const bf16x8 a = im->a3[kt][lane];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) out[nt] = mfma16(a, h2[kt][nt], out[nt]);
  }
  // photon 16 g + c finds its outputs in lane c of N-tile g
#pragma unroll
  for (int r = 0; r < kMlpOut; ++r) {
    float v = 0.f;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const float t = __shfl(out[nt][r], c, 64);
      v = (g == nt) ? t : v;
    }
    y[r] = fmaf(v, im->out_std[r], im->out_mean[r]);
  }
}

// True if all inputs lie in the training domain box.
__device__ __forceinline__ bool mlp_in_domain(const MlpImage* __restrict__ im, const float x[kMlpIn]) {
  bool ok = true;
#pragma unroll
  for (int j = 0; j < kMlpIn; ++j) ok = ok && (x[j] >= im->in_lo[j]) && (x[j] <= im->in_hi[j]);
  return ok;
}

}  // namespace cphot
