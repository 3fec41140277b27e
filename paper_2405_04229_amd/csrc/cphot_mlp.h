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
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef short s16x2 __attribute__((ext_vector_type(2)));

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

// ReLU of two FP32 values, rounded to bf16 and packed (a in the low half). The
// maximum with zero is taken on the bf16 bit patterns as signed 16-bit integers
// (a negative bf16 has its sign bit set, so it compares below zero): one packed
// integer instruction for two units. Rounding keeps the sign, so this equals
// rounding the FP32 ReLU.
__device__ __forceinline__ uint32_t relu_bf16x2(float a, float b) {
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  const bf16x2 v = __builtin_convertvector((f32x2){a, b}, bf16x2);  // one v_cvt_pk_bf16_f32
  const s16x2 r = __builtin_elementwise_max(__builtin_bit_cast(s16x2, v), (s16x2){0, 0});
  return __builtin_bit_cast(uint32_t, r);
}

// Forward pass for the 64 photons of a wave (one per lane). Must be called by
// all 64 lanes together. x = raw inputs (h_e, cos zenith, azimuth, wavelength,
// h_obs); y = de-standardised outputs (dx, dy, optical path excess, log T).
// `stage` is this wave's 64 x 16 B of LDS: the inputs go through it into the
// B-operand layout and the outputs back to one lane per photon (a write and a
// read each instead of cross-lane shuffles).
__device__ __forceinline__ void mlp_forward_wave(const MlpImage* __restrict__ im, const float x[kMlpIn],
                                                 float y[kMlpOut], uint4* stage) {
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, c = lane & 15;
  // layer 1: B operand = scaled inputs of photon 16 nt + c in lanes g == 0
  // (K slots 0..4; all other K slots are zero)
  {
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    float xs[kMlpIn];
#pragma unroll
    for (int j = 0; j < kMlpIn; ++j) xs[j] = fmaf(x[j] - im->in_lo[j], im->in_scale[j], -1.0f);
    u32x4 w;
    w[0] = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){xs[0], xs[1]}, bf16x2));
    w[1] = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){xs[2], xs[3]}, bf16x2));
    w[2] = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){xs[4], 0.0f}, bf16x2));
    w[3] = 0u;
    stage[lane] = __builtin_bit_cast(uint4, w);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  bf16x8 bx[4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const uint4 v = g == 0 ? stage[16 * nt + c] : make_uint4(0u, 0u, 0u, 0u);
    bx[nt] = __builtin_bit_cast(bf16x8, v);
  }
  // hidden activations as bf16 pairs: slot 4 (m & 1) + r of K-tile m >> 1 is in
  // word 2 (m & 1) + r / 2
  u32x4 h1[2][4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const bf16x8 a = im->a1[m][lane];
    f32x4 bias;
#pragma unroll
    for (int r = 0; r < 4; ++r) bias[r] = im->b1[16 * m + 4 * g + r];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const f32x4 z = mfma16(a, bx[nt], bias);
      h1[m >> 1][nt][2 * (m & 1)] = relu_bf16x2(z[0], z[1]);
      h1[m >> 1][nt][2 * (m & 1) + 1] = relu_bf16x2(z[2], z[3]);
    }
  }
  // layer 2
  u32x4 h2[2][4];
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
      for (int nt = 0; nt < 4; ++nt) acc[nt] = mfma16(a, __builtin_bit_cast(bf16x8, h1[kt][nt]), acc[nt]);
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      h2[m >> 1][nt][2 * (m & 1)] = relu_bf16x2(acc[nt][0], acc[nt][1]);
      h2[m >> 1][nt][2 * (m & 1) + 1] = relu_bf16x2(acc[nt][2], acc[nt][3]);
    }
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
    for (int nt = 0; nt < 4; ++nt) out[nt] = mfma16(a, __builtin_bit_cast(bf16x8, h2[kt][nt]), out[nt]);
  }
  // photon 16 nt + c finds its outputs in lane c (g == 0) of N-tile nt
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (g == 0) {
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) stage[16 * nt + c] = __builtin_bit_cast(uint4, out[nt]);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const f32x4 o = __builtin_bit_cast(f32x4, stage[lane]);
#pragma unroll
  for (int r = 0; r < kMlpOut; ++r) y[r] = fmaf(o[r], im->out_std[r], im->out_mean[r]);
}

// True if all inputs lie in the training domain box.
__device__ __forceinline__ bool mlp_in_domain(const MlpImage* __restrict__ im, const float x[kMlpIn]) {
  bool ok = true;
#pragma unroll
  for (int j = 0; j < kMlpIn; ++j) ok = ok && (x[j] >= im->in_lo[j]) && (x[j] <= im->in_hi[j]);
  return ok;
}

}  // namespace cphot
