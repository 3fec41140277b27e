// Transport surrogate: training-set generation with the exact layered tracer,
// output normalisation, training (forward + backward on bf16 matrix cores with
// FP32 accumulation, Adam on FP32 master weights) and batch inference.
//
// The surrogate replaces the layered tracer's correction to the straight line
// (the role of the thesis's precomputed correction table, Sec. 4.4.1) by a
// small network trained on photons the exact tracer generates: over planar
// layers, or over the spherical shells of a curved Earth (Sec. 3.3.4).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "cphot_device.h"
#include "cphot_internal.h"
#include "cphot_mlp.h"
#include "cphot_walk64.h"

namespace cphot {

namespace {

constexpr int kTrainWave = 64;  // samples per training block (one wave)

// c += A[16 x 32] * B[32 x 16] with A rows and B columns stored k-contiguous
// (row r of A at A + r * lda, column n of B at Bt + n * ldb).
__device__ __forceinline__ f32x4 mma_kc(const __bf16* A, int lda, const __bf16* Bt, int ldb, f32x4 c) {
  const int l = threadIdx.x & 63;
  const bf16x8 a = *reinterpret_cast<const bf16x8*>(A + (l & 15) * lda + (l >> 4) * 8);
  const bf16x8 b = *reinterpret_cast<const bf16x8*>(Bt + (l & 15) * ldb + (l >> 4) * 8);
  return mfma16(a, b, c);
}

__device__ __forceinline__ f32x4 zero4() { return f32x4{0.f, 0.f, 0.f, 0.f}; }

// ---------------------------------------------------------------------------- training set

struct TrainSetParams {
  float4 const* layers;
  float4 const* moments;  // closed-form layer-sum moments [obs][j][5] (planar targets)
  float2 const* lambins;
  int n_layers, n_lam;
  int geometry;  // CPHOT_SURROGATE_PLANAR | CPHOT_SURROGATE_CURVED
  double earth_radius;
  float dh, lam_min, lam_max;
  float lo[5], hi[5];
  uint32_t key0, key1;
  int64_t first, n;
  float* X;
  float* Y;
};

__global__ __launch_bounds__(256) void k_training_set(TrainSetParams p) {
  __shared__ float4 s_lay[kMaxLayers];
  __shared__ float2 s_lam[kMaxLambdaBins];
  for (int i = threadIdx.x; i < p.n_layers; i += 256) s_lay[i] = p.layers[i];
  for (int i = threadIdx.x; i < p.n_lam; i += 256) s_lam[i] = p.lambins[i];
  __syncthreads();
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= p.n) return;
  const uint64_t i = (uint64_t)(p.first + j);
  const uint4 w = philox((uint32_t)i, 0u, (uint32_t)(i >> 32), TAG_TRAIN, p.key0, p.key1);
  const uint4 v = philox((uint32_t)i, 1u, (uint32_t)(i >> 32), TAG_TRAIN, p.key0, p.key1);
  const float h_obs = p.lo[4] + (p.hi[4] - p.lo[4]) * u24(w.x);
  // start: the lower boundary of a layer (shell) above the observation layer, drawn
  // uniformly among those in the box (integer arithmetic on the word's top 24 bits);
  // inside its start layer a photon is straight, so the network learns the
  // correction from that boundary on, a smooth function of the boundary height
  const int j_obs = (int)floorf(h_obs / p.dh);
  const int j_lo = max((int)ceilf(p.lo[0] / p.dh), j_obs + 1);
  const int j_hi = (int)floorf(p.hi[0] / p.dh);
  const int m = max(j_hi - j_lo + 1, 1);
  const int jj = j_lo + (int)(((uint64_t)(w.y >> 8) * (uint64_t)m) >> 24);
  const float h_e = (float)jj * p.dh;
  const float ct = p.lo[1] + (p.hi[1] - p.lo[1]) * u24(w.z);
  const float phi = p.lo[2] + (p.hi[2] - p.lo[2]) * u24(w.w);
  int kb = (int)floorf(u24(v.x) * (float)p.n_lam);
  kb = min(kb, p.n_lam - 1);
  const float lam = p.lam_min + ((float)kb + 0.5f) * (p.lam_max - p.lam_min) / (float)p.n_lam;
  const float st = sqrtf((1.f - ct) * (1.f + ct));
  float sphi, cphi;
  sincosf(phi, &sphi, &cphi);
  const float ux = st * cphi, uy = st * sphi, uz = -ct;
  float* x = p.X + 5 * j;
  x[0] = h_e;
  x[1] = ct;
  x[2] = phi;
  x[3] = lam;
  x[4] = h_obs;
  float* y = p.Y + 4 * j;
  if (p.geometry == CPHOT_SURROGATE_CURVED) {
    // by the spherical symmetry the start is above the Earth point (0, 0); the
    // chord from there to the sphere R + h_obs, in FP64
    const double Re = p.earth_radius, he = h_e, ho = h_obs;
    double s_ch, psi_s;
    chord_f64(Re, ho, he, (double)ct, s_ch, psi_s);
    Walk64 w;
    if (!shell_walk_f64(s_lay, (double)p.dh, p.n_layers, ho, Re, he, (double)ct, w)) {
      y[0] = y[1] = y[2] = y[3] = __builtin_nanf("");
      return;
    }
    const float2 sp = s_lam[kb];
    const double tau = (double)sp.x * w.tR + (double)sp.y * w.tA;
    // per metre of chord: the absolute quantities grow with the slant distance
    y[0] = (float)((w.across - psi_s) * (Re + ho) / s_ch);
    y[1] = 0.f;  // across the plane of the start direction: zero by symmetry
    y[2] = (float)(((w.len - s_ch) + w.opt) / s_ch);
    y[3] = (float)(-tau / s_ch);
    return;
  }
  const int i0 = min((int)(h_e / p.dh), p.n_layers - 1);
  const int iobs = (int)floorf(h_obs / p.dh);
  LayerWalk lw;
  layer_walk<false, true>(s_lay, s_lam[kb], p.dh, i0, iobs, 0.f, 0.f, h_e, ux, uy, uz, 0.f, 0.f, -1.f, lw);
  // last leg inside the observation layer, then targets: landing offset from the
  // straight line, optical path excess sum (n - 1) l + (path - straight path), -tau
  const float span_last = lw.z - h_obs;
  const float s_last = -span_last / lw.vz;
  float dr = lw.dr, gex = lw.gex;
  leg_excess(lw, span_last, lw.last_delta, s_lay[iobs].y, dr, gex);
  const float opt = fmaf(lw.last_delta, s_last, lw.opt);
  const float tau = fmaf(lw.last_ext, s_last, lw.tau);
  // the straight line's own sums from the start boundary down to h_obs (full layers
  // from the moments, the observation layer's span directly): the network learns
  // only what refraction adds to them
  const float4* mr = p.moments + ((size_t)iobs * p.n_layers + i0) * 5;
  const float4 Lo = s_lay[iobs];
  const float top = (float)(iobs + 1) * p.dh - h_obs, ict = 1.0f / ct;
  const float2 sp = s_lam[kb];
  const float opt_s = ict * fmaf(Lo.x, top, mr[2].x);
  const float tau_s = ict * fmaf(sp.x, mr[2].w, fmaf(sp.y, mr[3].z, fmaf(Lo.z, sp.x, Lo.w * sp.y) * top));
  y[0] = dr;   // along the photon's horizontal direction
  y[1] = 0.f;  // across it: zero for horizontal layers
  y[2] = (gex + opt) - opt_s;
  y[3] = tau_s - tau;
}

// ---------------------------------------------------------------------------- normalisation

__global__ void k_zero_f64(double* a, int n) {
  if ((int)threadIdx.x < n) a[threadIdx.x] = 0.0;
}

__global__ __launch_bounds__(256) void k_output_sums(const float* __restrict__ Y, int64_t n, double* sums) {
  double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) {
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      const double v = Y[4 * j + o];
      s[o] += v;
      s[4 + o] += v * v;
    }
  }
  __shared__ double red[8][4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    double v = s[q];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    if (lane == 0) red[q][wid] = v;
  }
  __syncthreads();
  if (threadIdx.x < 8) {
    const double v = red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] + red[threadIdx.x][3];
    atomicAdd(sums + threadIdx.x, v);
  }
}

__global__ void k_output_norm(const double* sums, int64_t n, float* norm) {
  const int o = threadIdx.x;
  if (o >= 4) return;
  const double mean = sums[o] / (double)n;
  const double var = sums[4 + o] / (double)n - mean * mean;
  norm[16 + o] = (float)mean;
  norm[20 + o] = (float)sqrt(var > 1e-30 ? var : 1e-30);
}

// ---------------------------------------------------------------------------- packing

struct TrainWeights {  // bf16 operand layouts for the training kernel (k-contiguous)
  __bf16 w1t[64][32];  // [out unit][input k], k >= 5 zero
  __bf16 w2t[64][64];  // [out][in]
  __bf16 w2[64][64];   // [in][out]
  __bf16 w3t[16][64];  // [output o][in], o >= 4 zero
  __bf16 w3[64][32];   // [in][output o], o >= 4 zero
};

// Builds the training layouts and the inference image from the FP32 master
// weights and the normalisation (at creation, after new parameters or a new
// normalisation; a training step updates its own entries, see k_adam).
__global__ __launch_bounds__(256) void k_pack(const float* __restrict__ m, const float* __restrict__ norm,
                                             TrainWeights* tw, MlpImage* im) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  const int T = gridDim.x * 256;
  for (int e = t; e < 64 * 32; e += T) {
    const int o = e / 32, k = e % 32;
    tw->w1t[o][k] = (__bf16)(k < 5 ? m[kOffW1 + k * 64 + o] : 0.f);
  }
  for (int e = t; e < 64 * 64; e += T) {
    const int a = e / 64, b = e % 64;
    tw->w2t[a][b] = (__bf16)m[kOffW2 + b * 64 + a];
    tw->w2[a][b] = (__bf16)m[kOffW2 + a * 64 + b];
  }
  for (int e = t; e < 16 * 64; e += T) {
    const int o = e / 64, i = e % 64;
    tw->w3t[o][i] = (__bf16)(o < 4 ? m[kOffW3 + i * 4 + o] : 0.f);
  }
  for (int e = t; e < 64 * 32; e += T) {
    const int i = e / 32, o = e % 32;
    tw->w3[i][o] = (__bf16)(o < 4 ? m[kOffW3 + i * 4 + o] : 0.f);
  }
  // inference image
  for (int e = t; e < 4 * 64 * 8; e += T) {
    const int mt = e / 512, l = (e / 8) % 64, i = e % 8;
    const int g = l >> 4, c = l & 15;
    im->a1[mt][l][i] = (__bf16)((g == 0 && i < 5) ? m[kOffW1 + i * 64 + 16 * mt + c] : 0.f);
  }
  for (int e = t; e < 4 * 2 * 64 * 8; e += T) {
    const int mt = e / 1024, kt = (e / 512) % 2, l = (e / 8) % 64, i = e % 8;
    const int g = l >> 4, c = l & 15;
    im->a2[mt][kt][l][i] = (__bf16)m[kOffW2 + mlp_unit_of_slot(kt, g, i) * 64 + 16 * mt + c];
  }
  for (int e = t; e < 2 * 64 * 8; e += T) {
    const int kt = e / 512, l = (e / 8) % 64, i = e % 8;
    const int g = l >> 4, c = l & 15;
    im->a3[kt][l][i] = (__bf16)(c < 4 ? m[kOffW3 + mlp_unit_of_slot(kt, g, i) * 4 + c] : 0.f);
  }
  for (int e = t; e < 64; e += T) {
    im->b1[e] = m[kOffB1 + e];
    im->b2[e] = m[kOffB2 + e];
  }
  if (t < 4) im->b3[t] = m[kOffB3 + t];
  if (t < 5) {
    im->in_lo[t] = norm[t];
    im->in_hi[t] = norm[5 + t];
    im->in_scale[t] = norm[10 + t];
  }
  if (t < 4) {
    im->out_mean[t] = norm[16 + t];
    im->out_std[t] = norm[20 + t];
  }
  if (t == 0) im->pad0 = 0.f;
}

// Writes the bf16 copies of parameter i (new FP32 value v) into every slot of the
// training layouts and the inference image that holds it: the inverse of k_pack's
// index maps, so that one Adam thread refreshes its own parameter and a training
// step needs no separate packing pass. Slots that hold zero padding are untouched.
__device__ __forceinline__ void scatter_param(int i, float v, TrainWeights* tw, MlpImage* im) {
  const __bf16 b = (__bf16)v;
  if (i < kOffB1) {  // W1[k][o]
    const int k = i / 64, o = i % 64;
    tw->w1t[o][k] = b;
    im->a1[o / 16][o % 16][k] = b;  // lane c (g = 0) of M-tile o / 16, K slot k
  } else if (i < kOffW2) {
    im->b1[i - kOffB1] = v;
  } else if (i < kOffB2) {  // W2[a][c2]: K slot (kt, g, ii) of unit a, column c2
    const int e = i - kOffW2, a = e / 64, c2 = e % 64;
    tw->w2t[c2][a] = b;
    tw->w2[a][c2] = b;
    const int kt = (a / 16) >> 1, ii = 4 * ((a / 16) & 1) + (a & 3), g = (a % 16) >> 2;
    im->a2[c2 / 16][kt][16 * g + c2 % 16][ii] = b;
  } else if (i < kOffW3) {
    im->b2[i - kOffB2] = v;
  } else if (i < kOffB3) {  // W3[in][o]
    const int e = i - kOffW3, in = e / 4, o = e % 4;
    tw->w3t[o][in] = b;
    tw->w3[in][o] = b;
    const int kt = (in / 16) >> 1, ii = 4 * ((in / 16) & 1) + (in & 3), g = (in % 16) >> 2;
    im->a3[kt][16 * g + o][ii] = b;
  } else {
    im->b3[i - kOffB3] = v;
  }
}

// ---------------------------------------------------------------------------- training step

struct StepParams {
  const float* X;
  const float* Y;
  int64_t n;        // training-set size
  int64_t start;    // first sample of this batch (wraps modulo n)
  int batch;        // samples in the batch (multiple of 64)
  const float* norm;
  const float* master;
  const TrainWeights* tw;
  float* partial;   // [blocks][kMlpParams]
  float* loss_partial;
};

// One wave, 64 samples: forward, loss, backward; writes this block's share of
// the gradient of mean((y_hat - t_hat)^2) over the whole batch.
__global__ __launch_bounds__(64) void k_train_step(StepParams p) {
  __shared__ __attribute__((aligned(16))) __bf16 Xh[64][32];
  __shared__ __attribute__((aligned(16))) __bf16 XhT[32][64];
  __shared__ __attribute__((aligned(16))) __bf16 H1[64][64];
  __shared__ __attribute__((aligned(16))) __bf16 H1T[64][64];  // later dZ1^T
  __shared__ __attribute__((aligned(16))) __bf16 H2[64][64];   // later dZ2
  __shared__ __attribute__((aligned(16))) __bf16 H2T[64][64];  // later dZ2^T
  __shared__ __attribute__((aligned(16))) __bf16 dY[64][32];
  __shared__ __attribute__((aligned(16))) __bf16 dYT[16][64];
  const int l = threadIdx.x;
  const int g = l >> 4, c = l & 15;
  const float* norm = p.norm;
  const int64_t s0 = p.start + (int64_t)blockIdx.x * kTrainWave;
  // scaled inputs of sample l
  {
    const int64_t js = (s0 + l) % p.n;
    for (int k = 0; k < 32; ++k) {
      float v = 0.f;
      if (k < 5) v = fmaf(p.X[5 * js + k] - norm[k], norm[10 + k], -1.0f);
      const __bf16 b = (__bf16)v;
      Xh[l][k] = b;
      XhT[k][l] = b;
    }
    for (int o = 0; o < 32; ++o) dY[l][o] = (__bf16)0.f;
    for (int o = 0; o < 16; ++o) dYT[o][l] = (__bf16)0.f;
  }
  __syncthreads();
  const TrainWeights* tw = p.tw;
  const float* m = p.master;
  // ---- forward, rows = samples
  for (int mt = 0; mt < 4; ++mt)
    for (int nt = 0; nt < 4; ++nt) {
      f32x4 acc;
      for (int r = 0; r < 4; ++r) acc[r] = m[kOffB1 + 16 * nt + c];
      acc = mma_kc(&Xh[16 * mt][0], 32, &tw->w1t[16 * nt][0], 32, acc);
      for (int r = 0; r < 4; ++r) {
        const int s = 16 * mt + 4 * g + r, j = 16 * nt + c;
        const __bf16 h = (__bf16)fmaxf(acc[r], 0.f);
        H1[s][j] = h;
        H1T[j][s] = h;
      }
    }
  __syncthreads();
  for (int mt = 0; mt < 4; ++mt)
    for (int nt = 0; nt < 4; ++nt) {
      f32x4 acc;
      for (int r = 0; r < 4; ++r) acc[r] = m[kOffB2 + 16 * nt + c];
      for (int kt = 0; kt < 2; ++kt) acc = mma_kc(&H1[16 * mt][32 * kt], 64, &tw->w2t[16 * nt][32 * kt], 64, acc);
      for (int r = 0; r < 4; ++r) {
        const int s = 16 * mt + 4 * g + r, j = 16 * nt + c;
        const __bf16 h = (__bf16)fmaxf(acc[r], 0.f);
        H2[s][j] = h;
        H2T[j][s] = h;
      }
    }
  __syncthreads();
  float loss = 0.f;
  const float dscale = 2.0f / (4.0f * (float)p.batch);
  for (int mt = 0; mt < 4; ++mt) {
    f32x4 acc;
    for (int r = 0; r < 4; ++r) acc[r] = c < 4 ? m[kOffB3 + c] : 0.f;
    for (int kt = 0; kt < 2; ++kt) acc = mma_kc(&H2[16 * mt][32 * kt], 64, &tw->w3t[0][32 * kt], 64, acc);
    if (c < 4) {
      for (int r = 0; r < 4; ++r) {
        const int s = 16 * mt + 4 * g + r;
        const int64_t js = (s0 + s) % p.n;
        const float t = (p.Y[4 * js + c] - norm[16 + c]) / norm[20 + c];
        const float d = acc[r] - t;
        loss += d * d;
        const __bf16 db = (__bf16)(d * dscale);
        dY[s][c] = db;
        dYT[c][s] = db;
      }
    }
  }
  __syncthreads();
  float* part = p.partial + (size_t)blockIdx.x * kMlpParams;
  // ---- backward
  // dW3[j][o] = sum_s H2^T[j][s] dY^T[o][s]
  for (int mj = 0; mj < 4; ++mj) {
    f32x4 acc = zero4();
    for (int ks = 0; ks < 2; ++ks) acc = mma_kc(&H2T[16 * mj][32 * ks], 64, &dYT[0][32 * ks], 64, acc);
    if (c < 4)
      for (int r = 0; r < 4; ++r) part[kOffW3 + (16 * mj + 4 * g + r) * 4 + c] = acc[r];
  }
  if (l < 4) {
    float sb = 0.f;
    for (int s = 0; s < 64; ++s) sb += (float)dYT[l][s];
    part[kOffB3 + l] = sb;
  }
  __syncthreads();
  // dZ2[s][j] = (sum_o dY[s][o] W3[j][o]) * (H2[s][j] > 0), into H2 and H2T
  for (int mt = 0; mt < 4; ++mt)
    for (int nt = 0; nt < 4; ++nt) {
      f32x4 acc = zero4();
      acc = mma_kc(&dY[16 * mt][0], 32, &tw->w3[16 * nt][0], 32, acc);
      for (int r = 0; r < 4; ++r) {
        const int s = 16 * mt + 4 * g + r, j = 16 * nt + c;
        const bool on = (float)H2[s][j] > 0.f;
        const __bf16 d = (__bf16)(on ? acc[r] : 0.f);
        H2[s][j] = d;
        H2T[j][s] = d;
      }
    }
  __syncthreads();
  // dW2[i][j] = sum_s H1^T[i][s] dZ2^T[j][s]; db2 = row sums of dZ2^T
  for (int mi = 0; mi < 4; ++mi)
    for (int nj = 0; nj < 4; ++nj) {
      f32x4 acc = zero4();
      for (int ks = 0; ks < 2; ++ks) acc = mma_kc(&H1T[16 * mi][32 * ks], 64, &H2T[16 * nj][32 * ks], 64, acc);
      for (int r = 0; r < 4; ++r) part[kOffW2 + (16 * mi + 4 * g + r) * 64 + 16 * nj + c] = acc[r];
    }
  {
    float sb = 0.f;
    for (int s = 0; s < 64; ++s) sb += (float)H2T[l][s];
    part[kOffB2 + l] = sb;
  }
  // dZ1[s][i] = (sum_j dZ2[s][j] W2[i][j]) * (H1[s][i] > 0)
  float dz1[4][4][4];
  for (int mt = 0; mt < 4; ++mt)
    for (int ni = 0; ni < 4; ++ni) {
      f32x4 acc = zero4();
      for (int kt = 0; kt < 2; ++kt) acc = mma_kc(&H2[16 * mt][32 * kt], 64, &tw->w2[16 * ni][32 * kt], 64, acc);
      for (int r = 0; r < 4; ++r) {
        const int s = 16 * mt + 4 * g + r, i = 16 * ni + c;
        dz1[mt][ni][r] = ((float)H1[s][i] > 0.f) ? acc[r] : 0.f;
      }
    }
  __syncthreads();  // H1^T (read by dW2 above) is free now
  for (int mt = 0; mt < 4; ++mt)
    for (int ni = 0; ni < 4; ++ni)
      for (int r = 0; r < 4; ++r) H1T[16 * ni + c][16 * mt + 4 * g + r] = (__bf16)dz1[mt][ni][r];
  __syncthreads();
  // dW1[k][i] = sum_s Xh^T[k][s] dZ1^T[i][s] (k < 5 kept); db1 = row sums of dZ1^T
  for (int mk = 0; mk < 2; ++mk)
    for (int ni = 0; ni < 4; ++ni) {
      f32x4 acc = zero4();
      for (int ks = 0; ks < 2; ++ks) acc = mma_kc(&XhT[16 * mk][32 * ks], 64, &H1T[16 * ni][32 * ks], 64, acc);
      for (int r = 0; r < 4; ++r) {
        const int k = 16 * mk + 4 * g + r;
        if (k < 5) part[kOffW1 + k * 64 + 16 * ni + c] = acc[r];
      }
    }
  {
    float sb = 0.f;
    for (int s = 0; s < 64; ++s) sb += (float)H1T[l][s];
    part[kOffB1 + l] = sb;
  }
  // loss share
  for (int d = 32; d >= 1; d >>= 1) loss += __shfl_xor(loss, d, 64);
  if (l == 0) p.loss_partial[blockIdx.x] = loss;
}

// Sum of the block partials (fixed order: deterministic) -> grad; optionally
// the Adam update of the master weights (lr follows a cosine schedule).
struct AdamParams {
  const float* partial;
  const float* loss_partial;
  int blocks;
  float* master;
  float* m1;
  float* m2;
  TrainWeights* tw;  // bf16 layouts refreshed with each updated parameter
  MlpImage* img;
  int t;             // Adam steps done before this one
  int total_steps;
  float lr;
  float* grad_out;   // may be null
  float* loss_out;   // loss per step of this call, may be null
  int loss_index;    // step index within this call
  int batch;
  int update;
};

__global__ __launch_bounds__(256) void k_adam(AdamParams p) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int t = p.t;
  if (i < kMlpParams) {
    float gsum = 0.f;
    for (int b = 0; b < p.blocks; ++b) gsum += p.partial[(size_t)b * kMlpParams + i];
    if (p.grad_out) p.grad_out[i] = gsum;
    if (p.update) {
      const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
      const float tt = (float)(t + 1);
      const float prog = p.total_steps > 1 ? (float)p.loss_index / (float)(p.total_steps - 1) : 0.f;
      const float lr = p.lr * (0.01f + 0.99f * 0.5f * (1.f + cosf(3.14159265f * fminf(prog, 1.f))));
      const float m1 = b1 * p.m1[i] + (1.f - b1) * gsum;
      const float m2 = b2 * p.m2[i] + (1.f - b2) * gsum * gsum;
      p.m1[i] = m1;
      p.m2[i] = m2;
      const float mh = m1 / (1.f - powf(b1, tt));
      const float vh = m2 / (1.f - powf(b2, tt));
      const float w = p.master[i] - lr * mh / (sqrtf(vh) + eps);
      p.master[i] = w;
      scatter_param(i, w, p.tw, p.img);
    }
  }
  if (i == 0 && p.loss_out) {
    float ls = 0.f;
    for (int b = 0; b < p.blocks; ++b) ls += p.loss_partial[b];
    p.loss_out[p.loss_index] = ls / (4.0f * (float)p.batch);
  }
}

// ---------------------------------------------------------------------------- batch inference

__global__ __launch_bounds__(256) void k_forward(const MlpImage* __restrict__ img, const float* __restrict__ X,
                                                 float* __restrict__ Y, int64_t n) {
  __shared__ __attribute__((aligned(16))) MlpImage s_img;
  __shared__ uint4 s_stage[256];
  {
    const uint4* src = reinterpret_cast<const uint4*>(img);
    uint4* dst = reinterpret_cast<uint4*>(&s_img);
    for (int i = threadIdx.x; i < (int)(sizeof(MlpImage) / 16); i += 256) dst[i] = src[i];
  }
  __syncthreads();
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t jj = j < n ? j : n - 1;  // every lane takes part in the wave-wide product
  float x[kMlpIn], y[kMlpOut];
#pragma unroll
  for (int k = 0; k < kMlpIn; ++k) x[k] = X[5 * jj + k];
  mlp_forward_wave(&s_img, x, y, s_stage + (threadIdx.x & ~63u));
  if (j < n) {
#pragma unroll
    for (int o = 0; o < kMlpOut; ++o) Y[4 * j + o] = y[o];
  }
}

}  // namespace

}  // namespace cphot

// ================================================================================ host API

// Per-block partial gradients and loss shares of cphot_surrogate_gradient_noalloc:
// at most kNoAllocSamples samples, i.e. kNoAllocSamples / 64 single-wave blocks, each
// writing all kMlpParams entries of its row and its loss share (so nothing needs
// clearing between calls). 1.23 MB per device, held until the process ends. In host
// code `scratch` only names the symbol: its device address comes from
// hipGetSymbolAddress (once per device, kept in g_scratch_addr).
constexpr int kNoAllocSamples = 4096;
constexpr int kNoAllocBlocks = kNoAllocSamples / 64;
static __device__ __align__(256) float scratch[(size_t)kNoAllocBlocks * cphot::kMlpParams + kNoAllocBlocks];

struct cphot_surrogate {
  cphot_surrogate_desc d;
  int device = 0;
  int max_blocks = 0;
  float* master = nullptr;
  float* m1 = nullptr;
  float* m2 = nullptr;
  float* norm = nullptr;
  float* partial = nullptr;
  float* loss_partial = nullptr;
  int steps_done = 0;  // Adam steps enqueued so far (bias correction)
  double* sums = nullptr;
  cphot::TrainWeights* tw = nullptr;
  cphot::MlpImage* img = nullptr;
  bool normalised = false;
};

namespace {

int sfail(int code, const std::string& m) {
  cphot::set_last_error(m);
  return code;
}

int shfail(hipError_t e, const char* what) { return sfail(CPHOT_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e)); }

// splitmix64 -> uniform in [0, 1): initial weights only
double init_uniform(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

hipError_t pack(cphot_surrogate* s, hipStream_t st) {
  hipLaunchKernelGGL(cphot::k_pack, dim3(16), dim3(256), 0, st, s->master, s->norm, s->tw, s->img);
  return hipGetLastError();
}

// Device address of `scratch` on device `dev` (the current device), looked up on
// the first call per device and kept: each device holds its own copy of the array.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_addr[kMaxDevices] = {};

int scratch_address(int dev, float** out) {
  if (dev < 0 || dev >= kMaxDevices) return sfail(CPHOT_ERR_INVALID_ARG, "device index beyond 64");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return shfail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return sfail(CPHOT_ERR_HIP, "hipGetSymbolAddress(scratch) returned null");
    g_scratch_addr[dev] = static_cast<float*>(ptr);
  }
  *out = g_scratch_addr[dev];
  return CPHOT_OK;
}

}  // namespace

extern "C" {

int cphot_surrogate_create(const cphot_surrogate_desc* desc, cphot_surrogate** out) {
  if (!desc || !out) return sfail(CPHOT_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  for (int j = 0; j < 5; ++j)
    if (!std::isfinite(desc->in_lo[j]) || !std::isfinite(desc->in_hi[j]) || !(desc->in_hi[j] > desc->in_lo[j]))
      return sfail(CPHOT_ERR_INVALID_ARG, "domain box needs finite lo < hi on every input");
  if (desc->in_lo[1] < 0.0 || desc->in_hi[1] > 1.0)
    return sfail(CPHOT_ERR_INVALID_ARG, "cos(zenith) range must lie in [0, 1]");
  if (desc->max_batch < 64 || desc->max_batch % 64 || desc->max_batch > (1 << 22))
    return sfail(CPHOT_ERR_INVALID_ARG, "max_batch must be a positive multiple of 64 up to 2^22");
  if (desc->geometry != CPHOT_SURROGATE_PLANAR && desc->geometry != CPHOT_SURROGATE_CURVED)
    return sfail(CPHOT_ERR_INVALID_ARG, "unknown surrogate geometry");
  cphot_surrogate* s = new (std::nothrow) cphot_surrogate();
  if (!s) return sfail(CPHOT_ERR_OUT_OF_MEMORY, "host allocation");
  s->d = *desc;
  (void)hipGetDevice(&s->device);
  s->max_blocks = desc->max_batch / 64;
  hipError_t e;
  auto fail_free = [&](hipError_t err, const char* what) {
    cphot_surrogate_destroy(s);
    return err == hipErrorOutOfMemory ? sfail(CPHOT_ERR_OUT_OF_MEMORY, what) : shfail(err, what);
  };
  if ((e = hipMalloc(&s->master, cphot::kMlpParams * 4)) != hipSuccess) return fail_free(e, "hipMalloc");
  if ((e = hipMalloc(&s->m1, cphot::kMlpParams * 4)) != hipSuccess) return fail_free(e, "hipMalloc");
  if ((e = hipMalloc(&s->m2, cphot::kMlpParams * 4)) != hipSuccess) return fail_free(e, "hipMalloc");
  if ((e = hipMalloc(&s->norm, cphot::kMlpNorm * 4)) != hipSuccess) return fail_free(e, "hipMalloc");
  if ((e = hipMalloc(&s->partial, (size_t)s->max_blocks * cphot::kMlpParams * 4)) != hipSuccess)
    return fail_free(e, "hipMalloc");
  if ((e = hipMalloc(&s->loss_partial, (size_t)s->max_blocks * 4)) != hipSuccess) return fail_free(e, "hipMalloc");
  if ((e = hipMalloc(&s->sums, 8 * sizeof(double))) != hipSuccess) return fail_free(e, "hipMalloc");
  if ((e = hipMalloc(&s->tw, sizeof(cphot::TrainWeights))) != hipSuccess) return fail_free(e, "hipMalloc");
  if ((e = hipMalloc(&s->img, sizeof(cphot::MlpImage))) != hipSuccess) return fail_free(e, "hipMalloc");
  // He-uniform initial weights, zero biases
  std::vector<float> w(cphot::kMlpParams, 0.f);
  uint64_t rs = desc->init_seed;
  auto fill = [&](int off, int fan_in, int count) {
    const double lim = std::sqrt(6.0 / fan_in);
    for (int i = 0; i < count; ++i) w[off + i] = (float)((2.0 * init_uniform(rs) - 1.0) * lim);
  };
  fill(cphot::kOffW1, 5, 320);
  fill(cphot::kOffW2, 64, 4096);
  fill(cphot::kOffW3, 64, 256);
  std::vector<float> nrm(cphot::kMlpNorm, 0.f);
  for (int j = 0; j < 5; ++j) {
    nrm[j] = (float)desc->in_lo[j];
    nrm[5 + j] = (float)desc->in_hi[j];
    nrm[10 + j] = (float)(2.0 / (desc->in_hi[j] - desc->in_lo[j]));
  }
  for (int o = 0; o < 4; ++o) nrm[20 + o] = 1.f;
  std::vector<float> zeros(cphot::kMlpParams, 0.f);
  if ((e = hipMemcpy(s->master, w.data(), w.size() * 4, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(s->m1, zeros.data(), zeros.size() * 4, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(s->m2, zeros.data(), zeros.size() * 4, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(s->norm, nrm.data(), nrm.size() * 4, hipMemcpyHostToDevice)) != hipSuccess)
    return fail_free(e, "hipMemcpy");
  if ((e = pack(s, nullptr)) != hipSuccess) return fail_free(e, "pack");
  if ((e = hipDeviceSynchronize()) != hipSuccess) return fail_free(e, "synchronize");
  *out = s;
  return CPHOT_OK;
}

void cphot_surrogate_destroy(cphot_surrogate* s) {
  if (!s) return;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(s->device);
  for (void* ptr : {(void*)s->master, (void*)s->m1, (void*)s->m2, (void*)s->norm, (void*)s->partial,
                    (void*)s->loss_partial, (void*)s->sums, (void*)s->tw, (void*)s->img})
    if (ptr) (void)hipFree(ptr);
  (void)hipSetDevice(prev);
  delete s;
}

int cphot_surrogate_make_training_set(const cphot_surrogate* s, const cphot_atmosphere* atm, int64_t first,
                                      int64_t n, uint64_t seed, float* X, float* Y, void* stream) {
  if (!s || !atm) return sfail(CPHOT_ERR_INVALID_ARG, "null surrogate or atmosphere");
  if (n < 0 || first < 0) return sfail(CPHOT_ERR_INVALID_ARG, "negative n or first");
  if (n > 0 && (!X || !Y)) return sfail(CPHOT_ERR_INVALID_ARG, "null X or Y");
  cphot::TrainSetParams p;
  std::memset(&p, 0, sizeof(p));
  int rc = cphot::atmosphere_layer_view(atm, &p.layers, &p.lambins, &p.n_layers, &p.n_lam, &p.dh, &p.lam_min,
                                        &p.lam_max);
  if (rc) return sfail(rc, "the surrogate is trained on a layered atmosphere (n_layers > 0)");
  p.moments = cphot::atmosphere_layer_moments(atm);
  if (!p.moments) return sfail(CPHOT_ERR_INVALID_ARG, "the atmosphere has no layer-sum moments");
  const double top = (double)p.dh * p.n_layers;
  if (s->d.in_hi[0] > top || s->d.in_hi[4] > top || s->d.in_lo[4] < 0.0)
    return sfail(CPHOT_ERR_INVALID_ARG, "domain heights must lie inside the layered atmosphere");
  if (s->d.in_lo[3] > p.lam_min || s->d.in_hi[3] < p.lam_max)
    return sfail(CPHOT_ERR_INVALID_ARG, "domain wavelengths must cover the atmosphere's band");
  if (s->d.in_lo[0] < s->d.in_lo[4])
    return sfail(CPHOT_ERR_INVALID_ARG, "domain emission heights must start at or above the lowest observation level");
  {  // the starts are layer boundaries above the observation layer: the box must hold one for every h_obs
    const double dh = (double)p.dh;
    if (!((std::floor(s->d.in_hi[4] / dh) + 1.0) * dh <= s->d.in_hi[0]) ||
        !(std::ceil(s->d.in_lo[0] / dh) * dh <= s->d.in_hi[0]))
      return sfail(CPHOT_ERR_INVALID_ARG, "the emission-height range must hold a layer boundary above every "
                                          "observation layer of the box");
  }
  p.geometry = s->d.geometry;
  p.earth_radius = cphot::atmosphere_earth_radius(atm);
  if (p.geometry == CPHOT_SURROGATE_CURVED && !(p.earth_radius > 1e5 && std::isfinite(p.earth_radius)))
    return sfail(CPHOT_ERR_INVALID_ARG, "a curved surrogate needs the atmosphere's earth_radius");
  if (p.geometry == CPHOT_SURROGATE_CURVED) {
    // every ray of the box must meet the observation sphere on its straight chord (the
    // targets are per metre of that chord): (R + h_e,max) sin(zenith_max) < R + h_obs,min
    const double c = s->d.in_lo[1], sz = std::sqrt(std::max(0.0, (1.0 - c) * (1.0 + c)));
    if (!((p.earth_radius + s->d.in_hi[0]) * sz < p.earth_radius + s->d.in_lo[4]))
      return sfail(CPHOT_ERR_INVALID_ARG, "curved domain box reaches rays that miss the observation sphere: "
                                          "raise the lowest cos zenith or lower the highest emission height");
  }
  if (n == 0) return CPHOT_OK;
  for (int j = 0; j < 5; ++j) {
    p.lo[j] = (float)s->d.in_lo[j];
    p.hi[j] = (float)s->d.in_hi[j];
  }
  p.key0 = (uint32_t)seed;
  p.key1 = (uint32_t)(seed >> 32);
  p.first = first;
  p.n = n;
  p.X = X;
  p.Y = Y;
  hipLaunchKernelGGL(cphot::k_training_set, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, p);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? CPHOT_OK : shfail(e, "launch training set");
}

int cphot_surrogate_fit_normalization(cphot_surrogate* s, const float* Y, int64_t n, void* stream) {
  if (!s || !Y || n < 2) return sfail(CPHOT_ERR_INVALID_ARG, "need a surrogate and at least two targets");
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(cphot::k_zero_f64, dim3(1), dim3(64), 0, st, s->sums, 8);
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(cphot::k_output_sums, dim3(blocks), dim3(256), 0, st, Y, n, s->sums);
  hipLaunchKernelGGL(cphot::k_output_norm, dim3(1), dim3(64), 0, st, (const double*)s->sums, n, s->norm);
  hipError_t e = pack(s, st);
  if (e != hipSuccess) return shfail(e, "normalisation");
  s->normalised = true;
  return CPHOT_OK;
}

static int run_steps(cphot_surrogate* s, const float* X, const float* Y, int64_t n, int batch, int steps,
                     int total_steps, float lr, int64_t start, float* loss_out, float* grad_out, int update,
                     float* partial, float* loss_partial, hipStream_t st) {
  const int blocks = batch / 64;
  for (int k = 0; k < steps; ++k) {
    cphot::StepParams sp;
    sp.X = X;
    sp.Y = Y;
    sp.n = n;
    sp.start = (start + (int64_t)k * batch) % n;
    sp.batch = batch;
    sp.norm = s->norm;
    sp.master = s->master;
    sp.tw = s->tw;
    sp.partial = partial;
    sp.loss_partial = loss_partial;
    hipLaunchKernelGGL(cphot::k_train_step, dim3(blocks), dim3(64), 0, st, sp);
    cphot::AdamParams ap;
    ap.partial = partial;
    ap.loss_partial = loss_partial;
    ap.blocks = blocks;
    ap.master = s->master;
    ap.m1 = s->m1;
    ap.m2 = s->m2;
    ap.tw = s->tw;
    ap.img = s->img;
    ap.t = s->steps_done;
    ap.total_steps = total_steps;
    ap.lr = lr;
    ap.grad_out = grad_out;
    ap.loss_out = loss_out;
    ap.loss_index = k;
    ap.batch = batch;
    ap.update = update;
    hipLaunchKernelGGL(cphot::k_adam, dim3((cphot::kMlpParams + 255) / 256), dim3(256), 0, st, ap);
    if (update) ++s->steps_done;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return shfail(e, "training step");
  }
  return CPHOT_OK;
}

int cphot_surrogate_train(cphot_surrogate* s, const float* X, const float* Y, int64_t n, int32_t batch,
                          int32_t steps, float lr, float* loss_out, void* stream) {
  if (!s || !X || !Y) return sfail(CPHOT_ERR_INVALID_ARG, "null argument");
  if (!s->normalised) return sfail(CPHOT_ERR_UNSUPPORTED, "fit the output normalisation first");
  if (batch < 64 || batch % 64 || batch > s->d.max_batch)
    return sfail(CPHOT_ERR_INVALID_ARG, "batch must be a multiple of 64 up to max_batch");
  if (n < batch) return sfail(CPHOT_ERR_INVALID_ARG, "training set smaller than one batch");
  if (steps < 0 || !(lr > 0.f) || !std::isfinite(lr)) return sfail(CPHOT_ERR_INVALID_ARG, "bad steps or lr");
  return run_steps(s, X, Y, n, batch, steps, steps, lr, 0, loss_out, nullptr, 1, s->partial, s->loss_partial,
                   (hipStream_t)stream);
}

int cphot_surrogate_gradient(cphot_surrogate* s, const float* X, const float* Y, int64_t n, float* grad,
                             float* loss, void* stream) {
  if (!s || !X || !Y || !grad) return sfail(CPHOT_ERR_INVALID_ARG, "null argument");
  if (n < 64 || n % 64 || n > s->d.max_batch)
    return sfail(CPHOT_ERR_INVALID_ARG, "n must be a multiple of 64 up to max_batch");
  return run_steps(s, X, Y, n, (int)n, 1, 1, 1.f, 0, loss, grad, 0, s->partial, s->loss_partial,
                   (hipStream_t)stream);
}

int cphot_surrogate_gradient_noalloc(cphot_surrogate* s, const float* X, const float* Y, int64_t n, float* grad,
                                     float* loss, void* stream) {
  if (!s || !X || !Y || !grad) return sfail(CPHOT_ERR_INVALID_ARG, "null argument");
  if (n < 64 || n % 64 || n > kNoAllocSamples)
    return sfail(CPHOT_ERR_INVALID_ARG, "n must be a multiple of 64 up to 4096 (the static workspace)");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return shfail(e, "hipGetDevice");
  if (dev != s->device) return sfail(CPHOT_ERR_INVALID_ARG, "call on the device the surrogate was created on");
  float* ws = nullptr;
  const int rc = scratch_address(dev, &ws);
  if (rc) return rc;
  return run_steps(s, X, Y, n, (int)n, 1, 1, 1.f, 0, loss, grad, 0, ws, ws + (size_t)kNoAllocBlocks * cphot::kMlpParams,
                   (hipStream_t)stream);
}

int cphot_surrogate_forward(const cphot_surrogate* s, const float* X, float* Y, int64_t n, void* stream) {
  if (!s) return sfail(CPHOT_ERR_INVALID_ARG, "null surrogate");
  if (n < 0 || (n > 0 && (!X || !Y))) return sfail(CPHOT_ERR_INVALID_ARG, "bad buffers");
  if (n == 0) return CPHOT_OK;
  hipLaunchKernelGGL(cphot::k_forward, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                     (const cphot::MlpImage*)s->img, X, Y, n);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? CPHOT_OK : shfail(e, "launch forward");
}

int cphot_surrogate_get_params(const cphot_surrogate* s, float* params, float* norm) {
  if (!s) return sfail(CPHOT_ERR_INVALID_ARG, "null surrogate");
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess && params) e = hipMemcpy(params, s->master, cphot::kMlpParams * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess && norm) e = hipMemcpy(norm, s->norm, cphot::kMlpNorm * 4, hipMemcpyDeviceToHost);
  return e == hipSuccess ? CPHOT_OK : shfail(e, "get params");
}

int cphot_surrogate_set_params(cphot_surrogate* s, const float* params, const float* norm) {
  if (!s) return sfail(CPHOT_ERR_INVALID_ARG, "null surrogate");
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess && params) e = hipMemcpy(s->master, params, cphot::kMlpParams * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess && norm) {
    e = hipMemcpy(s->norm, norm, cphot::kMlpNorm * 4, hipMemcpyHostToDevice);
    s->normalised = true;
  }
  if (e == hipSuccess) e = pack(s, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  return e == hipSuccess ? CPHOT_OK : shfail(e, "set params");
}

}  // extern "C"

namespace cphot {
const MlpImage* surrogate_image(const cphot_surrogate* s) { return s ? s->img : nullptr; }
bool surrogate_ready(const cphot_surrogate* s) { return s && s->normalised; }
int surrogate_geometry(const cphot_surrogate* s) { return s ? s->d.geometry : CPHOT_SURROGATE_PLANAR; }
}  // namespace cphot
