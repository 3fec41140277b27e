// Device helpers shared by the photon and surrogate kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cphot_internal.h"

namespace cphot {

constexpr uint32_t TAG_SEGMENT = 0;
constexpr uint32_t TAG_CHERENKOV = 1;
constexpr uint32_t TAG_FLUOR = 2;  // + band (2, 3, 4)
constexpr uint32_t TAG_TRAIN = 8;
constexpr uint32_t TAG_POISSON = 12;  // + source (12 Cherenkov, 13..15 fluorescence bands)
constexpr int kMaxRecordsPerSegmentLog2 = 20;
constexpr float kCmPerNs = 0.299792458f;  // metres per ns

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 products.
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                        uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return make_uint4(c0, c1, c2, c3);
}

// Hardware reciprocal and square root (about 1 ulp for the normal, positive
// inputs they get here) where the correctly rounded sequences cost about ten
// instructions; used on the per-photon planar path, whose tolerances are far
// above an ulp.
__device__ __forceinline__ float rcp_fast(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float sqrt_fast(float x) { return __builtin_amdgcn_sqrtf(x); }

// exp(-x) for 0 <= x <= 64 from IEEE basic operations only, so that it comes out
// bit-identical on any IEEE machine (record counts are decided by it):
// x = k ln2 + r with ln2 split into a 29-bit head (k ln2_hi exact) and a tail
// (Cody and Waite's reduction), exp(-r) by its Taylor series to r^14 (first omitted
// term below 2e-19 for |r| <= ln2 / 2), then the exact scaling by 2^-k.
__device__ inline double exp_neg_exact(double x) {
#pragma clang fp contract(off)
  const double kLn2Hi = 0x1.62e42ffp-1, kLn2Lo = -0x1.718432a1b0e26p-35, kInvLn2 = 0x1.71547652b82fep+0;
  const double k = floor(x * kInvLn2 + 0.5);
  const double r = (x - k * kLn2Hi) - k * kLn2Lo;
  const double t = -r;
  double q = 0x1.93974a8c07c9dp-37;  // 1/14!
  q = q * t + 0x1.6124613a86d09p-33;
  q = q * t + 0x1.1eed8eff8d898p-29;
  q = q * t + 0x1.ae64567f544e4p-26;
  q = q * t + 0x1.27e4fb7789f5cp-22;
  q = q * t + 0x1.71de3a556c734p-19;
  q = q * t + 0x1.a01a01a01a01ap-16;
  q = q * t + 0x1.a01a01a01a01ap-13;
  q = q * t + 0x1.6c16c16c16c17p-10;
  q = q * t + 0x1.1111111111111p-7;
  q = q * t + 0x1.5555555555555p-5;
  q = q * t + 0x1.5555555555555p-3;
  q = q * t + 0.5;
  q = q * t + 1.0;
  q = q * t + 1.0;
  return ldexp(q, -(int)k);
}

// Poisson(mu) record count (0 <= mu < 2^20): inversion, in equal chunks of mean
// at most 64 (a sum of independent Poisson counts is Poisson): for each chunk the
// smallest n with u < sum_{j<=n} e^-m m^j / j!, the terms built as p <- p m / n.
// The first chunk uses the segment's own word w0, chunk c > 0 word 0 of the Philox
// block (c, id low, id high, tag). IEEE basic operations only (see exp_neg_exact).
__device__ inline int64_t poisson_count(double mu, uint32_t w0, uint64_t id, uint32_t tag, uint32_t k0,
                                        uint32_t k1) {
#pragma clang fp contract(off)
  if (!(mu > 0.0)) return 0;
  const int64_t nc = (int64_t)ceil(mu / 64.0);
  const double m = mu / (double)nc;
  const double e = exp_neg_exact(m);
  int64_t total = 0;
  for (int64_t c = 0; c < nc; ++c) {
    const uint32_t word = c == 0 ? w0 : philox((uint32_t)c, (uint32_t)id, (uint32_t)(id >> 32), tag, k0, k1).x;
    const double u = (double)word * (1.0 / 4294967296.0);
    double pk = e, F = e;
    int64_t n = 0;
    while (u >= F && n < 4096) {
      n += 1;
      pk = pk * m / (double)n;
      F = F + pk;
    }
    total += n;
  }
  return total;
}

// Random word -> uniform on [0, 1) with 24 bits (exact in FP32).
__device__ __forceinline__ float u24(uint32_t w) { return (float)(w >> 8) * 5.9604644775390625e-8f; }

template <int BS>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* s_wave, uint32_t& total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) s_wave[wid] = x;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int q = 0; q < BS / 64; ++q) {
    const uint32_t t = s_wave[q];
    pre += (q < wid) ? t : 0u;
    tot += t;
  }
  total = tot;
  return pre + x - v;
}

// Two exclusive block scans at once (one barrier): returns the exclusive prefixes
// of a and b, and their block totals. s_wave holds 2 * BS / 64 entries.
template <int BS>
__device__ __forceinline__ uint2 block_exclusive_scan2(uint32_t a, uint32_t b, uint32_t* s_wave, uint32_t& total_a,
                                                      uint32_t& total_b) {
  constexpr int kWaves = BS / 64;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t x = a, y = b;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t xu = __shfl_up(x, d, 64), yu = __shfl_up(y, d, 64);
    if (lane >= d) {
      x += xu;
      y += yu;
    }
  }
  if (lane == 63) {
    s_wave[wid] = x;
    s_wave[kWaves + wid] = y;
  }
  __syncthreads();
  uint32_t pa = 0, pb = 0, ta = 0, tb = 0;
#pragma unroll
  for (int q = 0; q < kWaves; ++q) {
    const uint32_t u = s_wave[q], v = s_wave[kWaves + q];
    pa += (q < wid) ? u : 0u;
    pb += (q < wid) ? v : 0u;
    ta += u;
    tb += v;
  }
  total_a = ta;
  total_b = tb;
  return make_uint2(pa + x - a, pb + y - b);
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}


// Walk of a downward photon through equal homogeneous layers (Sec. 3.4.2), from
// its start point in layer `i` down to the layer `obs_layer`. Within a layer
// the ray is straight; at a horizontal boundary the horizontal part of n u is
// conserved (the vector form of Snell's law, Eq. 3.15, with a vertical
// normal), so layer i is crossed with sine s_i = s_0 n_0 / n_i = s_0 (1 - e_i),
// e_i = (d_i - d_0) / (1 + d_i), d = n - 1. The cosine is carried without
// forming 1 - s^2 near s = 1 (which in FP32 would lose every digit of a
// near-horizontal photon's cosine): c_i^2 = c_0^2 + s_0^2 e_i (2 - e_i), with
// c_0 = -u_z and s_0 the horizontal part of the start direction. Layer data:
// lay[i] = (n - 1, 1/n, Rayleigh part, aerosol part); the extinction per metre
// at wavelength bin k is lay.z * sp.x + lay.w * sp.y with sp = (spectral
// Rayleigh, spectral aerosol). On return (x, y, z) is the entry point into the
// observation layer and (vx, vy, vz) the direction there.
struct LayerWalk {
  float x, y, z;
  float vx, vy, vz;
  float tau;         // optical depth accumulated above the observation layer
  float geo;         // sum of l (1 - u . axis)                               (NEED_TIME)
  float opt;         // sum of (n - 1) l                                       (NEED_TIME or NEED_EXCESS)
  float dr;          // horizontal travel beyond the straight line, along the azimuth (NEED_EXCESS)
  float gex;         // geometric path beyond the straight line                (NEED_EXCESS)
  float last_delta;  // n - 1 of the observation layer
  float last_ext;    // extinction per metre there
  float s0, c0, d0, hx, hy;  // start sine and cosine, start n - 1, azimuth
};

// Sine and squared cosine in a layer with n - 1 = d, 1/n = inv_n.
__device__ __forceinline__ void layer_angle(float s0, float c0, float d0, float d, float inv_n, float& s,
                                            float& c2, float& e) {
  e = (d - d0) * inv_n;
  s = fmaf(-s0, e, s0);
  c2 = fmaxf(fmaf(s0 * s0 * e, 2.0f - e, c0 * c0), 1e-30f);
}

// Excess of a leg of vertical extent `span` crossed at sine s (layer with
// n - 1 = d, 1/n = inv_n) over the same extent crossed at the start sine s0:
// returns horizontal and path excess without subtracting nearly equal
// lengths (s - s0 = -s0 e).
__device__ __forceinline__ void leg_excess(const LayerWalk& w, float span, float d, float inv_n, float& dr,
                                           float& gex) {
  float s, c2, e;
  layer_angle(w.s0, w.c0, w.d0, d, inv_n, s, c2, e);
  const float c = sqrtf(c2);
  const float dsq = -w.s0 * e * (s + w.s0);  // s^2 - s0^2
  const float den = s * w.c0 + w.s0 * c;     // zero only for a vertical photon, whose offset is zero
  if (den > 0.f) dr = fmaf(span, dsq / (den * c * w.c0), dr);
  gex = fmaf(span, dsq / (c * w.c0 * (c + w.c0)), gex);
}

template <bool NEED_TIME, bool NEED_EXCESS>
__device__ __forceinline__ void layer_walk(const float4* __restrict__ lay, float2 sp, float dh, int i,
                                           int obs_layer, float Px, float Py, float Pz, float ux, float uy,
                                           float uz, float axx, float axy, float axz, LayerWalk& w) {
  const float sh = sqrtf(ux * ux + uy * uy);
  float hx = 1.f, hy = 0.f;
  if (sh > 0.f) {
    const float ish = 1.0f / sh;
    hx = ux * ish;
    hy = uy * ish;
  }
  float4 L = lay[i];
  const float s0 = sh, c0 = -uz, d0 = L.x;
  w.d0 = d0;
  w.s0 = s0;
  w.c0 = c0;
  w.hx = hx;
  w.hy = hy;
  w.dr = 0.f;
  w.gex = 0.f;
  float x = Px, y = Py, z = Pz, tau = 0.f, geo2 = 0.f, opt = 0.f;
  // geometric delay per unit path 1 - v.a = |v - a|^2 / 2, v = (s h, -c), formed
  // from the differences so that no near-1 quantity is subtracted; the factor
  // 1/2 is applied once at the end
  const float nax = -axx, nay = -axy, naz = -axz;
  while (i > obs_layer) {
    const float zb = (float)i * dh;
    const float span = z - zb;
    float s, c2, e;
    layer_angle(s0, c0, d0, L.x, L.y, s, c2, e);
    const float ic = rsqrtf(c2);
    const float path = span * ic;
    const float adv = path * s;
    x = fmaf(hx, adv, x);
    y = fmaf(hy, adv, y);
    tau = fmaf(fmaf(L.z, sp.x, L.w * sp.y), path, tau);
    if constexpr (NEED_TIME) {
      const float ex = fmaf(s, hx, nax), ey = fmaf(s, hy, nay), ez = fmaf(-c2, ic, naz);
      geo2 = fmaf(path, fmaf(ex, ex, fmaf(ey, ey, ez * ez)), geo2);
    }
    if constexpr (NEED_TIME || NEED_EXCESS) opt = fmaf(L.x, path, opt);
    if constexpr (NEED_EXCESS) leg_excess(w, span, L.x, L.y, w.dr, w.gex);
    z = zb;
    --i;
    L = lay[i];
  }
  float s, c2, e;
  layer_angle(s0, c0, d0, L.x, L.y, s, c2, e);
  const float c = sqrtf(c2);
  w.x = x;
  w.y = y;
  w.z = z;
  w.vx = s * hx;
  w.vy = s * hy;
  w.vz = -c;
  w.tau = tau;
  w.geo = 0.5f * geo2;
  w.opt = opt;
  w.last_delta = L.x;
  w.last_ext = fmaf(L.z, sp.x, L.w * sp.y);
}

// Closed-form layer sums for planar layers. Below the start layer j every full
// layer i (obs < i < j, thickness dh) is crossed with 1/c_i = (1/c0) w_i,
// w_i = (1 + t u_i)^(-1/2), t = tan^2 of the start zenith angle and
// u_i = e_i (2 - e_i), e_i = (n_i - n_j) / n_i (Snell's law as in the crossing
// loop). Expanding w_i in powers of t u_i turns every sum the loop accumulates
// (travel, optical depth, optical path, geometric delay) into a polynomial in t
// whose coefficients depend only on (obs, j): moments of the layers' refractivity
// differences, tabulated once per atmosphere in FP64 (`mom`, five float4 per
// start layer, dh and the series coefficients folded in):
//   m0 = (a1 U1, a2 U2, a3 U3, EU0)   m1 = (a1 EU1, a2 EU2, E2U0, a1 E2U1)
//   m2 = (D0, a1 D1, a2 D2, R0)       m3 = (a1 R1, a2 R2, A0, a1 A1)
//   m4 = (a2 A2, N dh, 0, 0)
// with U_m = dh sum u^m, EU_m = dh sum e u^m, E2U_m = dh sum e^2 u^m,
// D_m = dh sum (n_i - 1) u^m, R_m / A_m = dh sum (Rayleigh / aerosol part) u^m,
// N = j - obs - 1 and a1 = -1/2, a2 = 3/8, a3 = -5/16. The geometric delay is
// expanded about the start direction v0, |v_i - a|^2 = |v0 - a|^2
// + 2 (v0 - a).(v_i - v0) + |v_i - v0|^2, so that no near-equal lengths are
// subtracted. With |t u| <= 5.4e-3 (the caller's bound) the truncated terms are
// below 2e-5 m over 32 km of layers. The start layer itself is crossed straight
// (e = 0). Outputs as layer_walk's at the top of the observation layer.
template <bool NEED_TIME>
__device__ __forceinline__ void layer_series(const float4* __restrict__ lay, const float4* __restrict__ mom,
                                             float2 sp, float dh, int j, int obs_layer, float Px, float Py,
                                             float Pz, float ux, float uy, float uz, float axx, float axy,
                                             float axz, LayerWalk& w) {
  const float sh = sqrt_fast(ux * ux + uy * uy);
  float hx = 1.f, hy = 0.f;
  if (sh > 0.f) {
    const float ish = rcp_fast(sh);
    hx = ux * ish;
    hy = uy * ish;
  }
  const float s0 = sh, c0 = -uz;
  const float4* m = mom + 5 * j;
  const float4 m0 = m[0], m1 = m[1], m2 = m[2], m3 = m[3], m4 = m[4];
  const float4 Lj = lay[j], Lo = lay[obs_layer];
  const float ic0 = rcp_fast(c0);
  const float tn = s0 * ic0, t = tn * tn;
  const float span = Pz - (float)j * dh;
  const float Ws = t * fmaf(t, fmaf(t, m0.z, m0.y), m0.x);  // dh sum (w - 1)
  const float Wd = m4.y + Ws;                                // dh sum w
  const float EWd = fmaf(t, fmaf(t, m1.y, m1.x), m0.w);      // dh sum e w
  const float adv = tn * (span + (Wd - EWd));
  w.x = fmaf(hx, adv, Px);
  w.y = fmaf(hy, adv, Py);
  w.z = (float)(obs_layer + 1) * dh;
  const float Rd = fmaf(t, fmaf(t, m3.y, m3.x), m2.w);
  const float Ad = fmaf(t, fmaf(t, m4.x, m3.w), m3.z);
  w.tau = ic0 * fmaf(fmaf(Lj.z, sp.x, Lj.w * sp.y), span, fmaf(sp.x, Rd, sp.y * Ad));
  w.geo = 0.f;
  w.opt = 0.f;
  if constexpr (NEED_TIME) {
    const float Dd = fmaf(t, fmaf(t, m2.z, m2.y), m2.x);
    w.opt = ic0 * fmaf(Lj.x, span, Dd);
    const float ex = fmaf(s0, hx, -axx), ey = fmaf(s0, hy, -axy), ez = -c0 - axz;
    const float G = fmaf(ex, ex, fmaf(ey, ey, ez * ez));
    const float gh = fmaf(hx, ex, hy * ey);
    const float E2Wd = fmaf(t, m1.w, m1.z);                                       // dh sum e^2 w
    const float Qd = t * t * fmaf(t, m0.z * 0.8f, m0.y * (2.0f / 3.0f));         // dh sum (1 - w)^2 / w
    const float inner = fmaf(G, span + Wd, fmaf(-2.0f * s0 * gh, EWd, s0 * s0 * E2Wd));
    w.geo = 0.5f * fmaf(ic0, inner, fmaf(2.0f * ez, Ws, c0 * Qd));
  }
  float s, c2, e;
  layer_angle(s0, c0, Lj.x, Lo.x, Lo.y, s, c2, e);
  const float c = sqrt_fast(c2);
  w.vx = s * hx;
  w.vy = s * hy;
  w.vz = -c;
  w.last_delta = Lo.x;
  w.last_ext = fmaf(Lo.z, sp.x, Lo.w * sp.y);
  w.s0 = s0;
  w.c0 = c0;
  w.d0 = Lj.x;
  w.hx = hx;
  w.hy = hy;
  w.dr = 0.f;
  w.gex = 0.f;
}

// Curved Earth (Sec. 3.3.4): the layers are spherical shells about the Earth
// centre. Within a shell a ray keeps its impact parameter; at a boundary the
// vector form of Snell's law with the radial normal conserves Bouguer's
// invariant n r sin(angle to the radial), so in shell i the impact parameter is
// p_i = n_0 (R + h_0) s_0 / n_i and the path stays in the plane of the Earth
// centre and the start direction. In FP32 a radius near R carries only half a
// metre, and the chord lengths of near-horizontal rays amplify that by
// tan^2 of the angle to the radial; so the walk never forms R + h - p_i by
// subtraction but carries the deficit
//   D_i(h) = (R + h) - p_i = (h - h_0) + (R + h_0) [(1 - s_0) - s_0 (d_0 - d_i) / (1 + d_i)],
// 1 - s_0 = c_0^2 / (1 + s_0), d = n - 1, whose terms are all small or exact. Then
// r cos(angle to the radial) = sqrt(D (2 r - D)) and a chord from ha down to hb is
//   l = (ha - hb)(2R + ha + hb) / (ra ca + rb cb),  dpsi = asin(p l / (ra rb)).
// A ray turns round inside a shell where D would become negative, and is
// totally reflected at a boundary where the next shell's D is not positive.
// The swept central angle is summed in FP64; the arrival point on the sphere
// R + h_obs is formed as a displacement from the emission point (below).
// Point of the sphere R + h_obs reached after sweeping the central angle psi
// from the emission point P (radial height h0) in the plane of the Earth centre
// and the direction u, moved by `across` metres normal to that plane. With the
// radial unit vector e_r at P, the unit tangent e_t (the direction's component
// across e_r) and r1 = R + h_obs, the point is C + r1 (cos psi e_r + sin psi e_t)
// and P = C + (R + h0) e_r, so
//   A - P = -((h0 - h_obs) + r1 (1 - cos psi)) e_r + r1 sin psi e_t,
// a sum of terms no larger than the path itself: FP32 carries it to about 1e-7 of
// the displacement (a few mm over tens of km), with no radius-sized value
// subtracted; A = P + (A - P) is formed in FP64 for the binning.
__device__ __forceinline__ void curved_arrival(double Re, float h_obs, float Px, float Py, float Pz, float h0,
                                               float ux, float uy, float uz, float psi, float across, double& ax,
                                               double& ay, double& az) {
  const float Rf = (float)Re;
  const float rq = Rf + h0;  // |P - C| (its rounding scales e_r by 1 +- 6e-8)
  const float irq = rcp_fast(rq);
  // e_r = (Px, Py, Pz + R) / rq, its z component kept as 1 + ez1 (Pz + R - rq = Pz - h0)
  const float erx = Px * irq, ery = Py * irq, ez1 = (Pz - h0) * irq;
  const float mu = fmaf(ux, erx, fmaf(uy, ery, fmaf(uz, ez1, uz)));
  float tx = fmaf(-mu, erx, ux), ty = fmaf(-mu, ery, uy), tz = fmaf(-mu, ez1, uz - mu);
  const float tn2 = fmaf(tx, tx, fmaf(ty, ty, tz * tz));
  if (tn2 > 0.f) {
    const float itn = __builtin_amdgcn_rsqf(tn2);
    tx *= itn;
    ty *= itn;
    tz *= itn;
  } else {
    tx = 1.f;
    ty = 0.f;
    tz = 0.f;
  }
  float sps, omc;  // sin psi and 1 - cos psi
  if (fabsf(psi) <= 0.5f) {
    // Taylor series: the first omitted terms are below 3e-9 and 2e-10 of the sums at |psi| = 0.5
    const float q = psi * psi;
    sps = psi * fmaf(q * (-1.0f / 6.0f), fmaf(q * (-1.0f / 20.0f), fmaf(q * (-1.0f / 42.0f), fmaf(q, -1.0f / 72.0f, 1.0f), 1.0f), 1.0f), 1.0f);
    omc = (0.5f * q) * fmaf(q * (-1.0f / 12.0f), fmaf(q * (-1.0f / 30.0f), fmaf(q * (-1.0f / 56.0f), fmaf(q, -1.0f / 90.0f, 1.0f), 1.0f), 1.0f), 1.0f);
  } else {
    const float sh = sinf(0.5f * psi);
    sps = sinf(psi);
    omc = 2.0f * sh * sh;
  }
  const float r1 = Rf + h_obs;
  const float rad = -fmaf(r1, omc, h0 - h_obs);  // along e_r
  const float tan = r1 * sps;                    // along e_t
  float dx = fmaf(rad, erx, tan * tx), dy = fmaf(rad, ery, tan * ty), dz = fmaf(rad, ez1, fmaf(tan, tz, rad));
  if (across != 0.f) {  // normal of the plane: e_r x e_t
    const float erz = 1.0f + ez1;
    dx = fmaf(across, ery * tz - erz * ty, dx);
    dy = fmaf(across, erz * tx - erx * tz, dy);
    dz = fmaf(across, erx * ty - ery * tx, dz);
  }
  ax = (double)Px + (double)dx;
  ay = (double)Py + (double)dy;
  az = (double)Pz + (double)dz;
}

struct CurvedWalk {
  double ax, ay, az;  // arrival point (core frame)
  float tau, geo, opt;
  int arrived;        // 0: left the top of the atmosphere
};

template <bool NEED_TIME>
__device__ __forceinline__ void curved_walk(const float4* __restrict__ lay, float2 sp, float dh, int n_layers,
                                            float h_obs, double Re, float Px, float Py, float Pz, float h0,
                                            float ux, float uy, float uz, float axx, float axy, float axz,
                                            CurvedWalk& w) {
  const float Rf = (float)Re, twoR = (float)(2.0 * Re);
  // emission frame: radial e_r, tangent e_t (photon's horizontal direction), normal e_n
  const float qz = Pz + Rf;
  const float rq = sqrt_fast(fmaf(Px, Px, fmaf(Py, Py, qz * qz)));
  const float irq = rcp_fast(rq);
  const float erx = Px * irq, ery = Py * irq, erz = qz * irq;
  const float mu = fmaf(ux, erx, fmaf(uy, ery, uz * erz));  // cos of the angle to the upward radial
  float etx = fmaf(-mu, erx, ux), ety = fmaf(-mu, ery, uy), etz = fmaf(-mu, erz, uz);
  const float s0 = sqrt_fast(fmaf(etx, etx, fmaf(ety, ety, etz * etz)));
  if (s0 > 0.f) {
    const float is = rcp_fast(s0);
    etx *= is;
    ety *= is;
    etz *= is;
  } else {
    etx = 1.f;
    ety = 0.f;
    etz = 0.f;
  }
  float a_r = 0.f, a_t = 0.f, a_n = 0.f;
  if constexpr (NEED_TIME) {
    const float enx = ery * etz - erz * ety, eny = erz * etx - erx * etz, enz = erx * ety - ery * etx;
    a_r = fmaf(axx, erx, fmaf(axy, ery, axz * erz));
    a_t = fmaf(axx, etx, fmaf(axy, ety, axz * etz));
    a_n = fmaf(axx, enx, fmaf(axy, eny, axz * enz));
  }
  int i = min((int)(h0 * (1.0f / dh)), n_layers - 1);
  const int obs = (int)floorf(h_obs / dh);
  const float A = Rf + h0;
  const float c1 = mu * mu / (1.0f + s0);  // 1 - s_0
  const float d0 = lay[i].x;
  // bracket of D_i for shell values (d_i, 1 / (1 + d_i))
  auto bracket = [&](float di, float inv_ni) { return fmaf(-s0, (d0 - di) * inv_ni, c1); };
  float h = h0, tau = 0.f, geo = 0.f, opt = 0.f;
  double psi = 0.0;
  bool down = mu < 0.f;
  int arrived = 0;
  for (int iter = 0; iter < 8 * n_layers; ++iter) {
    const float4 L = lay[i];
    const float br = bracket(L.x, L.y);
    const float ra = Rf + h;
    const float Da = fmaf(A, br, h - h0);
    const float rca = sqrt_fast(fmaxf(Da * (2.0f * ra - Da), 0.f));  // ra cos(angle to the radial)
    const float pa = ra - Da;                                     // impact parameter in this shell
    const float ext = fmaf(L.z, sp.x, L.w * sp.y);
    float ell, dpsi, cth;
    bool to_top = false;
    if (down) {
      const float hb = (i == obs) ? h_obs : (float)i * dh;
      const float Db = fmaf(A, br, hb - h0);
      if (Db > 0.f) {
        const float rb = Rf + hb;
        const float rcb = sqrt_fast(Db * (2.0f * rb - Db));
        ell = (h - hb) * (twoR + h + hb) * rcp_fast(rca + rcb);
        const float x = pa * ell * rcp_fast(ra * rb);
        dpsi = fmaf(x * x * (1.0f / 6.0f), x, x);
        cth = rca * rcp_fast(ra);
        h = hb;
      } else {  // the ray turns round inside the shell and leaves through its top
        const float ho = (float)(i + 1) * dh;
        const float ro = Rf + ho;
        const float Do = fmaf(A, br, ho - h0);
        const float rco = sqrt_fast(fmaxf(Do * (2.0f * ro - Do), 0.f));
        ell = rca + rco;
        dpsi = atan2f(rca, pa) + atan2f(rco, pa);
        cth = rca * rcp_fast(ra);
        h = ho;
        down = false;
        to_top = true;
      }
    } else {
      const float ho = (float)(i + 1) * dh;
      const float ro = Rf + ho;
      const float Do = fmaf(A, br, ho - h0);
      const float rco = sqrt_fast(fmaxf(Do * (2.0f * ro - Do), 0.f));
      ell = (ho - h) * (twoR + ho + h) * rcp_fast(rco + rca);
      const float x = pa * ell * rcp_fast(ra * ro);
      dpsi = fmaf(x * x * (1.0f / 6.0f), x, x);
      cth = -rca * rcp_fast(ra);
      h = ho;
      to_top = true;
    }
    tau = fmaf(ext, ell, tau);
    if constexpr (NEED_TIME) {
      const float sa = pa * rcp_fast(ra);
      float sp_, cp_;
      sincosf((float)psi, &sp_, &cp_);
      const float cphi = fmaf(cth, cp_, sa * sp_), sphi = fmaf(sa, cp_, -cth * sp_);
      const float gr = -cphi - a_r, gt = sphi - a_t;
      geo = fmaf(ell, 0.5f * fmaf(gr, gr, fmaf(gt, gt, a_n * a_n)), geo);
      opt = fmaf(L.x, ell, opt);
    }
    psi += (double)dpsi;
    if (!to_top) {
      if (i == obs) {
        arrived = 1;
        break;
      }
      const float4 Lb = lay[i - 1];
      if (!(fmaf(A, bracket(Lb.x, Lb.y), h - h0) > 0.f)) {
        down = false;  // total reflection at the boundary below: back up in shell i
        continue;
      }
      --i;
      continue;
    }
    if (i + 1 >= n_layers) break;  // left the atmosphere
    const float4 Lt = lay[i + 1];
    if (!(fmaf(A, bracket(Lt.x, Lt.y), h - h0) > 0.f)) {
      down = true;  // total reflection at the boundary above: back down in shell i
      continue;
    }
    ++i;
  }
  w.tau = tau;
  w.geo = geo;
  w.opt = opt;
  w.arrived = arrived;
  if (arrived) {
    curved_arrival(Re, h_obs, Px, Py, Pz, h0, ux, uy, uz, (float)psi, 0.f, w.ax, w.ay, w.az);
  } else {  // left the atmosphere: no arrival point
    w.ax = (double)Px;
    w.ay = (double)Py;
    w.az = (double)Pz;
  }
}

// Closed-form shell sums for a downward ray over spherical shells (Sec. 3.3.4;
// the evaluation of the shell walk's sums without one step per shell, as the
// planar layer sums above).
//
// With p the impact parameter in the start shell j (radius r0 = R + h0 there,
// local zenith cosine c0), Bouguer's invariant gives p_i^2 = p^2 (1 - u_i) in
// shell i, u_i = e_i (2 - e_i), e_i = (n_i - n_j) / n_i. With G(r) = r^2 - p^2
// (the straight line's squared distance from its perigee) the chord of shell i
// between radii ra > rb is sqrt(G(ra) + p^2 u_i) - sqrt(G(rb) + p^2 u_i). For the
// full shells between the observation shell and j, write G(b) = G_j - D(b),
// D(b) = b_j^2 - b^2 (b_j the start shell's lower radius), and expand
// sqrt(G_j - D + p^2 u) = sqrt(G_j) (1 - x + y)^(1/2) in x = D / G_j (curvature)
// and y = t u, t = p^2 / G_j (refraction; t is tan^2 of the straight line's
// zenith angle at b_j): every weighted sum of chords sum_i w_i l_i becomes
// sqrt(G_j) sum_km a_km t^k G_j^-m T_km(w), with shell moments
// T_km(w) = sum_i w_i u_i^k (D_{i+1}^m - D_i^m) tabulated per (observation
// shell, start shell) in FP64, the coefficients a_km = binom(1/2, k + m)
// binom(k + m, k) (-1)^m folded in and D scaled by S = 2 R dh. Weights: the
// Rayleigh and aerosol extinction parts (optical depth), the central angle per
// metre of chord R^2 / (b_i b_{i+1}) (its refraction part, k >= 1) and
// R^2 e_i / (b_i b_{i+1}) (the change of p), the path length (k >= 1) and n - 1
// (the delay). The straight line itself is never expanded: its chord L_s from r0
// to the observation sphere and its central angle asin(s0 L_s / r_obs) are
// formed directly, and the series add only the refraction terms to them. The
// partial start shell (straight, u = 0) and the partial observation shell
// (chord with p_obs, and its difference to the straight chord) are formed
// directly without subtracting near-equal lengths.
//
// Terms: k = 0 and 1 to m = 5, k = 2 to m = 3, k = 3 to m = 2 (15 pairs). The
// series serves rays with D_obs / G_j <= rho_max (0.1) and t <= t_max (the
// atmosphere's bound, t u_max <= 1.4e-2): there the omitted terms stay below
// 5e-4 m in path and arrival point and 1e-6 in optical depth (checked against
// the shell-by-shell chords in FP64). Other rays return false (the shell walk
// traces them). The delay uses the identity sum l_i (1 - v_i . a) = L - a.(E - P)
// split into the straight line's part L_s |u - a|^2 / 2, the path excess and the
// shift of the arrival point along the sphere.
// (kShellTerms, kShellRow and the row layout: cphot_internal.h)

// s += v . (b0, b1, b2, b3)
__device__ __forceinline__ float shell_acc4(float4 v, float b0, float b1, float b2, float b3, float s) {
  return fmaf(v.w, b3, fmaf(v.z, b2, fmaf(v.y, b1, fmaf(v.x, b0, s))));
}

template <bool NEED_TIME>
__device__ __forceinline__ bool curved_series(const float4* __restrict__ lay, const float* __restrict__ rows,
                                              float2 sp, float dh, int n_layers, int obs, float h_obs, double Re,
                                              float rho_max, float t_max, bool nb_rising, float Px, float Py,
                                              float Pz, float h0,
                                              float ux, float uy, float uz, float axx, float axy, float axz,
                                              CurvedWalk& w) {
  const float Rf = (float)Re, twoR = (float)(2.0 * Re);
  const float qz = Pz + Rf;
  const float rq = sqrt_fast(fmaf(Px, Px, fmaf(Py, Py, qz * qz)));
  const float irq = rcp_fast(rq);
  const float erx = Px * irq, ery = Py * irq, erz = qz * irq;
  const float mu = fmaf(ux, erx, fmaf(uy, ery, uz * erz));
  const float c0 = -mu;
  if (!(c0 > 0.f)) return false;
  const float etx0 = fmaf(-mu, erx, ux), ety0 = fmaf(-mu, ery, uy), etz0 = fmaf(-mu, erz, uz);
  const float s0 = sqrt_fast(fmaf(etx0, etx0, fmaf(ety0, ety0, etz0 * etz0)));
  const int j = min((int)(h0 * (1.0f / dh)), n_layers - 1);
  const float r0 = Rf + h0;
  const float rc0 = r0 * c0, p = r0 * s0;
  const float G0 = rc0 * rc0;
  const float robs = Rf + h_obs;
  // straight chord from r0 to the observation sphere
  const float dO = (h0 - h_obs) * (twoR + h0 + h_obs);
  const float Gobs = G0 - dO;
  const float4 Lj = lay[j];
  if (!(Gobs > 0.f)) {
    // The straight line misses the observation sphere. Refraction bends the ray
    // down, and it reaches the sphere iff its impact parameter in every shell,
    // n_j p / n_i, stays below that shell's lower radius (b_i, r_obs in the
    // observation shell); with n_i b_i increasing in i the binding shells are the
    // observation shell and the one above it. Rays failing this turn round above
    // the sphere and leave the atmosphere: they never arrive (no walk needed).
    if (!nb_rising) return false;
    const float gap = (h0 - h_obs) - r0 * (c0 * c0) * rcp_fast(1.0f + s0);  // p - r_obs
    float g = 0.f;                                                          // bound on p - r_obs
    if (j > obs) {
      const float hb1 = (float)(obs + 1) * dh - h_obs;                     // b_{obs+1} - r_obs
      g = fminf(robs * ((lay[obs].x - Lj.x) * Lj.y), fmaf(robs + hb1, (lay[obs + 1].x - Lj.x) * Lj.y, hb1));
    }
    if (gap < g) return false;  // bent onto the sphere: the shell walk traces it
    w.tau = 0.f;
    w.geo = 0.f;
    w.opt = 0.f;
    w.arrived = 0;
    w.ax = (double)Px;  // no arrival point
    w.ay = (double)Py;
    w.az = (double)Pz;
    return true;
  }
  const float Ls = dO * rcp_fast(rc0 + sqrt_fast(Gobs));
  const float extj = fmaf(Lj.z, sp.x, Lj.w * sp.y);
  float tau, dpsi = 0.f, dL = 0.f, opt = 0.f;
  if (j <= obs) {
    tau = extj * Ls;
    if constexpr (NEED_TIME) opt = Lj.x * Ls;
  } else {
    const float hj = (float)j * dh, ho1 = (float)(obs + 1) * dh;
    const float dJ = (h0 - hj) * (twoR + h0 + hj);           // r0^2 - b_j^2
    const float Gj = G0 - dJ;
    const float DO = (hj - h_obs) * (twoR + hj + h_obs);     // b_j^2 - r_obs^2
    const float iG = rcp_fast(Gj);
    const float t = (p * p) * iG;
    if (!(DO * iG <= rho_max && t <= t_max)) return false;
    const float sG = sqrt_fast(Gj);
    const float gam = (twoR * dh) * iG;
    // basis sqrt(G_j) t^k gam^m of the 15 terms, taken four at a time against the
    // rows' float4 groups (few live registers): q = 0..4 (k 0, m 1..5), 5..9 (k 1,
    // m 1..5), 10..12 (k 2, m 1..3), 13..14 (k 3, m 1..2)
    const float g1 = sG * gam, g2 = g1 * gam, g3 = g2 * gam, g4 = g3 * gam, g5 = g4 * gam;
    const float t2 = t * t, t3 = t2 * t;
    const float* r = rows + (size_t)j * kShellRow;
    const float4* r4 = reinterpret_cast<const float4*>(r);
    float sR = 0.f, sA = 0.f, sPe = 0.f, sP1 = 0.f, sL = 0.f, sD = 0.f;
    {
      const float b0 = g1, b1 = g2, b2 = g3, b3 = g4;
      sR = shell_acc4(r4[0], b0, b1, b2, b3, sR);
      sA = shell_acc4(r4[4], b0, b1, b2, b3, sA);
      sPe = shell_acc4(r4[8], b0, b1, b2, b3, sPe);
      if constexpr (NEED_TIME) sD = shell_acc4(r4[20], b0, b1, b2, b3, sD);
    }
    // the groups' loads stay with their products: hoisting all of them would hold
    // 64 (96 with the delay) table values at once
    __builtin_amdgcn_sched_barrier(0);
    {
      const float b0 = g5, b1 = t * g1, b2 = t * g2, b3 = t * g3;
      sR = shell_acc4(r4[1], b0, b1, b2, b3, sR);
      sA = shell_acc4(r4[5], b0, b1, b2, b3, sA);
      sPe = shell_acc4(r4[9], b0, b1, b2, b3, sPe);
      sP1 = shell_acc4(r4[13], b0, b1, b2, b3, sP1);
      if constexpr (NEED_TIME) {
        sL = shell_acc4(r4[17], b0, b1, b2, b3, sL);
        sD = shell_acc4(r4[21], b0, b1, b2, b3, sD);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    {
      const float b0 = t * g4, b1 = t * g5, b2 = t2 * g1, b3 = t2 * g2;
      sR = shell_acc4(r4[2], b0, b1, b2, b3, sR);
      sA = shell_acc4(r4[6], b0, b1, b2, b3, sA);
      sPe = shell_acc4(r4[10], b0, b1, b2, b3, sPe);
      sP1 = shell_acc4(r4[14], b0, b1, b2, b3, sP1);
      if constexpr (NEED_TIME) {
        sL = shell_acc4(r4[18], b0, b1, b2, b3, sL);
        sD = shell_acc4(r4[22], b0, b1, b2, b3, sD);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    {
      const float b0 = t2 * g3, b1 = t3 * g1, b2 = t3 * g2;  // the groups' fourth entries are zero
      sR = shell_acc4(r4[3], b0, b1, b2, 0.f, sR);
      sA = shell_acc4(r4[7], b0, b1, b2, 0.f, sA);
      sPe = shell_acc4(r4[11], b0, b1, b2, 0.f, sPe);
      sP1 = shell_acc4(r4[15], b0, b1, b2, 0.f, sP1);
      if constexpr (NEED_TIME) {
        sL = shell_acc4(r4[19], b0, b1, b2, 0.f, sL);
        sD = shell_acc4(r4[23], b0, b1, b2, 0.f, sD);
      }
    }
    // partial start shell (straight: u = 0 there) and partial observation shell
    const float lS = dJ * rcp_fast(rc0 + sG);
    const float4 Lo = lay[obs];
    const float eO = (Lo.x - Lj.x) * Lo.y;
    const float dd = (p * p) * (eO * (2.0f - eO));
    const float num = (ho1 - h_obs) * (twoR + ho1 + h_obs);  // b_{obs+1}^2 - r_obs^2
    const float A0 = Gj - (hj - ho1) * (twoR + hj + ho1), B0 = Gj - DO;
    const float qA = sqrt_fast(A0 + dd), qA0 = sqrt_fast(A0), qB = sqrt_fast(B0 + dd), qB0 = sqrt_fast(B0);
    const float lO = num * rcp_fast(qA + qB), lOs = num * rcp_fast(qA0 + qB0);
    const float dlO = -dd * (lO + lOs) * rcp_fast((qA + qA0) * (qB + qB0));  // lO - lOs
    tau = fmaf(extj, lS, fmaf(sp.x, sR, fmaf(sp.y, sA, fmaf(Lo.z, sp.x, Lo.w * sp.y) * lO)));
    dpsi = p * ((sP1 - sPe) * rcp_fast(Rf * Rf) + (dlO - eO * lO) * rcp_fast((Rf + ho1) * robs));
    if constexpr (NEED_TIME) {
      dL = sL + dlO;
      opt = fmaf(Lj.x, lS, fmaf(Lo.x, lO, sD));
    }
  }
  // straight central angle asin(s0 Ls / r_obs) (x <= 0.02: three terms)
  const float x = s0 * Ls * rcp_fast(robs), x2 = x * x;
  const float psi_s = x * fmaf(x2, fmaf(x2, 0.075f, 1.0f / 6.0f), 1.0f);
  w.tau = tau;
  w.opt = opt;
  w.geo = 0.f;
  if constexpr (NEED_TIME) {
    // delay: L_s |u - a|^2 / 2 + (L - L_s) - dpsi a.dE/dpsi at the straight arrival point
    const float is = s0 > 0.f ? rcp_fast(s0) : 0.f;
    const float etx = s0 > 0.f ? etx0 * is : 1.f, ety = s0 > 0.f ? ety0 * is : 0.f, etz = s0 > 0.f ? etz0 * is : 0.f;
    const float a_r = fmaf(axx, erx, fmaf(axy, ery, axz * erz)), a_t = fmaf(axx, etx, fmaf(axy, ety, axz * etz));
    const float gx = ux - axx, gy = uy - axy, gz = uz - axz;
    const float ps2 = psi_s * psi_s;  // |psi| <= 0.02: two terms each
    const float sps = psi_s * fmaf(ps2, -1.0f / 6.0f, 1.0f), cps = fmaf(ps2, -0.5f, 1.0f);
    w.geo = fmaf(0.5f * Ls, fmaf(gx, gx, fmaf(gy, gy, gz * gz)), dL) - dpsi * robs * fmaf(a_t, cps, -a_r * sps);
  }
  w.arrived = 1;
  curved_arrival(Re, h_obs, Px, Py, Pz, h0, ux, uy, uz, psi_s + dpsi, 0.f, w.ax, w.ay, w.az);
  return true;
}

}  // namespace cphot
