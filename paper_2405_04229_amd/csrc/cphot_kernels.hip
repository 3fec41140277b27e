// Photon generation and propagation kernels for gfx950.
//
// One persistent kernel per (block size, transport, detector, mode). Each block
// walks tiles of `BS` consecutive segments:
//   1. coalesced SoA load, one segment per thread; FP64 yield and the
//      stochastically rounded record count (Sec. 2.2.1); FP32 per-segment
//      geometry (cone angle, rotation bisector, start point, depth) into LDS;
//   2. block exclusive scan of the counts -> a flat record index space;
//   3. every thread takes records j = tid, tid + BS, ... and finds its segment
//      by binary search over the LDS offsets, then draws the record's Philox
//      block, builds the photon on the cone (Sec. 4.2), transports it
//      (Sec. 3.4.1 straight / Sec. 3.4.2 layered), applies absorption
//      (Sec. 2.3.2) and bins it (LDS-privatised grid histogram or global
//      atomics); upward photons leave first (Sec. 5.3.4).
// Photons live in registers only; nothing per photon touches HBM except the
// final bin increment.
#include "cphot_device.h"
#include "cphot_internal.h"
#include "cphot_mlp.h"

namespace cphot {

namespace {

struct SegResult {
  int32_t n;       // Cherenkov records
  int32_t status;  // 0 ok, 1 below the Cherenkov threshold, 2 skipped
  float cos_t, sin_t, a0, a1, a2;
  double mu;       // expected Cherenkov records
  int32_t nf[3];   // fluorescence records per band
  float inv_q;     // 1 / pre-emission reduction factor (1 without reduction)
  // DISPERSIVE: g(lambda) = beta n(lambda, h_mid) - 1 = disp_gm + disp_a (R(lambda) - R(lam_min))
  float disp_a, disp_gm;
};

// Per-segment yield in FP64 with IEEE basic operations only and no
// contraction, in the fixed order that makes the record count reproducible
// bit for bit on any IEEE machine. EXT: Poisson counts and the dispersive
// spectrum are compiled in (kernels without them never see those settings).
template <bool EXT>
__device__ __forceinline__ SegResult segment_setup(const KParams& p, float fx0, float fy0, float fz0, float fx1,
                                                float fy1, float fz1, float fbeta, float fq, float fdedx,
                                                uint64_t id) {
#pragma clang fp contract(off)
  SegResult r{0, 0, 0.f, 0.f, 0.f, 0.f, 0.f, 0.0, {0, 0, 0}, 1.f};
  const bool cher = (p.emission & CPHOT_EMIT_CHERENKOV) != 0;
  const bool fluor = (p.emission & CPHOT_EMIT_FLUORESCENCE) != 0;
  if (!__builtin_isfinite(fx0) || !__builtin_isfinite(fy0) || !__builtin_isfinite(fz0) ||
      !__builtin_isfinite(fx1) || !__builtin_isfinite(fy1) || !__builtin_isfinite(fz1) ||
      !__builtin_isfinite(fbeta) || !__builtin_isfinite(fq) || (fluor && !__builtin_isfinite(fdedx))) {
    r.status = 2;
    return r;
  }
  const double beta = (double)fbeta;
  if (!(beta > 0.0 && beta < 1.0)) {
    r.status = 2;
    return r;
  }
  const double dx = (double)fx1 - (double)fx0, dy = (double)fy1 - (double)fy0, dz = (double)fz1 - (double)fz0;
  const double L = sqrt(dx * dx + dy * dy + dz * dz);
  if (!(L > 0.0)) {
    r.status = 2;
    return r;
  }
  // pre-emission reduction (Sec. 4.3.1): the bound q of the layer holding the
  // segment's lowest point scales every expected count before rounding
  double q = 1.0;
  if (p.red) {
    const double hmin = (double)fz0 < (double)fz1 ? (double)fz0 : (double)fz1;
    double x = hmin / p.dh64;
    if (x < 0.0) x = 0.0;
    int64_t li = (int64_t)floor(x);
    if (li > p.n_layers - 1) li = p.n_layers - 1;
    q = p.red[li];
    r.inv_q = q > 0.0 ? (float)(1.0 / q) : 0.f;
  }
  // one Philox block per segment: word 0 rounds the Cherenkov yield, words 1..3
  // the fluorescence bands
  const uint4 w = philox(0u, (uint32_t)id, (uint32_t)(id >> 32), TAG_SEGMENT, p.key0, p.key1);
  if (cher) {
    // refractivity at the midpoint: direct index mapping into the FP64 table and
    // linear interpolation (Sec. 4.1), heights clamped to the table
    const double hm = 0.5 * ((double)fz0 + (double)fz1);
    double x = hm / p.step;
    if (x < 0.0) x = 0.0;
    if (x > (double)p.n_tab) x = (double)p.n_tab;
    double fi = floor(x);
    int64_t idx = (int64_t)fi;
    if (idx > p.n_tab - 1) {
      idx = p.n_tab - 1;
      fi = (double)idx;
    }
    const double frac = x - fi;
    double delta = (1.0 - frac) * p.tab[idx] + frac * p.tab[idx + 1];
    const double eps = 1.0 - beta;
    if (EXT && p.spectrum == CPHOT_SPECTRUM_DISPERSIVE) {
      // records are drawn for the largest cone, n at lam_min; each record's own
      // angle follows from its wavelength
      r.disp_a = (float)(delta * (1.0 - eps) * p.disp_inv_rref);
      delta = delta * p.disp_dmax;
    }
    // threshold beta n > 1 through g = beta n - 1 = delta - eps - eps delta, eps = 1 - beta
    const double g = delta - eps - eps * delta;
    if (!(g > 0.0)) {
      r.status = 1;
    } else {
      const double s2 = g * (g + 2.0) / ((1.0 + g) * (1.0 + g));
      r.disp_gm = (float)g;
      const double z2 = (double)fq * (double)fq;
      double mu = p.K * z2;
      mu = mu * L;
      mu = mu * s2;
      mu = mu / (double)p.bunch;
      if (!(mu < (double)(1 << kMaxRecordsPerSegmentLog2))) {
        r.status = 2;
        return r;
      }
      mu = mu * q;
      r.mu = mu;
      if (EXT && p.poisson) {
        const int64_t n = poisson_count(mu, w.x, id, TAG_POISSON, p.key0, p.key1);
        if (n >= (int64_t(1) << kMaxRecordsPerSegmentLog2)) {
          r.status = 2;
          r.n = 0;
          return r;
        }
        r.n = (int32_t)n;
      } else {
        const double fl = floor(mu);
        const double u = (double)w.x * (1.0 / 4294967296.0);
        r.n = (int32_t)fl + (u < mu - fl ? 1 : 0);
      }
      r.cos_t = (float)(1.0 / (1.0 + g));
      r.sin_t = (float)sqrt(s2);
    }
  }
  if (fluor && fdedx > 0.0f) {
    // per band: Y_b dE/dx L / 2 (lower hemisphere only)
    const uint32_t wb[3] = {w.y, w.z, w.w};
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      double mu = p.fl_yield[b] * (double)fdedx;
      mu = mu * L;
      mu = mu * 0.5;
      mu = mu / (double)p.bunch;
      if (!(mu < (double)(1 << kMaxRecordsPerSegmentLog2))) {
        SegResult bad{0, 2, 0.f, 0.f, 0.f, 0.f, 0.f, 0.0, {0, 0, 0}, 1.f};
        return bad;
      }
      mu = mu * q;
      if (EXT && p.poisson) {
        const int64_t n = poisson_count(mu, wb[b], id, TAG_POISSON + 1 + b, p.key0, p.key1);
        if (n >= (int64_t(1) << kMaxRecordsPerSegmentLog2)) {
          SegResult bad{0, 2, 0.f, 0.f, 0.f, 0.f, 0.f, 0.0, {0, 0, 0}, 1.f};
          return bad;
        }
        r.nf[b] = (int32_t)n;
      } else {
        const double fl = floor(mu);
        const double u = (double)wb[b] * (1.0 / 4294967296.0);
        r.nf[b] = (int32_t)fl + (u < mu - fl ? 1 : 0);
      }
    }
  }
  // bisector of the cone axis (0,0,-1) and the track direction; the rotation
  // is M = 2 a a^T - I (Euler-Rodrigues, 180 degrees, Sec. 4.2)
  const double P0 = dx / L, P1 = dy / L, P2 = dz / L;
  if (1.0 - P2 < 1e-6) {
    r.a0 = 1.f;  // 2 a a^T - I with a = x-hat: a half turn about x
  } else {
    const double b2 = P2 - 1.0;
    const double na = sqrt(P0 * P0 + P1 * P1 + b2 * b2);
    r.a0 = (float)(P0 / na);
    r.a1 = (float)(P1 / na);
    r.a2 = (float)(b2 / na);
  }
  return r;
}

// Per-block copy in LDS of the small kernel-argument arrays that records index
// per lane (Linsley pieces, fluorescence band wavelengths): indexing argument
// memory per lane would become vector loads from it, and holding the values in
// scalar registers would add to a scalar register file that is already full.
struct KConst {
  float4 lin[5];  // (lower bound (m), a, b, 1/c (1/cm)) per Linsley piece
  float4 fl;      // band wavelengths (nm)
};

__device__ __forceinline__ void load_kconst(const KParams& p, KConst& k, int tid) {
  if (tid < 5) k.lin[tid] = make_float4(p.hb[tid], p.la[tid], p.lb[tid], p.linv_c[tid]);
  if (tid == 5) k.fl = make_float4(p.fl_lambda[0], p.fl_lambda[1], p.fl_lambda[2], 0.f);
}

// Linsley vertical depth in FP32 (g/cm^2).
__device__ __forceinline__ float depth_f(const KConst& k, float h) {
  int i = 0;
#pragma unroll
  for (int j = 1; j < 5; ++j) i += (h >= k.lin[j].x) ? 1 : 0;
  const float4 c = k.lin[i];
  const float hcm = h * 100.0f;
  if (i < 4) return c.y + c.z * __expf(-hcm * c.w);
  return c.y - c.z * hcm * c.w;
}

// Squared horizontal distance from (qx, qy) on the observation level to the
// nearest sphere centre of the shower's array (indices clamped to the array).
__device__ __forceinline__ float nearest_sphere_d2(const KParams& p, float core_x, float core_y, float qx, float qy) {
  const float cx0 = core_x - 0.5f * (float)(p.snx - 1) * p.pitch;
  const float cy0 = core_y - 0.5f * (float)(p.sny - 1) * p.pitch;
  const float fi = fminf(fmaxf(rintf((qx - cx0) * p.inv_pitch), 0.f), (float)(p.snx - 1));
  const float fj = fminf(fmaxf(rintf((qy - cy0) * p.inv_pitch), 0.f), (float)(p.sny - 1));
  const float ex = qx - fmaf(fi, p.pitch, cx0), ey = qy - fmaf(fj, p.pitch, cy0);
  return fmaf(ex, ex, ey * ey);
}

// Data-reduction bounds (filter levels 1 and 3, Sec. 4.3.2 / 4.3.4), conservative:
// a photon reaching a sphere of radius r crosses the observation level within
// r / cos(final zenith) of its centre, and its crossing lies within the
// refraction bound of its straight line's: H tan(z) E (1 + 3 tan^2 z) x 1.1 + 0.5 m,
// E the largest |n_i - n_j| / n_i above the observation layer (|tan z_i - tan z| <=
// tan z (E + 0.77 x) with x = 2.2 tan^2 z E <= 0.25). Directions steeper than
// cos z = 0.2, or with x > 0.25, are never cut. `slack` covers FP32 rounding.
__device__ __forceinline__ float cut_slack(float qx, float qy, float core_x, float core_y, float H) {
  return 0.5f + 1e-5f * (fabsf(qx - core_x) + fabsf(qy - core_y) + H);
}

// Filter level 1: can any photon of this segment's Cherenkov cone (half-angle
// theta, from any point of the segment) reach a sphere? The cone's straight lines
// land within H theta / cos^2(zeta + theta) of the axis's landing point (the
// gnomonic projection stretches arcs by at most sec^2 of the largest zenith
// angle), the same point for every point of the segment.
__device__ __forceinline__ bool track_may_hit(const KParams& p, float x0, float y0, float z0, float x1, float y1,
                                              float z1, float cos_t, float sin_t, float core_x, float core_y) {
  const float dx = x1 - x0, dy = y1 - y0, dz = z1 - z0;
  const float L = sqrt_fast(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
  if (!(L > 0.f)) return true;
  const float iL = rcp_fast(L);
  const float cz = -dz * iL, sz = sqrt_fast(fmaxf((1.0f - cz) * (1.0f + cz), 0.f));
  const float cmin = fmaf(cz, cos_t, -sz * sin_t);  // cos of the steepest cone direction
  if (!(cmin > 0.2f)) return true;
  const float H = fmaxf(z0, z1) - p.h_obs;
  if (!(H > 0.f)) return true;
  const float ic = rcp_fast(cmin);
  const float t2 = (1.0f - cmin * cmin) * ic * ic, tmax = sqrt_fast(t2);
  const float x = 2.2f * t2 * p.cut_e;
  if (!(x <= 0.25f)) return true;
  const float Rfp = H * (1.01f * sin_t) * ic * ic;
  const float dref = fmaf(H * tmax * p.cut_e * fmaf(3.0f, t2, 1.0f), 1.1f, 0.5f);
  const float reff = p.radius * ic * rcp_fast(sqrt_fast(1.0f - x));
  const float s = (p.h_obs - z0) * rcp_fast(dz);  // in units of the segment vector from its start
  const float qx = fmaf(s, dx, x0), qy = fmaf(s, dy, y0);
  const float lim = Rfp + dref + reff + cut_slack(qx, qy, core_x, core_y, H);
  return nearest_sphere_d2(p, core_x, core_y, qx, qy) <= lim * lim;
}

// Filter level 3: can this photon, emitted at height Pz > h_obs going down, reach
// a sphere? Its straight line's crossing of the observation level against the
// nearest sphere centre.
__device__ __forceinline__ bool photon_may_hit(const KParams& p, float Px, float Py, float Pz, float ux, float uy,
                                               float uz, float core_x, float core_y) {
  const float c = -uz;
  if (!(c > 0.2f)) return true;
  const float H = Pz - p.h_obs;
  const float ic = rcp_fast(c);
  const float t2 = fmaf(ux, ux, uy * uy) * ic * ic;
  const float x = 2.2f * t2 * p.cut_e;
  if (!(x <= 0.25f)) return true;
  const float dref = fmaf(H * sqrt_fast(t2) * p.cut_e * fmaf(3.0f, t2, 1.0f), 1.1f, 0.5f);
  const float reff = p.radius * ic * rcp_fast(sqrt_fast(1.0f - x));
  const float s = H * ic;
  const float qx = fmaf(s, ux, Px), qy = fmaf(s, uy, Py);
  const float lim = reff + dref + cut_slack(qx, qy, core_x, core_y, H);
  return nearest_sphere_d2(p, core_x, core_y, qx, qy) <= lim * lim;
}

// Distance from (qx, qy) on the observation level to the shower's ground grid
// (zero inside it), squared.
__device__ __forceinline__ float grid_out_d2(const KParams& p, float core_x, float core_y, float qx, float qy) {
  const float gx0 = core_x - 0.5f * (float)p.nx * p.cell, gy0 = core_y - 0.5f * (float)p.ny * p.cell;
  const float gx1 = fmaf((float)p.nx, p.cell, gx0), gy1 = fmaf((float)p.ny, p.cell, gy0);
  const float dx = fmaxf(fmaxf(gx0 - qx, qx - gx1), 0.f), dy = fmaxf(fmaxf(gy0 - qy, qy - gy1), 0.f);
  return fmaf(dx, dx, dy * dy);
}

// Filter level 3 for the ground grid over planar layers: the photon's straight
// line against the grid rectangle, widened by the refraction bound of the sphere
// cut (the landing point moves by at most H tan(z) E (1 + 3 tan^2 z) x 1.1 + 0.5 m).
__device__ __forceinline__ bool grid_may_hit(const KParams& p, float Px, float Py, float Pz, float ux, float uy,
                                             float uz, float core_x, float core_y) {
  const float c = -uz;
  if (!(c > 0.2f)) return true;
  const float H = Pz - p.h_obs;
  const float ic = rcp_fast(c);
  const float t2 = fmaf(ux, ux, uy * uy) * ic * ic;
  if (!(2.2f * t2 * p.cut_e <= 0.25f)) return true;
  const float dref = fmaf(H * sqrt_fast(t2) * p.cut_e * fmaf(3.0f, t2, 1.0f), 1.1f, 0.5f);
  const float s = H * ic;
  const float qx = fmaf(s, ux, Px), qy = fmaf(s, uy, Py);
  const float lim = dref + cut_slack(qx, qy, core_x, core_y, H);
  return grid_out_d2(p, core_x, core_y, qx, qy) <= lim * lim;
}

// Filter level 3 for the ground grid over spherical shells, an exact bound. With the
// refractive index non-decreasing downwards, Bouguer's invariant n r sin(z) gives
// sin z <= sin z_s at every radius (z_s of the straight line from the same start), so
// the ray reaches the sphere R + h_obs whenever the straight line does, never turns,
// and tan z_s - tan z <= E tan z_s sec^2 z_s with E >= (n(r) - n_start) / n(r). The
// central angle swept falls short of the straight line's psi_s by at most
// E sec^2(z_end) psi_s (z_end the straight line's local zenith at the sphere, its
// largest), and the vertical projection onto the ground plane does not stretch arcs:
// the arrival lies within E sec^2(z_end) (R + h_obs) psi_s of the straight line's.
// Rays whose straight line misses the sphere are never cut.
__device__ __forceinline__ bool curved_may_land(const KParams& p, float Px, float Py, float Pz, float ux,
                                                float uy, float uz, float rq, float h0, float core_x,
                                                float core_y) {
  const float Rf = (float)p.earth_radius, r1 = Rf + p.h_obs;
  const float irq = rcp_fast(rq);
  const float c0 = -fmaf(ux, Px * irq, fmaf(uy, Py * irq, uz * ((Pz + Rf) * irq)));
  if (!(c0 > 0.f)) return true;
  const float drs = (h0 - p.h_obs) * (rq + r1);  // r0^2 - r1^2
  const float rc = rq * c0;
  const float disc = fmaf(rc, rc, -drs);
  if (!(disc > 0.f)) return true;
  const float s_ch = drs * rcp_fast(rc + sqrt_fast(disc));
  const float s0 = sqrt_fast(fmaxf((1.0f - c0) * (1.0f + c0), 0.f));
  const float se = fminf(rq * s0 * rcp_fast(r1), 1.0f);  // sin z_end
  const float sec2 = rcp_fast(fmaxf((1.0f - se) * (1.0f + se), 1e-30f));
  const float psi_s = asinf(fminf(s_ch * s0 * rcp_fast(r1), 1.0f));
  const float qx = fmaf(s_ch, ux, Px), qy = fmaf(s_ch, uy, Py);
  const float lim = fmaf(p.cut_e * sec2, r1 * psi_s * 1.1f, 1.0f) + 1e-5f * (fabsf(qx - core_x) + fabsf(qy - core_y) + s_ch);
  return grid_out_d2(p, core_x, core_y, qx, qy) <= lim * lim;
}

// Integral of n - 1 from height lo to height hi (m), closed form per profile.
__device__ __forceinline__ float opt_integral(const KParams& p, float lo, float hi, float X_lo, float X_hi) {
  if (p.profile == CPHOT_PROFILE_LINSLEY5) return p.opt_scale * (X_lo - X_hi);
  if (p.profile == CPHOT_PROFILE_HOMOGENEOUS) return p.opt_scale * (hi - lo);
  const float t = p.h_top;
  const float a = fminf(fmaxf(lo, 0.f), t), b = fminf(fmaxf(hi, 0.f), t);
  return p.opt_scale * ((b - a) - (b * b - a * a) / (2.f * t));
}

// Survival threshold of a record: exp(-tau), times the detector efficiency of
// its wavelength bin and divided by its segment's reduction factor when set
// (the detection probability over the probability the record was generated with).
// Without efficiency the table holds ones, without reduction 1/q is 1: no branches.
// Under the dispersive spectrum the uniform compared with it is u / p_emit.
__device__ __forceinline__ float survival_threshold(const KParams& p, const float* __restrict__ s_eff, float tau,
                                                    int kb, uint32_t inv_q_bits) {
  return __expf(-tau) * (s_eff[kb] * __uint_as_float(inv_q_bits));
}

template <int T>
constexpr bool kMlpTransport = (T == CPHOT_TRANSPORT_SURROGATE || T == kTransportCurvedSurrogate);

// A surrogate record outside the network's domain: its transport is redone by the
// exact tracer in a separate pass over compacted records.
constexpr int32_t kStateDeferred = 7;

struct Photon {
  int32_t state, bin, tbin, fallback, culled;
  int32_t ix, iy;  // grid cell
  float x, y, z, t, tau, lam, u3, ux, uy, uz;
};

// One record: emission, transport, absorption, detection. With the surrogate
// transport every lane of the wave must call this together (`valid` marks the
// lanes that carry a real record); the network is evaluated before any lane
// leaves.
template <int TRANSPORT, int DETECTOR, bool NEED_TIME, bool EXT>
__device__ __forceinline__ void trace(const KParams& p, const float4* __restrict__ s_lay,
                                      const float2* __restrict__ s_lam, const MlpImage* __restrict__ s_img,
                                      const KConst* __restrict__ s_k, const float* __restrict__ s_eff,
                                      uint4* s_stage,
                                      const float4 q0, const float4 q1, const float4 q2, const float4 q3,
                                      const float4 q4, const float axz, const uint4 q5, uint32_t k, bool valid,
                                      Photon& o) {
  const float sx = q0.x, sy = q0.y, sz = q0.z;
  const float dx = q1.x, dy = q1.y, dz = q1.z;
  const float ax = q2.x, ay = q2.y, az = q2.z, X0 = q2.w;
  const float dX = q3.x;
  const float core_x = q4.x, core_y = q4.y, axx = q4.z, axy = q4.w;
  // record k: Cherenkov records first (k < q5.x), then the fluorescence bands
  float f, lam, u3, ux, uy, uz;
  bool emitted = true;
  float inv_pe = 1.f;
  if (k < q5.x) {
    const uint4 w = philox(k, __float_as_uint(q3.y), __float_as_uint(q3.z), TAG_CHERENKOV, p.key0, p.key1);
    f = u24(w.x);
    float sphi, cphi;
    // the cone azimuth needs sin and cos only to about 2e-5: its error enters the
    // direction times sin(theta) < 0.025; the hardware sine takes revolutions
    const float ua = u24(w.y);
    sphi = __builtin_amdgcn_sinf(ua);
    cphi = __builtin_amdgcn_cosf(ua);
    const float u2 = u24(w.z);
    lam = (p.spectrum == CPHOT_SPECTRUM_UNIFORM)
              ? p.lam_min + (p.lam_max - p.lam_min) * u2
              : rcp_fast(p.inv_lam_min - u2 * (p.inv_lam_min - p.inv_lam_max));
    u3 = u24(w.w);
    float cos_t = q0.w, sin_t = q1.w;
    if (EXT && p.spectrum == CPHOT_SPECTRUM_DISPERSIVE) {
      // angle of this wavelength (Eq. 2.5) and the record's emission probability
      // sin^2(theta) / sin^2(theta_max) relative to the cone it was drawn for.
      // g = beta n - 1 is taken as its segment value at lam_min plus the change of
      // the dispersion sum, R(lambda) - R(lam_min) = (s^2 - s_min^2) (k1 / ((k0 - s^2)
      // (k0 - s_min^2)) + k3 / ((k2 - s^2) (k2 - s_min^2))), which FP32 resolves to
      // about 1e-12 in g where R itself would carry 1e-10.
      const float sg = 1000.0f * rcp_fast(lam), sg2 = sg * sg;
      const float dR = (sg2 - p.disp_s2m) *
                       fmaf(p.disp_k1c, rcp_fast(238.0185f - sg2), p.disp_k3c * rcp_fast(57.362f - sg2));
      const float gm = q1.w;
      const float g = fmaxf(fmaf(q0.w, dR, gm), 0.f);
      const float c = rcp_fast(1.0f + g), gg = g * (g + 2.0f);
      const float pe = (gg * (c * c)) * (((1.0f + gm) * (1.0f + gm)) * rcp_fast(gm * (gm + 2.0f)));
      emitted = u3 < pe;
      inv_pe = rcp_fast(pe);
      cos_t = c;
      sin_t = sqrt_fast(gg) * c;
    }
    // photon on the cone around (0,0,-1), turned onto the track: u = 2 a (a.p) - p
    const float plx = cphi * sin_t, ply = sphi * sin_t, plz = -cos_t;
    const float d2 = 2.0f * fmaf(ax, plx, fmaf(ay, ply, az * plz));
    ux = fmaf(d2, ax, -plx);
    uy = fmaf(d2, ay, -ply);
    uz = fmaf(d2, az, -plz);
  } else {
    // fluorescence (Sec. 4.2.2): isotropic in the lower hemisphere, cos(polar) uniform
    const uint32_t band = (k < q5.y) ? 0u : ((k < q5.z) ? 1u : 2u);
    const uint32_t kk = k - (band == 0u ? q5.x : (band == 1u ? q5.y : q5.z));
    const uint4 w = philox(kk, __float_as_uint(q3.y), __float_as_uint(q3.z), TAG_FLUOR + band, p.key0, p.key1);
    f = u24(w.x);
    const float cz = 1.0f - u24(w.y);
    float sphi, cphi;
    sincospif(2.0f * u24(w.z), &sphi, &cphi);
    const float sz = sqrtf((1.0f - cz) * (1.0f + cz));
    ux = sz * cphi;
    uy = sz * sphi;
    uz = -cz;
    lam = (&s_k->fl.x)[band];
    u3 = u24(w.w);
  }
  o.lam = lam;
  o.u3 = u3;
  // detected iff u < p_emit exp(-tau) efficiency / q: compare u / p_emit from here on
  if constexpr (EXT) u3 = u3 * inv_pe;
  o.bin = -1;
  o.tbin = -1;
  o.fallback = 0;
  o.culled = 0;
  o.t = 0.f;
  o.tau = 0.f;
  o.ux = ux;
  o.uy = uy;
  o.uz = uz;
  const float Px = fmaf(f, dx, sx), Py = fmaf(f, dy, sy), Pz = fmaf(f, dz, sz);
  o.x = Px;
  o.y = Py;
  o.z = Pz;
  if constexpr (EXT && !kMlpTransport<TRANSPORT>) {
    if (!emitted) {  // below the threshold at its wavelength: never emitted
      o.state = 4;
      return;
    }
  }
  int kb = 0;
  if (TRANSPORT != CPHOT_TRANSPORT_STRAIGHT || p.eff) {
    kb = (int)((lam - p.lam_min) * ((float)p.n_lam / (p.lam_max - p.lam_min)));
    kb = min(max(kb, 0), p.n_lam - 1);
  }
  if constexpr (TRANSPORT == CPHOT_TRANSPORT_CURVED || TRANSPORT == kTransportCurvedWalk ||
                TRANSPORT == kTransportCurvedExact || TRANSPORT == kTransportCurvedSurrogate ||
                TRANSPORT == kTransportCurvedTable) {
    // height above the sphere R without subtracting R: (x^2 + y^2 + z (2R + z)) / (|P - C| + R)
    const float Rf = (float)p.earth_radius;
    const float qz = Pz + Rf;
    const float rq = sqrt_fast(fmaf(Px, Px, fmaf(Py, Py, qz * qz)));
    const float h0 = fmaf(Px, Px, fmaf(Py, Py, Pz * (2.0f * Rf + Pz))) * rcp_fast(rq + Rf);
    bool cull = false;  // filter level 3: cannot land on the grid
    if constexpr (TRANSPORT != kTransportCurvedExact) {
      if ((p.cuts & CPHOT_CUT_PHOTON) && uz < 0.f && h0 >= p.h_obs)
        cull = !curved_may_land(p, Px, Py, Pz, ux, uy, uz, rq, h0, core_x, core_y);
    }
    float ym[kMlpOut] = {0.f, 0.f, 0.f, 0.f};
    bool use_mlp = false;
    float c0 = 0.f;    // cos of the local zenith angle (angle between -u and the upward radial)
    float leg = 0.f;   // straight path inside the start shell, down to its lower boundary
    int j0 = 0;        // start shell
    if constexpr (TRANSPORT == kTransportCurvedSurrogate) {
      const float irq = rcp_fast(rq);
      c0 = -fmaf(ux, Px * irq, fmaf(uy, Py * irq, uz * (qz * irq)));
      const bool alive = valid && emitted && (uz < 0.f) && (h0 >= p.h_obs) && !cull;
      // the network starts at the start shell's lower boundary R + h_b (the photon is
      // straight inside its homogeneous start shell); a start inside the observation
      // shell is straight all the way (h_b = h_obs, nothing left to correct)
      j0 = min((int)(h0 * p.inv_dh), p.n_layers - 1);
      const bool in_obs = j0 <= p.obs_layer;
      const float h_b = in_obs ? p.h_obs : (float)j0 * p.dh;
      const float rc0 = (Rf + h0) * c0;
      const float dJ = (h0 - h_b) * (2.0f * Rf + h0 + h_b);  // r0^2 - r_b^2
      const float gb = fmaf(rc0, rc0, -dJ);                   // r_b^2 cos^2 at the boundary
      const bool reach = c0 > 0.f && gb > 0.f;
      const float sgb = sqrt_fast(fmaxf(gb, 0.f));
      leg = reach ? dJ * rcp_fast(rc0 + sgb) : 0.f;
      float xin[kMlpIn] = {h_b, sgb * rcp_fast(Rf + h_b), atan2f(uy, ux),
                           p.lam_min + ((float)kb + 0.5f) * ((p.lam_max - p.lam_min) / (float)p.n_lam), p.h_obs};
      use_mlp = alive && reach && (in_obs || mlp_in_domain(s_img, xin));
      if (!use_mlp || in_obs) {
#pragma unroll
        for (int q = 0; q < kMlpIn; ++q) xin[q] = s_img->in_lo[q];  // finite filler for lanes that do not use it
      }
      // the whole wave evaluates the network together, or skips it when no lane needs it
      if (__ballot(use_mlp && !in_obs)) mlp_forward_wave(s_img, xin, ym, s_stage);
      if (in_obs) {
#pragma unroll
        for (int q = 0; q < kMlpOut; ++q) ym[q] = 0.f;
      }
      if (EXT && !emitted) {
        o.state = 4;
        return;
      }
    }
    if (!(uz < 0.f)) {
      o.state = 1;
      return;
    }
    if (h0 < p.h_obs) {
      o.state = 3;
      return;
    }
    if (cull) {
      o.state = 3;
      o.culled = 1;
      return;
    }
    if constexpr (TRANSPORT == kTransportCurvedTable) {
      // correction interpolated from the table (Sec. 4.4.1), in the start shell
      const float irq = rcp_fast(rq);
      c0 = -fmaf(ux, Px * irq, fmaf(uy, Py * irq, uz * (qz * irq)));
      float4 v;
      const float tz = sqrt_fast(fmaxf((1.0f - c0) * (1.0f + c0), 0.f)) * rcp_fast(c0);
      use_mlp = c0 > 0.f && table_lookup(p.ctab, min((int)(h0 * p.inv_dh), p.n_layers - 1), h0, tz, v);
      const float2 sp = s_lam[kb];
      ym[0] = v.x;
      ym[2] = v.y;
      ym[3] = -fmaf(v.z, sp.x, v.w * sp.y);
    }
    CurvedWalk cw;
    if (use_mlp) {
      // straight chord to the sphere R + h_obs (cancellation-free root), its
      // central angle, plus the predicted extra ground distance, offset across,
      // optical path excess and log T (the network predicts them per metre of chord)
      const float r0 = Rf + h0, r1 = Rf + p.h_obs;
      const float s0 = sqrt_fast(fmaxf((1.0f - c0) * (1.0f + c0), 0.f));
      const float drs = (h0 - p.h_obs) * (r0 + r1);
      const float rc = r0 * c0;
      const float s_ch = drs * rcp_fast(rc + sqrt_fast(fmaf(rc, rc, -drs)));
      const float xs = s_ch * s0 * rcp_fast(r1);
      const float psi_s = fmaf(xs * xs * (1.0f / 6.0f), xs, xs);
      // the network's outputs are per metre of the chord from the start shell's lower
      // boundary (the same straight line, shortened by the leg inside the start
      // shell, whose optical depth and n - 1 are added exactly); the table's are absolute
      const float scale = (TRANSPORT == kTransportCurvedTable) ? 1.0f : s_ch - leg;
      const float psi = fmaf(ym[0] * scale, rcp_fast(r1), psi_s);
      curved_arrival(p.earth_radius, p.h_obs, Px, Py, Pz, h0, ux, uy, uz, psi, ym[1] * scale, cw.ax, cw.ay, cw.az);
      const float4 Lj = s_lay[j0];
      cw.tau = fmaf(fmaf(Lj.z, s_lam[kb].x, Lj.w * s_lam[kb].y), leg, -ym[3] * scale);
      cw.arrived = 1;
      cw.geo = 0.f;
      cw.opt = 0.f;
      if constexpr (NEED_TIME) {
        // delay = chord (1 - u.a) + excess - (arrival - chord end) . a
        const float gx = ux - axx, gy = uy - axy, gz = uz - axz;
        const double ex = (double)Px + (double)s_ch * ux, ey = (double)Py + (double)s_ch * uy,
                     ez = (double)Pz + (double)s_ch * uz;
        const float shift = (float)((cw.ax - ex) * axx + (cw.ay - ey) * axy + (cw.az - ez) * axz);
        cw.geo = fmaf(s_ch * 0.5f, fmaf(gx, gx, fmaf(gy, gy, gz * gz)), -shift);
        cw.opt = fmaf(Lj.x, leg, ym[2] * scale);
      }
    } else {
      if constexpr (TRANSPORT == kTransportCurvedSurrogate || TRANSPORT == kTransportCurvedTable) {
        o.state = kStateDeferred;  // outside the domain: traced exactly in a compacted pass
        return;
      }
      if constexpr (TRANSPORT == CPHOT_TRANSPORT_CURVED || TRANSPORT == kTransportCurvedExact) {
        // closed-form shell sums; rays outside their domain are walked, in a
        // compacted pass (CURVED) or in place (records that are compacted already)
        if (!curved_series<NEED_TIME>(s_lay, p.shells, s_lam[kb], p.dh, p.n_layers, p.obs_layer, p.h_obs,
                                      p.earth_radius, p.shell_rho, p.shell_tmax, p.shell_nb_rising != 0, Px, Py, Pz,
                                      h0, ux, uy, uz, axx, axy, axz, cw)) {
          if constexpr (TRANSPORT == CPHOT_TRANSPORT_CURVED) {
            o.state = kStateDeferred;
            return;
          } else {
            curved_walk<NEED_TIME>(s_lay, s_lam[kb], p.dh, p.n_layers, p.h_obs, p.earth_radius, Px, Py, Pz, h0,
                                   ux, uy, uz, axx, axy, axz, cw);
          }
        }
      } else {
        curved_walk<NEED_TIME>(s_lay, s_lam[kb], p.dh, p.n_layers, p.h_obs, p.earth_radius, Px, Py, Pz, h0, ux, uy,
                               uz, axx, axy, axz, cw);
      }
    }
    o.x = (float)cw.ax;
    o.y = (float)cw.ay;
    o.z = (float)cw.az;
    o.tau = cw.tau;
    if constexpr (NEED_TIME) o.t = (cw.geo + cw.opt) * (1.0f / kCmPerNs);
    if (!cw.arrived) {
      o.state = 3;
      return;
    }
    if (!(u3 < survival_threshold(p, s_eff, cw.tau, kb, q5.w))) {
      o.state = 2;
      return;
    }
    // bins in the tangent plane at the core, in FP64
    const double gx0 = (double)core_x - 0.5 * (double)p.nx * (double)p.cell;
    const double gy0 = (double)core_y - 0.5 * (double)p.ny * (double)p.cell;
    const double fxc = floor((cw.ax - gx0) * p.inv_cell64), fyc = floor((cw.ay - gy0) * p.inv_cell64);
    if (!(fxc >= 0.0 && fyc >= 0.0 && fxc < (double)p.nx && fyc < (double)p.ny)) {
      o.state = 3;
      return;
    }
    o.state = 0;
    o.ix = (int)fxc;
    o.iy = (int)fyc;
    o.bin = o.iy * p.nx + o.ix;
    return;
  } else {
  float ym[kMlpOut] = {0.f, 0.f, 0.f, 0.f};
  bool use_mlp = false;
  float h_b = Pz;   // the network's start: the lower boundary of the start layer (no leg otherwise)
  int j0 = 0;       // start layer
  if constexpr (TRANSPORT == CPHOT_TRANSPORT_SURROGATE) {
    const bool alive = valid && emitted && (uz < 0.f) && (Pz >= p.h_obs);
    // straight inside the homogeneous start layer; the network takes over at its lower
    // boundary; a start inside the observation layer is straight all the way
    j0 = min((int)(Pz * p.inv_dh), p.n_layers - 1);
    const bool in_obs = j0 <= p.obs_layer;
    h_b = in_obs ? p.h_obs : (float)j0 * p.dh;
    float xin[kMlpIn] = {h_b, -uz, atan2f(uy, ux),
                         p.lam_min + ((float)kb + 0.5f) * ((p.lam_max - p.lam_min) / (float)p.n_lam), p.h_obs};
    use_mlp = alive && (in_obs || mlp_in_domain(s_img, xin));
    if (!use_mlp || in_obs) {
#pragma unroll
      for (int q = 0; q < kMlpIn; ++q) xin[q] = s_img->in_lo[q];  // finite filler for lanes that do not use it
    }
    // the whole wave evaluates the network together, or skips it when no lane needs it
    if (__ballot(use_mlp && !in_obs)) mlp_forward_wave(s_img, xin, ym, s_stage);
    if (in_obs) {
#pragma unroll
      for (int q = 0; q < kMlpOut; ++q) ym[q] = 0.f;
    }
    if (EXT && !emitted) {
      o.state = 4;
      return;
    }
  }
  if (!(uz < 0.f)) {
    o.state = 1;
    return;
  }
  if (Pz < p.h_obs) {
    o.state = 3;
    return;
  }
  if constexpr (DETECTOR == CPHOT_DETECTOR_SPHERES && !kMlpTransport<TRANSPORT>) {
    if ((p.cuts & CPHOT_CUT_PHOTON) && !photon_may_hit(p, Px, Py, Pz, ux, uy, uz, core_x, core_y)) {
      o.state = 3;  // filter level 3: cannot reach a sphere
      o.culled = 1;
      return;
    }
  }
  if constexpr (DETECTOR == CPHOT_DETECTOR_GRID && !kMlpTransport<TRANSPORT>) {
    if ((p.cuts & CPHOT_CUT_PHOTON) && !grid_may_hit(p, Px, Py, Pz, ux, uy, uz, core_x, core_y)) {
      o.state = 3;  // filter level 3: cannot land on the grid
      o.culled = 1;
      return;
    }
  }
  if constexpr (TRANSPORT == CPHOT_TRANSPORT_TABLE) {
    // correction interpolated from the table (Sec. 4.4.1), in the start layer
    float4 v;
    const float tz = sqrtf(fmaf(ux, ux, uy * uy)) / -uz;
    use_mlp = table_lookup(p.ctab, min((int)(Pz * p.inv_dh), p.n_layers - 1), Pz, tz, v);
    const float2 sp = s_lam[kb];
    ym[0] = v.x;
    ym[2] = v.y;
    ym[3] = -fmaf(v.z, sp.x, v.w * sp.y);
  }
  float x, y, z;     // start of the final leg
  float vx, vy, vz;  // direction of the final leg
  float tau = 0.f, geo = 0.f, opt = 0.f;
  float last_delta = 0.f, last_ext = 0.f;
  if constexpr (TRANSPORT != CPHOT_TRANSPORT_STRAIGHT) {
    if (TRANSPORT == CPHOT_TRANSPORT_LAYERED || !use_mlp) {
      if constexpr (TRANSPORT == CPHOT_TRANSPORT_SURROGATE || TRANSPORT == CPHOT_TRANSPORT_TABLE) {
        o.state = kStateDeferred;  // outside the domain: traced exactly in a compacted pass
        return;
      }
      LayerWalk lw;
      const int j0 = min((int)(Pz * p.inv_dh), p.n_layers - 1);
      // closed-form sums where the series holds, the crossing loop elsewhere
      if (j0 > p.obs_layer && fmaf(ux, ux, uy * uy) <= p.series_tmax * (uz * uz))
        layer_series<NEED_TIME>(s_lay, p.moments, s_lam[kb], p.dh, j0, p.obs_layer, Px, Py, Pz, ux, uy, uz, axx,
                                axy, axz, lw);
      else
        layer_walk<NEED_TIME, false>(s_lay, s_lam[kb], p.dh, j0, p.obs_layer, Px, Py, Pz, ux, uy, uz, axx, axy,
                                     axz, lw);
      x = lw.x;
      y = lw.y;
      z = lw.z;
      vx = lw.vx;
      vy = lw.vy;
      vz = lw.vz;
      tau = lw.tau;
      geo = lw.geo;
      opt = lw.opt;
      last_delta = lw.last_delta;
      last_ext = lw.last_ext;
    } else {
      // straight line to the observation level plus the predicted correction:
      // landing (dx, dy), optical path excess e and log T; the delay after the
      // plane front is [l (1 - u.a) + e - (dx a_x + dy a_y)] / c
      const float s_pl = (p.h_obs - Pz) / uz;
      // the predicted offset is along / across the photon's horizontal direction
      const float sh = sqrtf(fmaf(ux, ux, uy * uy));
      const float hx = sh > 0.f ? ux / sh : 1.f, hy = sh > 0.f ? uy / sh : 0.f;
      const float odx = fmaf(ym[0], hx, -ym[1] * hy), ody = fmaf(ym[0], hy, ym[1] * hx);
      x = fmaf(s_pl, ux, Px) + odx;
      y = fmaf(s_pl, uy, Py) + ody;
      z = p.h_obs;
      vx = ux;
      vy = uy;
      vz = uz;
      // the leg inside the start layer down to the network's start h_b, exactly, and
      // for the table its absolute sums; the network predicts what refraction adds to
      // the straight line's own sums below h_b (full layers from the layer-sum
      // moments, the observation layer's span directly)
      const float ic = 1.0f / -uz;
      const float leg = (Pz - h_b) * ic;
      const float4 Lj = s_lay[j0];
      const float2 sp = s_lam[kb];
      float tau_s = 0.f, opt_s = 0.f;
      if constexpr (TRANSPORT == CPHOT_TRANSPORT_SURROGATE) {
        if (j0 > p.obs_layer) {
          const float4* mr = p.moments + 5 * j0;
          const float4 Lo = s_lay[p.obs_layer];
          const float top = (float)(p.obs_layer + 1) * p.dh - p.h_obs;
          tau_s = ic * fmaf(sp.x, mr[2].w, fmaf(sp.y, mr[3].z, fmaf(Lo.z, sp.x, Lo.w * sp.y) * top));
          opt_s = ic * fmaf(Lo.x, top, mr[2].x);
        }
      }
      tau = fmaf(fmaf(Lj.z, sp.x, Lj.w * sp.y), leg, tau_s - ym[3]);
      if constexpr (NEED_TIME) {
        const float gx = ux - axx, gy = uy - axy, gz = uz - axz;
        geo = s_pl * 0.5f * (gx * gx + gy * gy + gz * gz) - (odx * axx + ody * axy);
        opt = fmaf(Lj.x, leg, opt_s + ym[2]);
      }
      const float4 L = s_lay[p.obs_layer];
      last_delta = L.x;
      last_ext = fmaf(L.z, sp.x, L.w * sp.y);
    }
  } else {
    x = Px;
    y = Py;
    z = Pz;
    vx = ux;
    vy = uy;
    vz = uz;
  }
  // final straight leg: crossing of the observation level
  const float s_plane = (p.h_obs - z) * rcp_fast(vz);
  const float Qx = fmaf(s_plane, vx, x), Qy = fmaf(s_plane, vy, y);
  float s_end = s_plane;
  int32_t bin = -1;
  if constexpr (DETECTOR == CPHOT_DETECTOR_GRID) {
    const float gx0 = core_x - 0.5f * (float)p.nx * p.cell;
    const float gy0 = core_y - 0.5f * (float)p.ny * p.cell;
    const float fxc = floorf((Qx - gx0) * p.inv_cell), fyc = floorf((Qy - gy0) * p.inv_cell);
    if (fxc >= 0.f && fyc >= 0.f && fxc < (float)p.nx && fyc < (float)p.ny) {
      o.ix = (int)fxc;
      o.iy = (int)fyc;
      bin = o.iy * p.nx + o.ix;
    }
  } else {
    const float cx0 = core_x - 0.5f * (float)(p.snx - 1) * p.pitch;
    const float cy0 = core_y - 0.5f * (float)(p.sny - 1) * p.pitch;
    const float fi = floorf((Qx - cx0) * p.inv_pitch + 0.5f), fj = floorf((Qy - cy0) * p.inv_pitch + 0.5f);
    if (fi >= 0.f && fj >= 0.f && fi < (float)p.snx && fj < (float)p.sny) {
      const float qx = Qx - (cx0 + fi * p.pitch), qy = Qy - (cy0 + fj * p.pitch);
      const float b = qx * vx + qy * vy;  // q_z = 0 on the observation level
      const float cc = qx * qx + qy * qy - p.radius * p.radius;
      const float disc = b * b - cc;
      if (disc >= 0.f) {
        s_end = s_plane + (-b - sqrt_fast(disc));
        bin = (int)fj * p.snx + (int)fi;
      }
    }
  }
  const float ex = fmaf(s_end, vx, x), ey = fmaf(s_end, vy, y), ez = fmaf(s_end, vz, z);
  if constexpr (TRANSPORT != CPHOT_TRANSPORT_STRAIGHT) {
    tau = fmaf(last_ext, s_end, tau);
    if constexpr (NEED_TIME) {
      const float gx = vx - axx, gy = vy - axy, gz = vz - axz;
      geo = fmaf(s_end, 0.5f * (gx * gx + gy * gy + gz * gz), geo);
      opt = fmaf(last_delta, s_end, opt);
    }
  } else {
    // straight line in a planar atmosphere: closed forms over the height span
    const float inv_uz = -1.0f / vz;  // 1/|u_z|
    const float Xe = fmaf(f, dX, X0);
    float X_end = p.X_obs;
    if constexpr (DETECTOR == CPHOT_DETECTOR_SPHERES) {
      if (p.profile == CPHOT_PROFILE_LINSLEY5) X_end = depth_f(*s_k, ez);
    }
    if (p.has_ray) {
      const float r = 400.0f / lam;
      const float r2 = r * r;
      tau = (X_end - Xe) * inv_uz * (r2 * r2 * p.inv_ray400);
    }
    if (p.has_aer) {
      const float taua = p.aer_tau350 * __powf(lam * (1.0f / 350.0f), -p.aer_ang);
      tau = fmaf(taua * (__expf(-ez * p.aer_inv_h) - __expf(-Pz * p.aer_inv_h)), inv_uz, tau);
    }
    if constexpr (NEED_TIME) {
      const float gx = vx - axx, gy = vy - axy, gz = vz - axz;
      geo = s_end * 0.5f * (gx * gx + gy * gy + gz * gz);
      opt = opt_integral(p, ez, Pz, X_end, Xe) * inv_uz;
    }
  }
  o.x = ex;
  o.y = ey;
  o.z = ez;
  o.tau = tau;
  if constexpr (NEED_TIME) o.t = (geo + opt) * (1.0f / kCmPerNs);
  if (!(u3 < survival_threshold(p, s_eff, tau, kb, q5.w))) {
    o.state = 2;
    return;
  }
  if (bin < 0) {
    o.state = 3;
    return;
  }
  o.state = 0;
  o.bin = bin;
  if constexpr (DETECTOR == CPHOT_DETECTOR_SPHERES) {
    if (p.n_t > 0) {
      const float tb = floorf(o.t * p.inv_dt);
      o.tbin = tb < 0.f ? 0 : (tb >= (float)p.n_t ? p.n_t : (int)tb);
    }
  }
  }
}

}  // namespace

// Shower of segment i: the largest s with offsets[s] <= i.
__device__ __forceinline__ int shower_of(const KParams& p, int64_t i) {
  if (p.n_showers <= 1) return 0;
  int lo = 0, hi = p.n_showers;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (p.offsets[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

// Adds the LDS window of shower `sh` (record counts) to the global bins with
// the bunch weight, and clears it. Called by the whole block. The window is a
// rectangle of grid cells, or the whole sphere array.
template <int BS, int DETECTOR>
__device__ void flush_window(const KParams& p, uint32_t* s_hist, int sh) {
  const int n = p.hist_w * p.hist_h;
  const int row = DETECTOR == CPHOT_DETECTOR_GRID ? p.nx : p.snx;
  const int64_t base = (int64_t)sh * row * (DETECTOR == CPHOT_DETECTOR_GRID ? p.ny : p.sny);
  for (int b = threadIdx.x; b < n; b += BS) {
    const uint32_t v = s_hist[b];
    if (v) {
      const int ly = b / p.hist_w, lx = b - ly * p.hist_w;
      const int64_t gb = base + (int64_t)(p.hist_y0 + ly) * row + (p.hist_x0 + lx);
      const unsigned long long w = (unsigned long long)v * (unsigned long long)p.bunch;
      if (p.bins_f64) atomicAdd(reinterpret_cast<double*>(p.bins) + gb, (double)w);
      else if (p.bins_u64) atomicAdd(reinterpret_cast<unsigned long long*>(p.bins) + gb, w);
      else atomicAdd(reinterpret_cast<uint32_t*>(p.bins) + gb, (uint32_t)w);
      s_hist[b] = 0u;
    }
  }
  if constexpr (DETECTOR == CPHOT_DETECTOR_SPHERES) {
    // leading time bins of every sphere, after the sphere counts
    const int nt = n * p.hist_tw;
    uint32_t* s_t = s_hist + n;
    for (int b = threadIdx.x; b < nt; b += BS) {
      const uint32_t v = s_t[b];
      if (v) {
        const int sph = b / p.hist_tw, tb = b - sph * p.hist_tw;
        atomicAdd(p.thist + (base + sph) * (p.n_t + 1) + tb, v * (uint32_t)p.bunch);
        s_t[b] = 0u;
      }
    }
  }
}

// Waves per SIMD the register allocation must leave room for. The curved-table
// kernel sits two registers above the three-wave limit without the bound; the
// curved walk runs 15 % faster at four waves with a few spilled registers than
// at three without.
template <int T>
constexpr int kMinWavesPerSimd =
    (T == kTransportCurvedTable || T == CPHOT_TRANSPORT_CURVED) ? 3
    : (T == kTransportCurvedWalk || T == CPHOT_TRANSPORT_LAYERED ||
       T == CPHOT_TRANSPORT_STRAIGHT || T == CPHOT_TRANSPORT_TABLE)
        ? 4
                                                                                                                     : 1;

// EXT: Poisson record counts and the dispersive spectrum (its per-record angle and
// emission decision), compiled only into the kernels that run them: as runtime
// branches their registers cost the default path spills and about a tenth of its
// time.
template <int BS, int TRANSPORT, int DETECTOR, int MODE, bool EXT>
__global__ __launch_bounds__(BS, kMinWavesPerSimd<TRANSPORT>) void k_propagate(KParams p) {
  constexpr bool kTime = (DETECTOR == CPHOT_DETECTOR_SPHERES) || (MODE == MODE_RECORDS);
  constexpr bool kLayers = (TRANSPORT != CPHOT_TRANSPORT_STRAIGHT);
  constexpr bool kMlp = (TRANSPORT == CPHOT_TRANSPORT_SURROGATE || TRANSPORT == kTransportCurvedSurrogate);
  // transports that defer some records to the exact tracer (compaction queue)
  constexpr bool kDefer = kMlp || TRANSPORT == CPHOT_TRANSPORT_TABLE || TRANSPORT == kTransportCurvedTable ||
                          TRANSPORT == CPHOT_TRANSPORT_CURVED;
  constexpr bool kSort = kLayers && (MODE != MODE_COUNTS);
  // ground-grid kernels number a tile's records Cherenkov first, then fluorescence,
  // so that a wave holds one kind of record (one emission branch, one Philox call)
  // except at the single boundary; straight rays cost too little per record for the
  // second scan and its LDS to pay
  constexpr bool kSplit =
      (DETECTOR == CPHOT_DETECTOR_GRID) && (MODE != MODE_COUNTS) && (TRANSPORT != CPHOT_TRANSPORT_STRAIGHT);
  // exact transport behind a surrogate: records outside the network's domain
  constexpr int kExact =
      (TRANSPORT == CPHOT_TRANSPORT_SURROGATE || TRANSPORT == CPHOT_TRANSPORT_TABLE)       ? CPHOT_TRANSPORT_LAYERED
      : (TRANSPORT == kTransportCurvedSurrogate || TRANSPORT == kTransportCurvedTable) ? kTransportCurvedExact
      : (TRANSPORT == CPHOT_TRANSPORT_CURVED)                                               ? kTransportCurvedWalk
                                                                                            : TRANSPORT;
  // per-segment state for the record loop, one slot per segment of the tile:
  // q0 = start point, cos(theta); q1 = end - start, sin(theta) (DISPERSIVE: the
  // terms of beta n(lambda) - 1 in place of the angle); q2 = rotation
  // bisector, depth at the start; q3 = depth change, id low, id high, shower
  // (bit patterns); q4 = core x, core y, axis x, axis y; axz = axis z
  __shared__ float4 s_q0[BS], s_q1[BS], s_q2[BS], s_q3[BS], s_q4[BS];
  __shared__ float s_axz[BS];
  __shared__ uint4 s_q5[BS];  // record boundaries: Cherenkov, + band 0, + band 1
  __shared__ uint32_t s_off[BS + 1];
  __shared__ uint32_t s_offf[kSplit ? BS + 1 : 1];  // fluorescence record offsets
  __shared__ uint32_t s_wave[2 * (BS / 64)];
  __shared__ uint32_t s_src[kSort ? BS : 1];          // tile-local segment index of each slot
  __shared__ uint32_t s_bucket[kSort ? kMaxLayers + 1 : 1];
  __shared__ float4 s_lay[kLayers ? kMaxLayers : 1];
  __shared__ float2 s_lam[kLayers ? kMaxLambdaBins : 1];
  __shared__ uint4 s_imgw[kMlp ? sizeof(MlpImage) / 16 : 1];
  // compaction queues of deferred records (slot, k), one ring of 128 entries per
  // wave: at most 64 enter per round and the wave drains 64 at a time once it
  // holds that many, so a ring never holds more than 127
  __shared__ uint16_t s_qlo[kDefer ? 2 * BS : 1];
  __shared__ uint32_t s_qk[kDefer ? 2 * BS : 1];
  __shared__ uint4 s_mlpx[kMlp ? BS : 1];  // per-wave staging of the network's inputs and outputs
  __shared__ KConst s_k;
  __shared__ float s_eff[kMaxLambdaBins];  // detector efficiency per wavelength bin
  const MlpImage* s_img = reinterpret_cast<const MlpImage*>(s_imgw);
  // Optional LDS window of the grid, or the whole sphere array (record counts of
  // one shower at a time). With it each block walks a contiguous range of tiles,
  // so the window changes shower only a few times per block; records outside the
  // window, or of another shower than the window's, go to the global bins
  // directly. Without it every hit is a device atomic, and hits on one sphere
  // serialise on its cache line.
  extern __shared__ uint32_t s_hist[];
  __shared__ int s_win_sh, s_tile_sh;
  __shared__ uint32_t s_since;  // records since the last flush (keeps LDS counts below 2^32)
  const int n_hist = (MODE == MODE_PROPAGATE && p.lds_hist)
                         ? p.hist_w * p.hist_h * (DETECTOR == CPHOT_DETECTOR_SPHERES ? 1 + p.hist_tw : 1)
                         : 0;
  const int tid = threadIdx.x;

  if constexpr (kLayers) {
    for (int i = tid; i < p.n_layers; i += BS) s_lay[i] = p.layers[i];
    for (int i = tid; i < p.n_lam; i += BS) s_lam[i] = p.lambins[i];
  }
  if constexpr (kMlp) {
    const uint4* src = reinterpret_cast<const uint4*>(p.mlp);
    for (int i = tid; i < (int)(sizeof(MlpImage) / 16); i += BS) s_imgw[i] = src[i];
  }
  load_kconst(p, s_k, tid);
  for (int i = tid; i < kMaxLambdaBins; i += BS) s_eff[i] = (p.eff && i < p.n_lam) ? (float)p.eff[i] : 1.0f;
  for (int i = tid; i < n_hist; i += BS) s_hist[i] = 0u;
  if (tid == 0) {
    s_win_sh = -1;
    s_since = 0u;
  }
  __syncthreads();

  uint32_t c_in = 0, c_skip = 0, c_below = 0, c_gen = 0, c_up = 0, c_abs = 0, c_out = 0, c_bin = 0, c_fb = 0;
  uint32_t c_fl = 0, c_cut1 = 0, c_cut3 = 0;
  const int64_t n_tiles = (p.n + BS - 1) / BS;
  int64_t t_first = blockIdx.x, t_end = n_tiles, t_step = gridDim.x;
  if (n_hist) {
    t_first = (int64_t)blockIdx.x * n_tiles / gridDim.x;
    t_end = ((int64_t)blockIdx.x + 1) * n_tiles / gridDim.x;
    t_step = 1;
  }
  for (int64_t tile = t_first; tile < t_end; tile += t_step) {
    const int64_t i = tile * BS + tid;
    if (n_hist) {
      if (tid == 0) s_tile_sh = shower_of(p, tile * BS);
      __syncthreads();
      // per tile at most BS << 20 records: flushing at 2^31 keeps counts below 2^32
      if (s_tile_sh != s_win_sh || s_since >= (1u << 31)) {
        if (s_win_sh >= 0) flush_window<BS, DETECTOR>(p, s_hist, s_win_sh);
        __syncthreads();
        if (tid == 0) {
          s_win_sh = s_tile_sh;
          s_since = 0u;
        }
        __syncthreads();
      }
    }
    uint32_t nrec = 0;
    float4 q0 = make_float4(0.f, 0.f, 0.f, 0.f), q1 = q0, q2 = q0, q3 = q0, q4 = q0;
    float axz = 0.f;
    uint4 q5 = make_uint4(0u, 0u, 0u, 0u);
    int key = kMaxLayers;  // segments without records sort last
    if (i < p.n) {
      const float fx0 = p.x0[i], fy0 = p.y0[i], fz0 = p.z0[i], fx1 = p.x1[i], fy1 = p.y1[i], fz1 = p.z1[i];
      const uint64_t id = p.first_id + (uint64_t)i * p.id_stride;
      SegResult r =
          segment_setup<EXT>(p, fx0, fy0, fz0, fx1, fy1, fz1, p.beta[i], p.charge[i], p.dedx ? p.dedx[i] : 0.0f, id);
      if constexpr (MODE == MODE_PROPAGATE && DETECTOR == CPHOT_DETECTOR_SPHERES && !kMlpTransport<TRANSPORT>) {
        if ((p.cuts & CPHOT_CUT_TRACK) && r.n > 0) {
          const double* gc = p.geom + 5 * shower_of(p, i);
          if (!track_may_hit(p, fx0, fy0, fz0, fx1, fy1, fz1, r.cos_t, r.sin_t, (float)gc[0], (float)gc[1])) {
            c_cut1 += (uint32_t)r.n;  // filter level 1: no photon of the cone can reach a sphere
            r.n = 0;
          }
        }
      }
      c_in += 1;
      c_skip += r.status == 2;
      c_below += r.status == 1;
      q5 = make_uint4((uint32_t)r.n, (uint32_t)(r.n + r.nf[0]), (uint32_t)(r.n + r.nf[0] + r.nf[1]),
                      __float_as_uint(r.inv_q));
      nrec = q5.z + (uint32_t)r.nf[2];
      c_fl += nrec - (uint32_t)r.n;
      if constexpr (MODE == MODE_COUNTS) {
        p.counts[i] = (int32_t)nrec;
        if (p.expected) p.expected[i] = r.status == 0 ? r.mu : 0.0;
      } else if (nrec) {
        const int sh = shower_of(p, i);
        float X0 = 0.f, dXs = 0.f;
        if (TRANSPORT == CPHOT_TRANSPORT_STRAIGHT && p.profile == CPHOT_PROFILE_LINSLEY5) {
          X0 = depth_f(s_k, fz0);
          dXs = depth_f(s_k, fz1) - X0;
        }
        const double* g = p.geom + 5 * sh;
        const bool disp = EXT && p.spectrum == CPHOT_SPECTRUM_DISPERSIVE;
        q0 = make_float4(fx0, fy0, fz0, disp ? r.disp_a : r.cos_t);
        q1 = make_float4(fx1 - fx0, fy1 - fy0, fz1 - fz0, disp ? r.disp_gm : r.sin_t);
        q2 = make_float4(r.a0, r.a1, r.a2, X0);
        q3 = make_float4(dXs, __uint_as_float((uint32_t)id), __uint_as_float((uint32_t)(id >> 32)),
                         __uint_as_float((uint32_t)sh));
        q4 = make_float4((float)g[0], (float)g[1], (float)g[2], (float)g[3]);
        axz = (float)g[4];
        if constexpr (kSort) key = min(max((int)(0.5f * (fz0 + fz1) * p.inv_dh), 0), p.n_layers - 1);
      }
    }
    if constexpr (MODE == MODE_COUNTS) continue;
    // slot of this segment in the tile: sorted by start layer under layered
    // transport, so that the lanes of a wave cross similar numbers of layers
    int slot = tid;
    if constexpr (kSort) {
      for (int b = tid; b <= kMaxLayers; b += BS) s_bucket[b] = 0u;
      __syncthreads();
      const uint32_t rank = atomicAdd(&s_bucket[key], 1u);
      __syncthreads();
      if (tid < 64) {  // exclusive scan of the bucket sizes by one wave
        uint32_t carry = 0;
        for (int base = 0; base <= kMaxLayers; base += 64) {
          const int b = base + tid;
          const uint32_t v = b <= kMaxLayers ? s_bucket[b] : 0u;
          uint32_t x = v;
#pragma unroll
          for (int d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(x, d, 64);
            if (tid >= d) x += y;
          }
          if (b <= kMaxLayers) s_bucket[b] = carry + x - v;
          carry += __shfl(x, 63, 64);
        }
      }
      __syncthreads();
      slot = (int)(s_bucket[key] + rank);
      s_src[slot] = (uint32_t)tid;
    }
    s_q0[slot] = q0;
    s_q1[slot] = q1;
    s_q2[slot] = q2;
    s_q3[slot] = q3;
    s_q4[slot] = q4;
    s_axz[slot] = axz;
    s_q5[slot] = q5;
    s_off[slot] = kSplit ? q5.x : nrec;
    if constexpr (kSplit) s_offf[slot] = nrec - q5.x;
    __syncthreads();
    uint32_t total, total_c = 0;
    if constexpr (kSplit) {
      uint32_t total_f;
      const uint2 excl = block_exclusive_scan2<BS>(s_off[tid], s_offf[tid], s_wave, total_c, total_f);
      __syncthreads();
      s_off[tid] = excl.x;
      s_offf[tid] = excl.y;
      total = total_c + total_f;
    } else {
      const uint32_t mine = s_off[tid];
      const uint32_t excl = block_exclusive_scan<BS>(mine, s_wave, total);
      __syncthreads();
      s_off[tid] = excl;
    }
    if (tid == BS - 1) s_since += total;
    __syncthreads();
    // with the surrogate every lane of a wave runs each round (the tail lanes
    // repeat the last record and discard it); otherwise lanes stop at `total`
    const uint32_t rounds_end = kDefer ? ((total + BS - 1) / BS) * BS : total;
    // one record: a parity dump, or counters and bins
    auto consume = [&](const Photon& ph, int lo, uint32_t k, const float4& r3) {
      if constexpr (MODE == MODE_RECORDS) {
        const uint32_t src = kSort ? s_src[lo] : (uint32_t)lo;
        const int64_t slot_out = p.rec_off[tile * BS + src] + (int64_t)k;
        if (slot_out < p.rec_cap) {
          cphot_photon_record rr;
          rr.seg = ((uint64_t)__float_as_uint(r3.z) << 32) | __float_as_uint(r3.y);
          rr.k = k;
          rr.state = ph.state;
          rr.bin = ph.bin;
          rr.tbin = ph.tbin;
          rr.x = ph.x; rr.y = ph.y; rr.z = ph.z;
          rr.t = ph.t; rr.tau = ph.tau; rr.lambda = ph.lam;
          rr.dx = ph.ux; rr.dy = ph.uy; rr.dz = ph.uz;
          rr.u_abs = ph.u3;
          p.rec[slot_out] = rr;
        }
      } else {
        c_gen += 1;
        c_fb += ph.fallback;
        c_cut3 += ph.culled;
        c_up += ph.state == 1;
        c_abs += ph.state == 2;
        c_out += ph.state == 3;
        if (ph.state == 0) {
          c_bin += 1;
          const uint32_t sh = __float_as_uint(r3.w);
          if constexpr (DETECTOR == CPHOT_DETECTOR_GRID) {
            const int lx = ph.ix - p.hist_x0, ly = ph.iy - p.hist_y0;
            if (n_hist && (int)sh == s_win_sh && (unsigned)lx < (unsigned)p.hist_w &&
                (unsigned)ly < (unsigned)p.hist_h) {
              atomicAdd(&s_hist[ly * p.hist_w + lx], 1u);
            } else {
              const int64_t gb = (int64_t)sh * p.nx * p.ny + ph.bin;
              if (p.bins_f64) atomicAdd(reinterpret_cast<double*>(p.bins) + gb, (double)(float)p.bunch);
              else if (p.bins_u64) atomicAdd(reinterpret_cast<unsigned long long*>(p.bins) + gb, (unsigned long long)p.bunch);
              else atomicAdd(reinterpret_cast<uint32_t*>(p.bins) + gb, p.bunch);
            }
          } else {
            const int64_t nsph = (int64_t)p.snx * p.sny;
            const int64_t gb = (int64_t)sh * nsph + ph.bin;
            const bool win = n_hist && (int)sh == s_win_sh;
            if (win) {
              atomicAdd(&s_hist[ph.bin], 1u);
            } else {
              if (p.bins_f64) atomicAdd(reinterpret_cast<double*>(p.bins) + gb, (double)(float)p.bunch);
              else if (p.bins_u64) atomicAdd(reinterpret_cast<unsigned long long*>(p.bins) + gb, (unsigned long long)p.bunch);
              else atomicAdd(reinterpret_cast<uint32_t*>(p.bins) + gb, p.bunch);
            }
            if (p.n_t > 0) {
              if (win && ph.tbin < p.hist_tw) atomicAdd(&s_hist[nsph + ph.bin * p.hist_tw + ph.tbin], 1u);
              else atomicAdd(p.thist + gb * (p.n_t + 1) + ph.tbin, p.bunch);
            }
          }
        }
      }
    };
    uint32_t q_head = 0, q_len = 0;  // this wave's ring of deferred records (same in every lane)
    for (uint32_t base = 0; base + tid < rounds_end; base += BS) {
      const uint32_t jr = base + tid;
      const bool valid = jr < total;
      const uint32_t j = valid ? jr : total - 1;
      // largest slot lo in [0, BS) with offset <= j (offsets never decrease); with
      // the split numbering, records from total_c on are the fluorescence records
      const bool fl = kSplit && j >= total_c;
      const uint32_t* offs = fl ? s_offf : s_off;
      const uint32_t jj = fl ? j - total_c : j;
      int lo = 0;
#pragma unroll
      for (int step = BS / 2; step >= 1; step >>= 1) lo += (offs[lo + step] <= jj) ? step : 0;
      const uint32_t k = jj - offs[lo] + (fl ? s_q5[lo].x : 0u);
      Photon ph;
      const float4 r3 = s_q3[lo];
      trace<TRANSPORT, DETECTOR, kTime, EXT>(p, s_lay, s_lam, s_img, &s_k, s_eff, s_mlpx + (kMlp ? (tid & ~63) : 0), s_q0[lo],
                                        s_q1[lo], s_q2[lo], r3, s_q4[lo], s_axz[lo], s_q5[lo], k, valid, ph);
      if constexpr (kDefer) {
        // wave-level compaction: deferred records take consecutive entries of this
        // wave's ring (ballot and prefix count of the lanes below); the wave traces
        // them exactly, 64 at a time, with no block barrier
        const bool push = valid && ph.state == kStateDeferred;
        const uint64_t mask = __ballot(push);
        const uint32_t lane = (uint32_t)(tid & 63);
        uint16_t* q_lo = s_qlo + 2 * (tid & ~63);
        uint32_t* q_k = s_qk + 2 * (tid & ~63);
        if (push) {
          const uint32_t pos = (q_head + q_len + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull))) & 127u;
          q_lo[pos] = (uint16_t)lo;
          q_k[pos] = k;
        }
        q_len += (uint32_t)__popcll(mask);
        if (valid && !push) consume(ph, lo, k, r3);
        const bool last = base + BS >= rounds_end;
        while (q_len >= 64u || (last && q_len > 0u)) {
          // the ring's entries written by other lanes of this wave are complete
          // (the fences order the LDS accesses; no other wave touches this ring)
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
          const uint32_t take = min(q_len, 64u);
          if (lane < take) {
            const uint32_t e = (q_head + lane) & 127u;
            const int qlo = q_lo[e];
            const uint32_t qk = q_k[e];
            const float4 q3 = s_q3[qlo];
            Photon pe;
            trace<kExact, DETECTOR, kTime, EXT>(p, s_lay, s_lam, s_img, &s_k, s_eff, s_mlpx, s_q0[qlo], s_q1[qlo], s_q2[qlo], q3,
                                           s_q4[qlo], s_axz[qlo], s_q5[qlo], qk, true, pe);
            pe.fallback = 1;
            consume(pe, qlo, qk, q3);
          }
          // every lane has read its entry before the ring takes new ones
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
          q_head = (q_head + take) & 127u;
          q_len -= take;
        }
      } else {
        if (valid) consume(ph, lo, k, r3);
      }
    }
    __syncthreads();
  }
  if constexpr (MODE == MODE_PROPAGATE) {
    if (n_hist) {
      __syncthreads();
      if (s_win_sh >= 0) flush_window<BS, DETECTOR>(p, s_hist, s_win_sh);
    }
    if (p.counters) {
      // block-level reduction: one global atomic per counter per block (same-address
      // device atomics serialise, so their number must stay small)
      __shared__ uint32_t s_cnt[13];
      if (tid < 13) s_cnt[tid] = 0u;
      __syncthreads();
      // every consumed record has exactly one final state; the records not emitted
      // (state 4) are the rest, so they need no accumulator of their own
      const uint32_t c_ne = c_gen - c_up - c_abs - c_out - c_bin;  // modulo 2^32: exact over the block
      const uint32_t v[13] = {c_in,  c_skip, c_below, c_gen, c_up,   c_abs, c_out,
                              c_bin, c_fb,   c_fl,    c_cut1, c_cut3, c_ne};
#pragma unroll
      for (int q = 0; q < 13; ++q) {
        const uint32_t sw = wave_sum(v[q]);
        if ((tid & 63) == 0 && sw) atomicAdd(&s_cnt[q], sw);
      }
      __syncthreads();
      if (tid < 8 && s_cnt[tid]) atomicAdd(p.counters + tid, (unsigned long long)s_cnt[tid]);
      if (tid == 8 && s_cnt[7]) atomicAdd(p.counters + CPHOT_C_PHOTONS_BINNED, (unsigned long long)s_cnt[7] * p.bunch);
      if (tid == 9 && s_cnt[8]) atomicAdd(p.counters + CPHOT_C_SURROGATE_FALLBACK, (unsigned long long)s_cnt[8]);
      if (tid == 10 && s_cnt[9]) atomicAdd(p.counters + CPHOT_C_RECORDS_FLUORESCENCE, (unsigned long long)s_cnt[9]);
      if (tid == 11 && s_cnt[10]) atomicAdd(p.counters + CPHOT_C_RECORDS_CULLED_TRACK, (unsigned long long)s_cnt[10]);
      if (tid == 12 && s_cnt[11]) atomicAdd(p.counters + CPHOT_C_RECORDS_CULLED_PHOTON, (unsigned long long)s_cnt[11]);
      if (tid == 13 && s_cnt[12]) atomicAdd(p.counters + CPHOT_C_RECORDS_NOT_EMITTED, (unsigned long long)s_cnt[12]);
    }
  }
}

namespace {

template <int BS, int T, int D, int M, bool EXT>
hipError_t launch_one(const KParams& p, int grid, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL((k_propagate<BS, T, D, M, EXT>), dim3(grid), dim3(BS), lds, s, p);
  return hipGetLastError();
}

template <int BS, int T, int D, int M>
hipError_t launch_ext(const KParams& p, int grid, size_t lds, hipStream_t s) {
  const bool ext = p.poisson || p.spectrum == CPHOT_SPECTRUM_DISPERSIVE;
  return ext ? launch_one<BS, T, D, M, true>(p, grid, lds, s) : launch_one<BS, T, D, M, false>(p, grid, lds, s);
}

template <int BS, int T, int D>
hipError_t launch_mode(const KParams& p, int mode, int grid, size_t lds, hipStream_t s) {
  switch (mode) {
    case MODE_PROPAGATE: return launch_ext<BS, T, D, MODE_PROPAGATE>(p, grid, lds, s);
    case MODE_COUNTS: return launch_ext<BS, T, D, MODE_COUNTS>(p, grid, lds, s);
    default: return launch_ext<BS, T, D, MODE_RECORDS>(p, grid, lds, s);
  }
}

template <int BS>
hipError_t launch_bs(const KParams& p, int mode, int grid, size_t lds, hipStream_t s) {
  const bool g = p.detector == CPHOT_DETECTOR_GRID;
  switch (p.transport) {
    case CPHOT_TRANSPORT_STRAIGHT: return g ? launch_mode<BS, 0, 0>(p, mode, grid, lds, s) : launch_mode<BS, 0, 1>(p, mode, grid, lds, s);
    case CPHOT_TRANSPORT_LAYERED: return g ? launch_mode<BS, 1, 0>(p, mode, grid, lds, s) : launch_mode<BS, 1, 1>(p, mode, grid, lds, s);
    case CPHOT_TRANSPORT_SURROGATE: return g ? launch_mode<BS, 2, 0>(p, mode, grid, lds, s) : launch_mode<BS, 2, 1>(p, mode, grid, lds, s);
    case CPHOT_TRANSPORT_CURVED: return launch_mode<BS, 3, 0>(p, mode, grid, lds, s);  // grid detector only
    case kTransportCurvedWalk: return launch_mode<BS, kTransportCurvedWalk, 0>(p, mode, grid, lds, s);
    case CPHOT_TRANSPORT_TABLE: return g ? launch_mode<BS, 4, 0>(p, mode, grid, lds, s) : launch_mode<BS, 4, 1>(p, mode, grid, lds, s);
    case kTransportCurvedTable: return launch_mode<BS, kTransportCurvedTable, 0>(p, mode, grid, lds, s);
    default: return launch_mode<BS, kTransportCurvedSurrogate, 0>(p, mode, grid, lds, s);
  }
}

template <int BS, int T, int D, int M>
size_t static_lds_one() {
  hipFuncAttributes a;
  // the EXT kernels declare the same static LDS
  if (hipFuncGetAttributes(&a, reinterpret_cast<const void*>(&k_propagate<BS, T, D, M, false>)) != hipSuccess) return 0;
  return a.sharedSizeBytes;
}

template <int BS, int T, int D>
size_t static_lds_mode(int mode) {
  switch (mode) {
    case MODE_PROPAGATE: return static_lds_one<BS, T, D, MODE_PROPAGATE>();
    case MODE_COUNTS: return static_lds_one<BS, T, D, MODE_COUNTS>();
    default: return static_lds_one<BS, T, D, MODE_RECORDS>();
  }
}

template <int BS>
size_t static_lds_bs(const KParams& p, int mode) {
  const bool g = p.detector == CPHOT_DETECTOR_GRID;
  switch (p.transport) {
    case CPHOT_TRANSPORT_STRAIGHT: return g ? static_lds_mode<BS, 0, 0>(mode) : static_lds_mode<BS, 0, 1>(mode);
    case CPHOT_TRANSPORT_LAYERED: return g ? static_lds_mode<BS, 1, 0>(mode) : static_lds_mode<BS, 1, 1>(mode);
    case CPHOT_TRANSPORT_SURROGATE: return g ? static_lds_mode<BS, 2, 0>(mode) : static_lds_mode<BS, 2, 1>(mode);
    case CPHOT_TRANSPORT_CURVED: return static_lds_mode<BS, 3, 0>(mode);
    case kTransportCurvedWalk: return static_lds_mode<BS, kTransportCurvedWalk, 0>(mode);
    case CPHOT_TRANSPORT_TABLE: return g ? static_lds_mode<BS, 4, 0>(mode) : static_lds_mode<BS, 4, 1>(mode);
    case kTransportCurvedTable: return static_lds_mode<BS, kTransportCurvedTable, 0>(mode);
    default: return static_lds_mode<BS, kTransportCurvedSurrogate, 0>(mode);
  }
}

}  // namespace

size_t propagate_static_lds(const KParams& p, int mode, int block_size) {
  switch (block_size) {
    case 128: return static_lds_bs<128>(p, mode);
    case 512: return static_lds_bs<512>(p, mode);
    default: return static_lds_bs<256>(p, mode);
  }
}

hipError_t launch_propagate(const KParams& p, int mode, int block_size, int grid_blocks, size_t lds_bytes,
                            hipStream_t stream) {
  switch (block_size) {
    case 128: return launch_bs<128>(p, mode, grid_blocks, lds_bytes, stream);
    case 512: return launch_bs<512>(p, mode, grid_blocks, lds_bytes, stream);
    default: return launch_bs<256>(p, mode, grid_blocks, lds_bytes, stream);
  }
}

}  // namespace cphot
