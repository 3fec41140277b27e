// Correction table of the interpolation tracing (Sec. 4.4.1): device view and
// the bilinear lookup used inside the propagation kernel.
#pragma once

#include <hip/hip_runtime.h>

namespace cphot {

// The exact layered result jumps where the emission height crosses a layer
// boundary (the start layer fixes Snell's invariant n0 sin(theta0) of a given
// direction), so heights are tabulated layer by layer and never interpolated
// across a boundary: layer layer0 + r (r < n_rows) holds m nodes from its bottom
// (h_obs for the observation layer) to its top, which counts as inside it.
// Direction nodes are uniform in tan of the zenith angle, j / inv_dt (j < n_c):
// the corrections are smooth polynomials of tan(theta) (about tan (1 + tan^2)),
// where in cos they have a square-root cusp at the vertical. Node (r, k, j) at
// data[j * n_rows * m + r * m + k] = (offset along the azimuth, optical path
// excess, Rayleigh path integral, aerosol path integral), absolute (m).
struct TableView {
  const float4* data;
  int m, n_rows, layer0, n_c;
  float dh, inv_dh, h_obs;
  float inv_dt;
  int geometry;  // CPHOT_SURROGATE_PLANAR | CPHOT_SURROGATE_CURVED
  int pad;
};

// Bilinear interpolation at (h, tan zenith) for a photon starting in layer `li`
// (the exact walk's start layer); false outside the tabulated range.
__device__ __forceinline__ bool table_lookup(const TableView& t, int li, float h, float tz, float4& v) {
  const int r = li - t.layer0;
  const float fc = tz * t.inv_dt;
  if (!(r >= 0 && r < t.n_rows && fc >= 0.f && fc <= (float)(t.n_c - 1) + 1e-3f)) return false;
  const float lower = r == 0 ? t.h_obs : (float)li * t.dh;
  const float span = (float)(li + 1) * t.dh - lower;
  const float fh = fminf(fmaxf((h - lower) / span, 0.f), 1.f) * (float)(t.m - 1);
  const int k = min((int)fh, t.m - 2), j = min((int)fc, t.n_c - 2);
  const float wh = fh - (float)k, wc = fminf(fc - (float)j, 1.f);
  const float4* r0 = t.data + ((size_t)j * t.n_rows + r) * t.m + k;
  const float4* r1 = r0 + (size_t)t.n_rows * t.m;
  const float4 a = r0[0], b = r0[1], cc = r1[0], d = r1[1];
  auto lerp = [](float x, float y, float w) { return fmaf(w, y - x, x); };
  const float4 lo = make_float4(lerp(a.x, b.x, wh), lerp(a.y, b.y, wh), lerp(a.z, b.z, wh), lerp(a.w, b.w, wh));
  const float4 hi = make_float4(lerp(cc.x, d.x, wh), lerp(cc.y, d.y, wh), lerp(cc.z, d.z, wh), lerp(cc.w, d.w, wh));
  v = make_float4(lerp(lo.x, hi.x, wc), lerp(lo.y, hi.y, wc), lerp(lo.z, hi.z, wc), lerp(lo.w, hi.w, wc));
  return true;
}

}  // namespace cphot
