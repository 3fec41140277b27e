// Exact walks of one photon in FP64, for tabulated corrections and training
// targets (not the propagation hot path, which walks in FP32). Both follow the
// same laws as the FP32 walks of cphot_device.h, carried in double so that the
// stored corrections are limited by the physics rather than by rounding.
// Layer data: lay[i] = (n - 1, 1/n, Rayleigh part, aerosol part) as float4;
// the optical depth is returned split into its Rayleigh and aerosol path
// integrals, sum R_i l_i and sum A_i l_i, so that tau = sp.x tR + sp.y tA for a
// wavelength with spectral factors sp.
#pragma once

#include <hip/hip_runtime.h>

namespace cphot {

struct Walk64 {
  double across;  // planar: horizontal travel along the azimuth; curved: central angle swept
  double len;     // geometric path length
  double opt;     // sum (n - 1) l
  double tR, tA;  // Rayleigh and aerosol path integrals
};

// Planar layers (Sec. 3.4.2): from height h0 with cos of the zenith angle c0
// (downward) to the observation level h_obs. Snell's law conserves the
// horizontal part of n u: in layer i the sine is s0 (1 - e_i), e_i =
// (d_i - d_0) / (1 + d_i), and the squared cosine c0^2 + s0^2 e_i (2 - e_i).
// The start layer is `i0` (its top boundary counts as inside it), or the layer
// containing h0 when i0 < 0.
__device__ inline void planar_walk_f64(const float4* __restrict__ lay, double dh, int n_layers, double h_obs,
                                       double h0, double c0, Walk64& w, int i0 = -1) {
  const double s0 = sqrt((1.0 - c0) * (1.0 + c0));
  int i = i0 >= 0 ? i0 : min((int)(h0 / dh), n_layers - 1);
  const int obs = (int)floor(h_obs / dh);
  const double d0 = (double)lay[i].x;
  w.across = w.len = w.opt = w.tR = w.tA = 0.0;
  double z = h0;
  for (;;) {
    const float4 L = lay[i];
    const double di = (double)L.x;
    const double e = (di - d0) / (1.0 + di);
    const double s = s0 * (1.0 - e);
    const double c = sqrt(c0 * c0 + s0 * s0 * e * (2.0 - e));
    const double zb = (i > obs) ? i * dh : h_obs;
    const double path = (z - zb) / c;
    w.across += path * s;
    w.len += path;
    w.opt += di * path;
    w.tR += (double)L.z * path;
    w.tA += (double)L.w * path;
    if (i <= obs) break;
    z = zb;
    --i;
  }
}

// Spherical shells of a curved Earth (Sec. 3.3.4): the impact-parameter deficit
// D = (R + h) - p = (h - h0) + (R + h0) [(1 - s0) - s0 (d0 - d_i) / (1 + d_i)]
// is carried without radius-sized subtractions; a chord from ha down to hb is
// (ha - hb)(2R + ha + hb) / (ra ca + rb cb) and sweeps asin(p l / (ra rb)); a ray
// turns round inside a shell where D would become negative and is totally
// reflected where the next shell's D is not positive. Start at height h0 with
// local zenith cosine c0 (downward), in shell i0 (or the shell containing h0 when
// i0 < 0). Returns false if the ray does not reach the sphere R + h_obs.
__device__ inline bool shell_walk_f64(const float4* __restrict__ lay, double dh, int n_layers, double h_obs,
                                      double Re, double h0, double c0, Walk64& w, int i0 = -1) {
  const double s0 = sqrt((1.0 - c0) * (1.0 + c0));
  int i = i0 >= 0 ? i0 : min((int)(h0 / dh), n_layers - 1);
  const int obs = (int)floor(h_obs / dh);
  const double A = Re + h0;
  const double c1 = c0 * c0 / (1.0 + s0);
  const double d0 = (double)lay[i].x;
  auto bracket = [&](int k) {
    const double dk = (double)lay[k].x;
    return c1 - s0 * (d0 - dk) / (1.0 + dk);
  };
  double h = h0;
  w.across = w.len = w.opt = w.tR = w.tA = 0.0;
  bool down = c0 > 0.0;
  for (int iter = 0; iter < 8 * n_layers; ++iter) {
    const double br = bracket(i);
    const double ra = Re + h;
    const double Da = A * br + (h - h0);
    const double rca = sqrt(fmax(Da * (2.0 * ra - Da), 0.0));
    const double pa = ra - Da;
    double ell, dpsi;
    bool to_top = false;
    if (down) {
      const double hb = (i == obs) ? h_obs : i * dh;
      const double Db = A * br + (hb - h0);
      if (Db > 0.0) {
        const double rb = Re + hb;
        const double rcb = sqrt(Db * (2.0 * rb - Db));
        ell = (h - hb) * (2.0 * Re + h + hb) / (rca + rcb);
        dpsi = asin(pa * ell / (ra * rb));
        h = hb;
      } else {
        const double ho = (i + 1) * dh;
        const double ro = Re + ho;
        const double Do = A * br + (ho - h0);
        const double rco = sqrt(fmax(Do * (2.0 * ro - Do), 0.0));
        ell = rca + rco;
        dpsi = atan2(rca, pa) + atan2(rco, pa);
        h = ho;
        down = false;
        to_top = true;
      }
    } else {
      const double ho = (i + 1) * dh;
      const double ro = Re + ho;
      const double Do = A * br + (ho - h0);
      const double rco = sqrt(fmax(Do * (2.0 * ro - Do), 0.0));
      ell = (ho - h) * (2.0 * Re + ho + h) / (rco + rca);
      dpsi = asin(pa * ell / (ra * ro));
      h = ho;
      to_top = true;
    }
    const float4 L = lay[i];
    w.len += ell;
    w.opt += (double)L.x * ell;
    w.tR += (double)L.z * ell;
    w.tA += (double)L.w * ell;
    w.across += dpsi;
    if (!to_top) {
      if (i == obs) return true;
      if (!(A * bracket(i - 1) + (h - h0) > 0.0)) {
        down = false;
        continue;
      }
      --i;
      continue;
    }
    if (i + 1 >= n_layers) return false;
    if (!(A * bracket(i + 1) + (h - h0) > 0.0)) {
      down = true;
      continue;
    }
    ++i;
  }
  return false;
}

// Straight chord from height h0 at local zenith cosine c0 to the sphere R + h_obs,
// cancellation-free root, and the central angle it sweeps.
__device__ inline void chord_f64(double Re, double h_obs, double h0, double c0, double& len, double& psi) {
  const double r0 = Re + h0, r1 = Re + h_obs, s0 = sqrt((1.0 - c0) * (1.0 + c0));
  const double drs = (h0 - h_obs) * (r0 + r1);
  len = drs / (r0 * c0 + sqrt(r0 * r0 * c0 * c0 - drs));
  psi = asin(len * s0 / r1);
}

}  // namespace cphot
