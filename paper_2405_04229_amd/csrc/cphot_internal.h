// Internal declarations shared by the host API and the kernels of libcphot.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/cphot.h"
#include "cphot_table.h"

namespace cphot {

struct MlpImage;

constexpr int kMaxLayers = 128;
constexpr int kMaxLambdaBins = 64;

// Closed-form shell sums (curved Earth, curved_series in cphot_device.h): 15 (k, m)
// pairs of the double series, one row of shell moments per (observation shell,
// start shell), one 16-float group per weight (16-byte aligned), entry q of a group
// for pair q (q = 0..4: k 0, m 1..5; 5..9: k 1, m 1..5; 10..12: k 2, m 1..3; 13, 14:
// k 3, m 1..2; entry 15 zero): [0, 16) Rayleigh, [16, 32) aerosol, [32, 48)
// R^2 e / (b b'), [48, 64) R^2 / (b b') (k >= 1: entries 0..4 zero), [64, 80) path
// (k >= 1), [80, 96) n - 1.
constexpr int kShellTerms = 15;
constexpr int kShellRow = 96;
constexpr double kShellRhoMax = 0.1;  // largest D_obs / G_j the series serves

// Device-side tables owned by an atmosphere handle.
struct AtmoDevice {
  double* delta_table = nullptr;   // n_tab + 1 entries, FP64 (per-segment yield)
  // per layer: (n - 1, 1/n, Rayleigh depth per metre in g/cm^2/m, aerosol column per metre);
  // the extinction of layer i at wavelength bin k is lay.z * lam[k].x + lay.w * lam[k].y
  float4* layers = nullptr;        // n_layers
  float2* lambins = nullptr;       // n_lam: (1 / Rayleigh length in g/cm^2, aerosol vertical depth)
  // closed-form layer sums: [obs][j][5] float4 moments of the full layers
  // between observation layer obs and start layer j (planar transport)
  float4* moments = nullptr;
  float series_tmax = 0.f;         // largest tan^2(zenith) the series may serve
  // closed-form shell sums (curved Earth): [obs][j][kShellRow] floats of shell moments
  float* shells = nullptr;
  float shell_tmax = 0.f;          // largest t = tan^2 of the straight zenith at b_j the series may serve
};

// Everything a launch needs, passed by value as the kernel argument.
struct KParams {
  // segments
  const float *x0, *y0, *z0, *x1, *y1, *z1, *beta, *charge;
  int64_t n;
  uint64_t first_id;
  uint64_t id_stride;  // global id of segment i: first_id + i * id_stride
  int32_t n_showers;
  const int64_t* offsets;
  const double* geom;
  // refractivity table (FP64) and Frank-Tamm constant
  const double* tab;
  int64_t n_tab;
  double step;
  double K;
  uint32_t bunch;
  uint32_t key0, key1;
  // atmosphere profile for the straight closed forms (FP32)
  int32_t profile;
  float hb[5], la[5], lb[5], linv_c[5];   // Linsley bounds (m), a, b, 1/c (1/cm)
  float opt_scale;                        // LINSLEY5: kappa/rho0/100 (m per g/cm^2); others: delta0
  float h_top;
  int32_t has_ray, has_aer;
  float inv_ray400, aer_tau350, aer_inv_h, aer_ang;
  float lam_min, lam_max, inv_lam_min, inv_lam_max;
  int32_t spectrum;
  // DISPERSIVE (R: the standard-air dispersion sum): R(lam_min) / R(lambda_ref) and
  // 1 / R(lambda_ref) in FP64 (segment setup); s_min^2 = (1000 / lam_min)^2,
  // k1 / (k0 - s_min^2) and k3 / (k2 - s_min^2) in FP32 (per-record angle)
  double disp_dmax, disp_inv_rref;
  float disp_s2m, disp_k1c, disp_k3c;
  // observation level quantities (FP32)
  float h_obs, X_obs, I_obs, A_obs;
  // transport / detector
  int32_t transport, detector;
  int32_t n_layers, n_lam;
  float dh, inv_dh;
  int32_t obs_layer;
  const float4* layers;
  const float4* moments;  // rows of the observation layer's slice, by start layer
  float series_tmax;      // 0: crossing loop only
  const float* shells;    // curved: shell-moment rows of the observation shell's slice, by start shell
  float shell_tmax, shell_rho;  // curved series domain (0: shell walk only)
  int32_t shell_nb_rising;      // n_i b_i increases with i over the shells: a closed-form arrival test holds
  int32_t cuts;           // CPHOT_CUT_* (SPHERES, propagate mode)
  const double* eff;      // detector efficiency per wavelength bin (NULL: 1)
  const double* red;      // pre-emission reduction bound per layer (NULL: none)
  double dh64;            // layer thickness in FP64 (the reduction's layer of a segment)
  int32_t poisson;        // record counts ~ Poisson(mu) instead of stochastic rounding
  float cut_e;            // largest |n_i - n_j| / n_i above the observation layer (0 for straight rays)
  const float2* lambins;
  int32_t nx, ny;
  float cell, inv_cell;
  double inv_cell64;      // 1 / cell in FP64 (curved arrival points)
  int32_t snx, sny;
  float pitch, inv_pitch, radius;
  int32_t n_t;
  float inv_dt;
  // surrogate transport
  const MlpImage* mlp;
  // table transport
  TableView ctab;  // correction table (interpolation tracing)
  // emission
  const float* dedx;
  int32_t emission;
  double fl_yield[3];
  float fl_lambda[3];
  // curved Earth
  double earth_radius;
  int32_t bins_f64;
  // outputs
  void* bins;
  int32_t bins_u64;
  int32_t lds_hist;                    // grid counts privatised in an LDS window
  int32_t hist_w, hist_h;              // window size in cells (x, y)
  int32_t hist_x0, hist_y0;            // window origin in cells
  int32_t hist_tw;                     // spheres: leading time bins of each sphere held in LDS too
  uint32_t* thist;
  unsigned long long* counters;
  // debug outputs
  int32_t* counts;
  double* expected;
  const int64_t* rec_off;
  cphot_photon_record* rec;
  int64_t rec_cap;
};

enum Mode { MODE_PROPAGATE = 0, MODE_COUNTS = 1, MODE_RECORDS = 2 };

// Text returned by cphot_last_error() on this thread.
void set_last_error(const std::string& msg);
// Device layer tables of an atmosphere (CPHOT_ERR_INVALID_ARG if it has no layers).
int atmosphere_layer_view(const cphot_atmosphere* atm, const float4** layers, const float2** lambins, int* n_layers,
                          int* n_lam, float* dh, float* lam_min, float* lam_max);
// Inference image of a surrogate and whether its normalisation is set.
const MlpImage* surrogate_image(const cphot_surrogate* s);
double atmosphere_earth_radius(const cphot_atmosphere* a);
// Closed-form layer-sum moments [obs][j][5] (null without layers): the m = 0 entries
// r[2].x, r[2].w, r[3].z hold dh sum (n_i - 1), dh sum of the Rayleigh and aerosol
// parts over the full layers between observation layer obs and layer j.
const float4* atmosphere_layer_moments(const cphot_atmosphere* a);
int surrogate_geometry(const cphot_surrogate* s);
bool surrogate_ready(const cphot_surrogate* s);
// internal transport ids: SURROGATE / TABLE transport over curved shells
constexpr int kTransportCurvedSurrogate = 16;
constexpr int kTransportCurvedTable = 17;
// the shell walk for every photon (CPHOT_TRANSPORT_CURVED_WALK)
constexpr int kTransportCurvedWalk = CPHOT_TRANSPORT_CURVED_WALK;
// the closed-form shell sums, the shell walk in place for rays outside their
// domain: the exact tracer behind the curved surrogate and table (their deferred
// records are already compacted, so nothing is deferred a second time)
constexpr int kTransportCurvedExact = 18;
// Correction table: device view, the atmosphere it was built from, its h_obs.
TableView table_view(const cphot_table* t);
const cphot_atmosphere* table_atmosphere(const cphot_table* t);
double table_h_obs(const cphot_table* t);

hipError_t launch_propagate(const KParams& p, int mode, int block_size, int grid_blocks, size_t lds_hist_bytes,
                            hipStream_t stream);
// Static LDS bytes of the propagate kernel that `p`, `mode` and `block_size` select.
// Static LDS bytes of the propagation kernel instance a launch would use (0 if
// it cannot be queried).
size_t propagate_static_lds(const KParams& p, int mode, int block_size);

}  // namespace cphot
