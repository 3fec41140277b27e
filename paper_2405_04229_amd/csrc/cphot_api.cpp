// Host side of libcphot: argument checks, atmosphere tables, launch set-up.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <array>
#include <vector>

#include "cphot_internal.h"

struct cphot_atmosphere {
  cphot_atmosphere_desc d;
  int device = 0;
  double rho0 = 1.0;
  int64_t n_tab = 0;
  cphot::AtmoDevice dev;
  std::vector<double> layer_delta;  // host copies (FP64) for checks
  std::vector<double> cut_e;        // per observation layer: largest |n_i - n_j| / n_i of the layers above
  bool delta_monotone = false;      // layer n - 1 non-increasing with height (curved grid cut)
  bool nb_rising = false;           // n_i b_i (index times lower radius) increasing with i (curved arrival test)
};

namespace {
thread_local std::string g_err;
}  // namespace

namespace cphot {
void set_last_error(const std::string& msg) { g_err = msg; }
}  // namespace cphot

namespace {

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return CPHOT_ERR_HIP;
}

constexpr double kPi = 3.14159265358979323846;
constexpr double kAlpha = 1.0 / 137.035999084;  // fine-structure constant, CODATA 2018

// ---- atmosphere closed forms (FP64, host) -------------------------------------------

int linsley_layer(const cphot_atmosphere_desc& d, double h) {
  int i = 0;
  while (i < 4 && h >= d.lin_hb[i + 1]) ++i;
  return i;
}

double depth(const cphot_atmosphere_desc& d, double h) {
  const int i = linsley_layer(d, h);
  const double hcm = h * 100.0;
  if (i < 4) return d.lin_a[i] + d.lin_b[i] * std::exp(-hcm / d.lin_c[i]);
  return d.lin_a[4] - d.lin_b[4] * hcm / d.lin_c[4];
}

// Dispersion sum of standard air, 1e8 (n - 1), at lambda nm (two-term formula of
// Ciddor, Appl. Opt. 35 (1996) 1566; wavenumber in 1/um).
constexpr double kDispK0 = 238.0185, kDispK1 = 5792105.0, kDispK2 = 57.362, kDispK3 = 167917.0;
double air_dispersion(double lambda_nm) {
  const double s = 1000.0 / lambda_nm, s2 = s * s;
  return kDispK1 / (kDispK0 - s2) + kDispK3 / (kDispK2 - s2);
}

double density(const cphot_atmosphere_desc& d, double h) {
  const int i = linsley_layer(d, h);
  if (i < 4) return (d.lin_b[i] / d.lin_c[i]) * std::exp(-(h * 100.0) / d.lin_c[i]);
  return d.lin_b[4] / d.lin_c[4];
}

// n - 1 of the profile. The expression order is fixed: the FP64 table built
// from it decides integer photon counts.
double refractivity(const cphot_atmosphere& a, double h) {
  const cphot_atmosphere_desc& d = a.d;
  if (d.profile == CPHOT_PROFILE_HOMOGENEOUS) return d.delta0;
  if (d.profile == CPHOT_PROFILE_LINEAR) {
    if (h >= d.h_top) return 0.0;
    if (h < 0.0) h = 0.0;
    return d.delta0 * (1.0 - h / d.h_top);
  }
  return d.kappa * (density(d, h) / a.rho0);
}

std::mutex g_dev_mu;
int g_cu_count[64] = {0};

int cu_count(int dev) {
  std::lock_guard<std::mutex> lk(g_dev_mu);
  if (dev < 0 || dev >= 64) return 256;
  if (!g_cu_count[dev]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
    g_cu_count[dev] = v;
  }
  return g_cu_count[dev];
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// ---- launch parameters ----------------------------------------------------------------

int fill_params(const cphot_segments* seg, const cphot_detector* det, cphot::KParams& p, bool need_bins,
                const cphot_bins* out) {
  if (!seg || !det) return fail(CPHOT_ERR_INVALID_ARG, "null segments or detector");
  const cphot_atmosphere* a = det->atm;
  if (!a) return fail(CPHOT_ERR_INVALID_ARG, "detector has no atmosphere");
  const cphot_atmosphere_desc& d = a->d;
  if (seg->n < 0) return fail(CPHOT_ERR_INVALID_ARG, "negative segment count");
  if (seg->first_id < 0) return fail(CPHOT_ERR_INVALID_ARG, "negative first_id");
  if (seg->id_stride < 0) return fail(CPHOT_ERR_INVALID_ARG, "negative id_stride");
  if (seg->n > 0 && (!seg->x0 || !seg->y0 || !seg->z0 || !seg->x1 || !seg->y1 || !seg->z1 || !seg->beta ||
                     !seg->charge))
    return fail(CPHOT_ERR_INVALID_ARG, "null segment array");
  if (seg->n_showers < 1) return fail(CPHOT_ERR_INVALID_ARG, "n_showers must be >= 1");
  if (seg->n_showers > 1 && !seg->shower_offsets)
    return fail(CPHOT_ERR_INVALID_ARG, "shower_offsets required for several showers");
  if (!seg->shower_geom) return fail(CPHOT_ERR_INVALID_ARG, "shower_geom is required");
  if (det->transport != CPHOT_TRANSPORT_STRAIGHT && det->transport != CPHOT_TRANSPORT_LAYERED &&
      det->transport != CPHOT_TRANSPORT_SURROGATE && det->transport != CPHOT_TRANSPORT_CURVED &&
      det->transport != CPHOT_TRANSPORT_TABLE && det->transport != CPHOT_TRANSPORT_CURVED_WALK)
    return fail(CPHOT_ERR_INVALID_ARG, "unknown transport");
  if (det->transport == CPHOT_TRANSPORT_TABLE) {
    if (!det->table) return fail(CPHOT_ERR_INVALID_ARG, "table transport needs a correction table");
    if (cphot::table_atmosphere(det->table) != a)
      return fail(CPHOT_ERR_INVALID_ARG, "the correction table was built for another atmosphere");
    if (std::fabs(cphot::table_h_obs(det->table) - det->h_obs) > 1e-6)
      return fail(CPHOT_ERR_INVALID_ARG, "the correction table was built for another h_obs");
  }
  if (det->transport == CPHOT_TRANSPORT_SURROGATE && !cphot::surrogate_ready(det->surrogate))
    return fail(CPHOT_ERR_UNSUPPORTED, "surrogate transport needs a surrogate with its normalisation set");
  const bool curved_sur = det->transport == CPHOT_TRANSPORT_SURROGATE &&
                          cphot::surrogate_geometry(det->surrogate) == CPHOT_SURROGATE_CURVED;
  const bool curved_tab = det->transport == CPHOT_TRANSPORT_TABLE &&
                          cphot::table_view(det->table).geometry == CPHOT_SURROGATE_CURVED;
  const bool curved = det->transport == CPHOT_TRANSPORT_CURVED || det->transport == CPHOT_TRANSPORT_CURVED_WALK ||
                      curved_sur || curved_tab;
  if (curved && det->detector != CPHOT_DETECTOR_GRID)
    return fail(CPHOT_ERR_UNSUPPORTED, "curved transport collects on a ground grid");
  if (curved && !(d.earth_radius > 1e5 && std::isfinite(d.earth_radius)))
    return fail(CPHOT_ERR_INVALID_ARG, "curved transport needs the atmosphere's earth_radius");
  if (det->emission & ~(CPHOT_EMIT_CHERENKOV | CPHOT_EMIT_FLUORESCENCE))
    return fail(CPHOT_ERR_INVALID_ARG, "unknown emission bits");
  if (det->cuts & ~(CPHOT_CUT_TRACK | CPHOT_CUT_PHOTON)) return fail(CPHOT_ERR_INVALID_ARG, "unknown cut bits");
  if ((det->efficiency || det->reduction) && d.n_layers < 1)
    return fail(CPHOT_ERR_INVALID_ARG, "efficiency and reduction need an atmosphere with layers and wavelength bins");
  if (det->cuts && det->detector == CPHOT_DETECTOR_SPHERES &&
      det->transport != CPHOT_TRANSPORT_STRAIGHT && det->transport != CPHOT_TRANSPORT_LAYERED &&
      det->transport != CPHOT_TRANSPORT_TABLE)
    return fail(CPHOT_ERR_UNSUPPORTED, "cuts on SPHERES need STRAIGHT, LAYERED or planar TABLE transport");
  if (det->cuts && det->detector == CPHOT_DETECTOR_GRID) {
    if (det->cuts & CPHOT_CUT_TRACK) return fail(CPHOT_ERR_UNSUPPORTED, "the track cut is for SPHERES");
    if (det->transport == CPHOT_TRANSPORT_SURROGATE && !curved_sur)
      return fail(CPHOT_ERR_UNSUPPORTED, "the grid photon cut takes no planar surrogate transport");
    if (curved && !a->delta_monotone)
      return fail(CPHOT_ERR_UNSUPPORTED, "the curved grid photon cut needs n - 1 non-increasing with height");
  }
  if ((det->emission & CPHOT_EMIT_FLUORESCENCE) && seg->n > 0 && !seg->dedx)
    return fail(CPHOT_ERR_INVALID_ARG, "fluorescence needs the dedx column");
  if (det->detector != CPHOT_DETECTOR_GRID && det->detector != CPHOT_DETECTOR_SPHERES)
    return fail(CPHOT_ERR_INVALID_ARG, "unknown detector");
  if (det->spectrum != CPHOT_SPECTRUM_UNIFORM && det->spectrum != CPHOT_SPECTRUM_FRANK_TAMM &&
      det->spectrum != CPHOT_SPECTRUM_DISPERSIVE)
    return fail(CPHOT_ERR_INVALID_ARG, "unknown spectrum");
  if (det->spectrum == CPHOT_SPECTRUM_DISPERSIVE &&
      (!(d.lambda_min_nm >= 150.0) || !(det->lambda_ref_nm >= 150.0 && det->lambda_ref_nm <= 1e5)))
    return fail(CPHOT_ERR_INVALID_ARG, "the dispersive spectrum needs lam_min >= 150 nm and lambda_ref_nm in "
                                       "[150, 1e5] nm");
  if (det->bunch < 1) return fail(CPHOT_ERR_INVALID_ARG, "bunch must be >= 1");
  if (!std::isfinite(det->h_obs) || det->h_obs < 0.0 || det->h_obs >= d.h_top)
    return fail(CPHOT_ERR_INVALID_ARG, "h_obs must lie in [0, h_top)");

  std::memset(&p, 0, sizeof(p));
  p.x0 = seg->x0; p.y0 = seg->y0; p.z0 = seg->z0;
  p.x1 = seg->x1; p.y1 = seg->y1; p.z1 = seg->z1;
  p.beta = seg->beta; p.charge = seg->charge;
  p.n = seg->n;
  p.first_id = (uint64_t)seg->first_id;
  p.id_stride = seg->id_stride > 0 ? (uint64_t)seg->id_stride : 1u;
  p.n_showers = seg->n_showers;
  p.offsets = seg->shower_offsets;
  p.geom = seg->shower_geom;
  p.tab = a->dev.delta_table;
  p.n_tab = a->n_tab;
  p.step = d.table_step;
  {
    const double l1 = d.lambda_min_nm * 1e-9, l2 = d.lambda_max_nm * 1e-9;
    p.K = 2.0 * kPi * kAlpha * (1.0 / l1 - 1.0 / l2);
  }
  p.bunch = (uint32_t)det->bunch;
  p.key0 = (uint32_t)det->seed;
  p.key1 = (uint32_t)(det->seed >> 32);
  p.profile = d.profile;
  for (int i = 0; i < 5; ++i) {
    p.hb[i] = (float)d.lin_hb[i];
    p.la[i] = (float)d.lin_a[i];
    p.lb[i] = (float)d.lin_b[i];
    p.linv_c[i] = d.profile == CPHOT_PROFILE_LINSLEY5 ? (float)(1.0 / d.lin_c[i]) : 0.f;
  }
  p.opt_scale = d.profile == CPHOT_PROFILE_LINSLEY5 ? (float)(d.kappa / a->rho0 / 100.0) : (float)d.delta0;
  p.h_top = (float)d.h_top;
  p.has_ray = d.rayleigh400 > 0.0;
  p.has_aer = d.aerosol_tau350 > 0.0;
  p.inv_ray400 = p.has_ray ? (float)(1.0 / d.rayleigh400) : 0.f;
  p.aer_tau350 = (float)d.aerosol_tau350;
  p.aer_inv_h = p.has_aer ? (float)(1.0 / d.aerosol_height) : 0.f;
  p.aer_ang = (float)d.aerosol_angstrom;
  p.lam_min = (float)d.lambda_min_nm;
  p.lam_max = (float)d.lambda_max_nm;
  p.inv_lam_min = (float)(1.0 / d.lambda_min_nm);
  p.inv_lam_max = (float)(1.0 / d.lambda_max_nm);
  p.spectrum = det->spectrum;
  if (det->spectrum == CPHOT_SPECTRUM_DISPERSIVE) {
    const double rmax = air_dispersion(d.lambda_min_nm), rref = air_dispersion(det->lambda_ref_nm);
    p.disp_dmax = rmax / rref;
    p.disp_inv_rref = 1.0 / rref;
    const double sm = 1000.0 / d.lambda_min_nm, s2m = sm * sm;
    p.disp_s2m = (float)s2m;
    p.disp_k1c = (float)(kDispK1 / (kDispK0 - s2m));
    p.disp_k3c = (float)(kDispK3 / (kDispK2 - s2m));
  }
  p.dedx = seg->dedx;
  p.emission = det->emission ? det->emission : CPHOT_EMIT_CHERENKOV;
  for (int b = 0; b < 3; ++b) {
    p.fl_yield[b] = det->fl_yield[b];
    p.fl_lambda[b] = (float)det->fl_lambda[b];
    if ((p.emission & CPHOT_EMIT_FLUORESCENCE) &&
        (!(det->fl_yield[b] >= 0.0) || !std::isfinite(det->fl_yield[b]) ||
         !(det->fl_lambda[b] >= d.lambda_min_nm && det->fl_lambda[b] <= d.lambda_max_nm)))
      return fail(CPHOT_ERR_INVALID_ARG, "fluorescence yields must be >= 0 and wavelengths inside the band");
  }
  p.earth_radius = d.earth_radius;
  p.h_obs = (float)det->h_obs;
  p.X_obs = d.profile == CPHOT_PROFILE_LINSLEY5 ? (float)depth(d, det->h_obs) : 0.f;
  p.transport = curved_sur ? cphot::kTransportCurvedSurrogate
                : curved_tab ? cphot::kTransportCurvedTable
                             : det->transport;
  if (det->transport == CPHOT_TRANSPORT_TABLE) p.ctab = cphot::table_view(det->table);
  p.detector = det->detector;
  if (det->counts_rule != CPHOT_COUNTS_ROUNDED && det->counts_rule != CPHOT_COUNTS_POISSON)
    return fail(CPHOT_ERR_INVALID_ARG, "unknown counts_rule");
  p.poisson = det->counts_rule == CPHOT_COUNTS_POISSON;
  p.eff = det->efficiency;
  p.red = det->reduction;
  if (d.n_layers > 0) p.dh64 = d.h_top / d.n_layers;
  if (det->efficiency || det->reduction) {  // wavelength bins and layers for straight rays too
    p.n_layers = d.n_layers;
    p.n_lam = d.n_lambda_bins;
    p.dh = (float)(d.h_top / d.n_layers);
    p.inv_dh = (float)(d.n_layers / d.h_top);
  }
  if (det->transport != CPHOT_TRANSPORT_STRAIGHT) {
    if (d.n_layers < 1) return fail(CPHOT_ERR_INVALID_ARG, "layered transport needs an atmosphere with layers");
    if (det->transport == CPHOT_TRANSPORT_SURROGATE) p.mlp = cphot::surrogate_image(det->surrogate);
    p.n_layers = d.n_layers;
    p.n_lam = d.n_lambda_bins;
    p.dh = (float)(d.h_top / d.n_layers);
    p.inv_dh = (float)(d.n_layers / d.h_top);
    p.obs_layer = (int)std::floor(det->h_obs / (d.h_top / d.n_layers));
    p.layers = a->dev.layers;
    p.lambins = a->dev.lambins;
    p.moments = a->dev.moments ? a->dev.moments + (size_t)p.obs_layer * d.n_layers * 5 : nullptr;
    p.series_tmax = a->dev.moments ? a->dev.series_tmax : 0.f;
    // closed-form shell sums: the curved exact transport, and the exact tracer
    // behind the curved surrogate and table
    if ((det->transport == CPHOT_TRANSPORT_CURVED || curved_sur || curved_tab) && a->dev.shells) {
      p.shells = a->dev.shells + (size_t)p.obs_layer * d.n_layers * cphot::kShellRow;
      p.shell_tmax = a->dev.shell_tmax;
      p.shell_rho = (float)cphot::kShellRhoMax;
      p.shell_nb_rising = a->nb_rising ? 1 : 0;
    }
  }
  const int64_t ns = seg->n_showers;
  if (det->detector == CPHOT_DETECTOR_GRID) {
    if (det->nx < 1 || det->ny < 1 || !finite_pos(det->cell))
      return fail(CPHOT_ERR_INVALID_ARG, "grid needs nx, ny >= 1 and cell > 0");
    p.nx = det->nx; p.ny = det->ny;
    p.cell = (float)det->cell;
    p.inv_cell = (float)(1.0 / det->cell);
    p.inv_cell64 = 1.0 / (double)det->cell;
    p.cuts = need_bins ? det->cuts : 0;  // the parity entry points trace every record
    if (det->transport != CPHOT_TRANSPORT_STRAIGHT && d.n_layers > 0)
      p.cut_e = (float)(a->cut_e[(size_t)p.obs_layer] * (1.0 + 1e-6));
    if (need_bins && out->bins_capacity < ns * (int64_t)det->nx * det->ny)
      return fail(CPHOT_ERR_INVALID_ARG, "bins_capacity below n_showers * nx * ny");
  } else {
    if (det->snx < 1 || det->sny < 1 || !finite_pos(det->pitch) || !finite_pos(det->radius))
      return fail(CPHOT_ERR_INVALID_ARG, "spheres need snx, sny >= 1, pitch > 0, radius > 0");
    if (4.0 * det->radius > det->pitch)
      return fail(CPHOT_ERR_INVALID_ARG, "spheres must satisfy pitch >= 4 radius (one candidate per cell)");
    if (det->transport != CPHOT_TRANSPORT_STRAIGHT) {
      const double dh = d.h_top / d.n_layers;
      const double lo = p.obs_layer * dh, hi = (p.obs_layer + 1) * dh;
      if (det->h_obs - det->radius < lo || det->h_obs + det->radius >= hi)
        return fail(CPHOT_ERR_INVALID_ARG, "spheres must lie inside the layer containing h_obs");
    }
    p.cuts = need_bins ? det->cuts : 0;  // the parity entry points trace every record
    if (det->transport != CPHOT_TRANSPORT_STRAIGHT && d.n_layers > 0)
      p.cut_e = (float)(a->cut_e[(size_t)p.obs_layer] * (1.0 + 1e-6));
    p.snx = det->snx; p.sny = det->sny;
    p.pitch = (float)det->pitch;
    p.inv_pitch = (float)(1.0 / det->pitch);
    p.radius = (float)det->radius;
    p.n_t = det->n_time_bins;
    if (p.n_t < 0) return fail(CPHOT_ERR_INVALID_ARG, "n_time_bins must be >= 0");
    if (p.n_t > 0 && !finite_pos(det->time_bin_ns)) return fail(CPHOT_ERR_INVALID_ARG, "time_bin_ns must be > 0");
    p.inv_dt = p.n_t > 0 ? (float)(1.0 / det->time_bin_ns) : 0.f;
    const int64_t nsph = (int64_t)det->snx * det->sny;
    if (need_bins) {
      if (out->bins_capacity < ns * nsph) return fail(CPHOT_ERR_INVALID_ARG, "bins_capacity below n_showers * spheres");
      if (p.n_t > 0 && (!out->time_hist || out->time_capacity < ns * nsph * (p.n_t + 1)))
        return fail(CPHOT_ERR_INVALID_ARG, "time_hist missing or below n_showers * spheres * (n_time_bins + 1)");
    }
  }
  if (need_bins) {
    if (!out) return fail(CPHOT_ERR_INVALID_ARG, "null bins");
    if (out->bins_dtype != CPHOT_BINS_U32 && out->bins_dtype != CPHOT_BINS_U64 && out->bins_dtype != CPHOT_BINS_F64)
      return fail(CPHOT_ERR_INVALID_ARG, "unknown bins dtype");
    if (!out->bins) return fail(CPHOT_ERR_INVALID_ARG, "null bins buffer");
    p.bins = out->bins;
    p.bins_u64 = out->bins_dtype == CPHOT_BINS_U64;
    p.bins_f64 = out->bins_dtype == CPHOT_BINS_F64;
    p.thist = out->time_hist;
    p.counters = out->counters;
  }
  return CPHOT_OK;
}

// Moments of the closed-form shell sums (curved Earth; cphot_device.h, curved_series).
// Row (obs, j) sums over the full shells i, obs < i < j, in FP64: for each weight w
// and pair (k, m), a_km sum_i w_i u_i^k (D'_{i+1}^m - D'_i^m) with
// e_i = (n_i - n_j) / n_i, u_i = e_i (2 - e_i), D'_i = (b_j^2 - b_i^2) / (2 R dh)
// = (j - i) (1 + (i + j) dh / (2 R)), a_km = binom(1/2, k + m) binom(k + m, k) (-1)^m.
// Weights (one 16-float group each, entry q for pair q): Rayleigh and aerosol parts of
// the extinction, R^2 e_i / (b_i b_{i+1}), R^2 / (b_i b_{i+1}) (k >= 1), 1 (k >= 1), n_i - 1.
// Returns the largest |u| over all pairs (it bounds the series' t).
double shell_moments(const std::vector<float4>& lay, int L, double dh, double Re, std::vector<float>& rows) {
  static const int kKM[cphot::kShellTerms][2] = {{0, 1}, {0, 2}, {0, 3}, {0, 4}, {0, 5}, {1, 1}, {1, 2}, {1, 3},
                                                 {1, 4}, {1, 5}, {2, 1}, {2, 2}, {2, 3}, {3, 1}, {3, 2}};
  double acoef[cphot::kShellTerms];
  for (int q = 0; q < cphot::kShellTerms; ++q) {
    const int k = kKM[q][0], m = kKM[q][1], n = k + m;
    double bh = 1.0;  // binom(1/2, n)
    for (int i = 0; i < n; ++i) bh *= (0.5 - i) / (i + 1);
    double bk = 1.0;  // binom(n, k)
    for (int i = 0; i < k; ++i) bk *= (double)(n - i) / (i + 1);
    acoef[q] = bh * bk * ((m & 1) ? -1.0 : 1.0);
  }
  rows.assign((size_t)L * L * cphot::kShellRow, 0.f);
  const double R2 = Re * Re;
  double umax = 0.0;
  for (int j = 1; j < L; ++j) {
    double S[6][cphot::kShellTerms] = {{0.0}};
    const double dj = (double)lay[j].x;
    for (int obs = j - 1; obs >= 0; --obs) {
      float* r = &rows[((size_t)obs * L + j) * cphot::kShellRow];
      for (int q = 0; q < cphot::kShellTerms; ++q) {
        r[q] = (float)(acoef[q] * S[0][q]);
        r[16 + q] = (float)(acoef[q] * S[1][q]);
        r[32 + q] = (float)(acoef[q] * S[2][q]);
        r[80 + q] = (float)(acoef[q] * S[5][q]);
        if (q >= 5) {  // k >= 1 only: the straight line's part is formed directly
          r[48 + q] = (float)(acoef[q] * S[3][q]);
          r[64 + q] = (float)(acoef[q] * S[4][q]);
        }
      }
      // shell i = obs joins the sums of the rows below it
      const int i = obs;
      const double di = (double)lay[i].x;
      const double e = (di - dj) / (1.0 + di), u = e * (2.0 - e);
      umax = std::max(umax, std::fabs(u));
      const double bi = Re + i * dh, bi1 = Re + (i + 1) * dh;
      const double w[6] = {(double)lay[i].z, (double)lay[i].w, R2 * e / (bi * bi1), R2 / (bi * bi1), 1.0, di};
      const double D0 = (double)(j - i) * (1.0 + (i + j) * dh / (2.0 * Re));
      const double D1 = (double)(j - i - 1) * (1.0 + (i + 1 + j) * dh / (2.0 * Re));
      for (int q = 0; q < cphot::kShellTerms; ++q) {
        const int k = kKM[q][0], m = kKM[q][1];
        const double diff = std::pow(D1, m) - std::pow(D0, m);
        const double f = std::pow(u, k) * diff;
        for (int c = 0; c < 6; ++c) S[c][q] += w[c] * f;
      }
    }
  }
  return umax;
}

struct LaunchShape {
  int block, grid;
  size_t lds;
};

// Launch shape. The grid histogram can be privatised in LDS: the whole grid
// when it fits, else a window of W x W cells around the grid centre (the core),
// where most photons of a shower land. Each block then walks a contiguous range
// of tiles and flushes its window when the shower changes, so global atomics are
// paid per window cell and block rather than per photon.
constexpr size_t kLdsBudget = 64 * 1024;  // per block, static + dynamic
constexpr size_t kLdsPerCu = 160 * 1024;

// LDS a block may hold while a CU still runs four waves per SIMD (the occupancy
// the exact tracers' registers allow; kernels with more registers run fewer
// waves and are then only more conservative): 160 KB over 16 / (BS / 64) blocks.
size_t lds_at_four_waves(int bs) {
  const int blocks = std::max(1, 16 / (bs / 64));
  return kLdsPerCu / (size_t)blocks - 1024;  // margin for the allocation granule
}

int choose_shape(const cphot_detector* det, cphot::KParams& p, int mode, LaunchShape& s) {
  int bs = det->block_size ? det->block_size : 256;
  if (bs != 128 && bs != 256 && bs != 512) return fail(CPHOT_ERR_INVALID_ARG, "block_size must be 0, 128, 256 or 512");
  if (det->hist_window < 0 || det->hist_window_h < 0)
    return fail(CPHOT_ERR_INVALID_ARG, "hist_window and hist_window_h must be >= 0");
  size_t lds = 0;
  p.lds_hist = 0;
  p.hist_w = p.hist_h = p.hist_x0 = p.hist_y0 = p.hist_tw = 0;
  const size_t stat =
      (mode == cphot::MODE_PROPAGATE && det->lds_hist != 0) ? cphot::propagate_static_lds(p, mode, bs) : 0;
  if (mode == cphot::MODE_PROPAGATE && p.detector == CPHOT_DETECTOR_GRID && det->lds_hist != 0) {
    const size_t room = stat < kLdsBudget ? (kLdsBudget - stat) / 4 : 0;  // cells that fit
    int w = p.nx, h = p.ny;
    if (det->hist_window > 0) {
      // the caller's window, shrunk (longer side first) until it fits
      w = std::min(p.nx, det->hist_window);
      h = std::min(p.ny, det->hist_window_h > 0 ? det->hist_window_h : det->hist_window);
      while ((size_t)w * h > room && w > 0 && h > 0) {
        if (w >= h) --w;
        else --h;
      }
    } else if ((size_t)w * h > room) {
      int side = (int)std::sqrt((double)room);
      while (side > 0 && (size_t)side * side > room) --side;
      w = std::min(p.nx, side);
      h = std::min(p.ny, side);
    }
    const bool usable = w >= 8 && h >= 8 && (size_t)w * h <= room;
    if (det->lds_hist == 1 && !usable) return fail(CPHOT_ERR_INVALID_ARG, "no LDS histogram window fits this launch");
    // Library choice: the whole grid when it fits; a partial window only for
    // straight rays, where a record costs about as much as its global atomic.
    // Refracting transports spend far more per record and lose more to the
    // window's lower occupancy than they save in atomics (the autotuner times both).
    const bool whole = w == p.nx && h == p.ny;
    const bool wanted = det->lds_hist == 1 || whole || p.transport == CPHOT_TRANSPORT_STRAIGHT;
    if (usable && wanted) {
      p.lds_hist = 1;
      p.hist_w = w;
      p.hist_h = h;
      p.hist_x0 = std::min(std::max((p.nx - w) / 2 + det->hist_window_dx, 0), p.nx - w);
      p.hist_y0 = std::min(std::max((p.ny - h) / 2 + det->hist_window_dy, 0), p.ny - h);
      lds = (size_t)w * h * 4;
    }
  }
  // spheres: the whole array of sphere counts in LDS when it fits (hits cluster
  // on the few spheres near the core, whose device atomics would serialise), and
  // with it the leading time bins of every sphere, where the hits of the spheres
  // near the core arrive (delays after the plane front of a few to tens of ns);
  // later bins stay global. The time part takes only the LDS that leaves the
  // occupancy the kernel's registers allow.
  if (mode == cphot::MODE_PROPAGATE && p.detector == CPHOT_DETECTOR_SPHERES && det->lds_hist != 0) {
    const size_t room = stat < kLdsBudget ? (kLdsBudget - stat) / 4 : 0;
    const size_t nsph = (size_t)p.snx * p.sny;
    if (nsph > room) {
      if (det->lds_hist == 1) return fail(CPHOT_ERR_INVALID_ARG, "the sphere counts do not fit in LDS");
    } else {
      p.lds_hist = 1;
      p.hist_w = p.snx;
      p.hist_h = p.sny;
      const size_t cap = std::min(kLdsBudget, lds_at_four_waves(bs));
      if (p.n_t > 0 && cap > stat + nsph * 4) {
        const size_t tb = std::min((cap - stat) / 4 - nsph, room - nsph) / nsph;
        p.hist_tw = (int)std::min<size_t>(tb, (size_t)p.n_t + 1);
      }
      lds = nsph * (1 + (size_t)p.hist_tw) * 4;
    }
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  const int64_t tiles = (p.n + bs - 1) / bs;
  // One block per tile lets the dispatcher balance uneven tiles. With an LDS
  // histogram a persistent grid (a few blocks per CU, each over a contiguous
  // range of tiles) amortises the window's zeroing and flushes.
  // Sphere counts are few, so their flush stays cheap at one block per tile.
  const bool persistent = p.lds_hist && p.detector == CPHOT_DETECTOR_GRID;
  int64_t g = det->grid_blocks > 0 ? det->grid_blocks : (persistent ? (int64_t)cu_count(dev) * 4 : tiles);
  if (g > tiles) g = tiles;
  if (g < 1) g = 1;
  s.block = bs;
  s.grid = (int)g;
  s.lds = lds;
  return CPHOT_OK;
}

}  // namespace

namespace cphot {
double atmosphere_earth_radius(const cphot_atmosphere* a) { return a ? a->d.earth_radius : 0.0; }

int atmosphere_layer_view(const cphot_atmosphere* a, const float4** layers, const float2** lambins, int* n_layers,
                          int* n_lam, float* dh, float* lam_min, float* lam_max) {
  if (!a || a->d.n_layers < 1) return CPHOT_ERR_INVALID_ARG;
  *layers = a->dev.layers;
  *lambins = a->dev.lambins;
  *n_layers = a->d.n_layers;
  *n_lam = a->d.n_lambda_bins;
  *dh = (float)(a->d.h_top / a->d.n_layers);
  *lam_min = (float)a->d.lambda_min_nm;
  *lam_max = (float)a->d.lambda_max_nm;
  return CPHOT_OK;
}
const float4* atmosphere_layer_moments(const cphot_atmosphere* a) { return a ? a->dev.moments : nullptr; }
}  // namespace cphot

extern "C" {

int cphot_version(void) { return CPHOT_ABI_VERSION; }

const char* cphot_status_string(int status) {
  switch (status) {
    case CPHOT_OK: return "ok";
    case CPHOT_ERR_INVALID_ARG: return "invalid argument";
    case CPHOT_ERR_OUT_OF_MEMORY: return "out of device memory";
    case CPHOT_ERR_HIP: return "HIP runtime error";
    case CPHOT_ERR_UNSUPPORTED: return "unsupported";
    case CPHOT_ERR_CAPACITY: return "capacity exceeded";
    default: return "unknown status";
  }
}

const char* cphot_last_error(void) { return g_err.c_str(); }

int cphot_make_atmosphere(const cphot_atmosphere_desc* desc, cphot_atmosphere** out) {
  if (!desc || !out) return fail(CPHOT_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  const cphot_atmosphere_desc& d = *desc;
  if (d.profile != CPHOT_PROFILE_LINSLEY5 && d.profile != CPHOT_PROFILE_HOMOGENEOUS &&
      d.profile != CPHOT_PROFILE_LINEAR)
    return fail(CPHOT_ERR_INVALID_ARG, "unknown profile");
  if (!finite_pos(d.h_top) || !finite_pos(d.table_step) || d.h_top / d.table_step > 1e8)
    return fail(CPHOT_ERR_INVALID_ARG, "h_top and table_step must be > 0 with at most 1e8 table entries");
  if (!(d.lambda_min_nm > 0 && d.lambda_max_nm > d.lambda_min_nm && std::isfinite(d.lambda_max_nm)))
    return fail(CPHOT_ERR_INVALID_ARG, "need 0 < lambda_min < lambda_max");
  if (d.profile == CPHOT_PROFILE_LINSLEY5) {
    for (int i = 0; i < 5; ++i)
      if (!finite_pos(d.lin_c[i]) || !std::isfinite(d.lin_a[i]) || !std::isfinite(d.lin_b[i]))
        return fail(CPHOT_ERR_INVALID_ARG, "Linsley parameters must be finite with c > 0");
    if (d.lin_hb[0] != 0.0) return fail(CPHOT_ERR_INVALID_ARG, "lin_hb[0] must be 0");
    for (int i = 1; i < 5; ++i)
      if (!(d.lin_hb[i] > d.lin_hb[i - 1])) return fail(CPHOT_ERR_INVALID_ARG, "lin_hb must ascend");
    if (!finite_pos(d.lin_b[0])) return fail(CPHOT_ERR_INVALID_ARG, "lin_b[0] must be > 0");
    if (!std::isfinite(d.kappa) || d.kappa < 0) return fail(CPHOT_ERR_INVALID_ARG, "kappa must be >= 0");
  } else {
    if (!std::isfinite(d.delta0) || d.delta0 < 0) return fail(CPHOT_ERR_INVALID_ARG, "delta0 must be >= 0");
    if (d.rayleigh400 > 0) return fail(CPHOT_ERR_INVALID_ARG, "Rayleigh absorption needs the LINSLEY5 profile");
  }
  if (d.rayleigh400 < 0 || !std::isfinite(d.rayleigh400)) return fail(CPHOT_ERR_INVALID_ARG, "bad rayleigh400");
  if (d.aerosol_tau350 < 0 || !std::isfinite(d.aerosol_tau350)) return fail(CPHOT_ERR_INVALID_ARG, "bad aerosol_tau350");
  if (d.aerosol_tau350 > 0 && !finite_pos(d.aerosol_height)) return fail(CPHOT_ERR_INVALID_ARG, "bad aerosol_height");
  if (d.n_layers < 0 || d.n_layers > cphot::kMaxLayers)
    return fail(CPHOT_ERR_INVALID_ARG, "n_layers must be in [0, 128]");
  if (d.n_layers > 0 && (d.n_lambda_bins < 1 || d.n_lambda_bins > cphot::kMaxLambdaBins))
    return fail(CPHOT_ERR_INVALID_ARG, "n_lambda_bins must be in [1, 64] with layers");

  cphot_atmosphere* a = new (std::nothrow) cphot_atmosphere();
  if (!a) return fail(CPHOT_ERR_OUT_OF_MEMORY, "host allocation");
  a->d = d;
  (void)hipGetDevice(&a->device);
  a->rho0 = d.profile == CPHOT_PROFILE_LINSLEY5 ? d.lin_b[0] / d.lin_c[0] : 1.0;
  a->n_tab = (int64_t)std::ceil(d.h_top / d.table_step);
  std::vector<double> tab((size_t)a->n_tab + 1);
  for (int64_t j = 0; j <= a->n_tab; ++j) tab[(size_t)j] = refractivity(*a, (double)j * d.table_step);
  // Layer tables. Each layer's extinction per metre factorises into a height
  // part and a wavelength part: Rayleigh (X(lo) - X(hi)) / dh times 1/Lambda(lambda_k),
  // plus the aerosol column (exp(-lo/H) - exp(-hi/H)) / dh times tau_A(lambda_k).
  std::vector<float4> lay, mom;
  std::vector<float2> lamb;
  std::vector<float> shells;
  float series_tmax = 0.f, shell_tmax = 0.f;
  if (d.n_layers > 0) {
    const int L = d.n_layers, K = d.n_lambda_bins;
    const double dh = d.h_top / L;
    a->layer_delta.resize(L);
    lay.resize(L);
    lamb.resize(K);
    for (int i = 0; i < L; ++i) {
      const double lo = i * dh, hi = (i + 1) * dh;
      const double dl = refractivity(*a, 0.5 * (lo + hi));
      a->layer_delta[i] = dl;
      const double ray = d.rayleigh400 > 0.0 ? (depth(d, lo) - depth(d, hi)) / dh : 0.0;
      const double aer = d.aerosol_tau350 > 0.0
                             ? (std::exp(-lo / d.aerosol_height) - std::exp(-hi / d.aerosol_height)) / dh
                             : 0.0;
      lay[i] = make_float4((float)dl, (float)(1.0 / (1.0 + dl)), (float)ray, (float)aer);
    }
    // Moments for the closed-form layer sums: row (obs, j) sums over the full
    // layers i, obs < i < j, in FP64 (e_i = (n_i - n_j) / n_i, u_i = e_i (2 - e_i)),
    // with dh and the coefficients a1 = -1/2, a2 = 3/8, a3 = -5/16 of
    // (1 + x)^(-1/2) folded in. The series serves photons with tan^2(zenith) up
    // to 5.4e-3 / max|u| (at most 9), where the truncated terms stay negligible.
    mom.assign((size_t)L * L * 5, make_float4(0.f, 0.f, 0.f, 0.f));
    const double a1 = -0.5, a2 = 0.375, a3 = -0.3125;
    double umax = 0.0;
    for (int j = 1; j < L; ++j) {
      double S[17] = {0.0};  // U1..3, EU0..2, E2U0..1, D0..2, R0..2, A0..2 (sums, without dh)
      for (int obs = j - 1; obs >= 0; --obs) {
        float4* r = &mom[((size_t)obs * L + j) * 5];
        r[0] = make_float4((float)(dh * a1 * S[0]), (float)(dh * a2 * S[1]), (float)(dh * a3 * S[2]), (float)(dh * S[3]));
        r[1] = make_float4((float)(dh * a1 * S[4]), (float)(dh * a2 * S[5]), (float)(dh * S[6]), (float)(dh * a1 * S[7]));
        r[2] = make_float4((float)(dh * S[8]), (float)(dh * a1 * S[9]), (float)(dh * a2 * S[10]), (float)(dh * S[11]));
        r[3] = make_float4((float)(dh * a1 * S[12]), (float)(dh * a2 * S[13]), (float)(dh * S[14]), (float)(dh * a1 * S[15]));
        r[4] = make_float4((float)(dh * a2 * S[16]), (float)(dh * (j - obs - 1)), 0.f, 0.f);
        // layer obs joins the sums of the rows below it
        const int i = obs;
        const double di = (double)lay[i].x, dj = (double)lay[j].x;
        const double e = (di - dj) / (1.0 + di), u = e * (2.0 - e);
        umax = std::max(umax, std::fabs(u));
        const double Ri = (double)lay[i].z, Ai = (double)lay[i].w;
        S[0] += u; S[1] += u * u; S[2] += u * u * u;
        S[3] += e; S[4] += e * u; S[5] += e * u * u;
        S[6] += e * e; S[7] += e * e * u;
        S[8] += di; S[9] += di * u; S[10] += di * u * u;
        S[11] += Ri; S[12] += Ri * u; S[13] += Ri * u * u;
        S[14] += Ai; S[15] += Ai * u; S[16] += Ai * u * u;
      }
    }
    series_tmax = (float)std::min(9.0, umax > 0.0 ? 5.4e-3 / umax : 9.0);
    if (finite_pos(d.earth_radius) && d.earth_radius > 1e5) {
      const double umax_c = shell_moments(lay, L, dh, d.earth_radius, shells);
      shell_tmax = (float)std::min(25.0, umax_c > 0.0 ? 1.4e-2 / umax_c : 25.0);
    }
    // refraction bound of the data-reduction cuts: for the layers from obs up,
    // |n_i - n_j| / n_i <= (max delta - min delta) / (1 + min delta)
    a->cut_e.assign(L, 0.0);
    a->delta_monotone = true;
    for (int i = 0; i + 1 < L; ++i) a->delta_monotone = a->delta_monotone && lay[i].x >= lay[i + 1].x;
    // Bouguer's invariant over the shells: with n_i b_i increasing in i the ray's
    // impact parameter in shell i, n_j p / n_i, falls below every lower radius b_i
    // on the way down exactly when it does so in the lowest full shell
    a->nb_rising = finite_pos(d.earth_radius);
    for (int i = 0; i + 1 < L && a->nb_rising; ++i)
      a->nb_rising = (1.0 + (double)lay[i + 1].x) * (d.earth_radius + (i + 1) * dh) >
                     (1.0 + (double)lay[i].x) * (d.earth_radius + i * dh);
    double dmin = 1e300, dmax = -1e300;
    for (int obs = L - 1; obs >= 0; --obs) {
      dmin = std::min(dmin, (double)lay[obs].x);
      dmax = std::max(dmax, (double)lay[obs].x);
      a->cut_e[(size_t)obs] = (dmax - dmin) / (1.0 + dmin);
    }
    for (int k = 0; k < K; ++k) {
      const double lam = d.lambda_min_nm + (k + 0.5) * (d.lambda_max_nm - d.lambda_min_nm) / K;
      const double r = lam / 400.0;
      const double inv_ray = d.rayleigh400 > 0.0 ? 1.0 / (d.rayleigh400 * r * r * r * r) : 0.0;
      const double taua = d.aerosol_tau350 > 0.0 ? d.aerosol_tau350 * std::pow(lam / 350.0, -d.aerosol_angstrom) : 0.0;
      lamb[k] = make_float2((float)inv_ray, (float)taua);
    }
  }
  auto cleanup = [&](int code, const char* what, hipError_t e) {
    cphot_destroy_atmosphere(a);
    if (e == hipErrorOutOfMemory) return fail(CPHOT_ERR_OUT_OF_MEMORY, what);
    return hip_fail(e, what);
  };
  hipError_t e;
  if ((e = hipMalloc(&a->dev.delta_table, tab.size() * sizeof(double))) != hipSuccess)
    return cleanup(0, "hipMalloc(delta_table)", e);
  if ((e = hipMemcpy(a->dev.delta_table, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice)) !=
      hipSuccess)
    return cleanup(0, "hipMemcpy(delta_table)", e);
  if (d.n_layers > 0) {
    if ((e = hipMalloc(&a->dev.layers, lay.size() * sizeof(float4))) != hipSuccess) return cleanup(0, "hipMalloc", e);
    if ((e = hipMalloc(&a->dev.lambins, lamb.size() * sizeof(float2))) != hipSuccess) return cleanup(0, "hipMalloc", e);
    if ((e = hipMemcpy(a->dev.layers, lay.data(), lay.size() * sizeof(float4), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(a->dev.lambins, lamb.data(), lamb.size() * sizeof(float2), hipMemcpyHostToDevice)) != hipSuccess)
      return cleanup(0, "hipMemcpy(layers)", e);
    if ((e = hipMalloc(&a->dev.moments, mom.size() * sizeof(float4))) != hipSuccess) return cleanup(0, "hipMalloc", e);
    if ((e = hipMemcpy(a->dev.moments, mom.data(), mom.size() * sizeof(float4), hipMemcpyHostToDevice)) != hipSuccess)
      return cleanup(0, "hipMemcpy(moments)", e);
    a->dev.series_tmax = series_tmax;
    if (!shells.empty()) {
      if ((e = hipMalloc(&a->dev.shells, shells.size() * sizeof(float))) != hipSuccess)
        return cleanup(0, "hipMalloc", e);
      if ((e = hipMemcpy(a->dev.shells, shells.data(), shells.size() * sizeof(float), hipMemcpyHostToDevice)) !=
          hipSuccess)
        return cleanup(0, "hipMemcpy(shells)", e);
      a->dev.shell_tmax = shell_tmax;
    }
  }
  *out = a;
  return CPHOT_OK;
}

void cphot_destroy_atmosphere(cphot_atmosphere* a) {
  if (!a) return;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(a->device);
  if (a->dev.delta_table) (void)hipFree(a->dev.delta_table);
  if (a->dev.layers) (void)hipFree(a->dev.layers);
  if (a->dev.lambins) (void)hipFree(a->dev.lambins);
  if (a->dev.moments) (void)hipFree(a->dev.moments);
  if (a->dev.shells) (void)hipFree(a->dev.shells);
  (void)hipSetDevice(prev);
  delete a;
}

int cphot_reduction_table(const cphot_atmosphere* a, double h_obs, const double* efficiency, double* out) {
  if (!a || !out) return fail(CPHOT_ERR_INVALID_ARG, "null argument");
  const cphot_atmosphere_desc& d = a->d;
  if (d.n_layers < 1 || d.n_lambda_bins < 1) return fail(CPHOT_ERR_INVALID_ARG, "atmosphere without layers");
  if (!(h_obs >= 0.0 && h_obs < d.h_top)) return fail(CPHOT_ERR_INVALID_ARG, "h_obs must lie in [0, h_top)");
  const int L = d.n_layers, K = d.n_lambda_bins;
  const double dh = d.h_top / L;
  const int obs = (int)std::floor(h_obs / dh);
  for (int k = 0; k < K; ++k)
    if (efficiency && !(efficiency[k] >= 0.0 && efficiency[k] <= 1.0))
      return fail(CPHOT_ERR_INVALID_ARG, "efficiency values must lie in [0, 1]");
  // vertical optical depth per wavelength bin from each layer's bottom down to
  // h_obs, accumulated upwards from the observation layer
  std::vector<double> tau((size_t)K, 0.0);
  for (int i = 0; i < L; ++i) {
    double best = 0.0;
    for (int k = 0; k < K; ++k)
      best = std::max(best, (efficiency ? efficiency[k] : 1.0) * std::exp(-tau[(size_t)k]));
    out[i] = best * (1.0 + 1e-6);
    if (i >= obs) {  // the part of layer i above h_obs joins the column below layer i + 1
      const double lo = std::max((double)i * dh, h_obs), hi = (i + 1) * dh, span = hi - lo;
      // Rayleigh depth and aerosol column of that part: the layer averages times
      // the span (layered transport) or the exact columns (straight rays), the
      // smaller of the two; over a whole layer they are equal
      const double ray_avg = d.rayleigh400 > 0.0 ? (depth(d, i * dh) - depth(d, hi)) / dh * span : 0.0;
      const double ray_ex = d.rayleigh400 > 0.0 ? depth(d, lo) - depth(d, hi) : 0.0;
      const double aer_avg = d.aerosol_tau350 > 0.0 ? (std::exp(-i * dh / d.aerosol_height) -
                                                       std::exp(-hi / d.aerosol_height)) / dh * span
                                                    : 0.0;
      const double aer_ex = d.aerosol_tau350 > 0.0
                                ? std::exp(-lo / d.aerosol_height) - std::exp(-hi / d.aerosol_height)
                                : 0.0;
      const double ray = std::min(ray_avg, ray_ex), aer = std::min(aer_avg, aer_ex);
      for (int k = 0; k < K; ++k) {
        // the bin's longest wavelength: the least extinction any photon of the bin sees
        const double lam = d.lambda_min_nm + (k + 1) * (d.lambda_max_nm - d.lambda_min_nm) / K;
        const double r = lam / 400.0;
        const double inv_ray = d.rayleigh400 > 0.0 ? 1.0 / (d.rayleigh400 * r * r * r * r) : 0.0;
        const double taua =
            d.aerosol_tau350 > 0.0 ? d.aerosol_tau350 * std::pow(lam / 350.0, -d.aerosol_angstrom) : 0.0;
        tau[(size_t)k] += ray * inv_ray + aer * taua;
      }
    }
  }
  return CPHOT_OK;
}

int cphot_propagate(const cphot_segments* seg, const cphot_detector* det, cphot_bins* out, void* stream) {
  if (!out) return fail(CPHOT_ERR_INVALID_ARG, "null bins");
  cphot::KParams p;
  int rc = fill_params(seg, det, p, true, out);
  if (rc) return rc;
  if (p.n == 0) return CPHOT_OK;
  LaunchShape s;
  if ((rc = choose_shape(det, p, cphot::MODE_PROPAGATE, s))) return rc;
  hipError_t e = cphot::launch_propagate(p, cphot::MODE_PROPAGATE, s.block, s.grid, s.lds, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "launch propagate");
  return CPHOT_OK;
}

int cphot_segment_counts(const cphot_segments* seg, const cphot_detector* det, int32_t* counts, double* expected,
                         void* stream) {
  if (!counts && seg && seg->n > 0) return fail(CPHOT_ERR_INVALID_ARG, "null counts");
  cphot::KParams p;
  int rc = fill_params(seg, det, p, false, nullptr);
  if (rc) return rc;
  if (p.n == 0) return CPHOT_OK;
  p.counts = counts;
  p.expected = expected;
  LaunchShape s;
  if ((rc = choose_shape(det, p, cphot::MODE_COUNTS, s))) return rc;
  hipError_t e = cphot::launch_propagate(p, cphot::MODE_COUNTS, s.block, s.grid, s.lds, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "launch counts");
  return CPHOT_OK;
}

int cphot_trace_records(const cphot_segments* seg, const cphot_detector* det, const int64_t* record_offsets,
                        cphot_photon_record* records, int64_t capacity, void* stream) {
  if (seg && seg->n > 0 && (!record_offsets || !records || capacity < 0))
    return fail(CPHOT_ERR_INVALID_ARG, "null record buffers or negative capacity");
  cphot::KParams p;
  int rc = fill_params(seg, det, p, false, nullptr);
  if (rc) return rc;
  if (p.n == 0) return CPHOT_OK;
  p.rec_off = record_offsets;
  p.rec = records;
  p.rec_cap = capacity;
  LaunchShape s;
  if ((rc = choose_shape(det, p, cphot::MODE_RECORDS, s))) return rc;
  hipError_t e = cphot::launch_propagate(p, cphot::MODE_RECORDS, s.block, s.grid, s.lds, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "launch records");
  return CPHOT_OK;
}

// ---------------------------------------------------------------- captured steps

struct cphot_step {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

}  // extern "C"

namespace {

__global__ void k_fill_u32(uint32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

hipError_t clear_words(void* ptr, int64_t bytes, hipStream_t st) {
  if (!ptr || bytes <= 0) return hipSuccess;
  const int64_t n = bytes / 4;
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill_u32, dim3(blocks), dim3(256), 0, st, (uint32_t*)ptr, n);
  return hipGetLastError();
}

hipError_t clear_outputs(const cphot_bins* out, hipStream_t st) {
  hipError_t e = clear_words(out->bins, out->bins_capacity * (out->bins_dtype == CPHOT_BINS_U32 ? 4 : 8), st);
  if (e == hipSuccess) e = clear_words(out->time_hist, out->time_capacity * 4, st);
  if (e == hipSuccess && out->counters) e = clear_words(out->counters, CPHOT_NCOUNTERS * 8, st);
  return e;
}

}  // namespace

extern "C" {

int cphot_step_create(const cphot_segments* seg, const cphot_detector* det, const cphot_bins* out,
                      int32_t clear, cphot_step** step) {
  if (!step || !out) return fail(CPHOT_ERR_INVALID_ARG, "null argument");
  *step = nullptr;
  cphot::KParams p;
  int rc = fill_params(seg, det, p, true, out);
  if (rc) return rc;
  LaunchShape sh{};
  if (p.n > 0 && (rc = choose_shape(det, p, cphot::MODE_PROPAGATE, sh))) return rc;
  hipStream_t cs = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
  cphot_step* s = new (std::nothrow) cphot_step();
  if (!s) {
    (void)hipStreamDestroy(cs);
    return fail(CPHOT_ERR_OUT_OF_MEMORY, "host allocation");
  }
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess && clear) e = clear_outputs(out, cs);
  if (e == hipSuccess && p.n > 0) e = cphot::launch_propagate(p, cphot::MODE_PROPAGATE, sh.block, sh.grid, sh.lds, cs);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(cs, &g);
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = hipGraphInstantiate(&s->exec, g, nullptr, nullptr, 0);
  s->graph = g;
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess) {
    cphot_step_destroy(s);
    return hip_fail(e, "graph capture");
  }
  *step = s;
  return CPHOT_OK;
}

int cphot_step_launch(cphot_step* s, void* stream) {
  if (!s || !s->exec) return fail(CPHOT_ERR_INVALID_ARG, "null step");
  hipError_t e = hipGraphLaunch(s->exec, (hipStream_t)stream);
  return e == hipSuccess ? CPHOT_OK : hip_fail(e, "hipGraphLaunch");
}

void cphot_step_destroy(cphot_step* s) {
  if (!s) return;
  if (s->exec) (void)hipGraphExecDestroy(s->exec);
  if (s->graph) (void)hipGraphDestroy(s->graph);
  delete s;
}

// ---------------------------------------------------------------- streamer

struct cphot_streamer {
  int64_t chunk = 0;
  int dev = 0;
  float* dbuf[2] = {nullptr, nullptr};   // 9 columns of `chunk` floats each
  float* hbuf[2] = {nullptr, nullptr};   // pinned staging, same layout
  hipStream_t copy = nullptr;
  hipEvent_t copied[2] = {nullptr, nullptr};
  hipEvent_t done[2] = {nullptr, nullptr};
};

void cphot_streamer_destroy(cphot_streamer* s) {
  if (!s) return;
  for (int b = 0; b < 2; ++b) {
    if (s->done[b]) (void)hipEventSynchronize(s->done[b]);
    if (s->copied[b]) (void)hipEventSynchronize(s->copied[b]);
  }
  for (int b = 0; b < 2; ++b) {
    if (s->dbuf[b]) (void)hipFree(s->dbuf[b]);
    if (s->hbuf[b]) (void)hipHostFree(s->hbuf[b]);
    if (s->copied[b]) (void)hipEventDestroy(s->copied[b]);
    if (s->done[b]) (void)hipEventDestroy(s->done[b]);
  }
  if (s->copy) (void)hipStreamDestroy(s->copy);
  delete s;
}

int cphot_streamer_create(int64_t chunk_segments, cphot_streamer** out) {
  if (!out) return fail(CPHOT_ERR_INVALID_ARG, "null output handle");
  *out = nullptr;
  if (chunk_segments < 1 || chunk_segments > (int64_t(1) << 31))
    return fail(CPHOT_ERR_INVALID_ARG, "chunk_segments must be in [1, 2^31]");
  cphot_streamer* s = new cphot_streamer();
  s->chunk = chunk_segments;
  (void)hipGetDevice(&s->dev);
  const size_t bytes = (size_t)chunk_segments * 9 * sizeof(float);
  hipError_t e = hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking);
  for (int b = 0; b < 2 && e == hipSuccess; ++b) {
    e = hipMalloc((void**)&s->dbuf[b], bytes);
    if (e == hipSuccess) e = hipHostMalloc((void**)&s->hbuf[b], bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->copied[b], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->done[b], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    cphot_streamer_destroy(s);
    return e == hipErrorOutOfMemory ? fail(CPHOT_ERR_OUT_OF_MEMORY, "streamer buffers")
                                    : hip_fail(e, "streamer create");
  }
  *out = s;
  return CPHOT_OK;
}

}  // extern "C"

namespace {

// Host threads that fill a pinned staging buffer: one copy thread reads pageable
// memory at ~10 GB/s, too slow to keep up with a chunk's propagation.
constexpr int kStageThreads = 8;

// Copies rows [c0, c0 + n) of each column into the staging buffer (column f at
// dst + f * C), the rows split over host threads.
void stage_columns(float* dst, const float* const* cols, int ncol, int64_t C, int64_t c0, int64_t n) {
  const int T = (int)std::max<int64_t>(1, std::min<int64_t>(kStageThreads, n / 65536));
  auto work = [&](int t) {
    const int64_t a = n * t / T, b = n * (t + 1) / T;
    for (int f = 0; f < ncol; ++f)
      std::memcpy(dst + (size_t)f * C + a, cols[f] + c0 + a, (size_t)(b - a) * sizeof(float));
  };
  std::vector<std::thread> th;
  int started = 1;  // share 0 is this thread's; shares without a thread are copied here too
  try {
    th.reserve((size_t)T);
    for (; started < T; ++started) th.emplace_back(work, started);
  } catch (...) {
  }
  for (int t = started; t < T; ++t) work(t);
  work(0);
  for (auto& x : th) x.join();
}

// Page-locked host memory known to HIP (hipHostMalloc, or a pinned tensor): the copy
// engine reads it directly. Other pointers leave an error that is cleared here.
bool host_pinned(const void* p) {
  hipPointerAttribute_t a;
  const hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeHost;
}

}  // namespace

extern "C" {

int cphot_streamer_run(cphot_streamer* s, const cphot_host_segments* host, const cphot_detector* det,
                       cphot_bins* out, void* stream) {
  if (!s || !host || !det || !out) return fail(CPHOT_ERR_INVALID_ARG, "null argument");
  if (host->n < 0 || host->first_id < 0) return fail(CPHOT_ERR_INVALID_ARG, "negative n or first_id");
  if (host->n > 0 && (!host->x0 || !host->y0 || !host->z0 || !host->x1 || !host->y1 || !host->z1 ||
                      !host->beta || !host->charge))
    return fail(CPHOT_ERR_INVALID_ARG, "null host segment array");
  if (!host->shower_geom) return fail(CPHOT_ERR_INVALID_ARG, "null shower geometry");
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (dev != s->dev) return fail(CPHOT_ERR_INVALID_ARG, "streamer used on another device than it was made on");
  const float* cols[9] = {host->x0, host->y0, host->z0, host->x1, host->y1, host->z1, host->beta, host->charge,
                          host->dedx};
  const int ncol = host->dedx ? 9 : 8;
  // validate the whole run once (the same checks as a single call over the set)
  cphot_segments whole{};
  whole.x0 = whole.y0 = whole.z0 = whole.x1 = whole.y1 = whole.z1 = whole.beta = whole.charge = s->dbuf[0];
  whole.dedx = host->dedx ? s->dbuf[0] : nullptr;
  whole.n = host->n;
  whole.first_id = host->first_id;
  whole.n_showers = 1;
  whole.shower_geom = host->shower_geom;
  {
    cphot::KParams p;
    int rc = fill_params(&whole, det, p, true, out);
    if (rc) return rc;
    LaunchShape sh;
    if ((rc = choose_shape(det, p, cphot::MODE_PROPAGATE, sh))) return rc;
  }
  hipStream_t st = (hipStream_t)stream;
  const int64_t C = s->chunk;
  // columns in page-locked memory are copied to the device directly, without staging
  bool direct = host->n > 0;
  for (int f = 0; f < ncol && direct; ++f)
    direct = host_pinned(cols[f]) && host_pinned(cols[f] + (host->n - 1));
  int last = -1;
  for (int64_t c0 = 0, k = 0; c0 < host->n; c0 += C, ++k) {
    const int b = (int)(k & 1);
    const int64_t n = std::min(C, host->n - c0);
    // staging buffer b is free once its previous copy has finished; device buffer b
    // once the propagation that read it has finished (the copy stream waits for it)
    hipError_t e = hipEventSynchronize(s->copied[b]);
    if (e != hipSuccess) return hip_fail(e, "streamer wait");
    if (!direct) stage_columns(s->hbuf[b], cols, ncol, C, c0, n);
    e = hipStreamWaitEvent(s->copy, s->done[b], 0);
    for (int f = 0; f < ncol && e == hipSuccess; ++f)
      e = hipMemcpyAsync(s->dbuf[b] + (size_t)f * C, direct ? cols[f] + c0 : s->hbuf[b] + (size_t)f * C,
                         (size_t)n * sizeof(float), hipMemcpyHostToDevice, s->copy);
    if (e == hipSuccess) e = hipEventRecord(s->copied[b], s->copy);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, s->copied[b], 0);
    if (e != hipSuccess) return hip_fail(e, "streamer copy");
    cphot_segments seg{};
    float* d = s->dbuf[b];
    seg.x0 = d; seg.y0 = d + C; seg.z0 = d + 2 * C; seg.x1 = d + 3 * C; seg.y1 = d + 4 * C; seg.z1 = d + 5 * C;
    seg.beta = d + 6 * C; seg.charge = d + 7 * C;
    seg.dedx = host->dedx ? d + 8 * C : nullptr;
    seg.n = n;
    seg.first_id = host->first_id + c0;
    seg.n_showers = 1;
    seg.shower_geom = host->shower_geom;
    int rc = cphot_propagate(&seg, det, out, stream);
    if (rc) return rc;
    e = hipEventRecord(s->done[b], st);
    if (e != hipSuccess) return hip_fail(e, "streamer record");
    last = b;
  }
  // direct copies read the caller's memory until they complete
  if (direct && last >= 0) {
    const hipError_t e = hipEventSynchronize(s->copied[last]);
    if (e != hipSuccess) return hip_fail(e, "streamer wait");
  }
  return CPHOT_OK;
}

// ---------------------------------------------------------------- autotuner

}  // extern "C"

namespace {

// An LDS window of the grid: width, height, and the shift of its centre from the
// grid centre (cells), as cphot_detector carries it.
struct Window {
  int w, h, dx, dy;
};

// Photon footprint of one pilot launch with global atomics only: counts per grid
// cell summed over showers (the window is the same for every shower of a launch).
int grid_footprint(const cphot_segments* seg, const cphot_detector* det, cphot_bins* out, hipStream_t st,
                   std::vector<double>& foot) {
  cphot_detector d = *det;
  d.lds_hist = 0;
  d.block_size = 256;
  d.grid_blocks = 0;
  cphot::KParams p;
  int rc = fill_params(seg, &d, p, true, out);
  if (rc) return rc;
  LaunchShape sh;
  if ((rc = choose_shape(&d, p, cphot::MODE_PROPAGATE, sh))) return rc;
  const int64_t cells = (int64_t)det->nx * det->ny, n = cells * seg->n_showers;
  const size_t esz = out->bins_dtype == CPHOT_BINS_U32 ? 4 : 8;
  std::vector<unsigned char> host((size_t)n * esz);
  hipError_t e = clear_outputs(out, st);
  if (e == hipSuccess && p.n > 0) e = cphot::launch_propagate(p, cphot::MODE_PROPAGATE, sh.block, sh.grid, sh.lds, st);
  if (e == hipSuccess) e = hipMemcpyAsync(host.data(), out->bins, host.size(), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "autotune footprint");
  foot.assign((size_t)cells, 0.0);
  for (int64_t i = 0; i < n; ++i) {
    double v;
    if (out->bins_dtype == CPHOT_BINS_U32) v = (double)reinterpret_cast<const uint32_t*>(host.data())[i];
    else if (out->bins_dtype == CPHOT_BINS_U64) v = (double)reinterpret_cast<const uint64_t*>(host.data())[i];
    else v = reinterpret_cast<const double*>(host.data())[i];
    foot[(size_t)(i % cells)] += v;
  }
  return CPHOT_OK;
}

// The rectangle of at most `area` cells (sides >= 8, aspect ratios 1:4 to 4:1)
// that holds the most footprint counts, by a summed-area table over every
// position. False when the footprint is empty.
bool fit_window(const std::vector<double>& foot, int nx, int ny, size_t area, Window& best) {
  const size_t W = (size_t)nx + 1;
  std::vector<double> S(W * ((size_t)ny + 1), 0.0);
  for (int y = 0; y < ny; ++y) {
    double row = 0.0;
    for (int x = 0; x < nx; ++x) {
      row += foot[(size_t)y * nx + x];
      S[(size_t)(y + 1) * W + x + 1] = S[(size_t)y * W + x + 1] + row;
    }
  }
  double top = 0.0;
  bool found = false;
  for (double r : {0.25, 1.0 / 3.0, 0.5, 2.0 / 3.0, 1.0, 1.5, 2.0, 3.0, 4.0}) {
    const int w = std::min(nx, (int)std::sqrt((double)area * r));
    if (w < 8) continue;
    const int h = std::min(ny, (int)(area / (size_t)w));
    if (h < 8) continue;
    for (int y0 = 0; y0 + h <= ny; ++y0)
      for (int x0 = 0; x0 + w <= nx; ++x0) {
        const double v = S[(size_t)(y0 + h) * W + x0 + w] - S[(size_t)y0 * W + x0 + w] -
                         S[(size_t)(y0 + h) * W + x0] + S[(size_t)y0 * W + x0];
        if (v > top) {
          top = v;
          found = true;
          best = {w, h, x0 - (nx - w) / 2, y0 - (ny - h) / 2};
        }
      }
  }
  return found;
}

}  // namespace

extern "C" {

int cphot_autotune(const cphot_segments* seg, const cphot_detector* det, cphot_bins* out,
                   const int32_t* bunch_candidates, int32_t n_bunch, int32_t reps, cphot_tuning* best,
                   void* stream) {
  if (!seg || !det || !out || !best) return fail(CPHOT_ERR_INVALID_ARG, "null argument");
  if (reps < 1) return fail(CPHOT_ERR_INVALID_ARG, "reps must be >= 1");
  if (n_bunch < 0 || (n_bunch > 0 && !bunch_candidates)) return fail(CPHOT_ERR_INVALID_ARG, "bad bunch list");
  if (!out->counters) return fail(CPHOT_ERR_INVALID_ARG, "autotune reads the record counter: counters required");
  std::vector<int32_t> bunches;
  for (int i = 0; i < n_bunch; ++i) {
    if (bunch_candidates[i] < 1) return fail(CPHOT_ERR_INVALID_ARG, "bunch candidates must be >= 1");
    bunches.push_back(bunch_candidates[i]);
  }
  if (bunches.empty()) bunches.push_back(det->bunch);
  hipStream_t st = (hipStream_t)stream;
  int dev = 0;
  (void)hipGetDevice(&dev);
  const int cus = cu_count(dev);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(CPHOT_ERR_HIP, "hipEventCreate");
  cphot_tuning top{};
  top.photons_per_s = -1.0;
  int rc = CPHOT_OK;
  // grids too large for LDS: windows fitted to the footprint of a pilot launch
  std::vector<double> foot;
  if (det->detector == CPHOT_DETECTOR_GRID && det->lds_hist != 0 && (int64_t)det->nx * det->ny > 4096)
    rc = grid_footprint(seg, det, out, st, foot);
  for (int32_t b : bunches) {
    for (int bs : {128, 256, 512}) {
      std::vector<std::array<int, 6>> tried;  // launches already timed at this block size
      // grids: one block per tile, or a persistent grid of 2, 3, 4 or 8 blocks per CU (more
      // blocks than fit at once: the dispatcher starts later ones as earlier ones finish)
      for (int gpol = 0; gpol < 5 && rc == CPHOT_OK; ++gpol) {
        // LDS histogram: off; the largest centred square that fits; a centred 64 x 64;
        // rectangles fitted to the footprint with up to 2304, 4096 and 9216 cells
        // and with all the room the block's LDS budget leaves
        std::vector<Window> wins = {{-1, 0, 0, 0}, {0, 0, 0, 0}, {64, 64, 0, 0}};
        if (!foot.empty()) {
          cphot_detector d = *det;
          d.block_size = bs;
          cphot::KParams p;
          if ((rc = fill_params(seg, &d, p, true, out))) break;
          const size_t stat = cphot::propagate_static_lds(p, cphot::MODE_PROPAGATE, bs);
          const size_t room = stat < kLdsBudget ? (kLdsBudget - stat) / 4 : 0;
          for (size_t area : {(size_t)2304, (size_t)4096, (size_t)9216, room}) {
            Window f;
            if (area <= room && fit_window(foot, det->nx, det->ny, area, f)) wins.push_back(f);
          }
        }
        for (const Window& win : wins) {
          if (rc != CPHOT_OK) break;
          cphot_detector d = *det;
          d.bunch = b;
          d.block_size = bs;
          d.grid_blocks = gpol == 0 ? 0 : cus * (gpol == 1 ? 2 : (gpol == 2 ? 3 : (gpol == 3 ? 4 : 8)));
          d.lds_hist = win.w < 0 ? 0 : 1;
          d.hist_window = win.w < 0 ? 0 : win.w;
          d.hist_window_h = win.w < 0 ? 0 : win.h;
          d.hist_window_dx = win.w < 0 ? 0 : win.dx;
          d.hist_window_dy = win.w < 0 ? 0 : win.dy;
          cphot::KParams p;
          if ((rc = fill_params(seg, &d, p, true, out))) break;
          if (p.n == 0) break;
          LaunchShape sh;
          if (choose_shape(&d, p, cphot::MODE_PROPAGATE, sh) != CPHOT_OK) {
            rc = CPHOT_OK;  // shape not applicable (e.g. no window fits)
            continue;
          }
          {  // skip shapes that came out the same as one already timed
            const std::array<int, 6> key = {sh.grid, p.lds_hist, p.hist_w, p.hist_h, p.hist_x0, p.hist_y0};
            bool seen = false;
            for (const auto& k : tried) seen = seen || k == key;
            if (seen) continue;
            tried.push_back(key);
          }
          hipError_t e = clear_outputs(out, st);
          if (e == hipSuccess) e = cphot::launch_propagate(p, cphot::MODE_PROPAGATE, sh.block, sh.grid, sh.lds, st);
          if (e == hipSuccess) e = clear_outputs(out, st);
          if (e == hipSuccess) e = hipEventRecord(e0, st);
          for (int r = 0; r < reps && e == hipSuccess; ++r)
            e = cphot::launch_propagate(p, cphot::MODE_PROPAGATE, sh.block, sh.grid, sh.lds, st);
          if (e == hipSuccess) e = hipEventRecord(e1, st);
          if (e == hipSuccess) e = hipEventSynchronize(e1);
          float ms = 0.f;
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
          unsigned long long gen = 0;
          if (e == hipSuccess)
            e = hipMemcpy(&gen, out->counters + CPHOT_C_RECORDS_GENERATED, sizeof(gen), hipMemcpyDeviceToHost);
          if (e != hipSuccess) {
            rc = hip_fail(e, "autotune trial");
            break;
          }
          const double t = ms / reps;
          const double pps = (double)gen / reps * b / (t * 1e-3);
          if (pps > top.photons_per_s) {
            top.block_size = bs;
            // a persistent grid by library choice is reported with its block count
            top.grid_blocks = (d.grid_blocks == 0 && p.lds_hist && p.detector == CPHOT_DETECTOR_GRID) ? sh.grid
                                                                                                     : d.grid_blocks;
            top.lds_hist = d.lds_hist;
            top.hist_window = d.lds_hist ? p.hist_w : 0;
            top.hist_window_h = d.lds_hist ? p.hist_h : 0;
            top.hist_window_dx = d.lds_hist ? p.hist_x0 - (p.nx - p.hist_w) / 2 : 0;
            top.hist_window_dy = d.lds_hist ? p.hist_y0 - (p.ny - p.hist_h) / 2 : 0;
            top.bunch = b;
            top.ms = t;
            top.photons_per_s = pps;
          }
        }
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  *best = top;
  return CPHOT_OK;
}

}  // extern "C"

namespace {

// Process-wide cache of tuning results by configuration signature, optionally
// mirrored in text files (one "signature|fields" line per entry).
struct TuneCache {
  std::mutex mu;
  std::vector<std::pair<std::string, cphot_tuning>> entries;
  std::vector<std::string> files_read;
};
TuneCache& tune_cache() {
  static TuneCache c;
  return c;
}

// Everything the best launch shape can depend on, except the launch shape itself:
// device, atmosphere layout, detector settings, segment and shower counts, the
// candidate bunches and the number of timed launches.
std::string tune_signature(const cphot_segments* seg, const cphot_detector* det, const int32_t* bunches,
                           int32_t n_bunch, int32_t reps) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  hipDeviceProp_t prop;
  std::string name = "unknown";
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) name = prop.gcnArchName;
  const cphot_atmosphere_desc& a = det->atm->d;
  char buf[1024];
  std::snprintf(buf, sizeof(buf),
                "abi%d;%s;cu%d;atm%d,%d,%d,%.9g,%.9g,%.9g;t%d;d%d;s%d;e%d;c%d;cuts%d;b%d;h%.9g;g%d,%d,%.9g;"
                "sp%d,%d,%.9g,%.9g;nt%d,%.9g;eff%d;red%d;sur%d;tab%d;n%lld;ns%lld;reps%d;bunches",
                CPHOT_ABI_VERSION, name.c_str(), cu_count(dev), a.profile, a.n_layers, a.n_lambda_bins, a.h_top,
                a.lambda_min_nm, a.lambda_max_nm, det->transport, det->detector, det->spectrum, det->emission,
                det->counts_rule, det->cuts, det->bunch, det->h_obs, det->nx, det->ny, det->cell, det->snx,
                det->sny, det->pitch, det->radius, det->n_time_bins, det->time_bin_ns, det->efficiency != nullptr,
                det->reduction != nullptr, det->surrogate != nullptr, det->table != nullptr, (long long)seg->n,
                (long long)seg->n_showers, reps);
  std::string sig = buf;
  for (int i = 0; i < n_bunch; ++i) sig += "," + std::to_string(bunches[i]);
  return sig;
}

void read_tune_file(TuneCache& c, const char* path) {
  for (const std::string& f : c.files_read)
    if (f == path) return;
  c.files_read.push_back(path);
  FILE* fp = std::fopen(path, "r");
  if (!fp) return;  // no file yet
  char line[2048];
  while (std::fgets(line, sizeof(line), fp)) {
    char* bar = std::strchr(line, '|');
    if (!bar) continue;
    *bar = 0;
    cphot_tuning t{};
    if (std::sscanf(bar + 1, "%d %d %d %d %d %d %d %d %lf %lf", &t.block_size, &t.grid_blocks, &t.lds_hist,
                    &t.bunch, &t.hist_window, &t.hist_window_h, &t.hist_window_dx, &t.hist_window_dy, &t.ms,
                    &t.photons_per_s) != 10)
      continue;
    bool have = false;
    for (auto& e : c.entries) have = have || e.first == line;
    if (!have) c.entries.emplace_back(line, t);
  }
  std::fclose(fp);
}

}  // namespace

extern "C" {

int cphot_autotune_cached(const cphot_segments* seg, const cphot_detector* det, cphot_bins* out,
                          const int32_t* bunch_candidates, int32_t n_bunch, int32_t reps, const char* cache_path,
                          cphot_tuning* best, int32_t* hit, void* stream) {
  if (!seg || !det || !det->atm || !out || !best) return fail(CPHOT_ERR_INVALID_ARG, "null argument");
  if (n_bunch < 0 || (n_bunch > 0 && !bunch_candidates)) return fail(CPHOT_ERR_INVALID_ARG, "bad bunch list");
  const std::string sig = tune_signature(seg, det, bunch_candidates, n_bunch, reps);
  if (sig.find('|') != std::string::npos || sig.find('\n') != std::string::npos)
    return fail(CPHOT_ERR_INVALID_ARG, "device name unusable in a cache signature");
  TuneCache& c = tune_cache();
  {
    std::lock_guard<std::mutex> lock(c.mu);
    if (cache_path) read_tune_file(c, cache_path);
    for (auto& e : c.entries)
      if (e.first == sig) {
        *best = e.second;
        if (hit) *hit = 1;
        return CPHOT_OK;
      }
  }
  cphot_tuning t{};
  const int rc = cphot_autotune(seg, det, out, bunch_candidates, n_bunch, reps, &t, stream);
  if (rc) return rc;
  std::lock_guard<std::mutex> lock(c.mu);
  c.entries.emplace_back(sig, t);
  if (cache_path) {
    FILE* fp = std::fopen(cache_path, "a");
    if (!fp) return fail(CPHOT_ERR_INVALID_ARG, std::string("cannot append to the tuning cache ") + cache_path);
    std::fprintf(fp, "%s|%d %d %d %d %d %d %d %d %.17g %.17g\n", sig.c_str(), t.block_size, t.grid_blocks,
                 t.lds_hist, t.bunch, t.hist_window, t.hist_window_h, t.hist_window_dx, t.hist_window_dy, t.ms,
                 t.photons_per_s);
    std::fclose(fp);
  }
  *best = t;
  if (hit) *hit = 0;
  return CPHOT_OK;
}

void cphot_autotune_cache_clear(void) {
  TuneCache& c = tune_cache();
  std::lock_guard<std::mutex> lock(c.mu);
  c.entries.clear();
  c.files_read.clear();
}


int cphot_autotune_accuracy(const cphot_segments* seg, const cphot_detector* det, cphot_bins* out,
                            const int32_t* bunch_candidates, int32_t n_bunch, int32_t reps, double max_error,
                            double min_count, double* bin_errors, cphot_tuning* best, void* stream) {
  if (!seg || !det || !out || !best) return fail(CPHOT_ERR_INVALID_ARG, "null argument");
  if (n_bunch < 1 || !bunch_candidates) return fail(CPHOT_ERR_INVALID_ARG, "need at least one bunch candidate");
  if (!(max_error >= 0.0) || !(min_count >= 1.0) || !std::isfinite(max_error) || !std::isfinite(min_count))
    return fail(CPHOT_ERR_INVALID_ARG, "max_error must be >= 0 and min_count >= 1");
  if (!out->bins) return fail(CPHOT_ERR_INVALID_ARG, "the bunch check compares bins: bins required");
  for (int i = 0; i < n_bunch; ++i)
    if (bunch_candidates[i] < 1) return fail(CPHOT_ERR_INVALID_ARG, "bunch candidates must be >= 1");
  hipStream_t st = (hipStream_t)stream;
  // bins of one propagation with bunch b, as doubles on the host
  const int64_t nb = out->bins_capacity;
  auto bins_of = [&](int32_t b, std::vector<double>& h) -> int {
    cphot_detector d = *det;
    d.bunch = b;
    hipError_t ce = clear_outputs(out, st);
    if (ce != hipSuccess) return hip_fail(ce, "bunch check clear");
    int rc = cphot_propagate(seg, &d, out, st);
    if (rc) return rc;
    h.assign((size_t)nb, 0.0);
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "bunch check");
    if (out->bins_dtype == CPHOT_BINS_F64) {
      e = hipMemcpy(h.data(), out->bins, (size_t)nb * 8, hipMemcpyDeviceToHost);
    } else if (out->bins_dtype == CPHOT_BINS_U64) {
      std::vector<unsigned long long> t((size_t)nb);
      e = hipMemcpy(t.data(), out->bins, (size_t)nb * 8, hipMemcpyDeviceToHost);
      for (int64_t i = 0; i < nb; ++i) h[(size_t)i] = (double)t[(size_t)i];
    } else {
      std::vector<uint32_t> t((size_t)nb);
      e = hipMemcpy(t.data(), out->bins, (size_t)nb * 4, hipMemcpyDeviceToHost);
      for (int64_t i = 0; i < nb; ++i) h[(size_t)i] = (double)t[(size_t)i];
    }
    return e == hipSuccess ? CPHOT_OK : hip_fail(e, "bunch check copy");
  };
  std::vector<double> ref, cur;
  int rc = bins_of(1, ref);
  if (rc) return rc;
  std::vector<int32_t> ok;
  for (int i = 0; i < n_bunch; ++i) {
    const int32_t b = bunch_candidates[i];
    double err = 0.0;
    if (b != 1) {
      if ((rc = bins_of(b, cur))) return rc;
      for (size_t c = 0; c < ref.size(); ++c)
        if (ref[c] >= min_count) err = std::max(err, std::fabs(cur[c] - ref[c]) / ref[c]);
    }
    if (bin_errors) bin_errors[i] = err;
    if (err <= max_error) ok.push_back(b);
  }
  if (ok.empty()) ok.push_back(1);  // the finest statistics are the reference: always admissible
  return cphot_autotune(seg, det, out, ok.data(), (int32_t)ok.size(), reps, best, stream);
}

}  // extern "C"
