// Correction table of the interpolation tracing (Sec. 4.4.1): built once per
// atmosphere and observation level from the exact walk in FP64, looked up
// bilinearly per photon in the propagation kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "cphot_internal.h"
#include "cphot_walk64.h"

struct cphot_table {
  cphot_table_desc d;
  const cphot_atmosphere* atm = nullptr;
  int device = 0;
  float4* data = nullptr;
  cphot::TableView view{};
};

namespace cphot {
namespace {

struct BuildParams {
  const float4* layers;
  int n_layers;
  double dh, h_obs, Re;
  TableView v;
  float4* out;
};

// One node per thread: the exact walk from (h, c) in layer li compared with the
// straight path (planar) or chord (curved), absolute.
__global__ __launch_bounds__(256) void k_table_build(BuildParams p) {
  const TableView& v = p.v;
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= v.m * v.n_rows * v.n_c) return;
  const int kk = k % v.m, r = (k / v.m) % v.n_rows, j = k / (v.m * v.n_rows);
  const int li = v.layer0 + r;
  const double lower = r == 0 ? p.h_obs : li * p.dh, upper = (li + 1) * p.dh;
  const double h = lower + (upper - lower) * kk / (double)(v.m - 1);
  const double tz = j / (double)v.inv_dt;
  const double c = 1.0 / sqrt(1.0 + tz * tz);
  Walk64 w;
  float4 res;
  if (!(h > p.h_obs)) {  // start on the observation level: nothing to correct
    p.out[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }
  if (v.geometry == CPHOT_SURROGATE_CURVED) {
    double L, psi_s;
    chord_f64(p.Re, p.h_obs, h, c, L, psi_s);
    if (!shell_walk_f64(p.layers, p.dh, p.n_layers, p.h_obs, p.Re, h, c, w, li)) {
      const float q = __builtin_nanf("");
      p.out[k] = make_float4(q, q, q, q);
      return;
    }
    res.x = (float)((w.across - psi_s) * (p.Re + p.h_obs));
    res.y = (float)((w.len - L) + w.opt);
  } else {
    planar_walk_f64(p.layers, p.dh, p.n_layers, p.h_obs, h, c, w, li);
    const double L = (h - p.h_obs) / c;
    const double s0 = sqrt((1.0 - c) * (1.0 + c));
    res.x = (float)(w.across - L * s0);
    res.y = (float)((w.len - L) + w.opt);
  }
  res.z = (float)w.tR;
  res.w = (float)w.tA;
  p.out[k] = res;
}

struct LookupParams {
  TableView v;
  const float2* lambins;
  int n_lam, n_layers;
  float lam_min, lam_max;
  double h_obs, Re;
  const float* X;
  float* Y;
  int64_t n;
};

__global__ __launch_bounds__(256) void k_table_lookup(LookupParams p) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= p.n) return;
  const float* x = p.X + 5 * j;
  float* y = p.Y + 4 * j;
  const float h = x[0], c = x[1], lam = x[3];
  const int li = p.v.geometry == CPHOT_SURROGATE_CURVED ? min((int)(h / p.v.dh), p.n_layers - 1)
                                                        : min((int)(h * p.v.inv_dh), p.n_layers - 1);
  float4 v;
  const float tz = sqrtf(fmaxf((1.0f - c) * (1.0f + c), 0.f)) / c;
  if (!(h >= p.v.h_obs) || !(c > 0.f) || !table_lookup(p.v, li, h, tz, v)) {
    const float q = __builtin_nanf("");
    y[0] = y[1] = y[2] = y[3] = q;
    return;
  }
  int kb = (int)((lam - p.lam_min) * ((float)p.n_lam / (p.lam_max - p.lam_min)));
  kb = min(max(kb, 0), p.n_lam - 1);
  const float2 sp = p.lambins[kb];
  y[0] = v.x;
  y[1] = 0.f;
  y[2] = v.y;
  y[3] = -fmaf(v.z, sp.x, v.w * sp.y);
}

}  // namespace

TableView table_view(const cphot_table* t) { return t ? t->view : TableView{}; }
const cphot_atmosphere* table_atmosphere(const cphot_table* t) { return t ? t->atm : nullptr; }
double table_h_obs(const cphot_table* t) { return t ? t->d.h_obs : -1.0; }

}  // namespace cphot

extern "C" {

void cphot_table_destroy(cphot_table* t) {
  if (!t) return;
  if (t->data) (void)hipFree(t->data);
  delete t;
}

int cphot_table_create(const cphot_table_desc* desc, const cphot_atmosphere* atm, cphot_table** out) {
  if (!desc || !atm || !out) {
    cphot::set_last_error("null argument");
    return CPHOT_ERR_INVALID_ARG;
  }
  *out = nullptr;
  auto bad = [](const char* m) {
    cphot::set_last_error(m);
    return CPHOT_ERR_INVALID_ARG;
  };
  const float4* layers;
  const float2* lambins;
  int n_layers, n_lam;
  float dh, lam_min, lam_max;
  if (cphot::atmosphere_layer_view(atm, &layers, &lambins, &n_layers, &n_lam, &dh, &lam_min, &lam_max))
    return bad("the table is built on a layered atmosphere (n_layers > 0)");
  const double h_top = (double)dh * n_layers;
  if (desc->geometry != CPHOT_SURROGATE_PLANAR && desc->geometry != CPHOT_SURROGATE_CURVED)
    return bad("unknown table geometry");
  if (desc->n_h < 2 || desc->n_c < 2 || (int64_t)desc->n_h * desc->n_c * n_layers > (int64_t(1) << 26))
    return bad("table needs 2 <= n_h (nodes per layer), 2 <= n_c and n_h * n_c * n_layers <= 2^26");
  if (!(desc->h_obs >= 0.0 && desc->h_obs < h_top)) return bad("h_obs must lie in [0, h_top)");
  if (!(desc->h_hi > desc->h_obs && desc->h_hi <= h_top)) return bad("h_hi must lie in (h_obs, h_top]");
  if (!(desc->c_lo > 0.0 && desc->c_lo < 1.0)) return bad("c_lo must lie in (0, 1)");
  const double Re = cphot::atmosphere_earth_radius(atm);
  if (desc->geometry == CPHOT_SURROGATE_CURVED && !(Re > 1e5 && std::isfinite(Re)))
    return bad("a curved table needs the atmosphere's earth_radius");
  cphot_table* t = new (std::nothrow) cphot_table();
  if (!t) {
    cphot::set_last_error("host allocation");
    return CPHOT_ERR_OUT_OF_MEMORY;
  }
  t->d = *desc;
  t->atm = atm;
  (void)hipGetDevice(&t->device);
  const size_t nodes = (size_t)desc->n_h * desc->n_c *
                       (std::min((int)std::floor(desc->h_hi / dh), n_layers - 1) - (int)std::floor(desc->h_obs / dh) + 1);
  hipError_t e = hipMalloc((void**)&t->data, nodes * sizeof(float4));
  if (e != hipSuccess) {
    cphot_table_destroy(t);
    cphot::set_last_error("table allocation");
    return e == hipErrorOutOfMemory ? CPHOT_ERR_OUT_OF_MEMORY : CPHOT_ERR_HIP;
  }
  // heights: layer by layer from the observation layer to the one containing
  // h_hi, n_h nodes each; cos zenith: n_c nodes on [c_lo, 1]
  const int layer0 = (int)std::floor(desc->h_obs / dh);
  const int top = std::min((int)std::floor(desc->h_hi / dh), n_layers - 1);
  cphot::TableView& v = t->view;
  v.data = t->data;
  v.m = desc->n_h;
  v.layer0 = layer0;
  v.n_rows = top - layer0 + 1;
  v.n_c = desc->n_c;
  v.dh = dh;
  v.inv_dh = (float)(n_layers / h_top);
  v.h_obs = (float)desc->h_obs;
  v.inv_dt = (float)((desc->n_c - 1) / (std::sqrt((1.0 - desc->c_lo) * (1.0 + desc->c_lo)) / desc->c_lo));
  v.geometry = desc->geometry;
  cphot::BuildParams bp;
  bp.layers = layers;
  bp.n_layers = n_layers;
  bp.dh = (double)dh;
  bp.h_obs = desc->h_obs;
  bp.Re = Re;
  bp.v = v;
  bp.out = t->data;
  hipLaunchKernelGGL(cphot::k_table_build, dim3((unsigned)((nodes + 255) / 256)), dim3(256), 0, nullptr, bp);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    cphot_table_destroy(t);
    cphot::set_last_error(std::string("table build: ") + hipGetErrorString(e));
    return CPHOT_ERR_HIP;
  }
  *out = t;
  return CPHOT_OK;
}

int cphot_table_lookup(const cphot_table* t, const cphot_atmosphere* atm, const float* X, float* Y, int64_t n,
                       void* stream) {
  if (!t || !atm || n < 0 || (n > 0 && (!X || !Y))) {
    cphot::set_last_error("null table, atmosphere or buffers, or negative n");
    return CPHOT_ERR_INVALID_ARG;
  }
  if (n == 0) return CPHOT_OK;
  cphot::LookupParams p;
  std::memset(&p, 0, sizeof(p));
  const float4* layers;
  int n_layers;
  float dh;
  if (cphot::atmosphere_layer_view(atm, &layers, &p.lambins, &n_layers, &p.n_lam, &dh, &p.lam_min, &p.lam_max)) {
    cphot::set_last_error("layered atmosphere required");
    return CPHOT_ERR_INVALID_ARG;
  }
  p.n_layers = n_layers;
  p.v = t->view;
  p.h_obs = t->d.h_obs;
  p.Re = cphot::atmosphere_earth_radius(atm);
  p.X = X;
  p.Y = Y;
  p.n = n;
  hipLaunchKernelGGL(cphot::k_table_lookup, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    cphot::set_last_error(std::string("table lookup: ") + hipGetErrorString(e));
    return CPHOT_ERR_HIP;
  }
  return CPHOT_OK;
}

}  // extern "C"
