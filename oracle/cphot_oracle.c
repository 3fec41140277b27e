/*
 * cphot_oracle.c -- plain, slow FP64 CPU oracle for Cherenkov photon generation
 * and atmospheric propagation (D. Baack, "Optical Photon Emission in Extended
 * Airshowers", arXiv 2405.04229).
 *
 * TEST INFRASTRUCTURE ONLY. Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library. It shares no code,
 * header, table or constant generator with the HIP library; both sides are
 * driven by the same seeded inputs and the same counter-based random words,
 * so every photon can be compared one to one.
 *
 * Every function follows the thesis step by step in FP64 with no blocking,
 * fusion or reordering. Readings taken where the thesis is silent or garbled
 * are stated next to the step. Build with -ffp-contract=off: the integer photon
 * count per segment is decided by floating point and must come out identical
 * to the GPU's.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846
#define ORC_ALPHA (1.0 / 137.035999084)  /* fine-structure constant, CODATA 2018 */
#define ORC_C_M_PER_NS 0.299792458

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), the counter-based      */
/* generator family the thesis adopts for reproducible, race-free streams    */
/* (Sec. 3.1). Written from the published round definition.                   */
/* ------------------------------------------------------------------------- */
void orc_philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Random word -> uniform on [0,1) with 24 bits, exactly representable in FP32. */
static double u24(uint32_t w) { return (double)(w >> 8) * (1.0 / 16777216.0); }
/* Random word -> uniform on [0,1) with 32 bits (segment count rounding). */
static double u32d(uint32_t w) { return (double)w * (1.0 / 4294967296.0); }

enum { TAG_SEGMENT = 0, TAG_CHERENKOV = 1, TAG_FLUOR = 2, TAG_TRAIN = 8, TAG_POISSON = 12 };

static void draw(uint64_t seed, uint32_t k, uint64_t seg, uint32_t tag, uint32_t out[4]) {
  uint32_t ctr[4] = {k, (uint32_t)seg, (uint32_t)(seg >> 32), tag};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  orc_philox(ctr, key, out);
}

/* ------------------------------------------------------------------------- */
/* Atmosphere (Sec. 2.3.1, 3.3, 4.1)                                          */
/* ------------------------------------------------------------------------- */
enum { PROFILE_LINSLEY5 = 0, PROFILE_HOMOGENEOUS = 1, PROFILE_LINEAR = 2 };

typedef struct {
  int32_t profile;
  int32_t n_layers;        /* equal homogeneous layers on [0, h_top) */
  double a[5], b[5], c[5]; /* Linsley X(h) = a + b exp(-h/c), c in cm */
  double hb[5];            /* layer lower bounds, m */
  double kappa;            /* n - 1 = kappa rho / rho(0) */
  double delta0;           /* homogeneous: n - 1; linear: n - 1 at h = 0 */
  double h_top;            /* m */
  double step;             /* refractivity table spacing, m */
  double rayleigh400;      /* Rayleigh attenuation length at 400 nm, g/cm^2 (0: none) */
  double aer_tau350;       /* vertical aerosol optical depth at 350 nm (0: none) */
  double aer_H;            /* aerosol scale height, m */
  double aer_angstrom;     /* aerosol wavelength exponent */
  double lam_min, lam_max; /* nm */
  int32_t n_lam;           /* wavelength bins of the layer absorption table */
  int32_t pad;
  double earth_radius;     /* m */
} orc_atmo_params;

typedef struct {
  orc_atmo_params p;
  double rho0;
  int64_t n_tab;  /* entries 0..n_tab */
  double* tab;
  double* layer_delta; /* n_layers */
  double* layer_ext;   /* n_layers * n_lam, extinction per metre */
} orc_atmo;

static int linsley_layer(const orc_atmo_params* p, double h) {
  int i = 0;
  while (i < 4 && h >= p->hb[i + 1]) ++i;
  return i;
}

/* Vertical depth X(h) in g/cm^2 (Linsley parametrisation). */
double orc_depth(const orc_atmo* A, double h) {
  const orc_atmo_params* p = &A->p;
  int i = linsley_layer(p, h);
  double hcm = h * 100.0;
  if (i < 4) return p->a[i] + p->b[i] * exp(-hcm / p->c[i]);
  return p->a[4] - p->b[4] * hcm / p->c[4];
}

/* Density rho(h) = -dX/dh in g/cm^3. */
double orc_density(const orc_atmo* A, double h) {
  const orc_atmo_params* p = &A->p;
  int i = linsley_layer(p, h);
  if (i < 4) return (p->b[i] / p->c[i]) * exp(-(h * 100.0) / p->c[i]);
  return p->b[4] / p->c[4];
}

/* Refractivity n - 1 from the closed-form profile. The thesis works with the
 * reduced refractive index n - 1 following density (Sec. 2.3.1, 5.2). */
double orc_delta_closed(const orc_atmo* A, double h) {
  const orc_atmo_params* p = &A->p;
  if (p->profile == PROFILE_HOMOGENEOUS) return p->delta0;
  if (p->profile == PROFILE_LINEAR) {
    if (h >= p->h_top) return 0.0;
    if (h < 0.0) h = 0.0;
    return p->delta0 * (1.0 - h / p->h_top);
  }
  return p->kappa * (orc_density(A, h) / A->rho0);
}

/* Constant-time lookup in the 1 m table by direct index mapping and linear
 * interpolation between neighbours (Sec. 4.1, Eq. 4.1). Heights outside the
 * table are clamped to its ends (the thesis assumes in-range heights). */
double orc_delta_table(const orc_atmo* A, double h) {
  double x = h / A->p.step;
  if (x < 0.0) x = 0.0;
  if (x > (double)A->n_tab) x = (double)A->n_tab;
  double fi = floor(x);
  int64_t idx = (int64_t)fi;
  if (idx > A->n_tab - 1) { idx = A->n_tab - 1; fi = (double)idx; }
  double frac = x - fi;
  return (1.0 - frac) * A->tab[idx] + frac * A->tab[idx + 1];
}

/* Integral of n - 1 over height between h_lo and h_hi (m * 1). */
static double delta_integral(const orc_atmo* A, double h_lo, double h_hi) {
  const orc_atmo_params* p = &A->p;
  if (p->profile == PROFILE_HOMOGENEOUS) return p->delta0 * (h_hi - h_lo);
  if (p->profile == PROFILE_LINEAR) {
    double lo = h_lo < 0 ? 0 : (h_lo > p->h_top ? p->h_top : h_lo);
    double hi = h_hi < 0 ? 0 : (h_hi > p->h_top ? p->h_top : h_hi);
    double F_hi = hi - hi * hi / (2.0 * p->h_top);
    double F_lo = lo - lo * lo / (2.0 * p->h_top);
    return p->delta0 * (F_hi - F_lo);
  }
  /* Linsley: integral of kappa rho/rho0 dh = kappa/rho0 * (X(lo) - X(hi)) / 100 */
  return p->kappa / A->rho0 * (orc_depth(A, h_lo) - orc_depth(A, h_hi)) / 100.0;
}

static double rayleigh_length(const orc_atmo* A, double lam_nm) {
  double r = lam_nm / 400.0;
  return A->p.rayleigh400 * r * r * r * r;
}

static double aerosol_tau(const orc_atmo* A, double lam_nm) {
  return A->p.aer_tau350 * pow(lam_nm / 350.0, -A->p.aer_angstrom);
}

/* Vertical optical depth between heights lo < hi at wavelength lam. */
static double vertical_tau(const orc_atmo* A, double lo, double hi, double lam) {
  double tau = 0.0;
  if (A->p.rayleigh400 > 0.0) tau += (orc_depth(A, lo) - orc_depth(A, hi)) / rayleigh_length(A, lam);
  if (A->p.aer_tau350 > 0.0)
    tau += aerosol_tau(A, lam) * (exp(-lo / A->p.aer_H) - exp(-hi / A->p.aer_H));
  return tau;
}

int orc_atmo_create(const orc_atmo_params* p, orc_atmo** out) {
  if (p->step <= 0 || p->h_top <= 0) return -1;
  if (p->profile != PROFILE_LINSLEY5 && p->rayleigh400 > 0) return -1;
  orc_atmo* A = (orc_atmo*)calloc(1, sizeof(orc_atmo));
  A->p = *p;
  A->rho0 = p->b[0] / p->c[0];
  A->n_tab = (int64_t)ceil(p->h_top / p->step);
  A->tab = (double*)malloc(sizeof(double) * (size_t)(A->n_tab + 1));
  for (int64_t j = 0; j <= A->n_tab; ++j) A->tab[j] = orc_delta_closed(A, (double)j * p->step);
  if (p->n_layers > 0) {
    int L = p->n_layers;
    double dh = p->h_top / L;
    A->layer_delta = (double*)malloc(sizeof(double) * (size_t)L);
    A->layer_ext = (double*)calloc((size_t)L * (size_t)(p->n_lam > 0 ? p->n_lam : 1), sizeof(double));
    for (int i = 0; i < L; ++i) {
      double lo = i * dh, hi = (i + 1) * dh;
      A->layer_delta[i] = orc_delta_closed(A, 0.5 * (lo + hi));
      for (int k = 0; k < p->n_lam; ++k) {
        double lam = p->lam_min + (k + 0.5) * (p->lam_max - p->lam_min) / p->n_lam;
        A->layer_ext[(size_t)i * p->n_lam + k] = vertical_tau(A, lo, hi, lam) / dh;
      }
    }
  }
  *out = A;
  return 0;
}

void orc_atmo_free(orc_atmo* A) {
  if (!A) return;
  free(A->tab); free(A->layer_delta); free(A->layer_ext); free(A);
}

void orc_layer_tables(const orc_atmo* A, double* delta_out, double* ext_out) {
  int L = A->p.n_layers, K = A->p.n_lam;
  for (int i = 0; i < L; ++i) delta_out[i] = A->layer_delta[i];
  for (int i = 0; i < L * K; ++i) ext_out[i] = A->layer_ext[i];
}

/* ------------------------------------------------------------------------- */
/* Run description                                                            */
/* ------------------------------------------------------------------------- */
enum { TRANSPORT_STRAIGHT = 0, TRANSPORT_LAYERED = 1, TRANSPORT_CURVED = 2 };
enum { EMIT_CHERENKOV = 1, EMIT_FLUORESCENCE = 2 };
enum { DETECTOR_GRID = 0, DETECTOR_SPHERES = 1 };
enum { SPECTRUM_UNIFORM = 0, SPECTRUM_FRANK_TAMM = 1, SPECTRUM_DISPERSIVE = 2 };

typedef struct {
  int32_t transport, detector, spectrum, bunch;
  uint64_t seed;
  double h_obs;
  int32_t nx, ny;       /* ground grid cells */
  double cell;          /* m */
  int32_t snx, sny;     /* sphere grid */
  double pitch, radius; /* m */
  int32_t n_t;          /* time bins per sphere (+1 overflow) */
  int32_t counts_rule;  /* 0: stochastic rounding of mu, 1: Poisson(mu) */
  double dt;            /* ns */
  int32_t emission;     /* bit 0: Cherenkov, bit 1: fluorescence */
  int32_t pad2;
  double fl_yield[3];   /* fluorescence photons per MeV deposited, per band */
  double fl_lambda[3];  /* band wavelengths, nm */
  /* detector efficiency per wavelength bin of the atmosphere (NULL: 1) and the
   * pre-emission reduction bound per layer (NULL: none), Sec. 4.3.1 */
  const double* efficiency;
  const double* reduction;
  double lambda_ref;    /* dispersive spectrum: wavelength (nm) at which the atmosphere's n - 1 holds */
} orc_run;

enum { ST_BINNED = 0, ST_UPWARD = 1, ST_ABSORBED = 2, ST_OUTSIDE = 3, ST_NOT_EMITTED = 4 };

typedef struct {
  int64_t seg;
  int32_t k, state;    /* k: record index within the segment (Cherenkov first, then the bands) */
  int32_t bin, tbin;
  double x, y, z;       /* arrival point: ground or sphere entry */
  double t;             /* ns after the plane front */
  double tau;           /* optical depth */
  double lambda;        /* nm */
  double u_abs;         /* survival uniform */
  double margin;        /* distance of the arrival point to the nearest bin edge, m */
  double tmargin;       /* distance of t to the nearest time-bin edge, ns */
  double ex, ey, ez;    /* emission point */
  double dx, dy, dz;    /* emission direction */
  int32_t source;       /* 0 Cherenkov, 1 + b fluorescence band b */
  int32_t pad;
  double p_emit;        /* dispersive spectrum: probability that the record is emitted (else 1) */
} orc_photon;

typedef struct {
  int32_t n;      /* Cherenkov records drawn */
  int32_t status; /* 0 ok, 1 below the Cherenkov threshold, 2 skipped (non-finite/degenerate/invalid beta) */
  double mu;      /* expected Cherenkov records */
  double cos_t, sin2_t;
  int32_t nf[3];  /* fluorescence records per band */
  int32_t pad;
  double muf[3];  /* expected fluorescence records per band */
  double q;       /* pre-emission reduction factor (1 without reduction) */
} orc_segment;

typedef struct { double core_x, core_y, ax, ay, az; } orc_geom;

/* ------------------------------------------------------------------------- */
/* Segment yield (Sec. 2.2.1, Eq. 2.2-2.4 and the track integral with the    */
/* Heaviside step)                                                            */
/* ------------------------------------------------------------------------- */
typedef struct {
  double S[3], E[3], L, beta, z2;
  double cos_t, sin_t, sin2;
  double delta_mid; /* n - 1 at the midpoint, at the reference wavelength (dispersive spectrum) */
  double M[3][3]; /* rotation taking the cone axis (0,0,-1) onto the track direction */
} seg_setup;

/* exp(-x), 0 <= x <= 64, from IEEE basic operations only (the count decisions
 * depend on it, so it must not vary with the C library): write x = k ln2 + r with
 * ln2 = L1 + L2, L1 carrying 29 significant bits so that k L1 is exact (the
 * reduction of Cody and Waite); exp(-r) = sum_{j=0}^{14} (-r)^j / j! (the first
 * omitted term is below 2e-19 for |r| <= ln2/2); exp(-x) = 2^-k exp(-r). */
static double exp_neg_basic(double x) {
  static const double L1 = 0x1.62e42ffp-1;         /* ln2 rounded to 29 bits */
  static const double L2 = -0x1.718432a1b0e26p-35; /* ln2 - L1 */
  static const double INV_LN2 = 0x1.71547652b82fep+0;
  static const double inv_fact[15] = {
      1.0, 1.0, 0.5, 0x1.5555555555555p-3, 0x1.5555555555555p-5, 0x1.1111111111111p-7,
      0x1.6c16c16c16c17p-10, 0x1.a01a01a01a01ap-13, 0x1.a01a01a01a01ap-16, 0x1.71de3a556c734p-19,
      0x1.27e4fb7789f5cp-22, 0x1.ae64567f544e4p-26, 0x1.1eed8eff8d898p-29, 0x1.6124613a86d09p-33,
      0x1.93974a8c07c9dp-37};
  double k = floor(x * INV_LN2 + 0.5);
  double r = (x - k * L1) - k * L2;
  double t = -r;
  double sum = inv_fact[14];
  for (int j = 13; j >= 0; --j) sum = sum * t + inv_fact[j];
  return ldexp(sum, -(int)k);
}

/* Poisson-distributed record count with mean mu (< 2^20), the alternative to
 * stochastic rounding (Sec. 2.2.1; a Poisson number of emissions per segment).
 * Inversion: the smallest n with u < P(N <= n), the probabilities built as
 * p_0 = e^-m, p_n = p_{n-1} m / n; for large means the count is a sum over equal
 * chunks of mean m = mu / ceil(mu / 64) (sums of independent Poisson counts are
 * Poisson), the first chunk using the segment's word w0 and chunk c > 0 word 0 of
 * the Philox block (c, id, tag). */
static int64_t poisson_draw(double mu, uint32_t w0, uint64_t seed, uint64_t seg_id, uint32_t tag) {
  if (!(mu > 0.0)) return 0;
  int64_t chunks = (int64_t)ceil(mu / 64.0);
  double m = mu / (double)chunks;
  double e = exp_neg_basic(m);
  int64_t total = 0;
  for (int64_t c = 0; c < chunks; ++c) {
    uint32_t word = w0;
    if (c > 0) {
      uint32_t w[4];
      draw(seed, (uint32_t)c, seg_id, tag, w);
      word = w[0];
    }
    double u = u32d(word);
    double p = e, F = e;
    int64_t n = 0;
    while (u >= F && n < 4096) {
      n = n + 1;
      p = p * m / (double)n;
      F = F + p;
    }
    total += n;
  }
  return total;
}

/* Dispersion of air: 1e8 (n - 1) of standard air at lambda nm, the two-term
 * formula of Ciddor (Appl. Opt. 35 (1996) 1566), wavenumber s in 1/um. Only its
 * ratio between two wavelengths is used: n(lambda, h) - 1 = (n(h) - 1) x
 * R(lambda) / R(lambda_ref), so the height profile keeps its own scale. */
static double air_dispersion_sum(double lambda_nm) {
  double s = 1000.0 / lambda_nm;
  double s2 = s * s;
  return 5792105.0 / (238.0185 - s2) + 167917.0 / (57.362 - s2);
}

static double frank_tamm_K(double lam_min_nm, double lam_max_nm) {
  /* integral over lambda of 2 pi alpha / lambda^2, lambda in metres */
  double l1 = lam_min_nm * 1e-9, l2 = lam_max_nm * 1e-9;
  return 2.0 * ORC_PI * ORC_ALPHA * (1.0 / l1 - 1.0 / l2);
}

/* Fills `st` and returns the segment record. The count is the expected number
 * of records mu = K z^2 L sin^2(theta) / bunch, rounded stochastically:
 * N = floor(mu) + [u < mu - floor(mu)]. The thesis computes the number of
 * photons from the yield rather than sampling it (Sec. 4.2); this rounding is
 * the reading that keeps the mean and needs only IEEE basic operations. */
static orc_segment segment_setup(const orc_atmo* A, const orc_run* R, double K,
                                 float x0, float y0, float z0, float x1, float y1, float z1,
                                 float beta_f, float charge_f, float dedx_f, uint64_t seg_id, seg_setup* st) {
  orc_segment out;
  memset(&out, 0, sizeof(out));
  int emit = R->emission ? R->emission : EMIT_CHERENKOV;
  int fluor = (emit & EMIT_FLUORESCENCE) != 0;
  if (!isfinite(x0) || !isfinite(y0) || !isfinite(z0) || !isfinite(x1) || !isfinite(y1) ||
      !isfinite(z1) || !isfinite(beta_f) || !isfinite(charge_f) || (fluor && !isfinite(dedx_f))) {
    out.status = 2;
    return out;
  }
  double beta = (double)beta_f;
  if (!(beta > 0.0 && beta < 1.0)) { out.status = 2; return out; }
  double dx = (double)x1 - (double)x0, dy = (double)y1 - (double)y0, dz = (double)z1 - (double)z0;
  double L = sqrt(dx * dx + dy * dy + dz * dz);
  if (!(L > 0.0)) { out.status = 2; return out; }
  /* Pre-emission reduction (Sec. 4.3.1): the expected numbers of records are
   * multiplied by an upper bound q of the detection probability of any photon
   * the segment can emit -- the bound of the layer holding its lowest point --
   * and every record later survives with probability (detection probability)/q,
   * so the expected detections are unchanged while fewer records are drawn. The
   * bound is input data (per layer), like the atmosphere's parameters. */
  double q = 1.0;
  if (R->reduction) {
    double hmin = (double)z0 < (double)z1 ? (double)z0 : (double)z1;
    double x = hmin / (A->p.h_top / A->p.n_layers);
    if (x < 0.0) x = 0.0;
    int64_t li = (int64_t)floor(x);
    if (li > A->p.n_layers - 1) li = A->p.n_layers - 1;
    q = R->reduction[li];
  }
  out.q = q;
  /* one Philox block per segment: word 0 rounds the Cherenkov yield, words
   * 1..3 the three fluorescence bands */
  uint32_t w[4];
  draw(R->seed, 0u, seg_id, TAG_SEGMENT, w);
  if (emit & EMIT_CHERENKOV) {
    /* refractivity at the segment midpoint from the 1 m table */
    double hm = 0.5 * ((double)z0 + (double)z1);
    double delta = orc_delta_table(A, hm);
    st->delta_mid = delta;
    /* Dispersion (Sec. 2.2.1: the threshold and the yield depend on the
     * wavelength through n(lambda, l)): the records are drawn for the largest
     * cone -- n at the shortest wavelength, where air refracts most -- and each
     * record is later emitted with the ratio of its own sin^2(theta) to that
     * cone's, which integrates the Frank-Tamm density with its Heaviside factor. */
    if (R->spectrum == SPECTRUM_DISPERSIVE)
      delta = delta * (air_dispersion_sum(A->p.lam_min) / air_dispersion_sum(R->lambda_ref));
    /* threshold beta n > 1, with g = beta n - 1 written through eps = 1 - beta */
    double eps = 1.0 - beta;
    double g = delta - eps - eps * delta;
    if (!(g > 0.0)) {
      out.status = 1;
    } else {
      /* sin^2(theta) = 1 - 1/(beta n)^2 (Eq. 2.3, 2.4) */
      double s2 = g * (g + 2.0) / ((1.0 + g) * (1.0 + g));
      double z2 = (double)charge_f * (double)charge_f;
      double mu = K * z2;
      mu = mu * L;
      mu = mu * s2;
      mu = mu / (double)R->bunch;
      /* A segment asking for 2^20 records or more (or a non-finite yield) is
       * rejected as invalid input rather than truncated. */
      if (!(mu < 1048576.0)) { memset(&out, 0, sizeof(out)); out.status = 2; return out; }
      mu = mu * q;
      if (R->counts_rule == 1) {
        int64_t n = poisson_draw(mu, w[0], R->seed, seg_id, TAG_POISSON);
        if (n >= 1048576) { memset(&out, 0, sizeof(out)); out.status = 2; return out; }
        out.n = (int32_t)n;
      } else {
        double fl = floor(mu);
        out.n = (int32_t)fl + (u32d(w[0]) < mu - fl ? 1 : 0);
      }
      out.mu = mu; out.cos_t = 1.0 / (1.0 + g); out.sin2_t = s2;
    }
  }
  if (fluor && dedx_f > 0.0f) {
    /* fluorescence yield per band (Eq. 2.6 folded into a per-band photons/MeV
     * constant), emitted into the lower hemisphere only (Sec. 4.2.2), hence 1/2 */
    for (int b = 0; b < 3; ++b) {
      double mu = R->fl_yield[b] * (double)dedx_f;
      mu = mu * L;
      mu = mu * 0.5;
      mu = mu / (double)R->bunch;
      if (!(mu < 1048576.0)) { memset(&out, 0, sizeof(out)); out.status = 2; return out; }
      mu = mu * q;
      if (R->counts_rule == 1) {
        int64_t n = poisson_draw(mu, w[1 + b], R->seed, seg_id, TAG_POISSON + 1 + (uint32_t)b);
        if (n >= 1048576) { memset(&out, 0, sizeof(out)); out.status = 2; return out; }
        out.nf[b] = (int32_t)n;
      } else {
        double fl = floor(mu);
        out.nf[b] = (int32_t)fl + (u32d(w[1 + b]) < mu - fl ? 1 : 0);
      }
      out.muf[b] = mu;
    }
  }
  st->S[0] = x0; st->S[1] = y0; st->S[2] = z0;
  st->E[0] = x1; st->E[1] = y1; st->E[2] = z1;
  st->L = L; st->beta = beta; st->z2 = (double)charge_f * (double)charge_f;
  st->cos_t = out.cos_t; st->sin_t = sqrt(out.sin2_t); st->sin2 = out.sin2_t;
  /* Rotation of the cone axis D = (0,0,-1) onto the track direction P by the
   * 180-degree Euler-Rodrigues rotation about the normalised bisector
   * A = (D + P)/|D + P| (Sec. 4.2, M = 1 + 2 R^2). The thesis leaves A
   * unnormalised; the matrix needs |A| = 1. When P is (nearly) opposite to D
   * the bisector vanishes; then the 180-degree turn about the x axis is used. */
  double P[3] = {dx / L, dy / L, dz / L};
  if (1.0 - P[2] < 1e-6) {
    double Md[3][3] = {{1, 0, 0}, {0, -1, 0}, {0, 0, -1}};
    memcpy(st->M, Md, sizeof(Md));
  } else {
    double a[3] = {P[0], P[1], P[2] - 1.0};
    double na = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    a[0] /= na; a[1] /= na; a[2] /= na;
    st->M[0][0] = -2.0 * a[1] * a[1] - 2.0 * a[2] * a[2] + 1.0;
    st->M[0][1] = 2.0 * a[0] * a[1];
    st->M[0][2] = 2.0 * a[0] * a[2];
    st->M[1][0] = 2.0 * a[0] * a[1];
    st->M[1][1] = -2.0 * a[0] * a[0] - 2.0 * a[2] * a[2] + 1.0;
    st->M[1][2] = 2.0 * a[1] * a[2];
    st->M[2][0] = 2.0 * a[0] * a[2];
    st->M[2][1] = 2.0 * a[1] * a[2];
    st->M[2][2] = -2.0 * a[0] * a[0] - 2.0 * a[1] * a[1] + 1.0;
  }
  return out;
}

static int32_t segment_records(const orc_segment* sg) { return sg->n + sg->nf[0] + sg->nf[1] + sg->nf[2]; }

/* ------------------------------------------------------------------------- */
/* Transport                                                                  */
/* ------------------------------------------------------------------------- */
typedef struct {
  double pos[3], dir[3];
  double len;   /* total geometric path */
  double geo;   /* sum of l (1 - u . axis) */
  double opt;   /* sum of (n - 1) l */
  double tau;   /* optical depth */
  int ok;       /* 0: does not reach the observation level */
} path_state;

static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Straight line to the horizontal plane z = h (Sec. 3.4.1, Eq. 3.3 with the
 * sign restored: I = A + ((h - A_z) / u_z) u, a finite point iff u_z != 0). */
static double straight_to_plane(const double* pos, const double* dir, double h) {
  return (h - pos[2]) / dir[2];
}

/* Advance the path state by a straight leg of length s in a medium with
 * refractivity delta and extinction ext (per metre). */
static void leg(path_state* ps, const double* axis, double s, double delta, double ext) {
  for (int j = 0; j < 3; ++j) ps->pos[j] += s * ps->dir[j];
  ps->len += s;
  ps->geo += s * (1.0 - dot3(ps->dir, axis));
  ps->opt += s * delta;
  ps->tau += s * ext;
}

/* Refraction at a horizontal boundary in the vector form of Snell's law
 * (Sec. 3.4.2, Eq. 3.15): A2' = A1' + (sqrt(n2^2 - n1^2 + n1^2 cos^2 a1) - n1 cos a1) N,
 * with optical vectors A' = n A and N the unit normal pointing along travel. */
static void refract(double* dir, const double* N, double n1, double n2) {
  double A1[3] = {n1 * dir[0], n1 * dir[1], n1 * dir[2]};
  double cos1 = dot3(dir, N);
  double c = sqrt(n2 * n2 - n1 * n1 + n1 * n1 * cos1 * cos1) - n1 * cos1;
  for (int j = 0; j < 3; ++j) dir[j] = (A1[j] + c * N[j]) / n2;
}

/* ------------------------------------------------------------------------- */
/* One photon record                                                          */
/* ------------------------------------------------------------------------- */
static void sphere_candidate(const orc_run* R, const orc_geom* G, double x, double y,
                             int* isph, double C[3]) {
  double cx0 = G->core_x - 0.5 * (R->snx - 1) * R->pitch;
  double cy0 = G->core_y - 0.5 * (R->sny - 1) * R->pitch;
  double fi = floor((x - cx0) / R->pitch + 0.5);
  double fj = floor((y - cy0) / R->pitch + 0.5);
  if (fi < 0 || fj < 0 || fi >= R->snx || fj >= R->sny) { *isph = -1; return; }
  *isph = (int)fj * R->snx + (int)fi;
  C[0] = cx0 + fi * R->pitch; C[1] = cy0 + fj * R->pitch; C[2] = R->h_obs;
}

static double min4(double a, double b, double c, double d) {
  double m = a < b ? a : b; m = m < c ? m : c; return m < d ? m : d;
}

/* Refraction at a spherical shell boundary (the vector form, Eq. 3.15, with
 * the radial normal N pointing along travel). Going outwards into thinner air
 * the radicand can turn negative: the ray is then totally reflected. Returns 1
 * if the ray crossed, 0 if it was reflected. */
static int refract_or_reflect(double* dir, const double* N, double n1, double n2) {
  double cos1 = dot3(dir, N);
  double rad = n2 * n2 - n1 * n1 + n1 * n1 * cos1 * cos1;
  if (rad < 0.0) {
    for (int j = 0; j < 3; ++j) dir[j] -= 2.0 * cos1 * N[j];
    return 0;
  }
  double c = sqrt(rad) - n1 * cos1;
  for (int j = 0; j < 3; ++j) dir[j] = (n1 * dir[j] + c * N[j]) / n2;
  return 1;
}

/* Distance along dir from pos to the sphere of radius r about C, first
 * crossing ahead (inward when `inward`), or -1 if there is none. Written as
 * c / (-b + sqrt(b^2 - c)) where the plain root would cancel. A point on (or,
 * by rounding, just inside) the sphere and moving inward crosses it at once. */
static double to_sphere(const double* pos, const double* dir, const double* C, double r, int inward) {
  double q[3] = {pos[0] - C[0], pos[1] - C[1], pos[2] - C[2]};
  double b = dot3(q, dir);
  double qq = dot3(q, q);
  double rq = sqrt(qq);
  double c = (rq - r) * (rq + r);
  double disc = b * b - c;
  if (disc < 0.0) return -1.0;
  double sq = sqrt(disc);
  if (inward) {
    if (!(b < 0.0)) return -1.0;
    if (!(c > 0.0)) return 0.0;
    return c / (-b + sq);
  }
  /* outward from inside (c < 0): the positive root */
  return b > 0.0 ? b + sq : -c / (sq - b);
}

/* Curved Earth (Sec. 3.3.4, spherical model): the layer refractivities become
 * shells about the Earth centre (0, 0, -R_E); the ray is straight inside a
 * shell and refracted with the vector form at every shell boundary. Ends on
 * the observation sphere r = R_E + h_obs (returns 1) or leaves the top of the
 * atmosphere (returns 0). */
static int curved_walk_rec(const orc_atmo* A, const orc_run* R, int kbin, const double* axis, path_state* ps,
                           double* inv_out, int cap, int* m_out);

static int curved_walk(const orc_atmo* A, const orc_run* R, int kbin, const double* axis, path_state* ps) {
  return curved_walk_rec(A, R, kbin, axis, ps, NULL, 0, NULL);
}

/* Bouguer's invariant n r sin(angle to the radial) of the ray in shell i. */
static double bouguer(const double* pos, const double* dir, const double* C, double n) {
  double q[3] = {pos[0] - C[0], pos[1] - C[1], pos[2] - C[2]};
  double cr[3] = {q[1] * dir[2] - q[2] * dir[1], q[2] * dir[0] - q[0] * dir[2], q[0] * dir[1] - q[1] * dir[0]};
  return n * sqrt(dot3(cr, cr));
}

static int curved_walk_rec(const orc_atmo* A, const orc_run* R, int kbin, const double* axis, path_state* ps,
                           double* inv_out, int cap, int* m_out) {
  const orc_atmo_params* p = &A->p;
  double Re = p->earth_radius;
  double C[3] = {0.0, 0.0, -Re};
  double dh = p->h_top / p->n_layers;
  double q[3] = {ps->pos[0] - C[0], ps->pos[1] - C[1], ps->pos[2] - C[2]};
  double h = sqrt(dot3(q, q)) - Re;
  int i = (int)floor(h / dh);
  if (i > p->n_layers - 1) i = p->n_layers - 1;
  int obs = (int)floor(R->h_obs / dh);
  double r_obs = Re + R->h_obs;
  int m = 0;
  for (int iter = 0; iter < 8 * p->n_layers; ++iter) {
    double delta = A->layer_delta[i], ext = A->layer_ext[(size_t)i * p->n_lam + kbin];
    if (inv_out && m < cap) inv_out[m] = bouguer(ps->pos, ps->dir, C, 1.0 + delta);
    ++m;
    if (m_out) *m_out = m;
    if (i == obs) {
      double s = to_sphere(ps->pos, ps->dir, C, r_obs, 1);
      if (s >= 0.0) { leg(ps, axis, s, delta, ext); return 1; }
    } else if (i > obs) {
      double s = to_sphere(ps->pos, ps->dir, C, Re + i * dh, 1);
      if (s >= 0.0) {
        leg(ps, axis, s, delta, ext);
        double qn[3] = {ps->pos[0] - C[0], ps->pos[1] - C[1], ps->pos[2] - C[2]};
        double nq = sqrt(dot3(qn, qn));
        double N[3] = {-qn[0] / nq, -qn[1] / nq, -qn[2] / nq};
        if (refract_or_reflect(ps->dir, N, 1.0 + delta, 1.0 + A->layer_delta[i - 1])) --i;
        continue;
      }
    }
    double s = to_sphere(ps->pos, ps->dir, C, Re + (i + 1) * dh, 0);
    leg(ps, axis, s, delta, ext);
    if (i + 1 >= p->n_layers) return 0;
    double qn[3] = {ps->pos[0] - C[0], ps->pos[1] - C[1], ps->pos[2] - C[2]};
    double nq = sqrt(dot3(qn, qn));
    double N[3] = {qn[0] / nq, qn[1] / nq, qn[2] / nq};
    if (refract_or_reflect(ps->dir, N, 1.0 + delta, 1.0 + A->layer_delta[i + 1])) ++i;
  }
  return 0;
}

/* Record k of a segment: Cherenkov records first, then the fluorescence bands. */
/* Survival threshold: the probability that a photon reaching the detector level
 * with optical depth tau is detected (transmission exp(-tau), times the detector
 * efficiency of its wavelength bin), over the probability q with which its
 * record was kept at generation (Sec. 2.3.2, 4.3.1). */
static double survival(const orc_run* R, const orc_segment* sg, double tau, int kbin, double p_emit) {
  double p = exp(-tau) * p_emit;
  if (R->efficiency) p = p * R->efficiency[kbin];
  if (R->reduction) p = p / sg->q;
  return p;
}

static void trace_photon(const orc_atmo* A, const orc_run* R, const orc_geom* G, double K,
                         const seg_setup* st, const orc_segment* sg, uint64_t seg_id, uint32_t k,
                         orc_photon* out) {
  (void)K;
  const orc_atmo_params* p = &A->p;
  memset(out, 0, sizeof(*out));
  out->seg = (int64_t)seg_id; out->k = (int32_t)k; out->bin = -1; out->tbin = -1;
  uint32_t w[4];
  double P[3], u[3], lam, u3, emit_p = 1.0;
  if ((int32_t)k < sg->n) {
    draw(R->seed, k, seg_id, TAG_CHERENKOV, w);
    double f = u24(w[0]);
    double phi = 2.0 * ORC_PI * u24(w[1]);
    if (R->spectrum == SPECTRUM_UNIFORM) lam = p->lam_min + (p->lam_max - p->lam_min) * u24(w[2]);
    else lam = 1.0 / (1.0 / p->lam_min - u24(w[2]) * (1.0 / p->lam_min - 1.0 / p->lam_max));
    u3 = u24(w[3]);
    double cos_t = st->cos_t, sin_t = st->sin_t;
    if (R->spectrum == SPECTRUM_DISPERSIVE) {
      /* n(lambda, h) at the segment midpoint; the angle of Eq. 2.5 and the
       * Frank-Tamm weight sin^2(theta) = 1 - 1/(beta n)^2 of this wavelength,
       * zero below the threshold (the Heaviside factor) */
      double dl = st->delta_mid * (air_dispersion_sum(lam) / air_dispersion_sum(R->lambda_ref));
      double eps = 1.0 - st->beta;
      double g = dl - eps - eps * dl;
      double s2 = g > 0.0 ? g * (g + 2.0) / ((1.0 + g) * (1.0 + g)) : 0.0;
      emit_p = s2 / st->sin2;
      /* below the threshold the record is never emitted; its direction is then
       * taken along the track (the cone of zero opening) */
      if (g > 0.0) { cos_t = 1.0 / (1.0 + g); sin_t = sqrt(s2); } else { cos_t = 1.0; sin_t = 0.0; }
    }
    /* photon on the cone around (0,0,-1) (Sec. 4.2), rotated onto the track */
    double pl[3] = {cos(phi) * sin_t, sin(phi) * sin_t, -cos_t};
    for (int i = 0; i < 3; ++i) u[i] = st->M[i][0] * pl[0] + st->M[i][1] * pl[1] + st->M[i][2] * pl[2];
    /* emission at a random point along the track (Sec. 4.2, third step) */
    for (int i = 0; i < 3; ++i) P[i] = st->S[i] + f * (st->E[i] - st->S[i]);
  } else {
    /* fluorescence (Sec. 4.2.2): isotropic, restricted to the lower hemisphere;
     * the thesis samples the polar angle uniformly, which is not isotropic -- the
     * cosine is drawn uniformly instead */
    int32_t kk = (int32_t)k - sg->n, band = 0;
    while (kk >= sg->nf[band]) { kk -= sg->nf[band]; ++band; }
    out->source = 1 + band;
    draw(R->seed, (uint32_t)kk, seg_id, TAG_FLUOR + (uint32_t)band, w);
    double f = u24(w[0]);
    double cz = 1.0 - u24(w[1]);
    double phi = 2.0 * ORC_PI * u24(w[2]);
    double sz = sqrt(1.0 - cz * cz);
    u[0] = sz * cos(phi); u[1] = sz * sin(phi); u[2] = -cz;
    lam = R->fl_lambda[band];
    u3 = u24(w[3]);
    for (int i = 0; i < 3; ++i) P[i] = st->S[i] + f * (st->E[i] - st->S[i]);
  }
  out->lambda = lam; out->u_abs = u3;
  out->ex = P[0]; out->ey = P[1]; out->ez = P[2];
  out->dx = u[0]; out->dy = u[1]; out->dz = u[2];
  out->p_emit = emit_p;
  double axis[3] = {G->ax, G->ay, G->az};
  /* a record of the largest cone that its wavelength does not emit */
  if (!(u3 < emit_p)) {
    out->state = ST_NOT_EMITTED;
    out->x = P[0]; out->y = P[1]; out->z = P[2];
    out->margin = 1e30; out->tmargin = 1e30;
    return;
  }
  /* upward photons are discarded first (Sec. 5.3.4) */
  if (!(u[2] < 0.0)) { out->state = ST_UPWARD; return; }
  double h_e = P[2];
  if (R->transport == TRANSPORT_CURVED) {
    double q[3] = {P[0], P[1], P[2] + p->earth_radius};
    h_e = sqrt(dot3(q, q)) - p->earth_radius;
  }
  if (h_e < R->h_obs) { out->state = ST_OUTSIDE; out->x = P[0]; out->y = P[1]; out->z = P[2]; return; }
  path_state ps;
  memset(&ps, 0, sizeof(ps));
  memcpy(ps.pos, P, sizeof(P));
  memcpy(ps.dir, u, sizeof(u));
  int kbin = 0;
  if (p->n_lam > 0) {
    kbin = (int)floor((lam - p->lam_min) / (p->lam_max - p->lam_min) * p->n_lam);
    if (kbin < 0) kbin = 0;
    if (kbin > p->n_lam - 1) kbin = p->n_lam - 1;
  }
  if (R->transport == TRANSPORT_CURVED) {
    int arrived = curved_walk(A, R, kbin, axis, &ps);
    out->x = ps.pos[0]; out->y = ps.pos[1]; out->z = ps.pos[2];
    out->tau = ps.tau;
    out->t = (ps.geo + ps.opt) / ORC_C_M_PER_NS;
    if (!arrived) { out->state = ST_OUTSIDE; out->margin = 1e30; return; }
    /* bins: the arrival point's coordinates in the tangent plane at the core */
    double gx0 = G->core_x - 0.5 * R->nx * R->cell, gy0 = G->core_y - 0.5 * R->ny * R->cell;
    double fx = (ps.pos[0] - gx0) / R->cell, fy = (ps.pos[1] - gy0) / R->cell;
    double ix = floor(fx), iy = floor(fy);
    out->margin = min4(fx - ix, ix + 1.0 - fx, fy - iy, iy + 1.0 - fy) * R->cell;
    if (!(u3 < survival(R, sg, ps.tau, kbin, out->p_emit))) { out->state = ST_ABSORBED; return; }
    if (!(ix >= 0 && iy >= 0 && ix < R->nx && iy < R->ny)) { out->state = ST_OUTSIDE; return; }
    out->state = ST_BINNED;
    out->bin = (int)iy * R->nx + (int)ix;
    return;
  }
  int layer = 0;
  double dh = 0.0;
  if (R->transport == TRANSPORT_LAYERED) {
    /* homogeneous layers with Snell's law at each boundary (Sec. 3.4.2) */
    dh = p->h_top / p->n_layers;
    layer = (int)floor(P[2] / dh);
    if (layer > p->n_layers - 1) layer = p->n_layers - 1;
    int obs_layer = (int)floor(R->h_obs / dh);
    double N[3] = {0.0, 0.0, -1.0};
    while (layer > obs_layer) {
      double zb = layer * dh;
      double s = straight_to_plane(ps.pos, ps.dir, zb);
      leg(&ps, axis, s, A->layer_delta[layer], A->layer_ext[(size_t)layer * p->n_lam + kbin]);
      ps.pos[2] = zb;
      refract(ps.dir, N, 1.0 + A->layer_delta[layer], 1.0 + A->layer_delta[layer - 1]);
      --layer;
    }
  }
  /* final straight leg to the observation level (ground grid) or a sphere */
  double s_plane = straight_to_plane(ps.pos, ps.dir, R->h_obs);
  double s_end = s_plane;
  double Q[3];
  for (int j = 0; j < 3; ++j) Q[j] = ps.pos[j] + s_plane * ps.dir[j];
  int bin = -1;
  double margin = 0.0;
  if (R->detector == DETECTOR_GRID) {
    double gx0 = G->core_x - 0.5 * R->nx * R->cell, gy0 = G->core_y - 0.5 * R->ny * R->cell;
    double fx = (Q[0] - gx0) / R->cell, fy = (Q[1] - gy0) / R->cell;
    double ix = floor(fx), iy = floor(fy);
    margin = min4(fx - ix, ix + 1.0 - fx, fy - iy, iy + 1.0 - fy) * R->cell;
    if (ix >= 0 && iy >= 0 && ix < R->nx && iy < R->ny) bin = (int)iy * R->nx + (int)ix;
  } else {
    int isph; double C[3];
    sphere_candidate(R, G, Q[0], Q[1], &isph, C);
    if (isph >= 0) {
      double q[3] = {Q[0] - C[0], Q[1] - C[1], Q[2] - C[2]};
      double b = dot3(q, ps.dir);
      double cc = dot3(q, q) - R->radius * R->radius;
      double disc = b * b - cc;
      double dperp2 = dot3(q, q) - b * b;
      margin = fabs(sqrt(dperp2 > 0 ? dperp2 : 0.0) - R->radius);
      if (disc >= 0.0) {
        double s_in = -b - sqrt(disc);
        s_end = s_plane + s_in;
        bin = isph;
      }
    } else {
      margin = 1e30;
    }
  }
  /* last leg up to the arrival point */
  double delta_last = (R->transport == TRANSPORT_LAYERED) ? A->layer_delta[layer] : 0.0;
  double ext_last = (R->transport == TRANSPORT_LAYERED) ? A->layer_ext[(size_t)layer * p->n_lam + kbin] : 0.0;
  double start_z = ps.pos[2], dir_z = ps.dir[2];
  leg(&ps, axis, s_end, delta_last, ext_last);
  if (R->transport == TRANSPORT_STRAIGHT) {
    /* straight line in a planar atmosphere: closed forms over the height span */
    double zlo = ps.pos[2], zhi = start_z;
    ps.opt = delta_integral(A, zlo, zhi) / fabs(dir_z);
    ps.tau = 0.0;
    if (p->rayleigh400 > 0.0 || p->aer_tau350 > 0.0) ps.tau = vertical_tau(A, zlo, zhi, lam) / fabs(dir_z);
  }
  out->x = ps.pos[0]; out->y = ps.pos[1]; out->z = ps.pos[2];
  out->tau = ps.tau;
  out->t = (ps.geo + ps.opt) / ORC_C_M_PER_NS;
  out->margin = margin;
  /* absorption and scattering remove the photon (Sec. 2.3.2): survival iff u < exp(-tau),
   * times the detector efficiency and over the reduction factor where set */
  if (!(u3 < survival(R, sg, ps.tau, kbin, out->p_emit))) { out->state = ST_ABSORBED; return; }
  if (bin < 0) { out->state = ST_OUTSIDE; return; }
  out->state = ST_BINNED;
  out->bin = bin;
  if (R->detector == DETECTOR_SPHERES && R->n_t > 0) {
    double tb = floor(out->t / R->dt);
    double e0 = fabs(out->t - tb * R->dt), e1 = fabs((tb + 1.0) * R->dt - out->t);
    out->tmargin = e0 < e1 ? e0 : e1;
    if (tb < 0) tb = 0;
    out->tbin = tb >= R->n_t ? R->n_t : (int32_t)tb;
  }
}

/* ------------------------------------------------------------------------- */
/* Exported drivers                                                           */
/* ------------------------------------------------------------------------- */
typedef struct {
  const float *x0, *y0, *z0, *x1, *y1, *z1, *beta, *charge;
  int64_t n;
  int64_t first_id;
  const float* dedx;  /* MeV/m, may be NULL (no fluorescence) */
  int64_t id_stride;  /* segment i has the global id first_id + i * id_stride (0 means 1) */
} orc_segments;

static uint64_t seg_id_of(const orc_segments* S, int64_t i) {
  return (uint64_t)(S->first_id + i * (S->id_stride > 0 ? S->id_stride : 1));
}

static float seg_dedx(const orc_segments* S, int64_t i) { return S->dedx ? S->dedx[i] : 0.0f; }

double orc_frank_tamm_K(double lam_min, double lam_max) { return frank_tamm_K(lam_min, lam_max); }
double orc_exp_neg(double x) { return exp_neg_basic(x); }
int64_t orc_poisson(double mu, uint32_t w0, uint64_t seed, uint64_t seg_id, uint32_t tag) {
  return poisson_draw(mu, w0, seed, seg_id, tag);
}

void orc_segment_counts(const orc_atmo* A, const orc_run* R, const orc_segments* S, orc_segment* out) {
  double K = frank_tamm_K(A->p.lam_min, A->p.lam_max);
  for (int64_t i = 0; i < S->n; ++i) {
    seg_setup st;
    out[i] = segment_setup(A, R, K, S->x0[i], S->y0[i], S->z0[i], S->x1[i], S->y1[i], S->z1[i],
                           S->beta[i], S->charge[i], seg_dedx(S, i), seg_id_of(S, i), &st);
  }
}

/* All photon records of segments [0, n). Returns the number of records, or
 * -(needed) when `cap` is too small (nothing written beyond cap). */
int64_t orc_trace(const orc_atmo* A, const orc_run* R, const orc_segments* S, const orc_geom* G,
                  orc_photon* out, int64_t cap) {
  double K = frank_tamm_K(A->p.lam_min, A->p.lam_max);
  int64_t m = 0;
  for (int64_t i = 0; i < S->n; ++i) {
    seg_setup st;
    orc_segment sg = segment_setup(A, R, K, S->x0[i], S->y0[i], S->z0[i], S->x1[i], S->y1[i], S->z1[i],
                                   S->beta[i], S->charge[i], seg_dedx(S, i), seg_id_of(S, i), &st);
    int32_t nrec = segment_records(&sg);
    for (int32_t k = 0; k < nrec; ++k) {
      if (m < cap) trace_photon(A, R, G, K, &st, &sg, seg_id_of(S, i), (uint32_t)k, &out[m]);
      ++m;
    }
  }
  return m <= cap ? m : -m;
}

enum {
  C_SEG_IN = 0, C_SEG_SKIPPED, C_SEG_BELOW, C_REC_GEN, C_REC_UP, C_REC_ABS, C_REC_OUT, C_REC_BIN,
  C_PHOT_BIN, C_SURR_FALLBACK, C_REC_NOT_EMITTED = 13, N_COUNTERS = 16
};

typedef struct {
  const orc_atmo* A; const orc_run* R; const orc_segments* S;
  int32_t n_showers; const int64_t* offsets; const orc_geom* geoms;
  int64_t begin, end;
  uint64_t* bins; uint64_t* thist; uint64_t counters[N_COUNTERS];
  int64_t bins_per_shower, thist_per_shower;
} worker_arg;

static void* worker(void* vp) {
  worker_arg* W = (worker_arg*)vp;
  const orc_atmo* A = W->A; const orc_run* R = W->R; const orc_segments* S = W->S;
  double K = frank_tamm_K(A->p.lam_min, A->p.lam_max);
  int32_t sh = 0;
  for (int64_t i = W->begin; i < W->end; ++i) {
    while (W->offsets && i >= W->offsets[sh + 1]) ++sh;
    seg_setup st;
    uint64_t sid = seg_id_of(S, i);
    orc_segment sg = segment_setup(A, R, K, S->x0[i], S->y0[i], S->z0[i], S->x1[i], S->y1[i], S->z1[i],
                                   S->beta[i], S->charge[i], seg_dedx(S, i), sid, &st);
    W->counters[C_SEG_IN] += 1;
    if (sg.status == 2) { W->counters[C_SEG_SKIPPED] += 1; continue; }
    if (sg.status == 1) W->counters[C_SEG_BELOW] += 1;
    int32_t nrec = segment_records(&sg);
    for (int32_t k = 0; k < nrec; ++k) {
      orc_photon ph;
      trace_photon(A, R, &W->geoms[sh], K, &st, &sg, sid, (uint32_t)k, &ph);
      W->counters[C_REC_GEN] += 1;
      switch (ph.state) {
        case ST_UPWARD: W->counters[C_REC_UP] += 1; break;
        case ST_ABSORBED: W->counters[C_REC_ABS] += 1; break;
        case ST_OUTSIDE: W->counters[C_REC_OUT] += 1; break;
        case ST_NOT_EMITTED: W->counters[C_REC_NOT_EMITTED] += 1; break;
        default:
          W->counters[C_REC_BIN] += 1;
          W->counters[C_PHOT_BIN] += (uint64_t)R->bunch;
          W->bins[(int64_t)sh * W->bins_per_shower + ph.bin] += (uint64_t)R->bunch;
          if (W->thist && ph.tbin >= 0)
            W->thist[(int64_t)sh * W->thist_per_shower + (int64_t)ph.bin * (R->n_t + 1) + ph.tbin] +=
                (uint64_t)R->bunch;
      }
    }
  }
  return NULL;
}

/* Full propagation: bins (u64, [n_showers][cells or spheres]), optional time
 * histograms (u64, [n_showers][spheres][n_t + 1]) and counters (u64 x 16) are
 * accumulated (+=). Threads split the segment range; counts are integers, so
 * the result does not depend on the thread count. */
int orc_propagate(const orc_atmo* A, const orc_run* R, const orc_segments* S, int32_t n_showers,
                  const int64_t* offsets, const orc_geom* geoms, uint64_t* bins, uint64_t* thist,
                  uint64_t* counters, int32_t n_threads) {
  if (n_threads < 1) n_threads = 1;
  int64_t bps = R->detector == DETECTOR_GRID ? (int64_t)R->nx * R->ny : (int64_t)R->snx * R->sny;
  int64_t tps = R->detector == DETECTOR_SPHERES && R->n_t > 0 ? bps * (R->n_t + 1) : 0;
  worker_arg* W = (worker_arg*)calloc((size_t)n_threads, sizeof(worker_arg));
  pthread_t* th = (pthread_t*)calloc((size_t)n_threads, sizeof(pthread_t));
  int64_t chunk = (S->n + n_threads - 1) / n_threads;
  for (int t = 0; t < n_threads; ++t) {
    W[t].A = A; W[t].R = R; W[t].S = S; W[t].n_showers = n_showers;
    W[t].offsets = n_showers > 1 ? offsets : NULL; W[t].geoms = geoms;
    W[t].begin = t * chunk < S->n ? t * chunk : S->n;
    W[t].end = (t + 1) * chunk < S->n ? (t + 1) * chunk : S->n;
    W[t].bins_per_shower = bps; W[t].thist_per_shower = tps;
    W[t].bins = (uint64_t*)calloc((size_t)(bps * n_showers), sizeof(uint64_t));
    W[t].thist = tps ? (uint64_t*)calloc((size_t)(tps * n_showers), sizeof(uint64_t)) : NULL;
    pthread_create(&th[t], NULL, worker, &W[t]);
  }
  for (int t = 0; t < n_threads; ++t) {
    pthread_join(th[t], NULL);
    for (int64_t j = 0; j < bps * n_showers; ++j) bins[j] += W[t].bins[j];
    if (tps && thist)
      for (int64_t j = 0; j < tps * n_showers; ++j) thist[j] += W[t].thist[j];
    for (int c = 0; c < N_COUNTERS; ++c) counters[c] += W[t].counters[c];
    free(W[t].bins); free(W[t].thist);
  }
  free(W); free(th);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Reference paths used by the pins                                           */
/* ------------------------------------------------------------------------- */

/* Trace one ray (start point, unit direction) through the layered atmosphere to
 * the plane z = h_end, for the analytic and closed-form checks. Writes the end
 * point and the n sin(theta) value of every layer crossed (max `cap`). */
int orc_layered_ray(const orc_atmo* A, const double* P, const double* u, double h_end,
                    double* end_out, double* snell_out, int cap) {
  const orc_atmo_params* p = &A->p;
  double dh = p->h_top / p->n_layers;
  double pos[3] = {P[0], P[1], P[2]}, dir[3] = {u[0], u[1], u[2]};
  int layer = (int)floor(pos[2] / dh);
  if (layer > p->n_layers - 1) layer = p->n_layers - 1;
  int end_layer = (int)floor(h_end / dh);
  double N[3] = {0.0, 0.0, -1.0};
  int m = 0;
  while (layer > end_layer) {
    double zb = layer * dh;
    double s = straight_to_plane(pos, dir, zb);
    for (int j = 0; j < 3; ++j) pos[j] += s * dir[j];
    pos[2] = zb;
    if (m < cap) snell_out[m] = (1.0 + A->layer_delta[layer]) * sqrt(dir[0] * dir[0] + dir[1] * dir[1]);
    ++m;
    refract(dir, N, 1.0 + A->layer_delta[layer], 1.0 + A->layer_delta[layer - 1]);
    --layer;
  }
  if (m < cap) snell_out[m] = (1.0 + A->layer_delta[layer]) * sqrt(dir[0] * dir[0] + dir[1] * dir[1]);
  ++m;
  double s = straight_to_plane(pos, dir, h_end);
  for (int j = 0; j < 3; ++j) end_out[j] = pos[j] + s * dir[j];
  return m;
}

/* ------------------------------------------------------------------------- */
/* Transport surrogate: training inputs and exact targets                     */
/* ------------------------------------------------------------------------- */
/* The MLP transport surrogate replaces the layered tracer's correction to
 * the straight line, the role the thesis gives to its precomputed correction
 * table (Sec. 4.4.1: the difference between the straight-line and the
 * iterative propagation). Inputs per photon: emission height h_e (m), cos of the
 * photon zenith angle, azimuth phi (rad), wavelength-bin centre (nm),
 * observation level h_obs (m). Targets: the landing offset (dx, dy) of the
 * layered path from the straight line started at the same point and direction,
 * expressed along and across the photon's horizontal direction (the frame the
 * configuration leaves open; in a planar atmosphere the offset lies along it),
 * and the parts of the optical path excess sum n_i l_i - l_straight (m) and of
 * log T = -tau that refraction adds to the straight line's own sums over the same
 * layers (sum (n_i - 1) and extinction times the straight line's slant span in each
 * layer): what the correction has to carry, the straight line's share being exact
 * and cheap. */

/* Training inputs i = first .. first+n-1 drawn from two Philox blocks with
 * counters (i low, 0, i high, 8) and (i low, 1, i high, 8): h_obs, cos(theta), phi uniform in
 * the domain box, the wavelength a uniformly drawn bin, and h_e the lower boundary of a
 * uniformly drawn layer above the observation layer. A photon is straight inside its
 * homogeneous start layer; the network is asked for the correction from that layer's
 * lower boundary on, which is a smooth function of the boundary height, whereas the
 * correction from the emission point jumps wherever the emission height crosses a layer
 * boundary (Snell's invariant takes the start layer's index). */
void orc_surrogate_inputs(const orc_atmo* A, uint64_t seed, const double* lo, const double* hi, int64_t first,
                          int64_t n, double* X) {
  for (int64_t j = 0; j < n; ++j) {
    uint64_t i = (uint64_t)(first + j);
    uint32_t ctr0[4] = {(uint32_t)i, 0u, (uint32_t)(i >> 32), TAG_TRAIN};
    uint32_t ctr1[4] = {(uint32_t)i, 1u, (uint32_t)(i >> 32), TAG_TRAIN};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4], v[4];
    orc_philox(ctr0, key, w);
    orc_philox(ctr1, key, v);
    double h_obs = lo[4] + (hi[4] - lo[4]) * u24(w[0]);
    /* the start: the lower boundary of a layer (shell) above the observation layer,
       drawn uniformly among those inside the box, j = j_lo + floor(u m) formed from
       the word's top 24 bits in integer arithmetic; inside its start layer a photon
       travels straight, so the correction from there is that of the whole path */
    double dh = A->p.h_top / A->p.n_layers;
    int64_t j_obs = (int64_t)floor(h_obs / dh);
    int64_t j_lo = (int64_t)ceil(lo[0] / dh);
    if (j_lo < j_obs + 1) j_lo = j_obs + 1;
    int64_t j_hi = (int64_t)floor(hi[0] / dh);
    int64_t m = j_hi - j_lo + 1;
    if (m < 1) m = 1;
    int64_t jj = j_lo + (int64_t)(((uint64_t)(w[1] >> 8) * (uint64_t)m) >> 24);
    double h_e = (double)jj * dh;
    double ct = lo[1] + (hi[1] - lo[1]) * u24(w[2]);
    double phi = lo[2] + (hi[2] - lo[2]) * u24(w[3]);
    int K = A->p.n_lam;
    int k = (int)floor(u24(v[0]) * K);
    if (k > K - 1) k = K - 1;
    double lam = A->p.lam_min + (k + 0.5) * (A->p.lam_max - A->p.lam_min) / K;
    double* x = X + 5 * j;
    x[0] = h_e; x[1] = ct; x[2] = phi; x[3] = lam; x[4] = h_obs;
  }
}

void orc_surrogate_targets(const orc_atmo* A, int64_t n, const double* X, double* Y) {
  const orc_atmo_params* p = &A->p;
  double dh = p->h_top / p->n_layers;
  double N[3] = {0.0, 0.0, -1.0};
  for (int64_t j = 0; j < n; ++j) {
    const double* x = X + 5 * j;
    double h_e = x[0], ct = x[1], phi = x[2], lam = x[3], h_obs = x[4];
    double st = sqrt(1.0 - ct * ct);
    double u[3] = {st * cos(phi), st * sin(phi), -ct};
    int kbin = (int)floor((lam - p->lam_min) / (p->lam_max - p->lam_min) * p->n_lam);
    if (kbin < 0) kbin = 0;
    if (kbin > p->n_lam - 1) kbin = p->n_lam - 1;
    double pos[3] = {0.0, 0.0, h_e}, dir[3] = {u[0], u[1], u[2]};
    double optical = 0.0, tau = 0.0;
    int layer = (int)floor(h_e / dh);
    if (layer > p->n_layers - 1) layer = p->n_layers - 1;
    int obs_layer = (int)floor(h_obs / dh);
    while (layer > obs_layer) {
      double zb = layer * dh;
      double s = straight_to_plane(pos, dir, zb);
      for (int q = 0; q < 3; ++q) pos[q] += s * dir[q];
      pos[2] = zb;
      optical += (1.0 + A->layer_delta[layer]) * s;
      tau += A->layer_ext[(size_t)layer * p->n_lam + kbin] * s;
      refract(dir, N, 1.0 + A->layer_delta[layer], 1.0 + A->layer_delta[layer - 1]);
      --layer;
    }
    double s = straight_to_plane(pos, dir, h_obs);
    for (int q = 0; q < 3; ++q) pos[q] += s * dir[q];
    optical += (1.0 + A->layer_delta[layer]) * s;
    tau += A->layer_ext[(size_t)layer * p->n_lam + kbin] * s;
    double s_straight = (h_obs - h_e) / u[2];
    /* the straight line's own sums over the same layers: n - 1 and extinction
     * times the slant length of each layer's span between h_obs and h_e */
    double opt_straight = 0.0, tau_straight = 0.0;
    int top_layer = (int)floor(h_e / dh);
    if (top_layer > p->n_layers - 1) top_layer = p->n_layers - 1;
    for (int i = obs_layer; i <= top_layer; ++i) {
      double lo = i * dh > h_obs ? i * dh : h_obs;
      double hi = (i + 1) * dh < h_e ? (i + 1) * dh : h_e;
      if (i == p->n_layers - 1) hi = h_e;
      if (!(hi > lo)) continue;
      opt_straight += A->layer_delta[i] * (hi - lo) / ct;
      tau_straight += A->layer_ext[(size_t)i * p->n_lam + kbin] * (hi - lo) / ct;
    }
    double* y = Y + 4 * j;
    /* landing offset in the photon's azimuthal frame: along and across its
     * horizontal direction (cos phi, sin phi) */
    double ox = pos[0] - s_straight * u[0], oy = pos[1] - s_straight * u[1];
    y[0] = ox * cos(phi) + oy * sin(phi);
    y[1] = -ox * sin(phi) + oy * cos(phi);
    y[2] = (optical - s_straight) - opt_straight;
    y[3] = -tau + tau_straight;
  }
}

/* Targets of the curved-Earth surrogate (Sec. 3.3.4 shells), each per metre of
 * the straight chord L from the start to the same observation sphere R + h_obs
 * (the absolute quantities grow with the slant distance; per metre of chord they
 * stay of one size across zenith angles). By the spherical symmetry a photon is
 * started at height h_e above the Earth point below it, P = (0, 0, h_e), with
 * local zenith angle acos(ct) and azimuth phi:
 *   y0 = (psi - psi_chord) (R + h_obs) / L   extra ground distance along the
 *                                            azimuth (psi: central angle swept),
 *   y1 = offset of the arrival point across the vertical plane of the start
 *        direction / L (zero by symmetry),
 *   y2 = ((path length - L) + sum (n - 1) l) / L   optical path excess,
 *   y3 = -tau / L.
 * A sample that does not reach the observation sphere gets NaN targets. */
void orc_surrogate_targets_curved(const orc_atmo* A, int64_t n, const double* X, double* Y) {
  const orc_atmo_params* p = &A->p;
  const double Re = p->earth_radius;
  const double C[3] = {0.0, 0.0, -Re};
  for (int64_t j = 0; j < n; ++j) {
    const double* x = X + 5 * j;
    double h_e = x[0], ct = x[1], phi = x[2], lam = x[3], h_obs = x[4];
    double st = sqrt(1.0 - ct * ct);
    double u[3] = {st * cos(phi), st * sin(phi), -ct};
    int kbin = (int)floor((lam - p->lam_min) / (p->lam_max - p->lam_min) * p->n_lam);
    if (kbin < 0) kbin = 0;
    if (kbin > p->n_lam - 1) kbin = p->n_lam - 1;
    orc_run R;
    memset(&R, 0, sizeof(R));
    R.h_obs = h_obs;
    path_state ps;
    memset(&ps, 0, sizeof(ps));
    ps.pos[2] = h_e;
    for (int q = 0; q < 3; ++q) ps.dir[q] = u[q];
    const double axis[3] = {0.0, 0.0, -1.0};
    double* y = Y + 4 * j;
    double P[3] = {0.0, 0.0, h_e};
    double s_ch = to_sphere(P, u, C, Re + h_obs, 1);
    if (!curved_walk(A, &R, kbin, axis, &ps) || !(s_ch >= 0.0)) {
      y[0] = y[1] = y[2] = y[3] = NAN;
      continue;
    }
    double q0[3] = {P[0] - C[0], P[1] - C[1], P[2] - C[2]};
    double q1[3] = {ps.pos[0] - C[0], ps.pos[1] - C[1], ps.pos[2] - C[2]};
    double qs[3] = {P[0] + s_ch * u[0] - C[0], P[1] + s_ch * u[1] - C[1], P[2] + s_ch * u[2] - C[2]};
    double c1[3] = {q0[1] * q1[2] - q0[2] * q1[1], q0[2] * q1[0] - q0[0] * q1[2], q0[0] * q1[1] - q0[1] * q1[0]};
    double cs[3] = {q0[1] * qs[2] - q0[2] * qs[1], q0[2] * qs[0] - q0[0] * qs[2], q0[0] * qs[1] - q0[1] * qs[0]};
    double psi = atan2(sqrt(dot3(c1, c1)), dot3(q0, q1));
    double psi_s = atan2(sqrt(dot3(cs, cs)), dot3(q0, qs));
    double en[3] = {-sin(phi), cos(phi), 0.0};
    y[0] = (psi - psi_s) * (Re + h_obs) / s_ch;
    y[1] = ((q1[0] - qs[0]) * en[0] + (q1[1] - qs[1]) * en[1] + (q1[2] - qs[2]) * en[2]) / s_ch;
    y[2] = ((ps.len - s_ch) + ps.opt) / s_ch;
    y[3] = -ps.tau / s_ch;
  }
}

/* One ray through the curved atmosphere from P along u (checks): end point
 * (3), path length excess unused; Bouguer invariant per shell visited. Returns
 * the number of shells visited (negative if the ray left the atmosphere). */
int orc_curved_ray(const orc_atmo* A, double h_obs, const double* P, const double* u, double* end_out,
                   double* inv_out, int cap) {
  orc_run R;
  memset(&R, 0, sizeof(R));
  R.h_obs = h_obs;
  path_state ps;
  memset(&ps, 0, sizeof(ps));
  memcpy(ps.pos, P, 3 * sizeof(double));
  memcpy(ps.dir, u, 3 * sizeof(double));
  double axis[3] = {0.0, 0.0, -1.0};
  int m = 0;
  int arrived = curved_walk_rec(A, &R, 0, axis, &ps, inv_out, cap, &m);
  memcpy(end_out, ps.pos, 3 * sizeof(double));
  return arrived ? m : -m;
}
