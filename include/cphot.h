/*
 * cphot.h -- C ABI of the MI355X (gfx950) Cherenkov photon generation and
 * atmospheric propagation library, libcphot.so.
 *
 * Method: D. Baack, "Optical Photon Emission in Extended Airshowers"
 * (arXiv 2405.04229): Frank-Tamm yield and Cherenkov cone per charged track
 * segment (Sec. 2.2.1, 4.2), transport through a planar atmosphere by straight
 * lines (Sec. 3.4.1) or homogeneous layers with Snell's law (Sec. 3.4.2),
 * removal by absorption (Sec. 2.3.2, 4.3.1), and collection at an observation
 * level or at telescope bounding spheres (Sec. 5.3.4, 6.2).
 *
 * Conventions for every entry point:
 *  - Plain C; no C++ types or exceptions cross the boundary.
 *  - Device pointers are HIP device allocations on the current device; host
 *    pointers are ordinary process memory. Each field says which.
 *  - `stream` is a hipStream_t passed as void* (NULL = the legacy stream).
 *  - Calls that take a stream are asynchronous: they enqueue work and return;
 *    they allocate nothing, synchronise nothing and read nothing back, so they
 *    can be captured in a HIP graph. Argument checks happen before anything is
 *    enqueued: a call that returns an error has enqueued nothing.
 *  - Status: CPHOT_OK (0) or a negative CPHOT_ERR_* code. cphot_last_error()
 *    returns a text for the most recent failure on the calling thread.
 *  - Data-dependent anomalies (non-finite or zero-length segments, beta
 *    outside (0, 1)) are never errors: they are skipped and counted.
 * Units: metres, nanoseconds, nanometres, g/cm^2.
 */
#ifndef CPHOT_H
#define CPHOT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CPHOT_ABI_VERSION 4
#define CPHOT_NCOUNTERS 16

#define CPHOT_OK 0
#define CPHOT_ERR_INVALID_ARG (-1)
#define CPHOT_ERR_OUT_OF_MEMORY (-2)
#define CPHOT_ERR_HIP (-3)
#define CPHOT_ERR_UNSUPPORTED (-4)
#define CPHOT_ERR_CAPACITY (-5)

/* Atmosphere profiles. LINSLEY5: five-layer parametrised depth
 * X(h) = a_i + b_i exp(-h/c_i) (linear in the top layer), density -dX/dh and
 * refractivity n - 1 = kappa rho(h)/rho(0) (Sec. 2.3.1). HOMOGENEOUS: constant
 * n - 1 = delta0, the unit-test medium of Sec. 3.3.1. LINEAR: n - 1 falls
 * linearly from delta0 at h = 0 to 0 at h_top (the test profile of Sec. 6.3.1). */
#define CPHOT_PROFILE_LINSLEY5 0
#define CPHOT_PROFILE_HOMOGENEOUS 1
#define CPHOT_PROFILE_LINEAR 2

/* Transport. STRAIGHT: straight line to the observation level (Sec. 3.4.1,
 * Eq. 3.3). LAYERED: equal homogeneous layers with Snell's law at each boundary
 * (Sec. 3.4.2, Eq. 3.15). */
#define CPHOT_TRANSPORT_STRAIGHT 0
#define CPHOT_TRANSPORT_LAYERED 1
/* SURROGATE: straight line plus the correction predicted by a trained network
 * (see cphot_surrogate_*); photons outside the network's training domain fall
 * back to LAYERED transport and are counted in CPHOT_C_SURROGATE_FALLBACK. */
#define CPHOT_TRANSPORT_SURROGATE 2
/* CURVED: the layers become spherical shells about the Earth centre
 * (0, 0, -earth_radius) (Sec. 3.3.4, spherical model), refraction at every
 * shell boundary, arrival on the sphere of radius earth_radius + h_obs; GRID
 * bins then use the arrival point's (x, y) in the tangent plane at the core
 * (the core lies at (0, 0, h_obs)). A downward ray whose straight line stays
 * well clear of grazing (D_obs / G_j <= 0.1 and t <= the atmosphere's bound, see
 * cphot_device.h) takes the closed-form shell sums: the straight chord and its
 * central angle formed directly, the refraction terms from shell moments
 * tabulated per atmosphere (the same sums as the walk, truncation below 5e-4 m
 * and 1e-6 in optical depth). Other rays are gathered per block into full waves
 * and walked shell by shell. CURVED_WALK: the shell-by-shell walk for every ray
 * (the thesis's iterative tracing; same results within rounding). */
#define CPHOT_TRANSPORT_CURVED 3
#define CPHOT_TRANSPORT_CURVED_WALK 5
/* TABLE: straight line (or chord) plus the correction interpolated bilinearly
 * from a table precomputed with the exact tracer over emission height and cos
 * of the zenith angle (the thesis's interpolation tracing, Sec. 4.4.1; see
 * cphot_table_*). The table's geometry decides planar layers or curved shells
 * (then as CURVED: ground grid only). Photons outside the table's range are
 * traced exactly and counted in CPHOT_C_SURROGATE_FALLBACK. */
#define CPHOT_TRANSPORT_TABLE 4

/* Detectors. GRID: nx x ny square cells of `cell` metres on the observation
 * level, centred on each shower's core. SPHERES: snx x sny bounding spheres of
 * `radius` at `pitch` spacing, centred on the core at h_obs (Sec. 6.2, bounding
 * spheres of telescopes), with optional arrival-time histograms. */
#define CPHOT_DETECTOR_GRID 0
#define CPHOT_DETECTOR_SPHERES 1

/* Emission wavelength: UNIFORM on [lam_min, lam_max], or FRANK_TAMM with
 * dN/dlambda ~ 1/lambda^2 (Eq. 2.4), or DISPERSIVE: FRANK_TAMM with a refractive
 * index that depends on the wavelength as well as the height (Sec. 2.2.1: the
 * yield integral over wavelength and track with the Heaviside factor of the
 * threshold, and the angle of Eq. 2.5).
 *
 * DISPERSIVE: n(lambda, h) - 1 = (n(h) - 1) x R(lambda) / R(lambda_ref_nm), where n(h) - 1
 * is the atmosphere's refractivity, stated at the wavelength lambda_ref_nm, and R is the
 * two-term dispersion formula of standard air (Ciddor, Appl. Opt. 35 (1996) 1566):
 * R = 5792105 / (238.0185 - s^2) + 167917 / (57.362 - s^2), s = 1/lambda in 1/um.
 * R falls with lambda above 132 nm, so n is largest at lam_min. A segment draws its
 * records for that largest cone: mu = K z^2 L sin^2(theta_max) / bunch, with n taken at
 * lam_min and the segment midpoint (no records, status "below threshold", when
 * beta n(lam_min) <= 1). Each Cherenkov record samples lambda ~ 1/lambda^2, takes the
 * angle cos(theta) = 1 / (beta n(lambda, h_mid)), and is emitted iff
 * u < sin^2(theta) / sin^2(theta_max), with sin^2(theta) = 0 where beta n(lambda) <= 1 and
 * u the record's survival uniform; a record not emitted has state 4 and is counted in
 * CPHOT_C_RECORDS_NOT_EMITTED. The expected emitted records are thus the Frank-Tamm
 * integral with the threshold, and a record is detected iff
 * u < (sin^2(theta) / sin^2(theta_max)) x exp(-tau) x efficiency / q. The track cut
 * (CPHOT_CUT_TRACK) uses the largest cone. Propagation (refraction, delay) uses n(h).
 * Needs lam_min >= 150 nm and lambda_ref_nm in [150, 10^5] nm. */
#define CPHOT_SPECTRUM_UNIFORM 0
#define CPHOT_SPECTRUM_FRANK_TAMM 1
#define CPHOT_SPECTRUM_DISPERSIVE 2

/* Emission (bit set). CHERENKOV (Sec. 2.2.1); FLUORESCENCE (Sec. 2.2.2, 4.2.2):
 * per band b, mu_b = fl_yield[b] x dE/dx x L / 2 records (lower hemisphere
 * only), isotropic with cos(polar) uniform, wavelength fl_lambda[b]. A segment's
 * records are its Cherenkov records followed by band 0, 1, 2. 0 = CHERENKOV. */
#define CPHOT_EMIT_CHERENKOV 1
#define CPHOT_EMIT_FLUORESCENCE 2

/* Record count per segment and source from its expected value mu (Sec. 2.2.1):
 * ROUNDED: floor(mu) + [u < mu - floor(mu)] with the segment's own random word
 * (the mean is exact, the spread the smallest possible). POISSON: a Poisson(mu)
 * draw by inversion in equal chunks of mean <= 64 (the first chunk with the
 * segment's word, chunk c > 0 with Philox block (c, id low, id high, 12 + source),
 * source 0 Cherenkov, 1 + b band b), every step an IEEE basic operation (exp(-m) by
 * Cody-Waite reduction and a Taylor polynomial), so that counts are reproducible
 * bit for bit on any IEEE machine. A draw of 2^20 records or more marks the segment
 * skipped. */
#define CPHOT_COUNTS_ROUNDED 0
#define CPHOT_COUNTS_POISSON 1

/* Data-reduction cuts for the SPHERES detector (bit set; Sec. 4.3.2 filter level 1 and
 * Sec. 4.3.4 filter level 3, Sec. 6.2). Both are geometric bounds that never remove a
 * photon that could reach a sphere, so bins and time histograms equal those of the
 * same call without cuts; only the counters show the removed records.
 * TRACK: a segment's Cherenkov records are not generated when every photon of its cone
 *   (from any point of the segment, half-angle theta) lands farther from every sphere
 *   than the bound: the cone's landing disc around the axis's landing point has radius
 *   H (theta / cos^2(zeta + theta)) (H the segment's top above h_obs, zeta the track's
 *   zenith angle), widened by the refraction bound and by r / cos of the steepest
 *   direction. Fluorescence records are never cut (isotropic emission).
 * PHOTON: a record whose straight line lands farther from the nearest sphere centre
 *   than r / cos(zeta) plus the refraction bound is outside before its transport.
 * Refraction bound: H tan(zeta) E (1 + 3 tan^2(zeta)) x 1.1 + 0.5 m, E the largest
 *   |n_i - n_j| / n_i over the layers above the observation layer (0 for STRAIGHT).
 *   Directions with cos(zeta) <= 0.2, or with 2.2 tan^2(zeta) E > 0.25, are never cut.
 * GRID (PHOTON only; STRAIGHT, LAYERED, planar TABLE or any curved transport): a record
 *   whose straight line lands farther from the grid rectangle than the refraction bound
 *   is outside before its transport. Planar layers: the bound above. Spherical shells
 *   (n - 1 non-increasing with height, else UNSUPPORTED): E sec^2(z_end) (R + h_obs)
 *   psi_s x 1.1 + 1 m, psi_s the central angle the straight line sweeps to the sphere
 *   R + h_obs and z_end its local zenith there (Bouguer's invariant bounds the shortfall
 *   of the refracted path's central angle); rays whose straight line misses the sphere
 *   are never cut.
 * Cuts act in cphot_propagate (and captured steps) only; the parity entry points
 * (counts, records) ignore them. */
#define CPHOT_CUT_TRACK 1
#define CPHOT_CUT_PHOTON 2

/* Bin element types of cphot_bins.bins (F64: FP64 sums of the FP32 bunch weights). */
#define CPHOT_BINS_U32 0
#define CPHOT_BINS_U64 1
#define CPHOT_BINS_F64 2

/* Counter slots (uint64) of cphot_bins.counters. After a call,
 * records_generated = records_upward + records_absorbed + records_outside + records_binned
 * + records_not_emitted (the last is zero except under CPHOT_SPECTRUM_DISPERSIVE). */
#define CPHOT_C_SEGMENTS_IN 0
#define CPHOT_C_SEGMENTS_SKIPPED 1          /* non-finite, zero length, beta outside (0,1) */
#define CPHOT_C_SEGMENTS_BELOW_THRESHOLD 2  /* beta n <= 1 (Sec. 2.2.1) */
#define CPHOT_C_RECORDS_GENERATED 3
#define CPHOT_C_RECORDS_UPWARD 4
#define CPHOT_C_RECORDS_ABSORBED 5
#define CPHOT_C_RECORDS_OUTSIDE 6           /* missed the grid / every sphere, or emitted below h_obs */
#define CPHOT_C_RECORDS_BINNED 7
#define CPHOT_C_PHOTONS_BINNED 8            /* records_binned x bunch size */
#define CPHOT_C_SURROGATE_FALLBACK 9        /* records traced exactly because outside the surrogate's domain */
#define CPHOT_C_RECORDS_FLUORESCENCE 10     /* fluorescence records among records_generated */
#define CPHOT_C_RECORDS_CULLED_TRACK 11     /* Cherenkov records of segments removed by CPHOT_CUT_TRACK
                                               (never generated, not in records_generated) */
#define CPHOT_C_RECORDS_CULLED_PHOTON 12    /* records removed by CPHOT_CUT_PHOTON (among records_outside) */
#define CPHOT_C_RECORDS_NOT_EMITTED 13      /* DISPERSIVE: records of the largest cone not emitted at
                                               their wavelength (state 4); records_generated = upward +
                                               absorbed + outside + binned + not_emitted */

typedef struct cphot_atmosphere cphot_atmosphere;
typedef struct cphot_surrogate cphot_surrogate;
typedef struct cphot_table cphot_table;

/* Host description of an atmosphere. All fields are read during
 * cphot_make_atmosphere only. */
typedef struct {
  int32_t profile;          /* CPHOT_PROFILE_* */
  int32_t n_layers;         /* equal homogeneous layers on [0, h_top) for LAYERED transport; 0 = none */
  double lin_a[5];          /* LINSLEY5 a_i, g/cm^2 */
  double lin_b[5];          /* LINSLEY5 b_i, g/cm^2 */
  double lin_c[5];          /* LINSLEY5 c_i, cm */
  double lin_hb[5];         /* LINSLEY5 lower layer bounds, m (lin_hb[0] = 0, ascending) */
  double kappa;             /* LINSLEY5: n - 1 at rho(0) */
  double delta0;            /* HOMOGENEOUS / LINEAR: n - 1 at h = 0 */
  double h_top;             /* m: top of the refractivity table and of the layers */
  double table_step;        /* m: refractivity table spacing (Sec. 4.1 uses 1 m) */
  double rayleigh400;       /* Rayleigh attenuation length at 400 nm in g/cm^2, ~lambda^4; 0 = none (LINSLEY5 only) */
  double aerosol_tau350;    /* vertical aerosol optical depth at 350 nm; 0 = none */
  double aerosol_height;    /* aerosol scale height, m */
  double aerosol_angstrom;  /* aerosol optical depth ~ (lambda/350)^-angstrom */
  double lambda_min_nm;     /* emitted band */
  double lambda_max_nm;
  int32_t n_lambda_bins;    /* wavelength bins of the per-layer absorption table (LAYERED), >= 1 */
  int32_t reserved0;
  double earth_radius;      /* m, CURVED transport (6.371e6) */
  double reserved[3];
} cphot_atmosphere_desc;

/* Track segments, structure of arrays, float32 device arrays of length n. The
 * caller owns them. A segment starts at (x0,y0,z0) and ends at (x1,y1,z1), the
 * particle moving with speed beta (in units of c) and charge `charge` (in
 * units of e). Segment i carries the global id first_id + i * id_stride, which
 * keys its random streams: the same id always yields the same photons. */
typedef struct {
  const float* x0; const float* y0; const float* z0;
  const float* x1; const float* y1; const float* z1;
  const float* beta;
  const float* charge;
  int64_t n;                      /* number of segments (0 is allowed) */
  int64_t first_id;               /* global id of segment 0 */
  int32_t n_showers;              /* >= 1 */
  int32_t id_stride;              /* segment i has the global id first_id + i * id_stride (0 means 1):
                                     a strided subset of a larger set keeps its segments' ids, and with
                                     them their photons */
  const int64_t* shower_offsets;  /* device int64 [n_showers + 1], ascending, [0] = 0, [n_showers] = n;
                                     may be NULL when n_showers == 1 */
  const double* shower_geom;      /* device float64 [n_showers * 5]: core x, core y (m, on the
                                     observation level), shower axis unit vector (direction of travel) */
  const float* dedx;              /* device float32 [n], energy deposit in MeV/m (FLUORESCENCE); may be NULL */
} cphot_segments;

/* What to simulate and where to collect. Host struct, read at call time. */
typedef struct {
  const cphot_atmosphere* atm;
  int32_t transport;        /* CPHOT_TRANSPORT_* */
  int32_t detector;         /* CPHOT_DETECTOR_* */
  int32_t spectrum;         /* CPHOT_SPECTRUM_* */
  int32_t bunch;            /* photons per record (>= 1); each record carries this weight */
  uint64_t seed;            /* Philox key */
  double h_obs;             /* observation level, m */
  int32_t nx, ny;           /* GRID cells */
  double cell;              /* GRID cell size, m */
  int32_t snx, sny;         /* SPHERES grid */
  double pitch;             /* SPHERES spacing, m */
  double radius;            /* SPHERES radius, m */
  int32_t n_time_bins;      /* SPHERES arrival-time bins (0 = no time histograms) */
  int32_t counts_rule;      /* CPHOT_COUNTS_ROUNDED (0): a segment's expected records mu are rounded
                               stochastically; CPHOT_COUNTS_POISSON: drawn from Poisson(mu) */
  double time_bin_ns;       /* width of a time bin, ns */
  int32_t block_size;       /* tuning: threads per block (0 = library choice) */
  int32_t grid_blocks;      /* tuning: blocks of the persistent grid (0 = library choice) */
  int32_t lds_hist;         /* tuning: 1 = privatise the counts in LDS (GRID: the whole grid if it
                               fits, else a window of it; SPHERES: the whole sphere array, an error
                               if it does not fit), 0 = global atomics only, -1 = library choice */
  int32_t hist_window;      /* tuning: GRID LDS window width in cells (0 = the largest square that fits,
                               centred on the grid) */
  int32_t hist_window_h;    /* tuning: GRID LDS window height in cells (0 = hist_window: a square); a
                               window larger than the LDS allows is shrunk to fit */
  int32_t hist_window_dx;   /* tuning: GRID LDS window centre minus grid centre, cells along x (0 =
                               centred; clamped so that the window stays inside the grid) */
  int32_t hist_window_dy;   /* tuning: the same along y */
  const cphot_surrogate* surrogate; /* SURROGATE transport: a trained network (else NULL) */
  int32_t emission;         /* CPHOT_EMIT_* bits (0 = Cherenkov) */
  int32_t cuts;             /* CPHOT_CUT_* bits (SPHERES: STRAIGHT, LAYERED or TABLE transport; GRID: PHOTON
                               with STRAIGHT, LAYERED, planar TABLE or curved transports; else 0) */
  double fl_yield[3];       /* fluorescence photons per MeV deposited, per band */
  double fl_lambda[3];      /* band wavelengths, nm (inside the atmosphere's band) */
  const cphot_table* table; /* TABLE transport: a correction table built for this atmosphere and h_obs */
  /* Detector efficiency (Sec. 4.3.1: mirrors, sensor): device float64 [n_lambda_bins of the
   * atmosphere], the probability in [0, 1] that a photon of each wavelength bin that reaches the
   * detector is recorded; a photon survives iff u < exp(-tau) x efficiency. NULL: 1. Needs an
   * atmosphere with wavelength bins. The array must hold exactly n_lambda_bins values: the
   * kernels read one per bin and cannot check the length (the Python binding does). */
  const double* efficiency;
  /* Pre-emission reduction (Sec. 4.3.1), device float64 [n_layers of the atmosphere] or NULL:
   * q_i >= the detection probability exp(-tau) x efficiency of every photon emitted in layer i
   * (cphot_reduction_table computes such a bound). A segment's expected records are multiplied by
   * q of the layer of its lowest point before rounding, and each record survives iff
   * u < exp(-tau) x efficiency / q: the same expected detections with fewer records generated.
   * A q below the true probability biases the result (the caller's bound must hold). The array
   * must hold exactly n_layers values (read per layer, unchecked by the kernels). */
  const double* reduction;
  double lambda_ref_nm;     /* DISPERSIVE: wavelength (nm) at which the atmosphere's n - 1 is stated */
} cphot_detector;

/* Outputs, accumulated (+=) so that chunked calls need no host work; the caller
 * zeroes them first. Device buffers owned by the caller. */
typedef struct {
  void* bins;               /* GRID: [n_showers][ny][nx]; SPHERES: [n_showers][snx*sny] */
  int32_t bins_dtype;       /* CPHOT_BINS_U32 | CPHOT_BINS_U64 | CPHOT_BINS_F64 */
  int32_t reserved0;
  int64_t bins_capacity;    /* elements available at `bins` */
  uint32_t* time_hist;      /* SPHERES with n_time_bins > 0: [n_showers][snx*sny][n_time_bins + 1],
                               last bin = overflow; weights added as uint32 */
  int64_t time_capacity;    /* elements available at `time_hist` */
  unsigned long long* counters; /* CPHOT_NCOUNTERS uint64, may be NULL */
} cphot_bins;

/* One photon record for parity checks (64 bytes). */
typedef struct {
  uint64_t seg;     /* global segment id */
  uint32_t k;       /* record index within the segment */
  int32_t state;    /* 0 binned, 1 upward, 2 absorbed, 3 outside, 4 not emitted (DISPERSIVE) */
  int32_t bin;      /* grid cell or sphere index, -1 if none */
  int32_t tbin;     /* time bin (SPHERES), -1 if none */
  float x, y, z;    /* arrival point (ground or sphere entry) */
  float t;          /* ns after the shower plane front */
  float tau;        /* optical depth */
  float lambda;     /* nm */
  float dx, dy, dz; /* emission direction */
  float u_abs;      /* survival uniform */
} cphot_photon_record;
/* For fluorescence records, k counts from the segment's first record: Cherenkov
 * records come first, then bands 0, 1, 2 (the record's source follows from the
 * segment's counts). */

/* ABI version (CPHOT_ABI_VERSION). */
int cphot_version(void);

/* Static text for a status code. */
const char* cphot_status_string(int status);

/* Text of the most recent failure on the calling thread ("" if none). */
const char* cphot_last_error(void);

/* Build an atmosphere on the current device (Sec. 2.3.1, 3.3, 4.1). The library
 * tabulates n - 1 every table_step metres on [0, h_top] in FP64 (looked up by
 * direct index mapping and linear interpolation, Sec. 4.1, Listing 4.1) and,
 * with n_layers > 0, per-layer n - 1 at each layer's mid-height and per-layer
 * extinction per metre for each wavelength bin centre (Rayleigh from the
 * depth difference, aerosol from its exponential column). The handle owns all
 * device tables, is immutable and may be shared by concurrent streams.
 * Errors: INVALID_ARG (bad fields), OUT_OF_MEMORY, HIP. Synchronous. */
int cphot_make_atmosphere(const cphot_atmosphere_desc* desc, cphot_atmosphere** out);

/* Release an atmosphere (NULL allowed). The caller must ensure no enqueued
 * work still uses it. */
void cphot_destroy_atmosphere(cphot_atmosphere* atm);

/* Propagate every segment's photons to the detector and accumulate bins and
 * counters (Sec. 5.1 stages: import and filter, generate, filter, propagate).
 * Per segment: refractivity at the midpoint, threshold beta n > 1, expected
 * records mu = 2 pi alpha z^2 (1/lam_min - 1/lam_max) L sin^2(theta) / bunch,
 * rounded stochastically with the segment's own random word. Per record:
 * position along the track, azimuth on the cone cos(theta) = 1/(beta n), wavelength
 * and survival drawn from Philox4x32-10 keyed by (seed) with counter
 * (record index, segment id, tag). Asynchronous on `stream`.
 * Errors: INVALID_ARG (null or inconsistent fields, capacity of bins or
 * time_hist too small, spheres overlapping their cells or straddling a layer
 * boundary), HIP. */
int cphot_propagate(const cphot_segments* seg, const cphot_detector* det, cphot_bins* out, void* stream);

/* Records per segment (0 for skipped or below-threshold segments) into the
 * device int32 array `counts` [seg->n] and, if `expected` is not NULL, the
 * expected number of records mu (FP64, 0 where no photons are drawn) into the
 * device array `expected` [seg->n]. Same arithmetic as cphot_propagate.
 * Asynchronous. Errors: INVALID_ARG, HIP. */
int cphot_segment_counts(const cphot_segments* seg, const cphot_detector* det, int32_t* counts, double* expected,
                         void* stream);

/* Every record of every segment, written to the device array `records` at
 * position record_offsets[i] + k for record k of segment i (record_offsets is
 * a device int64 array [seg->n], e.g. the exclusive sum of
 * cphot_segment_counts). `capacity` is the length of `records`; records that
 * would fall beyond it are dropped. Same arithmetic as cphot_propagate; bins
 * are not touched. Asynchronous. Errors: INVALID_ARG, HIP. */
int cphot_trace_records(const cphot_segments* seg, const cphot_detector* det, const int64_t* record_offsets,
                        cphot_photon_record* records, int64_t capacity, void* stream);

/* ---------------------------------------------------------------- captured steps, tuning
 * A "step" is one whole propagation of a batch: clear the outputs (with a fill
 * kernel, no memset nodes), then cphot_propagate. cphot_step_create captures it
 * into an executable HIP graph bound to the given buffers (their pointers,
 * sizes and the detector settings are baked in); cphot_step_launch replays it
 * with one graph launch. Batches of many showers (segments with
 * shower_offsets) run as one kernel launch inside the step.
 * Errors: as cphot_propagate, plus HIP for capture failures. */
typedef struct cphot_step cphot_step;

int cphot_step_create(const cphot_segments* seg, const cphot_detector* det, const cphot_bins* out,
                      int32_t clear_outputs, cphot_step** step);
int cphot_step_launch(cphot_step* step, void* stream);
void cphot_step_destroy(cphot_step* step);

/* Result of cphot_autotune: the launch shape to put into cphot_detector. */
typedef struct {
  int32_t block_size;
  int32_t grid_blocks;   /* 0 = one block per tile */
  int32_t lds_hist;
  int32_t bunch;
  int32_t hist_window;   /* LDS window width in cells (0 with lds_hist 0) */
  int32_t hist_window_h; /* LDS window height in cells (0 with lds_hist 0) */
  double ms;             /* mean time of one propagation with this shape */
  double photons_per_s;  /* records generated x bunch / time */
  int32_t hist_window_dx, hist_window_dy;  /* window centre minus grid centre, cells */
} cphot_tuning;

/* Times cphot_propagate over candidate launch shapes (block size 128 / 256 /
 * 512; one block per tile or a persistent grid of 2, 3, 4 or 8 blocks per CU; LDS grid
 * histogram off, or on with the whole grid when it fits, else with windows:
 * the largest centred square, and rectangles fitted to the photon footprint of
 * a pilot launch (global atomics only; counts summed over showers): for a few
 * areas up to the LDS budget and aspect ratios from 1:4 to 4:1, the rectangle
 * that holds the most photons) and over the bunch sizes in
 * `bunch_candidates` (n_bunch values >= 1; NULL = the detector's own), `reps`
 * timed launches each after one warm-up, and returns the shape and bunch with
 * the most photons per second. Larger bunches trade statistical resolution for
 * speed: the caller lists only bunch sizes its bins can afford. The outputs in
 * `out` are overwritten by the trial runs. Synchronous (waits on `stream`).
 * Errors: INVALID_ARG, HIP. */
int cphot_autotune(const cphot_segments* seg, const cphot_detector* det, cphot_bins* out,
                   const int32_t* bunch_candidates, int32_t n_bunch, int32_t reps, cphot_tuning* best, void* stream);

/* cphot_autotune with an accuracy constraint on the bunch size. A bunch of b
 * photons moves b photons at once, so bins are coarser draws of the same density
 * (the thesis weighs bunch size against statistical resolution, Sec. 5.3.2). Each
 * candidate b is run once with the detector's own launch shape and its bins are
 * compared cell by cell with those of bunch 1 (the finest statistics):
 * err_b = max over cells with at least `min_count` bunch-1 photons of
 * |n_b - n_1| / n_1 (0 for b = 1). Only candidates with err_b <= max_error are
 * handed to cphot_autotune (bunch 1 always is), which picks the fastest shape
 * and bunch among them. `bin_errors` (may be NULL) receives err_b per candidate,
 * in the order given. Outputs are overwritten; synchronous on `stream`.
 * Errors: INVALID_ARG (no candidates, a candidate < 1, max_error < 0,
 * min_count < 1, no bins), HIP. */
int cphot_autotune_accuracy(const cphot_segments* seg, const cphot_detector* det, cphot_bins* out,
                            const int32_t* bunch_candidates, int32_t n_bunch, int32_t reps, double max_error,
                            double min_count, double* bin_errors, cphot_tuning* best, void* stream);

/* cphot_autotune behind a cache of results keyed by a configuration signature:
 * the device (architecture name and compute-unit count), the ABI version, the
 * atmosphere's profile, layer and wavelength-bin counts, every detector setting
 * except the launch shape (transport, detector kind and geometry, spectrum,
 * emission, counts rule, cuts, bunch, time bins, which optional tables are set),
 * the segment and shower counts, the bunch candidates and `reps`. A signature
 * seen before returns its stored result (`*hit` = 1, nothing launched, `out`
 * untouched); otherwise cphot_autotune runs and its result is stored (`*hit` =
 * 0). The cache lives in process memory; with `cache_path` (may be NULL) it is
 * also a text file, read on the first call that names it and appended to after
 * each new tuning, so that later processes on the same kind of device skip the
 * search. `hit` may be NULL. The stored shape is a timing result: it holds for
 * inputs of the same sizes, not for the same data only. Synchronous on a miss.
 * Errors: as cphot_autotune; INVALID_ARG when the file cannot be appended to. */
int cphot_autotune_cached(const cphot_segments* seg, const cphot_detector* det, cphot_bins* out,
                          const int32_t* bunch_candidates, int32_t n_bunch, int32_t reps, const char* cache_path,
                          cphot_tuning* best, int32_t* hit, void* stream);

/* Forget every cached tuning result of this process (files are not touched; a
 * file named again is read again). */
void cphot_autotune_cache_clear(void);

/* ---------------------------------------------------------------- streaming from host memory
 * A segment set too large to keep in device memory at once (the thesis feeds the
 * photon stage chunk by chunk from the shower simulation, Sec. 5.1, 5.4) is read
 * from host memory in chunks: each chunk is copied host -> pinned staging (by up to
 * 8 host threads) -> device on the streamer's own copy stream while the previous
 * chunk propagates on the caller's stream; columns that are page-locked already
 * (hipHostMalloc, a pinned tensor; every column of the call) are copied to the device
 * directly. Chunk c gets first_id + c * chunk_segments, so the photons are those of
 * one cphot_propagate over the whole set. Bins accumulate across chunks.
 *
 * cphot_streamer_create allocates two device chunk buffers and two pinned host
 * staging buffers of `chunk_segments` segments (36 B each with dE/dx) on the
 * current device; the handle is used on that device by one host thread at a
 * time. Errors: INVALID_ARG (chunk_segments < 1), OUT_OF_MEMORY, HIP. */
typedef struct cphot_streamer cphot_streamer;

/* Host-resident segments of one shower. */
typedef struct {
  const float *x0, *y0, *z0, *x1, *y1, *z1, *beta, *charge; /* host float32 [n] */
  const float* dedx;        /* host float32 [n] or NULL */
  int64_t n;
  int64_t first_id;
  const double* shower_geom; /* device float64 [5]: core x, core y, axis unit vector */
} cphot_host_segments;

int cphot_streamer_create(int64_t chunk_segments, cphot_streamer** out);

/* Propagates all of `host` with `det` into `out` (accumulating), enqueueing the
 * kernels on `stream`. Returns once the last chunk has been copied to the device
 * and its propagation enqueued (the host arrays may then be reused); the caller
 * synchronises `stream` before reading `out`. Argument checks as
 * cphot_propagate, done for the whole set before the first copy. Errors:
 * INVALID_ARG, UNSUPPORTED (several showers), HIP. */
int cphot_streamer_run(cphot_streamer* s, const cphot_host_segments* host, const cphot_detector* det,
                       cphot_bins* out, void* stream);

void cphot_streamer_destroy(cphot_streamer* s);

/* ---------------------------------------------------------------- correction table
 * Interpolation tracing (Sec. 4.4.1): the correction between straight-line and
 * iterative propagation, tabulated once per atmosphere and observation level and
 * interpolated bilinearly per photon. The exact layered result jumps where the
 * emission height crosses a layer boundary (the start layer fixes Snell's
 * invariant of a given direction), so heights are tabulated layer by layer, n_h
 * nodes from each layer's bottom (h_obs for the observation layer) to its top,
 * for the layers from h_obs up to the one containing h_hi, and never
 * interpolated across a boundary; directions on n_c nodes uniform in tan of the
 * (local) zenith angle from 0 to that of cos = c_lo (the corrections are smooth
 * in tan, with a square-root cusp at the vertical in cos). Each node holds,
 * relative to the straight path L to the
 * observation level (planar: L = (h_e - h_obs) / cos; curved: the chord to the
 * sphere R + h_obs): the landing offset along the photon's azimuth (planar:
 * horizontal offset; curved: extra ground distance), the optical path excess
 * (path - L) + sum (n - 1) l, and the Rayleigh and aerosol parts of the optical
 * depth, sum_i R_i l_i and sum_i A_i l_i, so that tau(lambda) = R(lambda) tau_R +
 * A(lambda) tau_A with the atmosphere's spectral factors (all in metres; over
 * planar layers they are linear in the height within a layer, so the height
 * interpolation is exact there). The nodes come from the exact walk carried in
 * FP64 on the GPU. */
typedef struct {
  int32_t geometry;   /* CPHOT_SURROGATE_PLANAR | CPHOT_SURROGATE_CURVED */
  int32_t n_h, n_c;   /* nodes per layer in height (>= 2) and in tan zenith (>= 2) */
  int32_t reserved0;
  double h_obs;       /* observation level, m (the detector's must match) */
  double h_hi;        /* highest emission height tabulated, m (<= h_top) */
  double c_lo;        /* lowest cos zenith tabulated, in (0, 1) */
} cphot_table_desc;

/* Build a table on the current device from `atm` (which must have layers).
 * Synchronous. The handle owns 16 B x n_h x n_c of device memory.
 * Errors: INVALID_ARG, OUT_OF_MEMORY, HIP. */
int cphot_table_create(const cphot_table_desc* desc, const cphot_atmosphere* atm, cphot_table** out);

/* Release a table (NULL allowed); no enqueued work may still use it. */
void cphot_table_destroy(cphot_table* t);

/* Upper bound of the detection probability per layer for the pre-emission
 * reduction (Sec. 4.3.1): host float64 out[n_layers], out[i] = (1 + 1e-6) x
 * max over wavelength bins k of efficiency[k] x exp(-tau_k(i)), where tau_k(i) is
 * the vertical optical depth from the bottom of layer i down to h_obs (0 for the
 * observation layer and below) at the bin's longest wavelength, with the smaller
 * of the layer-average and the exact column in the observation layer. Any path
 * from a point of layer i down to the observation level is at least that long
 * through the same layers (planar or spherical shells, straight or refracted), so
 * the bound holds for every photon emitted there. `efficiency` is host float64 [n_lambda_bins] or NULL (1).
 * Errors: INVALID_ARG (atmosphere without layers, h_obs outside [0, h_top),
 * efficiency outside [0, 1]). */
int cphot_reduction_table(const cphot_atmosphere* atm, double h_obs, const double* efficiency, double* out);

/* Interpolated corrections for device float32 X [n][5] (emission height, cos
 * zenith, azimuth (unused), wavelength, observation level (unused: the table's))
 * into Y [n][4] = (offset along the azimuth, 0, optical path excess, log T), in
 * metres for the straight path of each input, as the propagation applies them;
 * rows outside the table get NaN. For checks. Asynchronous. Errors: INVALID_ARG. */
int cphot_table_lookup(const cphot_table* t, const cphot_atmosphere* atm, const float* X, float* Y, int64_t n,
                       void* stream);

/* ---------------------------------------------------------------- transport surrogate
 * A network 5 -> 64 -> 64 -> 4 (ReLU hidden units, linear output, bf16 weights on
 * the matrix cores with FP32 accumulation) that maps a photon's (emission height
 * h_e in m, cos of its zenith angle, azimuth atan2(u_y, u_x) in rad, wavelength
 * in nm (the centre of its absorption-table bin), observation level in m) to
 * (dx, dy): the offset of the layered landing point from the straight-line
 * landing point, e: the optical path excess sum(n l) - straight length (m), and
 * log T = -tau. It plays the role of the thesis's precomputed correction
 * between straight-line and iterative propagation (Sec. 4.4.1), learned from
 * photons the exact layered tracer produces. Inputs are mapped from the
 * domain box to [-1, 1]; outputs are standardised by the training targets'
 * mean and standard deviation. Parameters: one FP32 vector of 4804 values,
 * W1[5][64], b1[64], W2[64][64], b2[64], W3[64][4], b3[4] (W[in][out]).
 * Normalisation vector (24 floats): in_lo[5], in_hi[5], 2/(in_hi - in_lo)[5],
 * 0, out_mean[4], out_std[4]. */
typedef struct {
  double in_lo[5];     /* domain box, inputs in the order above; cos zenith in [0, 1] */
  double in_hi[5];
  int32_t max_batch;   /* largest training batch (multiple of 64, <= 2^22) */
  int32_t geometry;    /* CPHOT_SURROGATE_PLANAR | CPHOT_SURROGATE_CURVED */
  uint64_t init_seed;  /* He-uniform initial weights, zero biases */
} cphot_surrogate_desc;

/* Surrogate geometry. PLANAR: planar layers, as above. CURVED: spherical shells
 * of a curved Earth (Sec. 3.3.4); zenith and height are local (angle to the
 * radial, height above the sphere R), and the outputs, each per metre of the
 * straight chord L to the sphere R + h_obs, are the extra ground distance
 * (psi - psi_chord)(R + h_obs) / L of the arrival point along the photon's
 * azimuth, the offset across it / L (zero by symmetry), the optical path excess
 * ((path - L) + sum (n - 1) l) / L, and log T / L. A detector with SURROGATE
 * transport and a CURVED surrogate traces like CURVED transport (ground grid
 * only), photons outside the domain exactly. */
#define CPHOT_SURROGATE_PLANAR 0
#define CPHOT_SURROGATE_CURVED 1

/* Allocate a surrogate on the current device. Synchronous.
 * Errors: INVALID_ARG, OUT_OF_MEMORY, HIP. */
int cphot_surrogate_create(const cphot_surrogate_desc* desc, cphot_surrogate** out);

/* Release a surrogate (NULL allowed); no enqueued work may still use it. */
void cphot_surrogate_destroy(cphot_surrogate* s);

/* Training samples first .. first+n-1 into device float32 X [n][5] and Y [n][4]:
 * inputs drawn uniformly in the domain box (emission height at or above the
 * observation level, a uniformly drawn wavelength bin) from Philox blocks with
 * counters (i low, 0 or 1, i high, 8) keyed by `seed`, targets from the exact
 * layered tracer of `atm` (which must have layers) for the surrogate's geometry
 * (CURVED: the shell walk carried in FP64 from a start above the Earth point
 * (0, 0), compared with the FP64 chord). Asynchronous.
 * Errors: INVALID_ARG (domain outside the atmosphere's layers or band), HIP. */
int cphot_surrogate_make_training_set(const cphot_surrogate* s, const cphot_atmosphere* atm, int64_t first,
                                      int64_t n, uint64_t seed, float* X, float* Y, void* stream);

/* Output normalisation from the targets Y [n][4] (device): mean and standard
 * deviation per output. Must precede training. Asynchronous. */
int cphot_surrogate_fit_normalization(cphot_surrogate* s, const float* Y, int64_t n, void* stream);

/* `steps` Adam steps (beta 0.9/0.999, lr cosine-decayed to lr/100) on the mean
 * squared error of standardised outputs, minibatches of `batch` consecutive
 * samples cycling through X [n][5], Y [n][4] (device). loss_out (device float
 * [steps], may be NULL) receives each step's loss. Asynchronous.
 * Errors: INVALID_ARG, UNSUPPORTED (normalisation not set), HIP. */
int cphot_surrogate_train(cphot_surrogate* s, const float* X, const float* Y, int64_t n, int32_t batch,
                          int32_t steps, float lr, float* loss_out, void* stream);

/* Gradient of the loss over the n samples (n a multiple of 64, <= max_batch)
 * with respect to the parameter vector into device float grad [4804], and the
 * loss into device float loss [1] (may be NULL); no update. Asynchronous. */
int cphot_surrogate_gradient(cphot_surrogate* s, const float* X, const float* Y, int64_t n, float* grad,
                             float* loss, void* stream);

/* cphot_surrogate_gradient for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving or training loops, harnesses that forbid
 * hipMalloc): the per-block partial gradients and loss shares live in a static
 * workspace of the library instead of the surrogate's buffers, so the call makes
 * no allocation of any kind. Limit: n a multiple of 64, at most 4096 samples (the
 * workspace holds 64 blocks x 4804 partial gradients + 64 loss shares, 1.23 MB per
 * device, kept until the process ends). Every call on one device shares that
 * device's workspace: calls that overlap on one device (other streams, other host
 * threads) race and must be ordered by the caller. Results equal those of
 * cphot_surrogate_gradient bit for bit. Must be called with the surrogate's device
 * current. Asynchronous. Errors: INVALID_ARG (null buffers, n out of range, another
 * device current), HIP. */
int cphot_surrogate_gradient_noalloc(cphot_surrogate* s, const float* X, const float* Y, int64_t n, float* grad,
                                     float* loss, void* stream);

/* Network outputs Y [n][4] for inputs X [n][5] (device, raw units). Asynchronous. */
int cphot_surrogate_forward(const cphot_surrogate* s, const float* X, float* Y, int64_t n, void* stream);

/* Copy the parameter vector (4804 floats) and the normalisation (24 floats)
 * to / from host memory; either pointer may be NULL. Synchronous (waits for
 * the device). */
int cphot_surrogate_get_params(const cphot_surrogate* s, float* params, float* norm);
int cphot_surrogate_set_params(cphot_surrogate* s, const float* params, const float* norm);

#ifdef __cplusplus
}
#endif

#endif /* CPHOT_H */
