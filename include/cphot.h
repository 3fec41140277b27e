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

#define CPHOT_ABI_VERSION 1
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

/* Detectors. GRID: nx x ny square cells of `cell` metres on the observation
 * level, centred on each shower's core. SPHERES: snx x sny bounding spheres of
 * `radius` at `pitch` spacing, centred on the core at h_obs (Sec. 6.2, bounding
 * spheres of telescopes), with optional arrival-time histograms. */
#define CPHOT_DETECTOR_GRID 0
#define CPHOT_DETECTOR_SPHERES 1

/* Emission wavelength: UNIFORM on [lam_min, lam_max], or FRANK_TAMM with
 * dN/dlambda ~ 1/lambda^2 (Eq. 2.4). */
#define CPHOT_SPECTRUM_UNIFORM 0
#define CPHOT_SPECTRUM_FRANK_TAMM 1

/* Bin element types of cphot_bins.bins. */
#define CPHOT_BINS_U32 0
#define CPHOT_BINS_U64 1

/* Counter slots (uint64) of cphot_bins.counters. After a call,
 * records_generated = records_upward + records_absorbed + records_outside + records_binned. */
#define CPHOT_C_SEGMENTS_IN 0
#define CPHOT_C_SEGMENTS_SKIPPED 1          /* non-finite, zero length, beta outside (0,1) */
#define CPHOT_C_SEGMENTS_BELOW_THRESHOLD 2  /* beta n <= 1 (Sec. 2.2.1) */
#define CPHOT_C_RECORDS_GENERATED 3
#define CPHOT_C_RECORDS_UPWARD 4
#define CPHOT_C_RECORDS_ABSORBED 5
#define CPHOT_C_RECORDS_OUTSIDE 6           /* missed the grid / every sphere, or emitted below h_obs */
#define CPHOT_C_RECORDS_BINNED 7
#define CPHOT_C_PHOTONS_BINNED 8            /* records_binned x bunch size */

typedef struct cphot_atmosphere cphot_atmosphere;

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
  double reserved[4];
} cphot_atmosphere_desc;

/* Track segments, structure of arrays, float32 device arrays of length n. The
 * caller owns them. A segment starts at (x0,y0,z0) and ends at (x1,y1,z1), the
 * particle moving with speed beta (in units of c) and charge `charge` (in
 * units of e). Segment i carries the global id first_id + i, which keys its
 * random streams: the same id always yields the same photons. */
typedef struct {
  const float* x0; const float* y0; const float* z0;
  const float* x1; const float* y1; const float* z1;
  const float* beta;
  const float* charge;
  int64_t n;                      /* number of segments (0 is allowed) */
  int64_t first_id;               /* global id of segment 0 */
  int32_t n_showers;              /* >= 1 */
  int32_t reserved0;
  const int64_t* shower_offsets;  /* device int64 [n_showers + 1], ascending, [0] = 0, [n_showers] = n;
                                     may be NULL when n_showers == 1 */
  const double* shower_geom;      /* device float64 [n_showers * 5]: core x, core y (m, on the
                                     observation level), shower axis unit vector (direction of travel) */
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
  int32_t reserved0;
  double time_bin_ns;       /* width of a time bin, ns */
  int32_t block_size;       /* tuning: threads per block (0 = library choice) */
  int32_t grid_blocks;      /* tuning: blocks of the persistent grid (0 = library choice) */
  int32_t lds_hist;         /* tuning: 1 = privatise the grid histogram in LDS, 0 = global atomics, -1 = library choice */
  int32_t reserved1;
} cphot_detector;

/* Outputs, accumulated (+=) so that chunked calls need no host work; the caller
 * zeroes them first. Device buffers owned by the caller. */
typedef struct {
  void* bins;               /* GRID: [n_showers][ny][nx]; SPHERES: [n_showers][snx*sny] */
  int32_t bins_dtype;       /* CPHOT_BINS_U32 | CPHOT_BINS_U64 */
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
  int32_t state;    /* 0 binned, 1 upward, 2 absorbed, 3 outside */
  int32_t bin;      /* grid cell or sphere index, -1 if none */
  int32_t tbin;     /* time bin (SPHERES), -1 if none */
  float x, y, z;    /* arrival point (ground or sphere entry) */
  float t;          /* ns after the shower plane front */
  float tau;        /* optical depth */
  float lambda;     /* nm */
  float dx, dy, dz; /* emission direction */
  float u_abs;      /* survival uniform */
} cphot_photon_record;

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

#ifdef __cplusplus
}
#endif

#endif /* CPHOT_H */
