"""Thin ctypes binding of libcphot.so (include/cphot.h).

Argument marshalling only: every step of the photon path runs in the HIP
kernels. PyTorch supplies device memory and streams. Importing this module does
not touch the GPU; the first call loads the library and fails loudly if it has
not been built or cannot be loaded.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcphot.so")

OK = 0
ERR_INVALID_ARG = -1
ERR_OUT_OF_MEMORY = -2
ERR_HIP = -3
ERR_UNSUPPORTED = -4
ERR_CAPACITY = -5
NCOUNTERS = 16

PROFILE = {"linsley5": 0, "homogeneous": 1, "linear": 2}
TRANSPORT = {"straight": 0, "layered": 1, "surrogate": 2, "curved": 3, "table": 4, "curved_walk": 5}
COUNTS = {"rounded": 0, "poisson": 1}  # record count per segment from its expected value
CUTS = {"track": 1, "photon": 2}  # data-reduction bounds for spheres (never drop a possible hit)
EMISSION = {"cherenkov": 1, "fluorescence": 2, "both": 3}
DETECTOR = {"grid": 0, "spheres": 1}
SPECTRUM = {"uniform": 0, "frank_tamm": 1, "dispersive": 2}
BINS = {"u32": 0, "u64": 1, "f64": 2}
GEOMETRY = {"planar": 0, "curved": 1}
COUNTERS = ["segments_in", "segments_skipped", "segments_below_threshold", "records_generated",
            "records_upward", "records_absorbed", "records_outside", "records_binned", "photons_binned",
            "surrogate_fallback", "records_fluorescence"]


class CphotError(RuntimeError):
    def __init__(self, fn, status, text):
        super().__init__(f"{fn} failed with status {status}: {text}")
        self.status = status


class AtmosphereDesc(C.Structure):
    _fields_ = [("profile", C.c_int32), ("n_layers", C.c_int32),
                ("lin_a", C.c_double * 5), ("lin_b", C.c_double * 5), ("lin_c", C.c_double * 5),
                ("lin_hb", C.c_double * 5), ("kappa", C.c_double), ("delta0", C.c_double), ("h_top", C.c_double),
                ("table_step", C.c_double), ("rayleigh400", C.c_double), ("aerosol_tau350", C.c_double),
                ("aerosol_height", C.c_double), ("aerosol_angstrom", C.c_double), ("lambda_min_nm", C.c_double),
                ("lambda_max_nm", C.c_double), ("n_lambda_bins", C.c_int32), ("reserved0", C.c_int32),
                ("earth_radius", C.c_double), ("reserved", C.c_double * 3)]


class Segments(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in ("x0", "y0", "z0", "x1", "y1", "z1", "beta", "charge")] + \
               [("n", C.c_int64), ("first_id", C.c_int64), ("n_showers", C.c_int32), ("id_stride", C.c_int32),
                ("shower_offsets", C.c_void_p), ("shower_geom", C.c_void_p), ("dedx", C.c_void_p)]


class Detector(C.Structure):
    _fields_ = [("atm", C.c_void_p), ("transport", C.c_int32), ("detector", C.c_int32), ("spectrum", C.c_int32),
                ("bunch", C.c_int32), ("seed", C.c_uint64), ("h_obs", C.c_double), ("nx", C.c_int32),
                ("ny", C.c_int32), ("cell", C.c_double), ("snx", C.c_int32), ("sny", C.c_int32),
                ("pitch", C.c_double), ("radius", C.c_double), ("n_time_bins", C.c_int32),
                ("counts_rule", C.c_int32), ("time_bin_ns", C.c_double), ("block_size", C.c_int32),
                ("grid_blocks", C.c_int32), ("lds_hist", C.c_int32), ("hist_window", C.c_int32),
                ("hist_window_h", C.c_int32), ("hist_window_dx", C.c_int32), ("hist_window_dy", C.c_int32),
                ("surrogate", C.c_void_p), ("emission", C.c_int32), ("cuts", C.c_int32),
                ("fl_yield", C.c_double * 3), ("fl_lambda", C.c_double * 3), ("table", C.c_void_p),
                ("efficiency", C.c_void_p), ("reduction", C.c_void_p), ("lambda_ref_nm", C.c_double)]


class SurrogateDesc(C.Structure):
    _fields_ = [("in_lo", C.c_double * 5), ("in_hi", C.c_double * 5), ("max_batch", C.c_int32),
                ("geometry", C.c_int32), ("init_seed", C.c_uint64)]


class TableDesc(C.Structure):
    _fields_ = [("geometry", C.c_int32), ("n_h", C.c_int32), ("n_c", C.c_int32), ("reserved0", C.c_int32),
                ("h_obs", C.c_double), ("h_hi", C.c_double), ("c_lo", C.c_double)]


class Tuning(C.Structure):
    _fields_ = [("block_size", C.c_int32), ("grid_blocks", C.c_int32), ("lds_hist", C.c_int32),
                ("bunch", C.c_int32), ("hist_window", C.c_int32), ("hist_window_h", C.c_int32), ("ms", C.c_double),
                ("photons_per_s", C.c_double), ("hist_window_dx", C.c_int32), ("hist_window_dy", C.c_int32)]


# launch-shape fields of cphot_detector that cphot_autotune returns
SHAPE_KEYS = ("block_size", "grid_blocks", "lds_hist", "hist_window", "hist_window_h", "hist_window_dx",
              "hist_window_dy")


def shape_of(tuning: dict) -> dict:
    """The launch shape of an autotune result, as make_detector keywords."""
    return {k: tuning[k] for k in SHAPE_KEYS}


def _tuning_dict(t) -> dict:
    return dict(block_size=t.block_size, grid_blocks=t.grid_blocks, lds_hist=t.lds_hist, hist_window=t.hist_window,
                hist_window_h=t.hist_window_h, hist_window_dx=t.hist_window_dx, hist_window_dy=t.hist_window_dy,
                bunch=t.bunch, ms=t.ms, photons_per_s=t.photons_per_s)


class HostSegments(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in ("x0", "y0", "z0", "x1", "y1", "z1", "beta", "charge", "dedx")] + [
        ("n", C.c_int64), ("first_id", C.c_int64), ("shower_geom", C.c_void_p)]


class Bins(C.Structure):
    _fields_ = [("bins", C.c_void_p), ("bins_dtype", C.c_int32), ("reserved0", C.c_int32),
                ("bins_capacity", C.c_int64), ("time_hist", C.c_void_p), ("time_capacity", C.c_int64),
                ("counters", C.c_void_p)]


RECORD_FIELDS = [("seg", "u8"), ("k", "u4"), ("state", "i4"), ("bin", "i4"), ("tbin", "i4"), ("x", "f4"),
                 ("y", "f4"), ("z", "f4"), ("t", "f4"), ("tau", "f4"), ("lambda", "f4"), ("dx", "f4"),
                 ("dy", "f4"), ("dz", "f4"), ("u_abs", "f4")]
RECORD_BYTES = 64

_lock = threading.Lock()
_lib = None
ABI_VERSION = 4  # CPHOT_ABI_VERSION of include/cphot.h that the ctypes structs below mirror


def lib():
    """The loaded library; raises if it is missing (no fallback exists)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"libcphot.so is not built ({LIB_PATH}); run __graft_entry__.build()")
            L = C.CDLL(LIB_PATH)
            P = C.c_void_p
            L.cphot_version.restype = C.c_int
            if L.cphot_version() != ABI_VERSION:
                raise RuntimeError(f"libcphot.so has ABI version {L.cphot_version()}, this binding's structs are "
                                   f"version {ABI_VERSION}: rebuild with __graft_entry__.build()")
            L.cphot_status_string.argtypes = [C.c_int]
            L.cphot_status_string.restype = C.c_char_p
            L.cphot_last_error.restype = C.c_char_p
            L.cphot_make_atmosphere.argtypes = [C.POINTER(AtmosphereDesc), C.POINTER(C.c_void_p)]
            L.cphot_make_atmosphere.restype = C.c_int
            L.cphot_destroy_atmosphere.argtypes = [P]
            L.cphot_propagate.argtypes = [C.POINTER(Segments), C.POINTER(Detector), C.POINTER(Bins), P]
            L.cphot_propagate.restype = C.c_int
            L.cphot_segment_counts.argtypes = [C.POINTER(Segments), C.POINTER(Detector), P, P, P]
            L.cphot_segment_counts.restype = C.c_int
            L.cphot_trace_records.argtypes = [C.POINTER(Segments), C.POINTER(Detector), P, P, C.c_int64, P]
            L.cphot_trace_records.restype = C.c_int
            L.cphot_surrogate_create.argtypes = [C.POINTER(SurrogateDesc), C.POINTER(C.c_void_p)]
            L.cphot_surrogate_destroy.argtypes = [P]
            L.cphot_surrogate_make_training_set.argtypes = [P, P, C.c_int64, C.c_int64, C.c_uint64, P, P, P]
            L.cphot_surrogate_fit_normalization.argtypes = [P, P, C.c_int64, P]
            L.cphot_surrogate_train.argtypes = [P, P, P, C.c_int64, C.c_int32, C.c_int32, C.c_float, P, P]
            L.cphot_surrogate_gradient.argtypes = [P, P, P, C.c_int64, P, P, P]
            L.cphot_surrogate_gradient_noalloc.argtypes = [P, P, P, C.c_int64, P, P, P]
            L.cphot_surrogate_gradient_noalloc.restype = C.c_int
            L.cphot_surrogate_forward.argtypes = [P, P, P, C.c_int64, P]
            L.cphot_surrogate_get_params.argtypes = [P, P, P]
            L.cphot_surrogate_set_params.argtypes = [P, P, P]
            L.cphot_step_create.argtypes = [C.POINTER(Segments), C.POINTER(Detector), C.POINTER(Bins), C.c_int32,
                                            C.POINTER(C.c_void_p)]
            L.cphot_step_create.restype = C.c_int
            L.cphot_step_launch.argtypes = [P, P]
            L.cphot_step_launch.restype = C.c_int
            L.cphot_step_destroy.argtypes = [P]
            L.cphot_autotune.argtypes = [C.POINTER(Segments), C.POINTER(Detector), C.POINTER(Bins), P, C.c_int32,
                                         C.c_int32, C.POINTER(Tuning), P]
            L.cphot_autotune.restype = C.c_int
            L.cphot_autotune_cached.argtypes = [C.POINTER(Segments), C.POINTER(Detector), C.POINTER(Bins), P,
                                                C.c_int32, C.c_int32, C.c_char_p, C.POINTER(Tuning),
                                                C.POINTER(C.c_int32), P]
            L.cphot_autotune_cached.restype = C.c_int
            L.cphot_autotune_accuracy.argtypes = [C.POINTER(Segments), C.POINTER(Detector), C.POINTER(Bins), P,
                                                  C.c_int32, C.c_int32, C.c_double, C.c_double, P,
                                                  C.POINTER(Tuning), P]
            L.cphot_autotune_accuracy.restype = C.c_int
            L.cphot_autotune_cache_clear.argtypes = []
            L.cphot_autotune_cache_clear.restype = None
            L.cphot_streamer_create.argtypes = [C.c_int64, C.POINTER(C.c_void_p)]
            L.cphot_streamer_create.restype = C.c_int
            L.cphot_streamer_run.argtypes = [P, C.POINTER(HostSegments), C.POINTER(Detector), C.POINTER(Bins), P]
            L.cphot_streamer_run.restype = C.c_int
            L.cphot_streamer_destroy.argtypes = [P]
            L.cphot_table_create.argtypes = [C.POINTER(TableDesc), P, C.POINTER(C.c_void_p)]
            L.cphot_table_create.restype = C.c_int
            L.cphot_table_destroy.argtypes = [P]
            L.cphot_table_lookup.argtypes = [P, P, P, P, C.c_int64, P]
            L.cphot_table_lookup.restype = C.c_int
            for fn in ("create", "make_training_set", "fit_normalization", "train", "gradient", "forward",
                       "get_params", "set_params"):
                getattr(L, "cphot_surrogate_" + fn).restype = C.c_int
            _lib = L
    return _lib


def _check(fn, rc):
    if rc != OK:
        raise CphotError(fn, rc, lib().cphot_last_error().decode())


def _dptr(t, dtype=None, what="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{what} must be a CUDA (HIP) tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{what} must have dtype {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return t.data_ptr()


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Atmosphere:
    """Owns a cphot_atmosphere handle (device tables on the current device)."""

    def __init__(self, profile="linsley5", n_layers=0, a=None, b=None, c=None, hb=None, kappa=2.83e-4,
                 delta0=0.0, h_top=25000.0, step=1.0, rayleigh400=0.0, aer_tau350=0.0, aer_H=1200.0,
                 aer_angstrom=1.0, lam_min=300.0, lam_max=600.0, n_lam=1, earth_radius=6.371e6, **_ignored):
        d = AtmosphereDesc()
        d.profile = PROFILE[profile]
        d.n_layers = int(n_layers)
        for name, v in (("lin_a", a), ("lin_b", b), ("lin_c", c), ("lin_hb", hb)):
            if v is not None:
                getattr(d, name)[:] = tuple(float(x) for x in v)
        d.kappa, d.delta0, d.h_top, d.table_step = kappa, delta0, h_top, step
        d.rayleigh400, d.aerosol_tau350, d.aerosol_height, d.aerosol_angstrom = rayleigh400, aer_tau350, aer_H, aer_angstrom
        d.lambda_min_nm, d.lambda_max_nm = lam_min, lam_max
        d.n_lambda_bins = max(int(n_lam), 1)
        d.earth_radius = float(earth_radius)
        self.desc = d
        h = C.c_void_p()
        _check("cphot_make_atmosphere", lib().cphot_make_atmosphere(C.byref(d), C.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.cphot_destroy_atmosphere(self._h)
            self._h = None

    def __del__(self):
        self.close()


def make_detector(atm: Atmosphere, transport="straight", detector="grid", spectrum="uniform", bunch=1, seed=0,
                  h_obs=2200.0, nx=100, ny=100, cell=10.0, snx=10, sny=10, pitch=150.0, radius=6.0, n_t=0,
                  dt=1.0, block_size=0, grid_blocks=0, lds_hist=-1, hist_window=0, hist_window_h=0,
                  hist_window_dx=0, hist_window_dy=0, surrogate=None,
                  emission="cherenkov", fl_yield=(7.0, 5.0, 2.0), fl_lambda=(337.0, 357.0, 391.0), cuts=(),
                  table=None, efficiency=None, reduction=None, counts="rounded", lambda_ref=400.0) -> Detector:
    """Fields of cphot_detector by name. `spectrum`: "uniform", "frank_tamm" or
    "dispersive" (with `lambda_ref`, the wavelength in nm at which the
    atmosphere's n - 1 holds); `counts`: "rounded" (stochastic rounding of each
    segment's expected records) or "poisson"; `cuts`: any of "track", "photon";
    `efficiency` and `reduction`: float64 device tensors (per wavelength bin,
    per layer) or None."""
    d = Detector()
    d.atm = atm.handle
    d.transport, d.detector, d.spectrum = TRANSPORT[transport], DETECTOR[detector], SPECTRUM[spectrum]
    d.bunch, d.seed, d.h_obs = int(bunch), int(seed) & (2**64 - 1), float(h_obs)
    d.nx, d.ny, d.cell = int(nx), int(ny), float(cell)
    d.snx, d.sny, d.pitch, d.radius = int(snx), int(sny), float(pitch), float(radius)
    d.n_time_bins, d.time_bin_ns = int(n_t), float(dt)
    d.block_size, d.grid_blocks, d.lds_hist = int(block_size), int(grid_blocks), int(lds_hist)
    d.hist_window, d.hist_window_h = int(hist_window), int(hist_window_h)
    d.hist_window_dx, d.hist_window_dy = int(hist_window_dx), int(hist_window_dy)
    d.emission = EMISSION[emission]
    d.cuts = sum(CUTS[c] for c in cuts)
    d.counts_rule = COUNTS[counts]
    d.lambda_ref_nm = float(lambda_ref)
    d.fl_yield[:] = tuple(float(v) for v in fl_yield)
    d.fl_lambda[:] = tuple(float(v) for v in fl_lambda)
    if surrogate is not None:
        d.surrogate = surrogate.handle
    if table is not None:
        d.table = table.handle
    if efficiency is not None or reduction is not None:
        import torch
        # the kernels read one value per wavelength bin / per layer of the atmosphere
        if efficiency is not None:
            if efficiency.numel() != atm.desc.n_lambda_bins:
                raise ValueError(f"efficiency needs {atm.desc.n_lambda_bins} values (one per wavelength bin)")
            d.efficiency = _dptr(efficiency, torch.float64, "efficiency")
        if reduction is not None:
            if reduction.numel() != atm.desc.n_layers:
                raise ValueError(f"reduction needs {atm.desc.n_layers} values (one per layer)")
            d.reduction = _dptr(reduction, torch.float64, "reduction")
    d._refs = (atm, surrogate, table, efficiency, reduction)  # keep the handles and buffers alive
    return d


def reduction_table(atm: Atmosphere, h_obs: float, efficiency=None):
    """Per-layer upper bound of the detection probability (cphot_reduction_table)
    as a float64 numpy array; `efficiency`: per-wavelength-bin values or None."""
    import numpy as np
    n = atm.desc.n_layers
    out = np.zeros(n, dtype=np.float64)
    eff = None if efficiency is None else np.ascontiguousarray(efficiency, dtype=np.float64)
    _check("cphot_reduction_table",
           lib().cphot_reduction_table(atm.handle, C.c_double(float(h_obs)),
                                       None if eff is None else eff.ctypes.data_as(C.c_void_p),
                                       out.ctypes.data_as(C.c_void_p)))
    return out


def make_segments(seg: dict, geom, offsets=None, first_id: int = 0, id_stride: int = 1) -> Segments:
    """`seg`: dict of float32 CUDA tensors x0..z1, beta, charge; `geom`: float64 CUDA
    tensor [n_showers, 5]; `offsets`: int64 CUDA tensor [n_showers + 1] or None.
    Segment i carries the global id first_id + i * id_stride."""
    import torch
    s = Segments()
    n = int(seg["x0"].shape[0])
    for f in ("x0", "y0", "z0", "x1", "y1", "z1", "beta", "charge"):
        t = seg[f]
        if int(t.shape[0]) != n:
            raise ValueError(f"segment field {f} has length {t.shape[0]}, expected {n}")
        setattr(s, f, _dptr(t, torch.float32, f))
    s.n = n
    s.first_id = int(first_id)
    if int(id_stride) < 1 or int(id_stride) >= 2**31:
        raise ValueError("id_stride must be in [1, 2^31)")
    s.id_stride = int(id_stride)
    ns = int(geom.shape[0])
    s.n_showers = ns
    s.shower_geom = _dptr(geom, torch.float64, "geom")
    if seg.get("dedx") is not None:
        if int(seg["dedx"].shape[0]) != n:
            raise ValueError("dedx must have one value per segment")
        s.dedx = _dptr(seg["dedx"], torch.float32, "dedx")
    if geom.dim() != 2 or geom.shape[1] != 5:
        raise ValueError("geom must be [n_showers, 5]")
    if offsets is not None:
        if int(offsets.shape[0]) != ns + 1:
            raise ValueError("offsets must have n_showers + 1 entries")
        s.shower_offsets = _dptr(offsets, torch.int64, "offsets")
    elif ns > 1:
        raise ValueError("offsets are required for several showers")
    s._keep = (seg, geom, offsets)
    return s


def make_bins(bins, time_hist=None, counters=None) -> Bins:
    """Output descriptor: `bins` int32 (read as uint32) or int64 (read as uint64),
    `time_hist` int32 (read as uint32), `counters` int64 [16]."""
    import torch
    b = Bins()
    if bins.dtype == torch.int32:
        b.bins_dtype = BINS["u32"]
    elif bins.dtype == torch.int64:
        b.bins_dtype = BINS["u64"]
    elif bins.dtype == torch.float64:
        b.bins_dtype = BINS["f64"]
    else:
        raise TypeError("bins must be int32 (read as uint32), int64 (read as uint64) or float64")
    b.bins = _dptr(bins, None, "bins")
    b.bins_capacity = bins.numel()
    if time_hist is not None:
        b.time_hist = _dptr(time_hist, torch.int32, "time_hist")
        b.time_capacity = time_hist.numel()
    if counters is not None:
        if counters.numel() < NCOUNTERS:
            raise ValueError("counters needs 16 entries")
        b.counters = _dptr(counters, torch.int64, "counters")
    b._keep = (bins, time_hist, counters)
    return b


def propagate(seg: Segments, det: Detector, bins, time_hist=None, counters=None, stream=None):
    """Accumulates into `bins`, `time_hist` and `counters` (see make_bins)."""
    b = make_bins(bins, time_hist, counters)
    _check("cphot_propagate", lib().cphot_propagate(C.byref(seg), C.byref(det), C.byref(b), _stream_ptr(stream)))


class Table:
    """Correction table of the interpolation tracing (cphot_table_*), built on the
    GPU from the exact walk for one atmosphere and observation level."""

    def __init__(self, atm: Atmosphere, h_obs, geometry="planar", n_h=4, n_c=256, h_hi=None, c_lo=0.4):
        """n_h: nodes per layer in height (heights are never interpolated across a
        layer boundary); n_c: nodes in cos zenith on [c_lo, 1]."""
        d = TableDesc()
        d.geometry = GEOMETRY[geometry]
        d.n_h, d.n_c = int(n_h), int(n_c)
        d.h_obs = float(h_obs)
        d.h_hi = float(h_hi if h_hi is not None else atm.desc.h_top)
        d.c_lo = float(c_lo)
        self.desc, self._atm = d, atm
        h = C.c_void_p()
        _check("cphot_table_create", lib().cphot_table_create(C.byref(d), atm.handle, C.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def lookup(self, X, stream=None):
        """Interpolated (offset along the azimuth, 0, optical path excess, log T) for
        float32 CUDA X [n, 5]; NaN outside the table."""
        import torch
        Y = torch.empty((X.shape[0], 4), dtype=torch.float32, device="cuda")
        _check("cphot_table_lookup", lib().cphot_table_lookup(self._h, self._atm.handle,
                                                               C.c_void_p(_dptr(X, torch.float32, "X")),
                                                               C.c_void_p(_dptr(Y, torch.float32, "Y")),
                                                               int(X.shape[0]), _stream_ptr(stream)))
        return Y

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.cphot_table_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


class Streamer:
    """Chunked propagation of host-resident segments (cphot_streamer_*): copies of
    chunk c + 1 overlap the propagation of chunk c."""

    def __init__(self, chunk_segments: int):
        h = C.c_void_p()
        _check("cphot_streamer_create", lib().cphot_streamer_create(int(chunk_segments), C.byref(h)))
        self._h = h

    def run(self, seg_np: dict, geom, det: Detector, bins, time_hist=None, counters=None, first_id=0, stream=None):
        """`seg_np`: dict of host float32 arrays (x0..charge, optional dedx): numpy
        arrays, or CPU tensors (pinned ones are copied to the device without staging);
        `geom`: float64 CUDA tensor [1, 5]. Accumulates into the outputs."""
        import numpy as np
        import torch
        cols = {}
        hs = HostSegments()
        n = int(seg_np["x0"].shape[0])
        for f in SEGMENT_FIELDS + ("dedx",):
            if f == "dedx" and seg_np.get("dedx") is None:
                continue
            v = seg_np[f]
            if isinstance(v, torch.Tensor):
                if v.device.type != "cpu" or v.dtype != torch.float32 or not v.is_contiguous() or v.dim() != 1:
                    raise ValueError(f"segment field {f} must be a contiguous 1-D float32 CPU tensor")
                a, ptr = v, v.data_ptr()
            else:
                a = np.ascontiguousarray(v, dtype=np.float32)
                ptr = a.ctypes.data
            if a.shape[0] != n:
                raise ValueError(f"segment field {f} has length {a.shape[0]}, expected {n}")
            cols[f] = a
            setattr(hs, f, ptr)
        hs.n = n
        hs.first_id = int(first_id)
        if not isinstance(geom, torch.Tensor) or tuple(geom.shape) != (1, 5):
            raise ValueError("geom must be a [1, 5] float64 CUDA tensor")
        hs.shower_geom = _dptr(geom, torch.float64, "geom")
        b = make_bins(bins, time_hist, counters)
        _check("cphot_streamer_run", lib().cphot_streamer_run(self._h, C.byref(hs), C.byref(det), C.byref(b),
                                                               _stream_ptr(stream)))
        del cols  # copied (or, pinned, read by the copy engine) before run returns

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.cphot_streamer_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


class Step:
    """A captured propagation step (HIP graph): clear outputs + propagate."""

    def __init__(self, seg: Segments, det: Detector, bins, time_hist=None, counters=None, clear=True):
        self._b = make_bins(bins, time_hist, counters)
        self._refs = (seg, det)
        h = C.c_void_p()
        _check("cphot_step_create", lib().cphot_step_create(C.byref(seg), C.byref(det), C.byref(self._b),
                                                            1 if clear else 0, C.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _check("cphot_step_launch", lib().cphot_step_launch(self._h, _stream_ptr(stream)))

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.cphot_step_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


def autotune(seg: Segments, det: Detector, bins, time_hist=None, counters=None, bunches=None, reps=3, stream=None,
             cache=False, cache_path=None):
    """Fastest launch shape (and bunch among `bunches`) for these inputs; the
    outputs are overwritten by the trials. With `cache` (or a `cache_path`),
    cphot_autotune_cached: a configuration tuned before in this process (or
    recorded in the file) returns its stored result, with "cached": True."""
    import numpy as np
    b = make_bins(bins, time_hist, counters)
    t = Tuning()
    bc = None if not bunches else np.ascontiguousarray(bunches, dtype=np.int32)
    bp = None if bc is None else bc.ctypes.data_as(C.c_void_p)
    nb = 0 if bc is None else len(bc)
    hit = C.c_int32(0)
    if cache or cache_path:
        path = None if cache_path is None else os.fsencode(cache_path)
        _check("cphot_autotune_cached", lib().cphot_autotune_cached(C.byref(seg), C.byref(det), C.byref(b), bp, nb,
                                                                    int(reps), path, C.byref(t), C.byref(hit),
                                                                    _stream_ptr(stream)))
    else:
        _check("cphot_autotune", lib().cphot_autotune(C.byref(seg), C.byref(det), C.byref(b), bp, nb, int(reps),
                                                      C.byref(t), _stream_ptr(stream)))
    return dict(_tuning_dict(t), cached=bool(hit.value))


def autotune_accuracy(seg: Segments, det: Detector, bins, time_hist=None, counters=None, bunches=(1,), reps=3,
                      max_error=0.01, min_count=1000.0, stream=None):
    """cphot_autotune over the bunch sizes whose bins stay within max_error of the
    bunch-1 bins (cells with >= min_count photons); "bin_errors" holds each
    candidate's error, in the order of `bunches`."""
    import numpy as np
    b = make_bins(bins, time_hist, counters)
    t = Tuning()
    bc = np.ascontiguousarray(bunches, dtype=np.int32)
    errs = np.zeros(len(bc), dtype=np.float64)
    _check("cphot_autotune_accuracy",
           lib().cphot_autotune_accuracy(C.byref(seg), C.byref(det), C.byref(b), bc.ctypes.data_as(C.c_void_p),
                                         len(bc), int(reps), float(max_error), float(min_count),
                                         errs.ctypes.data_as(C.c_void_p), C.byref(t), _stream_ptr(stream)))
    return dict(_tuning_dict(t),
                bin_errors={int(k): float(e) for k, e in zip(bc, errs)}, max_error=float(max_error),
                min_count=float(min_count))


def autotune_cache_clear():
    """Forget the tuning results cached in this process."""
    lib().cphot_autotune_cache_clear()


def segment_counts(seg: Segments, det: Detector, counts, expected=None, stream=None):
    import torch
    ex = C.c_void_p(_dptr(expected, torch.float64, "expected")) if expected is not None else C.c_void_p()
    _check("cphot_segment_counts", lib().cphot_segment_counts(C.byref(seg), C.byref(det),
                                                               C.c_void_p(_dptr(counts, torch.int32, "counts")),
                                                               ex, _stream_ptr(stream)))


def trace_records(seg: Segments, det: Detector, record_offsets, records, stream=None):
    """`records`: uint8 CUDA tensor of capacity * 64 bytes."""
    import torch
    cap = records.numel() // RECORD_BYTES
    _check("cphot_trace_records",
           lib().cphot_trace_records(C.byref(seg), C.byref(det),
                                     C.c_void_p(_dptr(record_offsets, torch.int64, "record_offsets")),
                                     C.c_void_p(_dptr(records, torch.uint8, "records")), cap, _stream_ptr(stream)))


def records_to_numpy(records_u8_cpu):
    import numpy as np
    dt = np.dtype([(n, t) for n, t in RECORD_FIELDS])
    assert dt.itemsize == RECORD_BYTES
    return records_u8_cpu.numpy().view(dt)


SEGMENT_FIELDS = ("x0", "y0", "z0", "x1", "y1", "z1", "beta", "charge")


def upload(seg_np: dict, geom_np, offsets_np=None, device="cuda"):
    """Copy host segment arrays (float32 SoA), the per-shower geometry and the
    offsets to device tensors."""
    import numpy as np
    import torch
    seg = {k: torch.from_numpy(np.ascontiguousarray(seg_np[k], dtype=np.float32)).to(device) for k in SEGMENT_FIELDS}
    if seg_np.get("dedx") is not None:
        seg["dedx"] = torch.from_numpy(np.ascontiguousarray(seg_np["dedx"], dtype=np.float32)).to(device)
    geom = torch.from_numpy(np.ascontiguousarray(np.atleast_2d(geom_np), dtype=np.float64)).to(device)
    off = None
    if offsets_np is not None:
        off = torch.from_numpy(np.ascontiguousarray(offsets_np, dtype=np.int64)).to(device)
    return seg, geom, off


N_PARAMS = 4804
N_NORM = 24


class Surrogate:
    """Transport surrogate network (cphot_surrogate_*): training and inference
    run in the library's kernels; tensors are plain device buffers."""

    def __init__(self, lo, hi, max_batch=8192, init_seed=0, geometry="planar"):
        d = SurrogateDesc()
        d.in_lo[:] = tuple(float(v) for v in lo)
        d.in_hi[:] = tuple(float(v) for v in hi)
        d.max_batch, d.init_seed = int(max_batch), int(init_seed)
        d.geometry = GEOMETRY[geometry]
        self.desc = d
        h = C.c_void_p()
        _check("cphot_surrogate_create", lib().cphot_surrogate_create(C.byref(d), C.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.cphot_surrogate_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def make_training_set(self, atm: Atmosphere, n, seed, first=0, stream=None):
        import torch
        X = torch.empty((int(n), 5), dtype=torch.float32, device="cuda")
        Y = torch.empty((int(n), 4), dtype=torch.float32, device="cuda")
        _check("cphot_surrogate_make_training_set",
               lib().cphot_surrogate_make_training_set(self._h, atm.handle, int(first), int(n), int(seed),
                                                       C.c_void_p(_dptr(X, torch.float32, "X")),
                                                       C.c_void_p(_dptr(Y, torch.float32, "Y")), _stream_ptr(stream)))
        return X, Y

    def fit_normalization(self, Y, stream=None):
        import torch
        _check("cphot_surrogate_fit_normalization",
               lib().cphot_surrogate_fit_normalization(self._h, C.c_void_p(_dptr(Y, torch.float32, "Y")),
                                                       Y.shape[0], _stream_ptr(stream)))

    def train(self, X, Y, batch, steps, lr, stream=None):
        import torch
        loss = torch.zeros(max(int(steps), 1), dtype=torch.float32, device="cuda")
        _check("cphot_surrogate_train",
               lib().cphot_surrogate_train(self._h, C.c_void_p(_dptr(X, torch.float32, "X")),
                                           C.c_void_p(_dptr(Y, torch.float32, "Y")), X.shape[0], int(batch),
                                           int(steps), float(lr), C.c_void_p(loss.data_ptr()), _stream_ptr(stream)))
        return loss

    def gradient(self, X, Y, stream=None):
        import torch
        g = torch.zeros(N_PARAMS, dtype=torch.float32, device="cuda")
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        _check("cphot_surrogate_gradient",
               lib().cphot_surrogate_gradient(self._h, C.c_void_p(_dptr(X, torch.float32, "X")),
                                              C.c_void_p(_dptr(Y, torch.float32, "Y")), X.shape[0],
                                              C.c_void_p(g.data_ptr()), C.c_void_p(loss.data_ptr()),
                                              _stream_ptr(stream)))
        return g, loss

    def gradient_noalloc(self, X, Y, grad, loss, stream=None):
        """cphot_surrogate_gradient_noalloc into caller-owned device buffers: grad
        float32 [4804], loss float32 [1]."""
        import torch
        if grad.numel() < N_PARAMS or loss.numel() < 1:
            raise ValueError(f"grad needs {N_PARAMS} elements and loss one")
        _check("cphot_surrogate_gradient_noalloc",
               lib().cphot_surrogate_gradient_noalloc(self._h, C.c_void_p(_dptr(X, torch.float32, "X")),
                                                      C.c_void_p(_dptr(Y, torch.float32, "Y")), X.shape[0],
                                                      C.c_void_p(_dptr(grad, torch.float32, "grad")),
                                                      C.c_void_p(_dptr(loss, torch.float32, "loss")),
                                                      _stream_ptr(stream)))

    def forward(self, X, stream=None):
        import torch
        Y = torch.empty((X.shape[0], 4), dtype=torch.float32, device="cuda")
        _check("cphot_surrogate_forward",
               lib().cphot_surrogate_forward(self._h, C.c_void_p(_dptr(X, torch.float32, "X")),
                                             C.c_void_p(Y.data_ptr()), X.shape[0], _stream_ptr(stream)))
        return Y

    def get_params(self):
        import numpy as np
        p = np.zeros(N_PARAMS, dtype=np.float32)
        n = np.zeros(N_NORM, dtype=np.float32)
        _check("cphot_surrogate_get_params", lib().cphot_surrogate_get_params(
            self._h, p.ctypes.data_as(C.c_void_p), n.ctypes.data_as(C.c_void_p)))
        return p, n

    def set_params(self, params=None, norm=None):
        import numpy as np
        pa = None if params is None else np.ascontiguousarray(params, dtype=np.float32)
        na = None if norm is None else np.ascontiguousarray(norm, dtype=np.float32)
        _check("cphot_surrogate_set_params", lib().cphot_surrogate_set_params(
            self._h, None if pa is None else pa.ctypes.data_as(C.c_void_p),
            None if na is None else na.ctypes.data_as(C.c_void_p)))
