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
TRANSPORT = {"straight": 0, "layered": 1}
DETECTOR = {"grid": 0, "spheres": 1}
SPECTRUM = {"uniform": 0, "frank_tamm": 1}
BINS = {"u32": 0, "u64": 1}
COUNTERS = ["segments_in", "segments_skipped", "segments_below_threshold", "records_generated",
            "records_upward", "records_absorbed", "records_outside", "records_binned", "photons_binned"]


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
                ("reserved", C.c_double * 4)]


class Segments(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in ("x0", "y0", "z0", "x1", "y1", "z1", "beta", "charge")] + \
               [("n", C.c_int64), ("first_id", C.c_int64), ("n_showers", C.c_int32), ("reserved0", C.c_int32),
                ("shower_offsets", C.c_void_p), ("shower_geom", C.c_void_p)]


class Detector(C.Structure):
    _fields_ = [("atm", C.c_void_p), ("transport", C.c_int32), ("detector", C.c_int32), ("spectrum", C.c_int32),
                ("bunch", C.c_int32), ("seed", C.c_uint64), ("h_obs", C.c_double), ("nx", C.c_int32),
                ("ny", C.c_int32), ("cell", C.c_double), ("snx", C.c_int32), ("sny", C.c_int32),
                ("pitch", C.c_double), ("radius", C.c_double), ("n_time_bins", C.c_int32),
                ("reserved0", C.c_int32), ("time_bin_ns", C.c_double), ("block_size", C.c_int32),
                ("grid_blocks", C.c_int32), ("lds_hist", C.c_int32), ("reserved1", C.c_int32)]


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
                 aer_angstrom=1.0, lam_min=300.0, lam_max=600.0, n_lam=1, **_ignored):
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
                  dt=1.0, block_size=0, grid_blocks=0, lds_hist=-1) -> Detector:
    d = Detector()
    d.atm = atm.handle
    d.transport, d.detector, d.spectrum = TRANSPORT[transport], DETECTOR[detector], SPECTRUM[spectrum]
    d.bunch, d.seed, d.h_obs = int(bunch), int(seed) & (2**64 - 1), float(h_obs)
    d.nx, d.ny, d.cell = int(nx), int(ny), float(cell)
    d.snx, d.sny, d.pitch, d.radius = int(snx), int(sny), float(pitch), float(radius)
    d.n_time_bins, d.time_bin_ns = int(n_t), float(dt)
    d.block_size, d.grid_blocks, d.lds_hist = int(block_size), int(grid_blocks), int(lds_hist)
    d._atm_ref = atm  # keep the handle alive
    return d


def make_segments(seg: dict, geom, offsets=None, first_id: int = 0) -> Segments:
    """`seg`: dict of float32 CUDA tensors x0..z1, beta, charge; `geom`: float64 CUDA
    tensor [n_showers, 5]; `offsets`: int64 CUDA tensor [n_showers + 1] or None."""
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
    ns = int(geom.shape[0])
    s.n_showers = ns
    s.shower_geom = _dptr(geom, torch.float64, "geom")
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


def propagate(seg: Segments, det: Detector, bins, time_hist=None, counters=None, stream=None):
    """Accumulates into `bins` (uint32 -> int32 tensor view or int64 tensor),
    `time_hist` (int32 tensor viewed as uint32) and `counters` (int64 [16])."""
    import torch
    b = Bins()
    if bins.dtype in (torch.int32,):
        b.bins_dtype = BINS["u32"]
    elif bins.dtype in (torch.int64,):
        b.bins_dtype = BINS["u64"]
    else:
        raise TypeError("bins must be int32 (read as uint32) or int64 (read as uint64)")
    b.bins = _dptr(bins, None, "bins")
    b.bins_capacity = bins.numel()
    if time_hist is not None:
        b.time_hist = _dptr(time_hist, torch.int32, "time_hist")
        b.time_capacity = time_hist.numel()
    if counters is not None:
        if counters.numel() < NCOUNTERS:
            raise ValueError("counters needs 16 entries")
        b.counters = _dptr(counters, torch.int64, "counters")
    _check("cphot_propagate", lib().cphot_propagate(C.byref(seg), C.byref(det), C.byref(b), _stream_ptr(stream)))


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
    geom = torch.from_numpy(np.ascontiguousarray(np.atleast_2d(geom_np), dtype=np.float64)).to(device)
    off = None
    if offsets_np is not None:
        off = torch.from_numpy(np.ascontiguousarray(offsets_np, dtype=np.int64)).to(device)
    return seg, geom, off
