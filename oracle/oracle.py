"""ctypes front end of the FP64 CPU oracle (cphot_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py, never by the product library. It imports nothing
from the product package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cphot_oracle.c")
_LIB = os.path.join(_HERE, "libcphot_oracle.so")
_lock = threading.Lock()
_lib = None


def build() -> str:
    """Compile the oracle with gcc (strict IEEE: no contraction, no fast math)."""
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-o", tmp, _SRC, "-lm", "-lpthread"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


class AtmoParams(C.Structure):
    _fields_ = [("profile", C.c_int32), ("n_layers", C.c_int32),
                ("a", C.c_double * 5), ("b", C.c_double * 5), ("c", C.c_double * 5), ("hb", C.c_double * 5),
                ("kappa", C.c_double), ("delta0", C.c_double), ("h_top", C.c_double), ("step", C.c_double),
                ("rayleigh400", C.c_double), ("aer_tau350", C.c_double), ("aer_H", C.c_double),
                ("aer_angstrom", C.c_double), ("lam_min", C.c_double), ("lam_max", C.c_double),
                ("n_lam", C.c_int32), ("pad", C.c_int32), ("earth_radius", C.c_double)]


class Run(C.Structure):
    _fields_ = [("transport", C.c_int32), ("detector", C.c_int32), ("spectrum", C.c_int32),
                ("bunch", C.c_int32), ("seed", C.c_uint64), ("h_obs", C.c_double),
                ("nx", C.c_int32), ("ny", C.c_int32), ("cell", C.c_double),
                ("snx", C.c_int32), ("sny", C.c_int32), ("pitch", C.c_double), ("radius", C.c_double),
                ("n_t", C.c_int32), ("counts_rule", C.c_int32), ("dt", C.c_double),
                ("emission", C.c_int32), ("pad2", C.c_int32), ("fl_yield", C.c_double * 3),
                ("fl_lambda", C.c_double * 3), ("efficiency", C.c_void_p), ("reduction", C.c_void_p),
                ("lambda_ref", C.c_double)]


class Segments(C.Structure):
    _fields_ = [(f, C.POINTER(C.c_float)) for f in ("x0", "y0", "z0", "x1", "y1", "z1", "beta", "charge")] + \
               [("n", C.c_int64), ("first_id", C.c_int64), ("dedx", C.POINTER(C.c_float)), ("id_stride", C.c_int64)]


class Geom(C.Structure):
    _fields_ = [("core_x", C.c_double), ("core_y", C.c_double), ("ax", C.c_double), ("ay", C.c_double),
                ("az", C.c_double)]


PHOTON_DTYPE = np.dtype([
    ("seg", np.int64), ("k", np.int32), ("state", np.int32), ("bin", np.int32), ("tbin", np.int32),
    ("x", np.float64), ("y", np.float64), ("z", np.float64), ("t", np.float64), ("tau", np.float64),
    ("lambda", np.float64), ("u_abs", np.float64), ("margin", np.float64), ("tmargin", np.float64),
    ("ex", np.float64), ("ey", np.float64), ("ez", np.float64),
    ("dx", np.float64), ("dy", np.float64), ("dz", np.float64), ("source", np.int32), ("pad", np.int32),
    ("p_emit", np.float64)])

SEGMENT_DTYPE = np.dtype([("n", np.int32), ("status", np.int32), ("mu", np.float64),
                          ("cos_t", np.float64), ("sin2_t", np.float64), ("nf", np.int32, 3), ("pad", np.int32),
                          ("muf", np.float64, 3), ("q", np.float64)])

STATE = {"binned": 0, "upward": 1, "absorbed": 2, "outside": 3}
COUNTERS = ["segments_in", "segments_skipped", "segments_below_threshold", "records_generated",
            "records_upward", "records_absorbed", "records_outside", "records_binned", "photons_binned",
            "surrogate_fallback"]
N_COUNTERS = 16

PROFILES = {"linsley5": 0, "homogeneous": 1, "linear": 2}
TRANSPORTS = {"straight": 0, "layered": 1, "curved": 2}
EMISSION = {"cherenkov": 1, "fluorescence": 2, "both": 3}
# synthetic fluorescence bands (nm) and yields (photons per MeV deposited)
FL_LAMBDA = (337.0, 357.0, 391.0)
FL_YIELD = (7.0, 5.0, 2.0)
DETECTORS = {"grid": 0, "spheres": 1}
SPECTRA = {"uniform": 0, "frank_tamm": 1, "dispersive": 2}


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            L = C.CDLL(_LIB)
            P = C.POINTER
            L.orc_philox.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
            L.orc_atmo_create.argtypes = [P(AtmoParams), P(C.c_void_p)]
            L.orc_atmo_create.restype = C.c_int
            L.orc_atmo_free.argtypes = [C.c_void_p]
            for fn in ("orc_depth", "orc_density", "orc_delta_closed", "orc_delta_table"):
                getattr(L, fn).argtypes = [C.c_void_p, C.c_double]
                getattr(L, fn).restype = C.c_double
            L.orc_layer_tables.argtypes = [C.c_void_p, P(C.c_double), P(C.c_double)]
            L.orc_frank_tamm_K.argtypes = [C.c_double, C.c_double]
            L.orc_frank_tamm_K.restype = C.c_double
            L.orc_exp_neg.restype = C.c_double
            L.orc_exp_neg.argtypes = [C.c_double]
            L.orc_poisson.restype = C.c_int64
            L.orc_poisson.argtypes = [C.c_double, C.c_uint32, C.c_uint64, C.c_uint64, C.c_uint32]
            L.orc_segment_counts.argtypes = [C.c_void_p, P(Run), P(Segments), C.c_void_p]
            L.orc_trace.argtypes = [C.c_void_p, P(Run), P(Segments), P(Geom), C.c_void_p, C.c_int64]
            L.orc_trace.restype = C.c_int64
            L.orc_propagate.argtypes = [C.c_void_p, P(Run), P(Segments), C.c_int32, P(C.c_int64), P(Geom),
                                        P(C.c_uint64), P(C.c_uint64), P(C.c_uint64), C.c_int32]
            L.orc_propagate.restype = C.c_int
            L.orc_layered_ray.argtypes = [C.c_void_p, P(C.c_double), P(C.c_double), C.c_double,
                                          P(C.c_double), P(C.c_double), C.c_int]
            L.orc_layered_ray.restype = C.c_int
            L.orc_surrogate_inputs.argtypes = [C.c_void_p, C.c_uint64, P(C.c_double), P(C.c_double), C.c_int64,
                                               C.c_int64, P(C.c_double)]
            L.orc_surrogate_targets.argtypes = [C.c_void_p, C.c_int64, P(C.c_double), P(C.c_double)]
            L.orc_surrogate_targets_curved.argtypes = [C.c_void_p, C.c_int64, P(C.c_double), P(C.c_double)]
            L.orc_curved_ray.argtypes = [C.c_void_p, C.c_double, P(C.c_double), P(C.c_double), P(C.c_double),
                                         P(C.c_double), C.c_int]
            L.orc_curved_ray.restype = C.c_int
            _lib = L
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


# --------------------------------------------------------------------------------------

def philox(ctr, key):
    """Philox4x32-10 block: 4 counter words, 2 key words -> 4 output words."""
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(out, C.c_uint32))
    return out


class Atmosphere:
    """The oracle's own atmosphere: 1 m refractivity table, layer tables."""

    def __init__(self, profile="linsley5", n_layers=0, a=None, b=None, c=None, hb=None, kappa=2.83e-4,
                 delta0=0.0, h_top=25000.0, step=1.0, rayleigh400=0.0, aer_tau350=0.0, aer_H=1200.0,
                 aer_angstrom=1.0, lam_min=300.0, lam_max=600.0, n_lam=0, earth_radius=6.371e6):
        p = AtmoParams()
        p.profile = PROFILES[profile]
        p.n_layers = int(n_layers)
        zeros = (0.0,) * 5
        for name, v in (("a", a), ("b", b), ("c", c), ("hb", hb)):
            getattr(p, name)[:] = tuple(v) if v is not None else zeros
        if profile == "linsley5":
            p.c[:] = tuple(c)  # required
        p.kappa, p.delta0, p.h_top, p.step = kappa, delta0, h_top, step
        p.rayleigh400, p.aer_tau350, p.aer_H, p.aer_angstrom = rayleigh400, aer_tau350, aer_H, aer_angstrom
        p.lam_min, p.lam_max, p.n_lam, p.earth_radius = lam_min, lam_max, int(n_lam), earth_radius
        if profile != "linsley5":
            p.b[0], p.c[0] = 1.0, 1.0  # rho0 unused; avoid a division by zero
        self.params = p
        h = C.c_void_p()
        rc = lib().orc_atmo_create(C.byref(p), C.byref(h))
        if rc != 0:
            raise ValueError("oracle atmosphere rejected the parameters")
        self._h = h

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_atmo_free(self._h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def depth(self, h):
        return np.array([lib().orc_depth(self._h, float(x)) for x in np.atleast_1d(h)])

    def density(self, h):
        return np.array([lib().orc_density(self._h, float(x)) for x in np.atleast_1d(h)])

    def delta_closed(self, h):
        return np.array([lib().orc_delta_closed(self._h, float(x)) for x in np.atleast_1d(h)])

    def delta_table(self, h):
        return np.array([lib().orc_delta_table(self._h, float(x)) for x in np.atleast_1d(h)])

    def layer_tables(self):
        L, K = self.params.n_layers, max(self.params.n_lam, 0)
        d = np.zeros(L)
        e = np.zeros(max(L * K, 1))
        lib().orc_layer_tables(self._h, _ptr(d, C.c_double), _ptr(e, C.c_double))
        return d, e[: L * K].reshape(L, K)


def make_run(transport="straight", detector="grid", spectrum="uniform", bunch=1, seed=0, h_obs=2200.0,
             nx=100, ny=100, cell=10.0, snx=10, sny=10, pitch=150.0, radius=6.0, n_t=0, dt=1.0,
             emission="cherenkov", fl_yield=FL_YIELD, fl_lambda=FL_LAMBDA, efficiency=None, reduction=None,
             counts="rounded", lambda_ref=400.0, **_ignored) -> Run:
    """`efficiency` (per wavelength bin) and `reduction` (per layer): float64
    arrays or None (Sec. 4.3.1)."""
    r = Run()
    r.transport, r.detector, r.spectrum = TRANSPORTS[transport], DETECTORS[detector], SPECTRA[spectrum]
    r.bunch, r.seed, r.h_obs = int(bunch), int(seed) & (2**64 - 1), float(h_obs)
    r.nx, r.ny, r.cell = int(nx), int(ny), float(cell)
    r.snx, r.sny, r.pitch, r.radius = int(snx), int(sny), float(pitch), float(radius)
    r.n_t, r.dt = int(n_t), float(dt)
    r.emission = EMISSION[emission]
    r.counts_rule = {"rounded": 0, "poisson": 1}[counts]
    r.lambda_ref = float(lambda_ref)
    r.fl_yield[:] = tuple(float(v) for v in fl_yield)
    r.fl_lambda[:] = tuple(float(v) for v in fl_lambda)
    keep = []
    if efficiency is not None:
        e = np.ascontiguousarray(efficiency, dtype=np.float64)
        r.efficiency = e.ctypes.data
        keep.append(e)
    if reduction is not None:
        q = np.ascontiguousarray(reduction, dtype=np.float64)
        r.reduction = q.ctypes.data
        keep.append(q)
    r._keep = keep
    return r


def _segments(seg: dict, first_id: int, id_stride: int = 1):
    arrs = {k: np.ascontiguousarray(seg[k], dtype=np.float32) for k in
            ("x0", "y0", "z0", "x1", "y1", "z1", "beta", "charge")}
    s = Segments()
    for k, v in arrs.items():
        setattr(s, k, _ptr(v, C.c_float))
    s.n = int(arrs["x0"].shape[0])
    s.first_id = int(first_id)
    s.id_stride = int(id_stride)
    if seg.get("dedx") is not None:
        arrs["dedx"] = np.ascontiguousarray(seg["dedx"], dtype=np.float32)
        s.dedx = _ptr(arrs["dedx"], C.c_float)
    return s, arrs  # keep arrays alive


def _geom(core, axis):
    g = Geom()
    g.core_x, g.core_y = float(core[0]), float(core[1])
    g.ax, g.ay, g.az = (float(v) for v in axis)
    return g


def frank_tamm_K(lam_min=300.0, lam_max=600.0) -> float:
    return lib().orc_frank_tamm_K(lam_min, lam_max)


def segment_counts(atm: Atmosphere, run: Run, seg: dict, first_id: int = 0, id_stride: int = 1) -> np.ndarray:
    s, keep = _segments(seg, first_id, id_stride)
    out = np.zeros(s.n, dtype=SEGMENT_DTYPE)
    lib().orc_segment_counts(atm.handle, C.byref(run), C.byref(s), out.ctypes.data_as(C.c_void_p))
    return out


def trace(atm: Atmosphere, run: Run, seg: dict, core=(0.0, 0.0), axis=(0.0, 0.0, -1.0),
          first_id: int = 0, id_stride: int = 1) -> np.ndarray:
    """Every photon record of the given segments, in (segment, k) order; segment i
    has the global id first_id + i * id_stride."""
    s, keep = _segments(seg, first_id, id_stride)
    g = _geom(core, axis)
    cap = 1024
    while True:
        out = np.zeros(cap, dtype=PHOTON_DTYPE)
        m = lib().orc_trace(atm.handle, C.byref(run), C.byref(s), C.byref(g), out.ctypes.data_as(C.c_void_p), cap)
        if m >= 0:
            return out[:m]
        cap = -m


def propagate(atm: Atmosphere, run: Run, seg: dict, geoms, offsets=None, first_id: int = 0,
              threads: int = 1, id_stride: int = 1):
    """Bins, time histograms and counters for a batch of showers.

    geoms: sequence of (core_x, core_y, axis_x, axis_y, axis_z), one per shower;
    offsets: int64 [n_showers + 1] segment offsets (None for one shower)."""
    s, keep = _segments(seg, first_id, id_stride)
    geoms = np.atleast_2d(np.asarray(geoms, dtype=np.float64))
    ns = geoms.shape[0]
    G = (Geom * ns)()
    for i in range(ns):
        G[i] = _geom(geoms[i, :2], geoms[i, 2:5])
    if offsets is None:
        offsets = np.array([0, s.n], dtype=np.int64)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    per = run.nx * run.ny if run.detector == 0 else run.snx * run.sny
    bins = np.zeros((ns, per), dtype=np.uint64)
    tper = per * (run.n_t + 1) if (run.detector == 1 and run.n_t > 0) else 0
    thist = np.zeros((ns, max(tper, 1)), dtype=np.uint64)
    counters = np.zeros(N_COUNTERS, dtype=np.uint64)
    lib().orc_propagate(atm.handle, C.byref(run), C.byref(s), ns, _ptr(offsets, C.c_int64), G,
                        _ptr(bins, C.c_uint64), _ptr(thist, C.c_uint64), _ptr(counters, C.c_uint64),
                        int(threads))
    if tper:
        thist = thist.reshape(ns, per, run.n_t + 1)
    else:
        thist = None
    return bins, thist, counters


def layered_ray(atm: Atmosphere, start, direction, h_end, cap=4096):
    P = np.ascontiguousarray(start, dtype=np.float64)
    u = np.ascontiguousarray(direction, dtype=np.float64)
    end = np.zeros(3)
    snell = np.zeros(cap)
    m = lib().orc_layered_ray(atm.handle, _ptr(P, C.c_double), _ptr(u, C.c_double), float(h_end),
                              _ptr(end, C.c_double), _ptr(snell, C.c_double), cap)
    return end, snell[: min(m, cap)]


def surrogate_inputs(atm: Atmosphere, seed, lo, hi, first, n):
    """Training inputs [n, 5] = (h_e, cos zenith, azimuth, wavelength-bin centre, h_obs)."""
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    X = np.zeros((int(n), 5))
    lib().orc_surrogate_inputs(atm.handle, int(seed) & (2**64 - 1), _ptr(lo, C.c_double), _ptr(hi, C.c_double),
                               int(first), int(n), _ptr(X, C.c_double))
    return X


def surrogate_targets(atm: Atmosphere, X, geometry="planar"):
    """Exact targets [n, 4] for inputs X [n, 5]: planar layers (landing offset
    along / across the azimuth, optical path excess, log T) or curved shells
    (extra ground distance along / across the azimuth, optical path excess, log T,
    each per metre of the straight chord to the observation sphere)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    Y = np.zeros((X.shape[0], 4))
    fn = lib().orc_surrogate_targets if geometry == "planar" else lib().orc_surrogate_targets_curved
    fn(atm.handle, X.shape[0], _ptr(X, C.c_double), _ptr(Y, C.c_double))
    return Y


def curved_ray(atm: Atmosphere, h_obs, start, direction, cap=4096):
    """(arrived, end point, Bouguer invariant per shell visited)."""
    P = np.ascontiguousarray(start, dtype=np.float64)
    u = np.ascontiguousarray(direction, dtype=np.float64)
    end = np.zeros(3)
    inv = np.zeros(cap)
    m = lib().orc_curved_ray(atm.handle, float(h_obs), _ptr(P, C.c_double), _ptr(u, C.c_double),
                             _ptr(end, C.c_double), _ptr(inv, C.c_double), cap)
    return m > 0, end, inv[: min(abs(m), cap)]


def exp_neg(x):
    """exp(-x) of the count sampler (IEEE basic operations only), 0 <= x <= 64."""
    return lib().orc_exp_neg(float(x))


def poisson(mu, w0, seed=0, seg_id=0, tag=12):
    """Poisson record count of the oracle's sampler for mean mu and first word w0."""
    return lib().orc_poisson(float(mu), int(w0), int(seed), int(seg_id), int(tag))
