"""Seeded synthetic workloads: charged track segments of air showers, as float32 SoA.

This module holds inputs only. It takes no step of the photon method (no yield,
no cone, no transport, no absorption, no binning); both the CPU oracle and the
HIP library receive what it produces. The thesis simulates photons from CORSIKA
track segments (Sec. 5.3.1 lists position, direction, charge and energy); no such
shower files exist here, so segments are drawn from a Gaisser-Hillas longitudinal
profile with a Gaussian lateral spread.

The 5-layer parametrised atmosphere (the CORSIKA "US standard after Linsley"
model, a public parametrisation; the thesis shows the profiles only as plots,
Fig. 2.8) is stated here as data. Segment placement needs the inverse of its
vertical depth X(h); that inverse lives here and is used for nothing else.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# X(h) = a_i + b_i exp(-h/c_i) for layers 0..3, X = a_4 - b_4 h / c_4 in layer 4;
# X in g/cm^2, h and c in cm. Layer i starts at LINSLEY_HB_M[i] metres.
LINSLEY_A = (-186.555305, -94.919, 0.61289, 0.0, 0.01128292)
LINSLEY_B = (1222.6562, 1144.9069, 1305.5948, 540.1778, 1.0)
LINSLEY_C = (994186.38, 878153.55, 636143.04, 772170.16, 1.0e9)
LINSLEY_HB_M = (0.0, 4.0e3, 10.0e3, 40.0e3, 100.0e3)
KAPPA = 2.83e-4              # n - 1 = KAPPA * rho / rho(0)

SEGMENT_FIELDS = ("x0", "y0", "z0", "x1", "y1", "z1", "beta", "charge")

BETA_RANGES = {
    # beta ~ U[lo, 1): the literal configuration text, and the variant whose
    # photon totals match the stated ~1e6 / ~1e8 photons.
    "literal": 0.99,
    "R": 0.99999,
}


def _vertical_depth(h_m: np.ndarray) -> np.ndarray:
    h = np.asarray(h_m, dtype=np.float64)
    out = np.empty_like(h)
    hcm = h * 100.0
    for i in range(5):
        lo = LINSLEY_HB_M[i]
        hi = LINSLEY_HB_M[i + 1] if i < 4 else np.inf
        m = (h >= lo) & (h < hi)
        if i < 4:
            out[m] = LINSLEY_A[i] + LINSLEY_B[i] * np.exp(-hcm[m] / LINSLEY_C[i])
        else:
            out[m] = LINSLEY_A[i] - LINSLEY_B[i] * hcm[m] / LINSLEY_C[i]
    out[h < 0] = LINSLEY_A[0] + LINSLEY_B[0] * np.exp(-hcm[h < 0] / LINSLEY_C[0])
    return out


def _height_of_depth(xv: np.ndarray) -> np.ndarray:
    """Inverse of the vertical depth, layer by layer (monotone, so layers are
    identified by their boundary depths)."""
    xv = np.asarray(xv, dtype=np.float64)
    xb = _vertical_depth(np.array(LINSLEY_HB_M[1:], dtype=np.float64))
    h = np.empty_like(xv)
    for i in range(5):
        upper = np.inf if i == 0 else xb[i - 1]
        lower = xb[i] if i < 4 else -np.inf
        m = (xv <= upper) & (xv > lower)
        if i < 4:
            h[m] = LINSLEY_C[i] * np.log(LINSLEY_B[i] / (xv[m] - LINSLEY_A[i])) / 100.0
        else:
            h[m] = (LINSLEY_A[i] - xv[m]) * LINSLEY_C[i] / LINSLEY_B[i] / 100.0
    return h


@dataclasses.dataclass
class Shower:
    """One synthetic shower: segments (float32 SoA) and its axis geometry."""
    seg: dict                 # field -> np.ndarray(float32, n)
    core: tuple               # (x, y) where the axis meets the observation level, m
    axis: tuple               # unit direction of travel (downward), 3 floats
    zenith_deg: float
    azimuth_deg: float
    h_obs: float
    first_id: int = 0         # global id of segment 0 (counter-based RNG key)

    @property
    def n(self) -> int:
        return int(self.seg["x0"].shape[0])

    def subset(self, idx: np.ndarray) -> "Shower":
        return dataclasses.replace(self, seg={k: v[idx] for k, v in self.seg.items()})


def axis_vector(zenith_deg: float, azimuth_deg: float) -> tuple:
    z = math.radians(zenith_deg)
    a = math.radians(azimuth_deg)
    return (math.sin(z) * math.cos(a), math.sin(z) * math.sin(a), -math.cos(z))


def make_shower(n_segments: int, *, seed: int, xmax: float = 600.0, lam: float = 70.0,
                zenith_deg: float = 0.0, azimuth_deg: float = 0.0,
                beta: str = "literal", h_start: float = 20000.0, h_obs: float = 2200.0,
                sigma0: float = 5.0, length=(1.0, 5.0), core=(0.0, 0.0),
                dedx=None, first_id: int = 0) -> Shower:
    """Draw `n_segments` track segments.

    Slant depth X - X0 ~ Gamma(k = (Xmax - X0)/lam + 1, scale = lam) is the
    Gaisser-Hillas shape, with X0 the slant depth of the axis start at
    `h_start`; draws beyond the observation level are redrawn. The centre sits
    on the axis at that depth (flat Earth: vertical depth = X cos zenith), offset
    laterally by N(0, sigma^2) on two axes normal to the shower axis with
    sigma = sigma0 * X / Xmax. Directions follow the axis; length ~ U[length];
    beta ~ U[lo, 1) with lo from BETA_RANGES; charge = +-1. With `dedx=(lo, hi)`
    an energy-deposit column dE/dx ~ U[lo, hi] MeV/m is added.
    """
    rng = np.random.default_rng(seed)
    n = int(n_segments)
    cz = math.cos(math.radians(zenith_deg))
    ax = np.array(axis_vector(zenith_deg, azimuth_deg))
    x0_slant = float(_vertical_depth(np.array([h_start]))[0]) / cz
    xg_slant = float(_vertical_depth(np.array([h_obs]))[0]) / cz
    k = (xmax - x0_slant) / lam + 1.0
    X = x0_slant + rng.gamma(k, lam, size=n)
    bad = X >= xg_slant
    while bad.any():
        X[bad] = x0_slant + rng.gamma(k, lam, size=int(bad.sum()))
        bad = X >= xg_slant
    h = _height_of_depth(X * cz)
    # point on the axis at height h: core + s * (-axis) with s the distance above h_obs
    s = (h - h_obs) / cz
    centre = np.empty((n, 3))
    centre[:, 0] = core[0] - s * ax[0]
    centre[:, 1] = core[1] - s * ax[1]
    centre[:, 2] = h
    # lateral offsets in the plane normal to the axis
    e1 = np.cross(ax, [0.0, 1.0, 0.0] if abs(ax[1]) < 0.9 else [1.0, 0.0, 0.0])
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(ax, e1)
    sig = sigma0 * X / xmax
    off1 = rng.normal(0.0, 1.0, n) * sig
    off2 = rng.normal(0.0, 1.0, n) * sig
    centre += off1[:, None] * e1[None, :] + off2[:, None] * e2[None, :]
    L = rng.uniform(length[0], length[1], n)
    half = 0.5 * L[:, None] * ax[None, :]
    start = centre - half
    end = centre + half
    lo = BETA_RANGES[beta]
    b = rng.uniform(lo, 1.0, n).astype(np.float32)
    b = np.minimum(b, np.float32(np.nextafter(np.float32(1.0), np.float32(0.0))))
    q = np.where(rng.random(n) < 0.5, -1.0, 1.0).astype(np.float32)
    seg = {
        "x0": start[:, 0].astype(np.float32), "y0": start[:, 1].astype(np.float32),
        "z0": start[:, 2].astype(np.float32), "x1": end[:, 0].astype(np.float32),
        "y1": end[:, 1].astype(np.float32), "z1": end[:, 2].astype(np.float32),
        "beta": b, "charge": q,
    }
    if dedx is not None:
        seg["dedx"] = rng.uniform(dedx[0], dedx[1], n).astype(np.float32)
    return Shower(seg=seg, core=(float(core[0]), float(core[1])), axis=tuple(float(v) for v in ax),
                  zenith_deg=float(zenith_deg), azimuth_deg=float(azimuth_deg), h_obs=float(h_obs),
                  first_id=int(first_id))


def make_batch(n_showers: int, *, seed: int, log_range=(3.0, 6.0), zenith_range=(0.0, 60.0),
               xmax_range=(350.0, 750.0), beta: str = "literal", h_obs: float = 2200.0,
               scale: float = 1.0):
    """Many showers of uneven size (segment counts log-uniform in 10**log_range,
    times `scale`), zenith and Xmax uniform, azimuth uniform. Returns a list of
    Shower whose first_id values make segment ids unique across the batch."""
    rng = np.random.default_rng(seed)
    counts = np.floor(10.0 ** rng.uniform(log_range[0], log_range[1], n_showers) * scale).astype(np.int64)
    counts = np.maximum(counts, 1)
    zen = rng.uniform(zenith_range[0], zenith_range[1], n_showers)
    azi = rng.uniform(0.0, 360.0, n_showers)
    xm = rng.uniform(xmax_range[0], xmax_range[1], n_showers)
    seeds = rng.integers(0, 2**62, n_showers)
    out = []
    first = 0
    for i in range(n_showers):
        sh = make_shower(int(counts[i]), seed=int(seeds[i]), xmax=float(xm[i]), zenith_deg=float(zen[i]),
                         azimuth_deg=float(azi[i]), beta=beta, h_obs=h_obs, first_id=first)
        out.append(sh)
        first += int(counts[i])
    return out


def concat_showers(showers):
    """Flatten a list of showers into one SoA plus offsets [n_showers + 1] and a
    per-shower geometry array [n_showers, 5] = core_x, core_y, axis_x, axis_y, axis_z."""
    fields = list(showers[0].seg.keys())
    seg = {k: np.concatenate([s.seg[k] for s in showers]) for k in fields}
    offs = np.zeros(len(showers) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([s.n for s in showers])
    geom = np.array([[s.core[0], s.core[1], *s.axis] for s in showers], dtype=np.float64)
    return seg, offs, geom


# ---- the five workload recipes ------------------------------------------------------
# Plain parameter dictionaries: each side (oracle, library) builds its own objects
# from them.

_LINSLEY = dict(a=LINSLEY_A, b=LINSLEY_B, c=LINSLEY_C, hb=LINSLEY_HB_M, kappa=KAPPA)
# straight rays, Rayleigh only, continuous wavelength (tiny vertical and batched workloads)
ATMO_STRAIGHT = dict(profile="linsley5", h_top=25000.0, step=1.0, rayleigh400=2974.0, **_LINSLEY)
# 100 layers of 250 m, Rayleigh + aerosol tables on 64 wavelength bins (telescope,
# surrogate and inclined workloads; the inclined one bends them into shells)
ATMO_LAYERED = dict(profile="linsley5", h_top=25000.0, step=1.0, rayleigh400=2974.0, aer_tau350=0.05,
                    aer_H=1200.0, aer_angstrom=1.0, n_layers=100, n_lam=64, **_LINSLEY)

RUN_TINY = dict(transport="straight", detector="grid", spectrum="uniform", bunch=1, h_obs=2200.0,
                nx=100, ny=100, cell=10.0)
RUN_TELESCOPE = dict(transport="layered", detector="spheres", spectrum="frank_tamm", bunch=5, h_obs=2200.0,
                     snx=10, sny=10, pitch=150.0, radius=6.0, n_t=512, dt=1.0)
RUN_BATCH = dict(transport="straight", detector="grid", spectrum="frank_tamm", bunch=1, h_obs=2200.0,
                 nx=200, ny=200, cell=5.0)
RUN_INCLINED = dict(transport="curved", detector="grid", spectrum="frank_tamm", emission="both", bunch=1,
                    h_obs=2200.0, nx=1000, ny=1000, cell=10.0)


def efficiency_curve(n_bins: int = 64, lam_min: float = 300.0, lam_max: float = 600.0):
    """Synthetic detector efficiency per wavelength bin (Sec. 4.3.1 names mirror
    reflectivity and sensor efficiency; the curves themselves are not printed):
    a silicon-photomultiplier-like detection efficiency peaking at 0.45 near
    420 nm with a Gaussian fall-off of 110 nm, times a mirror reflectivity of 0.9."""
    import numpy as np
    lam = lam_min + (np.arange(n_bins) + 0.5) * (lam_max - lam_min) / n_bins
    return 0.9 * 0.45 * np.exp(-0.5 * ((lam - 420.0) / 110.0) ** 2)


# surrogate training domain: emission height, cos zenith, azimuth, wavelength, observation level
SURROGATE_LO = (2000.0, math.cos(math.radians(60.0)), -math.pi, 300.0, 1000.0)
SURROGATE_HI = (20000.0, 1.0, math.pi, 600.0, 3000.0)
# curved-Earth surrogate (inclined workload): local zenith up to 66 deg, heights to 22 km
SURROGATE_CURVED_LO = (2000.0, 0.4, -math.pi, 300.0, 1000.0)
SURROGATE_CURVED_HI = (22000.0, 1.0, math.pi, 600.0, 3000.0)


def workload_tiny_vertical(beta: str = "literal", n: int = 10_000) -> Shower:
    """1e4 segments, vertical, Xmax 600, straight rays to a 100 x 100 grid of 10 m at 2200 m."""
    return make_shower(n, seed=1001, xmax=600.0, zenith_deg=0.0, beta=beta)


def workload_telescope(beta: str = "R", n: int = 1_000_000) -> Shower:
    """1e6 segments, zenith 20 deg, Xmax 400; refraction, bunches of 5, 100 spheres."""
    return make_shower(n, seed=1002, xmax=400.0, zenith_deg=20.0, beta=beta)


def workload_inclined_chunk(chunk: int, beta: str = "R", chunk_size: int = 10_000_000) -> Shower:
    """One chunk of the large inclined shower: zenith 60 deg, Xmax 600, dE/dx ~ U[0.1, 2] MeV/m."""
    return make_shower(chunk_size, seed=1005 * 1000 + chunk, xmax=600.0, zenith_deg=60.0, beta=beta,
                       dedx=(0.1, 2.0), first_id=chunk * chunk_size)
