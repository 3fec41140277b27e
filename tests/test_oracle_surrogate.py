"""Pins of the oracle's surrogate pieces: training inputs, exact targets, the FP64 network."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import mlp
from oracle import oracle as O
from tests import cases

LO = [2000.0, math.cos(math.radians(60.0)), -math.pi, 300.0, 1000.0]
HI = [20000.0, 1.0, math.pi, 600.0, 3000.0]


@pytest.fixture(scope="module")
def atm():
    return O.Atmosphere(**cases.ATMO_LAYERED)


def test_inputs_in_box_and_counter_based(atm):
    X = O.surrogate_inputs(atm, 7, LO, HI, 0, 20000)
    for j in range(5):
        assert X[:, j].min() >= LO[j] and X[:, j].max() <= HI[j]
    assert np.all(X[:, 0] >= X[:, 4])
    # starts are lower layer boundaries above the observation layer, each allowed
    # boundary equally likely
    dh = 250.0
    j = X[:, 0] / dh
    np.testing.assert_array_equal(j, np.round(j))
    j_lo = np.maximum(np.ceil(LO[0] / dh), np.floor(X[:, 4] / dh) + 1)
    j_hi = np.floor(HI[0] / dh)
    assert np.all(j >= j_lo) and np.all(j <= j_hi)
    assert stats.kstest((j - j_lo + np.random.default_rng(1).random(len(j))) / (j_hi - j_lo + 1),
                        "uniform").pvalue > 1e-3
    centres = 300.0 + (np.arange(64) + 0.5) * 300.0 / 64
    assert np.all(np.isin(X[:, 3], centres))
    # counter-based: a window reproduces the same rows
    np.testing.assert_array_equal(O.surrogate_inputs(atm, 7, LO, HI, 1234, 10), X[1234:1244])
    assert stats.kstest((X[:, 2] + math.pi) / (2 * math.pi), "uniform").pvalue > 1e-3
    assert stats.kstest((X[:, 1] - LO[1]) / (HI[1] - LO[1]), "uniform").pvalue > 1e-3


def test_targets_homogeneous_medium():
    """No refraction in a homogeneous medium: the straight line is the path, so the
    landing offset and the refraction's shares of the optical path excess and of
    the optical depth all vanish (the straight line's own sums, (n - 1) l and the
    aerosol depth over the slant path, are what the kernel adds itself)."""
    atm = O.Atmosphere(profile="homogeneous", delta0=2.5e-4, h_top=25000.0, n_layers=100, n_lam=8,
                       aer_tau350=0.1, aer_H=1500.0)
    X = O.surrogate_inputs(atm, 3, LO, HI, 0, 500)
    Y = O.surrogate_targets(atm, X)
    np.testing.assert_allclose(Y[:, :2], 0.0, atol=1e-8)
    ell = (X[:, 0] - X[:, 4]) / X[:, 1]
    np.testing.assert_allclose(Y[:, 2], 0.0, atol=1e-9 * ell.max())
    np.testing.assert_allclose(Y[:, 3], 0.0, atol=1e-12)
    # homogeneous layers carry constant extinction; full layers hold the exact aerosol
    # column at the bin centre (the straight-line sums the kernel forms from them)
    d, ext = atm.layer_tables()
    lam = X[:, 3]
    k = np.floor((lam - 300.0) / 300.0 * 8).astype(int)
    dh = 250.0
    i_full = 40
    col = 0.1 * (lam / 350.0) ** -1.0 * (math.exp(-i_full * dh / 1500.0) - math.exp(-(i_full + 1) * dh / 1500.0))
    np.testing.assert_allclose(ext[i_full, k] * dh, col, rtol=1e-12)


def test_targets_by_snell_closed_form(atm):
    """Landing offset, optical path excess and optical depth from Snell's law in
    its scalar form, layer by layer."""
    d, ext = atm.layer_tables()
    dh = 250.0
    X = O.surrogate_inputs(atm, 11, LO, HI, 0, 300)
    Y = O.surrogate_targets(atm, X)
    for x, y in zip(X, Y):
        he, ct, phi, lam, ho = x
        st = math.sqrt(1 - ct * ct)
        i0 = min(int(he // dh), 99)
        iobs = int(ho // dh)
        K = (1 + d[i0]) * st
        k = int((lam - 300.0) / 300.0 * 64)
        spans = {i: dh for i in range(iobs + 1, i0)}
        if i0 > iobs:
            spans[i0] = he - i0 * dh
            spans[iobs] = (iobs + 1) * dh - ho
        else:
            spans[i0] = he - ho
        r = opt = tau = 0.0
        for i, sp in spans.items():
            n = 1 + d[i]
            si = K / n
            ci = math.sqrt(1 - si * si)
            r += sp * si / ci
            opt += n * sp / ci
            tau += ext[i, k] * sp / ci
        ls = (he - ho) / ct
        r_straight = (he - ho) * st / ct
        # the straight line's own sums over the same spans
        opt_s = sum(d[i] * sp for i, sp in spans.items()) / ct
        tau_s = sum(ext[i, k] * sp for i, sp in spans.items()) / ct
        assert y[0] == pytest.approx(r - r_straight, abs=1e-7)   # along the photon's azimuth
        assert y[1] == pytest.approx(0.0, abs=1e-7)              # planar layers: no sideways offset
        assert y[2] == pytest.approx((opt - ls) - opt_s, rel=1e-7, abs=1e-9)
        assert y[3] == pytest.approx(-tau + tau_s, rel=1e-7, abs=1e-12)


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(0)
    a = np.concatenate([rng.normal(0, 1, 5000), rng.normal(0, 1e-3, 5000), [0.0, -0.0, 1.0, 3.0]])
    want = torch.from_numpy(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16(a), want)


def test_mlp_gradient_by_finite_differences():
    rng = np.random.default_rng(2)
    theta = mlp.init(5) + rng.normal(0, 0.05, mlp.N_PARAMS)
    X = np.column_stack([rng.uniform(lo, hi, 40) for lo, hi in zip(LO, HI)])
    Y = rng.normal(0, 1, (40, 4))
    mean, std = np.zeros(4), np.ones(4)
    loss, g = mlp.loss_and_grad(theta, X, Y, LO, HI, mean, std, quantize=False)
    idx = rng.choice(mlp.N_PARAMS, 60, replace=False)
    for i in idx:
        e = np.zeros_like(theta)
        h = 1e-6
        e[i] = h
        lp, _ = mlp.loss_and_grad(theta + e, X, Y, LO, HI, mean, std, quantize=False)
        lm, _ = mlp.loss_and_grad(theta - e, X, Y, LO, HI, mean, std, quantize=False)
        fd = (lp - lm) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-5, abs=1e-9)


def test_mlp_constant_network():
    theta = np.zeros(mlp.N_PARAMS)
    P = mlp.unpack(theta)
    P["b3"] = np.array([1.0, -2.0, 0.5, 3.0])
    theta = mlp.pack(P)
    X = np.column_stack([np.linspace(lo, hi, 7) for lo, hi in zip(LO, HI)])
    y = mlp.forward(theta, X, LO, HI, mean=[10, 20, 30, 40], std=[2, 2, 2, 2])
    np.testing.assert_allclose(y, np.tile([12, 16, 31, 46], (7, 1)))


# ---------------------------------------------------------------------------- curved shells

def _chord(re, h_e, h_obs, ct):
    """Straight chord from height h_e at local zenith cosine ct to the sphere
    re + h_obs, in 50-digit decimal arithmetic."""
    from decimal import Decimal, getcontext
    getcontext().prec = 50
    r0, r1, c = Decimal(re) + Decimal(h_e), Decimal(re) + Decimal(h_obs), Decimal(ct)
    return float(r0 * c - (r0 * r0 * c * c - (r0 * r0 - r1 * r1)).sqrt())


def test_curved_targets_homogeneous_medium():
    """Shells of one refractive index bend nothing: zero extra ground distance,
    optical path excess per metre of chord = n - 1, and the optical depth is the
    sum of each shell's extinction times the chord's length inside that shell."""
    re = 6.371e6
    hom = O.Atmosphere(profile="homogeneous", delta0=2e-4, h_top=25000.0, n_layers=100, n_lam=16,
                       aer_tau350=0.1, aer_H=1500.0, earth_radius=re)
    d, ext = hom.layer_tables()
    assert np.ptp(d) == 0.0
    X = O.surrogate_inputs(hom, 11, [2500.0, 0.4, -math.pi, 300.0, 1000.0], HI, 0, 300)
    Y = O.surrogate_targets(hom, X, "curved")
    dh = 250.0
    for x, y in zip(X, Y):
        h_e, ct, h_obs = x[0], x[1], x[4]
        s = _chord(re, h_e, h_obs, ct)
        k = int((x[3] - 300.0) / 300.0 * 16)
        assert abs(y[0]) < 1e-10 and abs(y[1]) < 1e-10
        assert y[2] == pytest.approx(2e-4, rel=1e-7)
        # distance along the chord from the start down to radius re + h
        r0, s0 = re + h_e, math.sqrt(1.0 - ct * ct)
        along = lambda h: r0 * ct - math.sqrt((re + h) ** 2 - (r0 * s0) ** 2)
        tau = 0.0
        for layer in range(int(h_obs // dh), min(int(h_e // dh), 99) + 1):
            lo_, hi_ = max(layer * dh, h_obs), min((layer + 1) * dh, h_e)
            tau += ext[layer, k] * (along(lo_) - along(hi_))
        assert -y[3] * s == pytest.approx(tau, rel=1e-8)


def test_curved_targets_flat_earth_limit(atm):
    """With an Earth radius of 1e12 m the shells are planar layers: the curved
    targets reduce to the planar ones."""
    flat = O.Atmosphere(**{**cases.ATMO_LAYERED, "earth_radius": 1e12})
    X = O.surrogate_inputs(flat, 12, LO, HI, 0, 400)
    # starts are layer boundaries (both walks begin in the layer above it); keep the
    # observation level clear of boundaries, where the planar and spherical walks may
    # end in different layers
    dh = 250.0
    m = lambda h: np.abs(h / dh - np.round(h / dh)) * dh
    X = X[m(X[:, 4]) > 0.05]
    assert len(X) > 300
    Yc = O.surrogate_targets(flat, X, "curved") * ((X[:, 0] - X[:, 4]) / X[:, 1])[:, None]
    Yp = O.surrogate_targets(flat, X, "planar")  # absolute; the chord is (h_e - h_obs) / cos in the limit
    # the planar excess and log T are the refraction's shares: add the straight line's own sums back
    d, ext = flat.layer_tables()
    k = np.floor((X[:, 3] - 300.0) / 300.0 * ext.shape[1]).astype(int)
    for n_, (he, ct, _, _, ho) in enumerate(X):
        spans = [(i, min((i + 1) * dh, he) - max(i * dh, ho)) for i in range(int(ho // dh), min(int(he // dh), 99) + 1)]
        Yp[n_, 2] += sum(d[i] * sp for i, sp in spans if sp > 0) / ct
        Yp[n_, 3] -= sum(ext[i, k[n_]] * sp for i, sp in spans if sp > 0) / ct
    # what is left of the curvature: the sphere sags by x^2 / 2R below the plane
    # over the horizontal span x (2e-4 m at 20 km), which moves lengths by about as
    # much; and FP64 resolves positions 1e12 m from the centre to 1.2e-4 m
    span = (X[:, 0] - X[:, 4]) * np.sqrt(1.0 - X[:, 1] ** 2) / X[:, 1]
    sag = span ** 2 / (2.0 * 1e12)
    ulp = np.spacing(1e12)
    tol = 4.0 * sag / X[:, 1] + 8.0 * ulp
    assert np.all(np.abs(Yc[:, 0] - Yp[:, 0]) <= tol)
    assert np.all(np.abs(Yc[:, 2] - Yp[:, 2]) <= tol)
    assert np.median(np.abs(Yc[:, 0] - Yp[:, 0])) < 1e-6
    np.testing.assert_allclose(Yc[:, 3], Yp[:, 3], rtol=1e-6)
    assert np.abs(Yc[:, 1]).max() < 1e-6


def test_curved_targets_earth_curvature_effect(atm):
    """On the real Earth the same photon bends a little more than over planar
    layers (the local vertical turns under it): the extra ground distance keeps
    its sign, and the curvature correction grows with zenith angle."""
    X = np.array([[12000.0, ct, 0.3, 405.46875, 2200.0] for ct in (0.95, 0.8, 0.6, 0.45)])
    Yc = O.surrogate_targets(atm, X, "curved") * ((X[:, 0] - X[:, 4]) / X[:, 1])[:, None]
    Yp = O.surrogate_targets(atm, X, "planar")
    assert np.all(np.sign(Yc[:, 0]) == np.sign(Yp[:, 0]))
    rel = np.abs(Yc[:, 0] - Yp[:, 0]) / np.abs(Yp[:, 0])
    assert np.all(np.diff(rel) > 0) and rel[-1] < 0.1


def test_curved_targets_nan_when_the_sphere_is_missed(atm):
    X = np.array([[20000.0, 0.01, 0.0, 405.46875, 2200.0]])
    assert np.all(np.isnan(O.surrogate_targets(atm, X, "curved")))


@pytest.mark.parametrize("geometry", ["planar", "curved"])
def test_targets_from_the_start_layer_boundary(atm, geometry):
    """The network starts at the start layer's lower boundary: the exact correction
    from an emission point inside layer j equals the correction from that layer's
    lower boundary (same straight line) plus the straight leg through layer j, whose
    optical depth and n - 1 part are ext_j l and delta_j l."""
    rng = np.random.default_rng(5)
    n = 300
    dh, R, h_obs = 250.0, 6.371e6, 2200.0
    j = rng.integers(10, 70, n)
    he = (j + rng.uniform(0.05, 0.95, n)) * dh
    ct = rng.uniform(0.45, 0.98, n)
    lam = 300.0 + (rng.integers(0, 64, n) + 0.5) * 300.0 / 64
    X = np.stack([he, ct, rng.uniform(-3, 3, n), lam, np.full(n, h_obs)], 1)
    hb = j * dh
    if geometry == "planar":
        leg = (he - hb) / ct
        cb = ct
    else:
        r0, rb = R + he, R + hb
        g = (r0 * ct) ** 2 - (r0 ** 2 - rb ** 2)
        cb = np.sqrt(g) / rb
        leg = (r0 ** 2 - rb ** 2) / (r0 * ct + np.sqrt(g))
    Xb = X.copy()
    Xb[:, 0], Xb[:, 1] = hb, cb
    Y = O.surrogate_targets(atm, X, geometry)
    Yb = O.surrogate_targets(atm, Xb, geometry)
    d, ext = atm.layer_tables()
    k = np.floor((lam - 300.0) / 300.0 * 64).astype(int)
    if geometry == "curved":   # per metre of chord: back to absolute values
        def chord(h, c):
            r, r1 = R + h, R + h_obs
            return (r ** 2 - r1 ** 2) / (r * c + np.sqrt((r * c) ** 2 - (r ** 2 - r1 ** 2)))
        Y = Y * chord(he, ct)[:, None]
        Yb = Yb * chord(hb, cb)[:, None]
    np.testing.assert_allclose(Y[:, 0], Yb[:, 0], rtol=1e-6, atol=1e-6)                    # landing offset (m)
    if geometry == "planar":   # the refraction's shares: the straight leg adds nothing to them
        np.testing.assert_allclose(Y[:, 2], Yb[:, 2], rtol=1e-6, atol=1e-7)
        np.testing.assert_allclose(Y[:, 3], Yb[:, 3], rtol=1e-6, atol=1e-12)
    else:                      # absolute sums: the leg adds its own
        np.testing.assert_allclose(Y[:, 2], Yb[:, 2] + d[j] * leg, rtol=1e-6, atol=1e-6)       # path excess (m)
        np.testing.assert_allclose(Y[:, 3], Yb[:, 3] - ext[j, k] * leg, rtol=1e-9, atol=1e-9)  # log T
