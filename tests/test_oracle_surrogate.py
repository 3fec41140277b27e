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
    centres = 300.0 + (np.arange(64) + 0.5) * 300.0 / 64
    assert np.all(np.isin(X[:, 3], centres))
    # counter-based: a window reproduces the same rows
    np.testing.assert_array_equal(O.surrogate_inputs(atm, 7, LO, HI, 1234, 10), X[1234:1244])
    assert stats.kstest((X[:, 2] + math.pi) / (2 * math.pi), "uniform").pvalue > 1e-3
    assert stats.kstest((X[:, 1] - LO[1]) / (HI[1] - LO[1]), "uniform").pvalue > 1e-3


def test_targets_homogeneous_medium():
    """No refraction in a homogeneous medium: zero offset, excess = (n-1) l, and
    the aerosol optical depth over the slant path."""
    atm = O.Atmosphere(profile="homogeneous", delta0=2.5e-4, h_top=25000.0, n_layers=100, n_lam=8,
                       aer_tau350=0.1, aer_H=1500.0)
    X = O.surrogate_inputs(atm, 3, LO, HI, 0, 500)
    Y = O.surrogate_targets(atm, X)
    np.testing.assert_allclose(Y[:, :2], 0.0, atol=1e-8)
    ell = (X[:, 0] - X[:, 4]) / X[:, 1]
    np.testing.assert_allclose(Y[:, 2], 2.5e-4 * ell, rtol=1e-9)
    # homogeneous layers carry constant extinction: tau = sum over spans of ext_i span_i / cos(theta),
    # and full layers hold the exact aerosol column at the bin centre
    d, ext = atm.layer_tables()
    lam = X[:, 3]
    k = np.floor((lam - 300.0) / 300.0 * 8).astype(int)
    dh = 250.0
    i_full = 40
    col = 0.1 * (lam / 350.0) ** -1.0 * (math.exp(-i_full * dh / 1500.0) - math.exp(-(i_full + 1) * dh / 1500.0))
    np.testing.assert_allclose(ext[i_full, k] * dh, col, rtol=1e-12)
    tau_closed = []
    for i in range(len(X)):
        he, ho = X[i, 0], X[i, 4]
        tau = 0.0
        for layer in range(int(ho // dh), min(int(he // dh), 99) + 1):
            lo_, hi_ = max(layer * dh, ho), min((layer + 1) * dh, he)
            tau += ext[layer, k[i]] * (hi_ - lo_)
        tau_closed.append(tau / X[i, 1])
    np.testing.assert_allclose(-Y[:, 3], tau_closed, rtol=1e-9)


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
        assert y[0] == pytest.approx(r - r_straight, abs=1e-7)   # along the photon's azimuth
        assert y[1] == pytest.approx(0.0, abs=1e-7)              # planar layers: no sideways offset
        assert y[2] == pytest.approx(opt - ls, rel=1e-9, abs=1e-9)
        assert y[3] == pytest.approx(-tau, rel=1e-10)


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
