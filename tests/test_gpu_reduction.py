"""Detector efficiency and pre-emission reduction (Sec. 4.3.1) on the GPU, through
the C ABI, against the oracle given the same efficiency and reduction tables."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_04229_amd import workload as W
from tests import cases, parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2405_04229_amd import cphot  # noqa: E402

ATMO = cases.ATMO_LAYERED
EFF = W.efficiency_curve(ATMO["n_lam"])


def _tables(h_obs=2200.0):
    atm = cphot.Atmosphere(**ATMO)
    q = cphot.reduction_table(atm, h_obs, EFF)
    return atm, q


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _thresholds(orc, q, n_lam=ATMO["n_lam"]):
    k = np.clip(np.floor((orc["lambda"] - 300.0) / 300.0 * n_lam).astype(int), 0, n_lam - 1)
    return np.exp(-orc["tau"]) * EFF[k]


def test_reduction_table_bounds_the_oracle_columns():
    """The library's bound against one built from the oracle's own layer
    extinction (bin centres): never below it, and within 1 % above it."""
    atm, q = _tables()
    oatm = O.Atmosphere(**ATMO)
    _, ext = oatm.layer_tables()
    L = ext.shape[0]
    dh = ATMO["h_top"] / L
    obs = int(2200.0 // dh)
    tau = np.zeros(ext.shape[1])
    ref = np.zeros(L)
    for i in range(L):
        ref[i] = np.max(EFF * np.exp(-tau))
        if i >= obs:
            tau = tau + ext[i] * ((i + 1) * dh - max(i * dh, 2200.0))
    assert np.all(q >= ref * (1.0 - 1e-12))
    assert np.all(q <= ref * 1.01)
    with pytest.raises(cphot.CphotError):
        cphot.reduction_table(atm, 2200.0, np.full(ATMO["n_lam"], 1.5))


@pytest.mark.parametrize("n", [1, 300, 5000])
def test_counts_bit_exact_with_reduction(n):
    atm, q = _tables()
    sh = W.make_shower(n, seed=905, xmax=450.0, zenith_deg=30.0, beta="R")
    g = np.array([[*sh.core, *sh.axis]])
    run = {**cases.RUN_TELESCOPE, "seed": 6}
    det = cphot.make_detector(atm, **run, efficiency=_dev(EFF), reduction=_dev(q))
    seg, gg, off = cphot.upload(sh.seg, g)
    S = cphot.make_segments(seg, gg, off)
    counts = torch.zeros(S.n, dtype=torch.int32, device="cuda")
    mu = torch.zeros(S.n, dtype=torch.float64, device="cuda")
    cphot.segment_counts(S, det, counts, mu)
    torch.cuda.synchronize()
    oc = O.segment_counts(O.Atmosphere(**ATMO), O.make_run(**run, efficiency=EFF, reduction=q), sh.seg)
    total = oc["n"] + oc["nf"].sum(1)
    np.testing.assert_array_equal(counts.cpu().numpy(), total)
    ok = oc["status"] == 0
    np.testing.assert_array_equal(mu.cpu().numpy()[ok], oc["mu"][ok])


@pytest.mark.parametrize("transport", ["layered", "straight"])
def test_records_with_efficiency_and_reduction(transport):
    atm, q = _tables()
    sh = W.make_shower(2000, seed=906, xmax=500.0, zenith_deg=40.0, azimuth_deg=70.0, beta="R")
    g = np.array([[*sh.core, *sh.axis]])
    run = dict(transport=transport, detector="grid", spectrum="frank_tamm", bunch=1, h_obs=2200.0, nx=300,
               ny=300, cell=4.0, seed=24)
    det = cphot.make_detector(atm, **run, efficiency=_dev(EFF), reduction=_dev(q))
    seg, gg, off = cphot.upload(sh.seg, g)
    S = cphot.make_segments(seg, gg, off)
    counts = torch.zeros(S.n, dtype=torch.int32, device="cuda")
    cphot.segment_counts(S, det, counts)
    offs = torch.cumsum(counts.to(torch.int64), 0) - counts.to(torch.int64)
    tot = int(counts.sum().item())
    rec = torch.zeros(max(tot, 1) * cphot.RECORD_BYTES, dtype=torch.uint8, device="cuda")
    cphot.trace_records(S, det, offs.contiguous(), rec)
    torch.cuda.synchronize()
    gr = cphot.records_to_numpy(rec.cpu())[:tot]
    oatm = O.Atmosphere(**ATMO)
    orun = O.make_run(**run, efficiency=EFF, reduction=q)
    o = O.trace(oatm, orun, sh.seg, core=sh.core, axis=sh.axis)
    qs = O.segment_counts(oatm, orun, sh.seg)["q"][o["seg"].astype(np.int64)]
    thr = _thresholds(o, q) / qs
    assert np.all(thr[np.isin(o["state"], [0, 2])] <= 1.0)
    flips, rep = parity.compare_records(gr, o, sh.core, ATMO, run, surv_thr=thr)
    print(rep)
    assert (o["state"] == 0).sum() > 1000
    assert flips <= max(3, parity.MAX_FLIP_FRACTION * len(o))


def test_reduction_preserves_the_detected_photons():
    """Full telescope workload, efficiency on both sides: the reduced call draws
    about a third of the records and detects the same photons per sphere within
    their statistical spread."""
    atm, q = _tables()
    sh = W.workload_telescope("R")
    g = np.array([[*sh.core, *sh.axis]])
    seg, gg, off = cphot.upload(sh.seg, g)
    S = cphot.make_segments(seg, gg, off)
    run = {**cases.RUN_TELESCOPE, "bunch": 1, "n_t": 0, "seed": 31}
    out = []
    for red in (None, _dev(q)):
        bins = torch.zeros(100, dtype=torch.int64, device="cuda")
        cnt = torch.zeros(cphot.NCOUNTERS, dtype=torch.int64, device="cuda")
        cphot.propagate(S, cphot.make_detector(atm, **run, efficiency=_dev(EFF), reduction=red), bins, None, cnt)
        torch.cuda.synchronize()
        out.append((bins.cpu().numpy().astype(np.float64), cnt.cpu().numpy()))
    (b0, c0), (b1, c1) = out
    print(dict(records=(int(c0[3]), int(c1[3])), binned=(b0.sum(), b1.sum())))
    assert c1[3] < 0.5 * c0[3]
    assert abs(b1.sum() - b0.sum()) < 5.0 * np.sqrt(b0.sum() + b1.sum())
    chi2, dof, p = parity.chi2_two_sample(b0, b1)
    assert p > 1e-4, (chi2, dof, p)


def test_efficiency_and_reduction_argument_errors():
    atm = cphot.Atmosphere(**cases.ATMO_STRAIGHT)  # no layers, no wavelength bins
    sh = W.make_shower(100, seed=907, beta="R")
    g = np.array([[*sh.core, *sh.axis]])
    seg, gg, off = cphot.upload(sh.seg, g)
    S = cphot.make_segments(seg, gg, off)
    bins = torch.zeros(100 * 100, dtype=torch.int64, device="cuda")
    # the binding checks the lengths the kernels read (one value per wavelength bin / layer)
    with pytest.raises(ValueError, match="efficiency"):
        cphot.make_detector(atm, **cases.RUN_TINY, efficiency=_dev(EFF))
    # the library refuses an efficiency on an atmosphere without wavelength bins
    eff = _dev(EFF)
    det = cphot.make_detector(atm, **cases.RUN_TINY)
    det.efficiency = eff.data_ptr()
    with pytest.raises(cphot.CphotError, match="efficiency"):
        cphot.propagate(S, det, bins)
    with pytest.raises(cphot.CphotError):
        cphot.reduction_table(atm, 2200.0, None)
