"""Data-reduction cuts (filter levels 1 and 3, Sec. 4.3.2, 4.3.4, 6.2): geometric
bounds that must never remove a photon that could reach a telescope sphere or land
on the ground grid. With the cuts on, bins and time histograms equal those of the
same call without them bit for bit; only the counters show the removed records."""
import numpy as np
import pytest

from paper_2405_04229_amd import workload as W
from tests import cases

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2405_04229_amd import cphot  # noqa: E402

C_GEN, C_UP, C_ABS, C_OUT, C_BIN = 3, 4, 5, 6, 7
C_FALLBACK, C_TRACK, C_PHOTON = 9, 11, 12


def _run(atm, S, ns, run, cuts, table=None):
    nsph = run["snx"] * run["sny"]
    n_t = run.get("n_t", 0)
    bins = torch.zeros(ns * nsph, dtype=torch.int64, device="cuda")
    th = torch.zeros(ns * nsph * (n_t + 1), dtype=torch.int32, device="cuda") if n_t else None
    cnt = torch.zeros(cphot.NCOUNTERS, dtype=torch.int64, device="cuda")
    det = cphot.make_detector(atm, **run, cuts=cuts, table=table)
    cphot.propagate(S, det, bins, th, cnt)
    torch.cuda.synchronize()
    return bins.cpu().numpy(), None if th is None else th.cpu().numpy(), cnt.cpu().numpy()


def _check(atm, S, ns, run, table=None, expect_track=True):
    b0, t0, c0 = _run(atm, S, ns, run, (), table)
    assert c0[C_BIN] > 0
    for cuts in (("track",), ("photon",), ("track", "photon")):
        b, t, c = _run(atm, S, ns, run, cuts, table)
        np.testing.assert_array_equal(b, b0, err_msg=str(cuts))
        if t0 is not None:
            np.testing.assert_array_equal(t, t0, err_msg=str(cuts))
        assert c[C_BIN] == c0[C_BIN]
        assert c[C_GEN] == c[C_UP] + c[C_ABS] + c[C_OUT] + c[C_BIN]
        assert c[C_GEN] + c[C_TRACK] == c0[C_GEN]
        assert c[C_FALLBACK] == 0  # records compacted after the photon cut are no fallbacks
        if "track" in cuts and expect_track:
            assert c[C_TRACK] > 0, cuts
        if "photon" in cuts:
            assert c[C_PHOTON] > 0, cuts
        else:
            assert c[C_PHOTON] == 0
    return c0, c


def _segments(sh):
    g = np.array([[*sh.core, *sh.axis]])
    seg, gg, off = cphot.upload(sh.seg, g)
    return cphot.make_segments(seg, gg, off)


def test_cuts_exact_on_the_telescope_workload():
    """Full telescope workload (1e6 segments, 512 time bins): nothing that hits is lost."""
    atm = cphot.Atmosphere(**cases.ATMO_LAYERED)
    S = _segments(W.workload_telescope("R"))
    c0, c = _check(atm, S, 1, {**cases.RUN_TELESCOPE, "seed": 21})
    # most records of the telescope workload miss the 10 x 10 spheres; the two filters
    # remove most of them (the last call above ran both)
    print(dict(generated=int(c0[C_GEN]), outside=int(c0[C_OUT]), track=int(c[C_TRACK]), photon=int(c[C_PHOTON])))
    assert c[C_TRACK] + c[C_PHOTON] > 0.5 * c0[C_OUT]


@pytest.mark.parametrize("transport", ["straight", "layered", "table"])
def test_cuts_exact_where_the_light_pool_clips_the_array(transport):
    """An inclined shower whose light pool edge crosses a dense array of large
    spheres, so that photons pass close to every bound."""
    atm = cphot.Atmosphere(**(cases.ATMO_STRAIGHT if transport == "straight" else cases.ATMO_LAYERED))
    sh = W.make_shower(300_000, seed=803, xmax=450.0, zenith_deg=50.0, azimuth_deg=30.0, beta="R")
    S = _segments(sh)
    run = {**cases.RUN_TELESCOPE, "transport": transport, "snx": 9, "sny": 7, "pitch": 40.0, "radius": 10.0,
           "n_t": 64, "dt": 2.0, "seed": 22}
    tab = cphot.Table(atm, run["h_obs"], "planar", h_hi=20000.0, c_lo=0.2) if transport == "table" else None
    _check(atm, S, 1, run, table=tab)


def test_cuts_exact_across_showers():
    """A batch of showers with their own sphere arrays; tiles mix showers."""
    atm = cphot.Atmosphere(**cases.ATMO_LAYERED)
    seg, offs, geom = W.concat_showers(W.make_batch(16, seed=29, beta="R", scale=0.05))
    sg, g, off = cphot.upload(seg, geom, offs)
    S = cphot.make_segments(sg, g, off)
    run = {**cases.RUN_TELESCOPE, "snx": 6, "sny": 6, "pitch": 60.0, "radius": 8.0, "n_t": 32, "dt": 2.0,
           "seed": 23}
    _check(atm, S, geom.shape[0], run)


def _grid_run(atm, S, run, cuts, table=None, dtype=torch.float64):
    bins = torch.zeros(run["nx"] * run["ny"], dtype=dtype, device="cuda")
    cnt = torch.zeros(cphot.NCOUNTERS, dtype=torch.int64, device="cuda")
    cphot.propagate(S, cphot.make_detector(atm, **run, cuts=cuts, table=table), bins, None, cnt)
    torch.cuda.synchronize()
    return bins.cpu().numpy(), cnt.cpu().numpy()


def _grid_check(atm, S, run, table=None, dtype=torch.float64, min_cut=0.05):
    b0, c0 = _grid_run(atm, S, run, (), table, dtype)
    b, c = _grid_run(atm, S, run, ("photon",), table, dtype)
    np.testing.assert_array_equal(b, b0)
    assert c[C_BIN] == c0[C_BIN] > 0
    assert c[C_GEN] == c0[C_GEN] and c[C_TRACK] == 0
    assert c[C_GEN] == c[C_UP] + c[C_ABS] + c[C_OUT] + c[C_BIN]
    assert c[C_PHOTON] > min_cut * c[C_GEN], (int(c[C_PHOTON]), int(c[C_GEN]))
    # a culled record counts as outside, also where the uncut call absorbed it on the way
    assert c[C_OUT] + c[C_ABS] == c0[C_OUT] + c0[C_ABS] and c[C_UP] == c0[C_UP]
    return c0, c


def test_grid_photon_cut_exact_on_the_inclined_chunk():
    """The large inclined shower's resident chunk (1e7 segments, curved shells,
    Cherenkov + fluorescence, FP64 bins): records whose straight line lands beyond
    the refraction bound of the grid are outside before transport, and the bins
    equal those of the uncut call bit for bit."""
    atm = cphot.Atmosphere(**cases.ATMO_LAYERED)
    sh = W.workload_inclined_chunk(0)
    g = np.array([[*sh.core, *sh.axis]])
    seg, gg, off = cphot.upload(sh.seg, g)
    S = cphot.make_segments(seg, gg, off, first_id=sh.first_id)
    c0, c = _grid_check(atm, S, {**cases.RUN_INCLINED, "seed": 5}, min_cut=0.15)
    print(dict(generated=int(c0[C_GEN]), culled=int(c[C_PHOTON]), walked_uncut=int(c0[9]), walked_cut=int(c[9])))
    assert c[9] < 0.5 * c0[9]   # most records outside the shell sums' domain never reach the walk


@pytest.mark.parametrize("transport", ["curved_walk", "table_curved", "layered", "table", "straight"])
def test_grid_photon_cut_exact_other_transports(transport):
    """The same bound for the shell walk and the curved table, and the planar
    bound for planar layers, the planar table and straight rays, on an inclined
    shower whose light pool is clipped by a small grid."""
    curved = transport in ("curved_walk", "table_curved")
    atm = cphot.Atmosphere(**(cases.ATMO_STRAIGHT if transport == "straight" else cases.ATMO_LAYERED))
    sh = W.make_shower(200_000, seed=811, xmax=500.0, zenith_deg=55.0 if curved else 40.0, azimuth_deg=20.0,
                       beta="R", dedx=(0.1, 2.0) if curved else None)
    S = _segments(sh)
    tab = None
    if transport == "table_curved":
        tab = cphot.Table(atm, 2200.0, "curved", n_c=512, c_lo=0.15)
    elif transport == "table":
        tab = cphot.Table(atm, 2200.0, "planar", h_hi=20000.0, c_lo=0.2)
    # planar: a grid smaller than the Cherenkov light pool, so that its edges cut through it
    grid = dict(nx=300, ny=200, cell=4.0) if curved else dict(nx=100, ny=60, cell=2.0)
    run = dict(transport="table" if tab is not None else transport, detector="grid", spectrum="frank_tamm",
               emission="both" if curved else "cherenkov", bunch=1, h_obs=2200.0, seed=24, **grid)
    _grid_check(atm, S, run, table=tab, dtype=torch.int64)


def test_cut_argument_errors():
    atm = cphot.Atmosphere(**cases.ATMO_LAYERED)
    S = _segments(W.make_shower(100, seed=804, beta="R"))
    bins = torch.zeros(100 * 100, dtype=torch.int64, device="cuda")
    with pytest.raises(cphot.CphotError, match="track cut"):  # grid detector: photon cut only
        cphot.propagate(S, cphot.make_detector(atm, **{**cases.RUN_TINY, "transport": "layered"},
                                               cuts=("track",)), bins)
    sur = cphot.Surrogate(cases.SURROGATE_LO, cases.SURROGATE_HI)
    norm = np.zeros(cphot.N_NORM, dtype=np.float32)
    norm[0:5], norm[5:10] = cases.SURROGATE_LO, cases.SURROGATE_HI
    norm[10:15] = 2.0 / (np.array(cases.SURROGATE_HI) - np.array(cases.SURROGATE_LO))
    norm[20:24] = 1.0
    sur.set_params(None, norm)
    with pytest.raises(cphot.CphotError, match="planar surrogate"):
        cphot.propagate(S, cphot.make_detector(atm, **{**cases.RUN_TINY, "transport": "surrogate"},
                                               surrogate=sur, cuts=("photon",)), bins)
    d = cphot.make_detector(atm, **{**cases.RUN_TELESCOPE, "n_t": 0})
    d.cuts = 4
    with pytest.raises(cphot.CphotError, match="cut bits"):
        cphot.propagate(S, d, bins)
