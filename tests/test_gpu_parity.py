"""HIP library against the FP64 oracle, through the C ABI, on the same seeded inputs.

Bars: integer record counts bit-exact; per-photon positions, times and optical
depths within the tolerances in tests/parity.py; decisions (survival, bin,
time bin) identical except where the oracle's value lies within rounding
distance of the decision boundary; bins equal up to those flips; counters
conserved.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_04229_amd import workload as W
from tests import cases, parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def _geom(sh):
    return np.array([[*sh.core, *sh.axis]])


def _orc_run(run_kw, seed):
    return O.make_run(**{**run_kw, "seed": seed})


# ---------------------------------------------------------------------------- counts

@pytest.mark.parametrize("beta", ["literal", "R"])
@pytest.mark.parametrize("n", [1, 255, 256, 257, 10_000])
def test_counts_bit_exact_tiny(beta, n):
    sh = W.workload_tiny_vertical(beta, n=n)
    run = {**cases.RUN_TINY, "seed": 17}
    g = parity.device_counts(cases.ATMO_STRAIGHT, run, sh.seg, _geom(sh))
    o = O.segment_counts(parity.oracle_atm(cases.ATMO_STRAIGHT), _orc_run(cases.RUN_TINY, 17), sh.seg)
    np.testing.assert_array_equal(g, o["n"])


def test_counts_bit_exact_telescope_full_size():
    """All 1e6 segments of the telescope workload, bunches of 5, in the launch
    configuration the benchmark uses."""
    sh = W.workload_telescope("R")
    run = {**cases.RUN_TELESCOPE, "seed": 2}
    g, mu = parity.device_counts(cases.ATMO_LAYERED, run, sh.seg, _geom(sh), with_mu=True)
    o = O.segment_counts(parity.oracle_atm(cases.ATMO_LAYERED), _orc_run(cases.RUN_TELESCOPE, 2), sh.seg)
    np.testing.assert_array_equal(g, o["n"])
    # the FP64 yield itself is bit-identical, not only its rounding
    omu = np.where(o["status"] == 0, o["mu"], 0.0)
    np.testing.assert_array_equal(mu.view(np.uint64), omu.view(np.uint64))
    assert g.sum() > 1e7


# ---------------------------------------------------------------------------- records

@pytest.mark.parametrize("beta", ["literal", "R"])
def test_records_tiny_vertical(beta):
    sh = W.workload_tiny_vertical(beta, n=3000 if beta == "R" else 10_000)
    run = {**cases.RUN_TINY, "seed": 5}
    g = parity.device_records(cases.ATMO_STRAIGHT, run, sh.seg, _geom(sh))
    o = O.trace(parity.oracle_atm(cases.ATMO_STRAIGHT), _orc_run(cases.RUN_TINY, 5), sh.seg, core=sh.core,
                axis=sh.axis)
    flips, rep = parity.compare_records(g, o, sh.core, cases.ATMO_STRAIGHT, run)
    print(rep)
    assert flips <= max(3, parity.MAX_FLIP_FRACTION * len(o))


def test_records_telescope_layered_spheres():
    sh = W.make_shower(6000, seed=1002, xmax=400.0, zenith_deg=20.0, beta="R")
    run = {**cases.RUN_TELESCOPE, "pitch": 25.0, "seed": 9}
    g = parity.device_records(cases.ATMO_LAYERED, run, sh.seg, _geom(sh))
    o = O.trace(parity.oracle_atm(cases.ATMO_LAYERED), _orc_run(run, 9), sh.seg, core=sh.core, axis=sh.axis)
    flips, rep = parity.compare_records(g, o, sh.core, cases.ATMO_LAYERED, run)
    print(rep)
    assert (o["state"] == 0).sum() > 500
    assert flips <= max(3, parity.MAX_FLIP_FRACTION * len(o))


def test_records_layered_grid_inclined():
    sh = W.make_shower(2000, seed=44, xmax=500.0, zenith_deg=45.0, azimuth_deg=130.0, beta="R")
    run = dict(transport="layered", detector="grid", spectrum="frank_tamm", bunch=1, h_obs=2200.0,
               nx=300, ny=300, cell=4.0, seed=21)
    g = parity.device_records(cases.ATMO_LAYERED, run, sh.seg, _geom(sh))
    o = O.trace(parity.oracle_atm(cases.ATMO_LAYERED), _orc_run(run, 21), sh.seg, core=sh.core, axis=sh.axis)
    flips, rep = parity.compare_records(g, o, sh.core, cases.ATMO_LAYERED, run)
    print(rep)
    assert flips <= max(3, parity.MAX_FLIP_FRACTION * len(o))


def test_records_sampled_at_full_telescope_size():
    """Sampled slices of the 1e6-segment telescope workload: the oracle traces
    each slice's photons one by one with the slice's global segment ids."""
    sh = W.workload_telescope("R")
    run = {**cases.RUN_TELESCOPE, "seed": 2}
    for start in (0, 123_457, 500_000, 999_900):
        sl = slice(start, start + 100)
        seg = {k: v[sl] for k, v in sh.seg.items()}
        g = parity.device_records(cases.ATMO_LAYERED, run, seg, _geom(sh), first_id=start)
        o = O.trace(parity.oracle_atm(cases.ATMO_LAYERED), _orc_run(run, 2), seg, core=sh.core, axis=sh.axis,
                    first_id=start)
        flips, rep = parity.compare_records(g, o, sh.core, cases.ATMO_LAYERED, run)
        assert flips <= 3


# ---------------------------------------------------------------------------- bins

@pytest.mark.parametrize("lds_hist", [1, 0])
@pytest.mark.parametrize("beta", ["literal", "R"])
def test_bins_tiny_vertical(beta, lds_hist):
    sh = W.workload_tiny_vertical(beta)
    run = {**cases.RUN_TINY, "seed": 3}
    gb, _, gc = parity.device_run(cases.ATMO_STRAIGHT, {**run, "lds_hist": lds_hist}, sh.seg, _geom(sh))
    ob, _, oc = O.propagate(parity.oracle_atm(cases.ATMO_STRAIGHT), _orc_run(cases.RUN_TINY, 3), sh.seg,
                            _geom(sh), threads=8)
    gc = gc.astype(np.uint64)
    # segment-level counters and record totals are exact
    np.testing.assert_array_equal(gc[:4], oc[:4])
    assert gc[3] == gc[4] + gc[5] + gc[6] + gc[7]
    assert int(gb.sum()) == int(gc[8]) == int(gc[7])
    diff = np.abs(gb.astype(np.int64) - ob.astype(np.int64)).sum()
    assert diff <= max(4, 2e-4 * ob.sum()), diff
    # per-bin counts within 0.1 % + flips
    assert np.all(np.abs(gb.astype(np.int64) - ob.astype(np.int64)) <= 0.001 * ob + 2)


def test_bins_and_time_histograms_telescope_subset():
    sh = W.make_shower(40_000, seed=1002, xmax=400.0, zenith_deg=20.0, beta="R")
    run = {**cases.RUN_TELESCOPE, "pitch": 40.0, "seed": 4}
    gb, gt, gc = parity.device_run(cases.ATMO_LAYERED, run, sh.seg, _geom(sh))
    ob, ot, oc = O.propagate(parity.oracle_atm(cases.ATMO_LAYERED), _orc_run(run, 4), sh.seg, _geom(sh), threads=8)
    gc = gc.astype(np.uint64)
    np.testing.assert_array_equal(gc[:4], oc[:4])
    assert gc[3] == gc[4] + gc[5] + gc[6] + gc[7]
    assert int(gb.sum()) == int(gc[8]) == 5 * int(gc[7])
    assert int(gt.astype(np.int64).sum()) == int(gb.sum())
    assert np.abs(gb.astype(np.int64) - ob.astype(np.int64)).sum() <= max(10, 2e-4 * ob.sum())
    assert np.abs(gt.astype(np.int64) - ot.astype(np.int64)).sum() <= max(20, 4e-4 * ot.sum())
    assert ob.sum() > 1000


def test_independent_seeds_chi2():
    sh = W.workload_tiny_vertical("R")
    gb, _, _ = parity.device_run(cases.ATMO_STRAIGHT, {**cases.RUN_TINY, "seed": 101}, sh.seg, _geom(sh))
    ob, _, _ = O.propagate(parity.oracle_atm(cases.ATMO_STRAIGHT), _orc_run(cases.RUN_TINY, 202), sh.seg,
                           _geom(sh), threads=8)
    chi2, dof, p = parity.chi2_two_sample(gb, ob)
    assert dof > 100 and p > 1e-3, (chi2, dof, p)


def test_multi_shower_batch_matches_oracle():
    shs = W.make_batch(6, seed=77, log_range=(2.0, 3.5), beta="R")
    seg, offs, geom = W.concat_showers(shs)
    run = dict(transport="straight", detector="grid", spectrum="uniform", bunch=1, h_obs=2200.0, nx=200, ny=200,
               cell=5.0, seed=12)
    gb, _, gc = parity.device_run(cases.ATMO_STRAIGHT, run, seg, geom, offsets=offs)
    ob, _, oc = O.propagate(parity.oracle_atm(cases.ATMO_STRAIGHT), _orc_run(run, 12), seg, geom, offsets=offs,
                            threads=8)
    np.testing.assert_array_equal(gc[:4].astype(np.uint64), oc[:4])
    assert np.abs(gb.astype(np.int64) - ob.astype(np.int64)).sum() <= max(4, 2e-4 * ob.sum())


# ---------------------------------------------------------------------------- edge cases

def test_degenerate_segments_are_counted_not_errors():
    n = 300
    sh = W.workload_tiny_vertical("R", n=n)
    seg = {k: v.copy() for k, v in sh.seg.items()}
    seg["x0"][0] = np.nan            # non-finite
    seg["beta"][1] = 1.0             # beta outside (0, 1)
    seg["beta"][2] = -0.5
    seg["x1"][3], seg["y1"][3], seg["z1"][3] = seg["x0"][3], seg["y0"][3], seg["z0"][3]  # zero length
    seg["charge"][4] = 0.0           # no charge: no photons
    seg["z0"][5], seg["z1"][5] = seg["z1"][5], seg["z0"][5]  # upward track
    seg["z0"][6], seg["z1"][6] = 1500.0, 1498.0               # below the observation level
    seg["z0"][7], seg["z1"][7] = 30000.0, 29998.0             # above the table: clamped
    run = {**cases.RUN_TINY, "seed": 8}
    gb, _, gc = parity.device_run(cases.ATMO_STRAIGHT, run, seg, _geom(sh))
    ob, _, oc = O.propagate(parity.oracle_atm(cases.ATMO_STRAIGHT), _orc_run(cases.RUN_TINY, 8), seg, _geom(sh))
    np.testing.assert_array_equal(gc[:4].astype(np.uint64), oc[:4])
    assert int(gc[1]) == 4
    np.testing.assert_array_equal(gb, ob)
    g = parity.device_records(cases.ATMO_STRAIGHT, run, seg, _geom(sh))
    o = O.trace(parity.oracle_atm(cases.ATMO_STRAIGHT), _orc_run(cases.RUN_TINY, 8), seg, core=sh.core,
                axis=sh.axis)
    parity.compare_records(g, o, sh.core, cases.ATMO_STRAIGHT, run)


def test_empty_input_and_bad_arguments():
    from paper_2405_04229_amd import cphot
    sh = W.workload_tiny_vertical("R", n=10)
    empty = {k: v[:0] for k, v in sh.seg.items()}
    gb, _, gc = parity.device_run(cases.ATMO_STRAIGHT, cases.RUN_TINY, empty, _geom(sh))
    assert gb.sum() == 0 and gc.sum() == 0
    atm = cphot.Atmosphere(**cases.ATMO_STRAIGHT)
    seg, g, off = cphot.upload(sh.seg, _geom(sh))
    S = cphot.make_segments(seg, g, off)
    small = torch.zeros(10, dtype=torch.int64, device="cuda")
    with pytest.raises(cphot.CphotError):
        cphot.propagate(S, cphot.make_detector(atm, **cases.RUN_TINY), small)
    with pytest.raises(cphot.CphotError):
        cphot.propagate(S, cphot.make_detector(atm, **{**cases.RUN_TINY, "bunch": 0}),
                        torch.zeros(10000, dtype=torch.int64, device="cuda"))
    with pytest.raises(cphot.CphotError):  # layered transport without layers
        cphot.propagate(S, cphot.make_detector(atm, **{**cases.RUN_TINY, "transport": "layered"}),
                        torch.zeros(10000, dtype=torch.int64, device="cuda"))
    with pytest.raises(cphot.CphotError):
        cphot.Atmosphere(**{**cases.ATMO_STRAIGHT, "step": 0.0})


def test_deterministic_across_launch_shapes():
    sh = W.workload_tiny_vertical("R")
    base = {**cases.RUN_TINY, "seed": 31}
    ref = None
    for bs, grid, lds in [(256, 0, -1), (128, 7, 0), (512, 1, 1), (256, 3, 1)]:
        gb, _, gc = parity.device_run(cases.ATMO_STRAIGHT, {**base, "block_size": bs, "grid_blocks": grid,
                                                            "lds_hist": lds}, sh.seg, _geom(sh))
        if ref is None:
            ref = (gb, gc)
        else:
            np.testing.assert_array_equal(gb, ref[0])
            np.testing.assert_array_equal(gc, ref[1])
