"""Batched showers in one launch, captured HIP-graph steps and the autotuner."""
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

RUN_BATCH = dict(transport="straight", detector="grid", spectrum="frank_tamm", bunch=1, h_obs=2200.0, nx=200,
                 ny=200, cell=5.0)


def _batch(n=12, scale=0.05, seed=5):
    shs = W.make_batch(n, seed=seed, beta="R", scale=scale)
    return W.concat_showers(shs)


def test_batch_matches_oracle_per_shower():
    seg, offs, geom = _batch()
    run = {**RUN_BATCH, "seed": 3}
    gb, _, gc = parity.device_run(cases.ATMO_STRAIGHT, run, seg, geom, offsets=offs)
    ob, _, oc = O.propagate(parity.oracle_atm(cases.ATMO_STRAIGHT), O.make_run(**run), seg, geom, offsets=offs,
                            threads=8)
    np.testing.assert_array_equal(gc[:4].astype(np.uint64), oc[:4])
    atm = parity.oracle_atm(cases.ATMO_STRAIGHT)
    for s in range(len(geom)):
        d = np.abs(gb[s].astype(np.int64) - ob[s].astype(np.int64)).sum()
        # bins differ only through photons whose landing point lies within the
        # position tolerance of a cell edge (inclined showers: long paths)
        sl = slice(int(offs[s]), int(offs[s + 1]))
        o = O.trace(atm, O.make_run(**run), {k: v[sl] for k, v in seg.items()}, core=geom[s, :2],
                    axis=geom[s, 2:5], first_id=int(offs[s]))
        assert d <= max(4, parity.flip_budget(o, geom[s, :2], cases.ATMO_STRAIGHT, run)), (s, d)


def _setup(seg, offs, geom, run, atm):
    det = cphot.make_detector(atm, **run)
    sg, g, off = cphot.upload(seg, geom, offs)
    S = cphot.make_segments(sg, g, off)
    ns = geom.shape[0]
    bins = torch.zeros(ns * run["nx"] * run["ny"], dtype=torch.int32, device="cuda")
    cnt = torch.zeros(16, dtype=torch.int64, device="cuda")
    return det, S, bins, cnt


def test_graph_replays_equal_eager():
    seg, offs, geom = _batch(seed=9)
    atm = cphot.Atmosphere(**cases.ATMO_STRAIGHT)
    run = {**RUN_BATCH, "seed": 4}
    det, S, bins, cnt = _setup(seg, offs, geom, run, atm)
    cphot.propagate(S, det, bins, None, cnt)
    torch.cuda.synchronize()
    ref_b, ref_c = bins.clone(), cnt.clone()
    step = cphot.Step(S, det, bins, None, cnt, clear=True)
    other = torch.randn(1 << 20, device="cuda")
    for r in range(4):
        bins.fill_(7)        # garbage the step must clear
        cnt.fill_(3)
        step.launch()
        torch.cuda.synchronize()
        assert torch.equal(bins, ref_b), r
        assert torch.equal(cnt, ref_c), r
        other.mul_(1.0001).sum().item()  # eager work and a synchronisation between replays


def test_autotune_returns_equivalent_shape():
    seg, offs, geom = _batch(seed=11)
    atm = cphot.Atmosphere(**cases.ATMO_STRAIGHT)
    run = {**RUN_BATCH, "seed": 6}
    det, S, bins, cnt = _setup(seg, offs, geom, run, atm)
    best = cphot.autotune(S, det, bins, None, cnt, bunches=[1], reps=2)
    assert best["block_size"] in (128, 256, 512) and best["bunch"] == 1 and best["ms"] > 0
    bins.zero_()
    cnt.zero_()
    cphot.propagate(S, det, bins, None, cnt)
    ref = bins.clone()
    tuned = cphot.make_detector(atm, **run, **cphot.shape_of(best))
    bins.zero_()
    cphot.propagate(S, tuned, bins, None, cnt)
    torch.cuda.synchronize()
    assert torch.equal(bins, ref)


@pytest.mark.parametrize("bs", [128, 256, 512])
def test_lds_window_bins_identical_to_global_atomics(bs):
    """Grid counts privatised in an LDS window (around each shower's core, the
    rest global) give the same integer bins as global atomics alone, for window
    sizes, persistent-grid sizes and block sizes, across shower boundaries
    inside tiles and blocks."""
    seg, offs, geom = _batch(n=20, seed=13)
    atm = cphot.Atmosphere(**cases.ATMO_STRAIGHT)
    run = {**RUN_BATCH, "seed": 8}
    det, S, bins, cnt = _setup(seg, offs, geom, run, atm)
    ref_det = cphot.make_detector(atm, **run, block_size=bs, lds_hist=0)
    cphot.propagate(S, ref_det, bins, None, cnt)
    torch.cuda.synchronize()
    ref_b, ref_c = bins.clone(), cnt.clone()
    assert int(ref_c[7]) > 10_000
    # square windows, rectangles shifted off the centre (clamped at the grid's edges), and a
    # rectangle larger than the LDS budget (shrunk to fit)
    windows = [(0, 0, 0, 0), (9, 0, 0, 0), (16, 0, 0, 0), (40, 0, 0, 0), (48, 12, 5, -3), (12, 40, -7, 9),
               (30, 20, 10_000, -10_000), (400, 300, 0, 0)]
    for w, h, dx, dy in windows:
        for grid in (0, 7, 1024):
            d = cphot.make_detector(atm, **run, block_size=bs, grid_blocks=grid, lds_hist=1, hist_window=w,
                                    hist_window_h=h, hist_window_dx=dx, hist_window_dy=dy)
            bins.zero_()
            cnt.zero_()
            cphot.propagate(S, d, bins, None, cnt)
            torch.cuda.synchronize()
            assert torch.equal(bins, ref_b), (w, h, dx, dy, grid)
            assert torch.equal(cnt, ref_c), (w, h, dx, dy, grid)


@pytest.mark.parametrize("bs", [128, 256, 512])
def test_lds_sphere_counts_identical_to_global_atomics(bs):
    """Sphere counts privatised in LDS (flushed when a block's shower changes)
    give the same bins and time histograms as global atomics alone, for u32, u64
    and FP64 bins, several grid sizes and block sizes, across shower boundaries
    inside tiles and blocks."""
    seg, offs, geom = _batch(n=20, seed=17)
    atm = cphot.Atmosphere(**cases.ATMO_LAYERED)
    run = {**cases.RUN_TELESCOPE, "snx": 12, "sny": 9, "pitch": 20.0, "radius": 5.0, "n_t": 64, "dt": 0.1,
           "seed": 12}
    sg, g, off = cphot.upload(seg, geom, offs)
    S = cphot.make_segments(sg, g, off)
    ns, nsph = geom.shape[0], 12 * 9
    for dtype in (torch.int32, torch.int64, torch.float64):
        bins = torch.zeros(ns * nsph, dtype=dtype, device="cuda")
        th = torch.zeros(ns * nsph * 65, dtype=torch.int32, device="cuda")
        cnt = torch.zeros(16, dtype=torch.int64, device="cuda")
        cphot.propagate(S, cphot.make_detector(atm, **run, block_size=bs, lds_hist=0), bins, th, cnt)
        torch.cuda.synchronize()
        ref_b, ref_t, ref_c = bins.clone(), th.clone(), cnt.clone()
        assert int(ref_c[7]) > 2_000
        # hits inside and beyond the leading time bins held in LDS, and overflow
        t = ref_t.view(ns * nsph, 65).sum(0).cpu().numpy()
        assert t[:20].sum() > 0 and t[40:64].sum() > 0 and t[64] > 0, t
        for grid in (0, 7, 1024):
            bins.zero_()
            th.zero_()
            cnt.zero_()
            d = cphot.make_detector(atm, **run, block_size=bs, grid_blocks=grid, lds_hist=1)
            cphot.propagate(S, d, bins, th, cnt)
            torch.cuda.synchronize()
            assert torch.equal(bins, ref_b), (dtype, grid)
            assert torch.equal(th, ref_t), (dtype, grid)
            assert torch.equal(cnt, ref_c), (dtype, grid)


def test_lds_sphere_counts_that_do_not_fit():
    """A sphere array too large for LDS: an error when LDS is demanded, global
    atomics under the library's choice, with the same bins."""
    sh = W.make_shower(20_000, seed=22, xmax=500.0, zenith_deg=20.0, beta="R")
    g = np.array([[*sh.core, *sh.axis]])
    atm = cphot.Atmosphere(**cases.ATMO_LAYERED)
    run = {**cases.RUN_TELESCOPE, "snx": 200, "sny": 200, "pitch": 2.0, "radius": 0.5, "n_t": 0, "seed": 5}
    seg, gg, off = cphot.upload(sh.seg, g)
    S = cphot.make_segments(seg, gg, off)
    bins = torch.zeros(200 * 200, dtype=torch.int64, device="cuda")
    with pytest.raises(cphot.CphotError, match="LDS"):
        cphot.propagate(S, cphot.make_detector(atm, **run, lds_hist=1), bins)
    out = []
    for lds in (-1, 0):
        bins.zero_()
        cphot.propagate(S, cphot.make_detector(atm, **run, lds_hist=lds), bins)
        torch.cuda.synchronize()
        out.append(bins.clone())
    assert torch.equal(out[0], out[1]) and int(out[0].sum()) > 1000


def test_lds_window_f64_and_large_single_grid():
    """One shower on a grid far larger than LDS (window in the middle), FP64 and
    u64 bins: identical to global atomics."""
    sh = W.make_shower(20_000, seed=21, xmax=500.0, zenith_deg=45.0, azimuth_deg=10.0, beta="R")
    g = np.array([[*sh.core, *sh.axis]])
    atm = cphot.Atmosphere(**cases.ATMO_STRAIGHT)
    run = {**RUN_BATCH, "nx": 700, "ny": 500, "cell": 2.0, "bunch": 3, "seed": 9}
    seg, gg, off = cphot.upload(sh.seg, g)
    S = cphot.make_segments(seg, gg, off)
    out = []
    for dtype in (torch.int64, torch.float64):
        for lds in (0, 1):
            d = cphot.make_detector(atm, **run, lds_hist=lds)
            bins = torch.zeros(700 * 500, dtype=dtype, device="cuda")
            cphot.propagate(S, d, bins, None, None)
            torch.cuda.synchronize()
            out.append(bins.cpu().numpy().astype(np.float64))
    for b in out[1:]:
        np.testing.assert_array_equal(b, out[0])
    assert out[0].sum() > 1e5


@pytest.mark.parametrize("bunch", [1, 5])
def test_batched_workload_at_full_size(bunch):
    """The benchmark's batch (256 showers, 3.3e7 segments): every segment's record
    count bit-exact, and slices of three showers traced record by record with
    their global segment ids and their own geometry."""
    seg, offs, geom = W.concat_showers(W.make_batch(256, seed=1003, beta="R"))
    run = {**RUN_BATCH, "bunch": bunch, "seed": 3}
    # counts depend on the segments only: one shower's geometry serves the whole set
    g = parity.device_counts(cases.ATMO_STRAIGHT, run, seg, geom[:1])
    o = O.segment_counts(parity.oracle_atm(cases.ATMO_STRAIGHT), O.make_run(**run), seg)
    np.testing.assert_array_equal(g, o["n"])
    assert len(g) > 3e7
    atm = parity.oracle_atm(cases.ATMO_STRAIGHT)
    for s in (0, 131, 255):
        start = int(offs[s]) + (int(offs[s + 1]) - int(offs[s])) // 2
        sl = slice(start, min(start + 100, int(offs[s + 1])))
        part = {k: v[sl] for k, v in seg.items()}
        gr = parity.device_records(cases.ATMO_STRAIGHT, run, part, geom[s:s + 1], first_id=start)
        orr = O.trace(atm, O.make_run(**run), part, core=geom[s, :2], axis=geom[s, 2:5], first_id=start)
        flips, rep = parity.compare_records(gr, orr, geom[s, :2], cases.ATMO_STRAIGHT, run)
        assert flips <= 3, rep


def test_autotune_cache_in_memory_and_file(tmp_path):
    seg, offs, geom = _batch(n=4, scale=0.02, seed=13)
    atm = cphot.Atmosphere(**cases.ATMO_STRAIGHT)
    run = {**RUN_BATCH, "seed": 6}
    det, S, bins, cnt = _setup(seg, offs, geom, run, atm)
    path = tmp_path / "tuning.txt"
    cphot.autotune_cache_clear()
    a = cphot.autotune(S, det, bins, None, cnt, bunches=[1, 2], reps=1, cache_path=path)
    assert not a["cached"]
    b = cphot.autotune(S, det, bins, None, cnt, bunches=[1, 2], reps=1, cache_path=path)
    assert b == {**a, "cached": True}
    c = cphot.autotune(S, det, bins, None, cnt, bunches=[1], reps=1, cache_path=path)  # another signature
    assert not c["cached"]
    assert len(path.read_text().splitlines()) == 2
    cphot.autotune_cache_clear()  # as a new process would: the file answers
    d = cphot.autotune(S, det, bins, None, cnt, bunches=[1, 2], reps=1, cache_path=path)
    assert d == {**a, "cached": True}
    assert cphot.autotune(S, det, bins, None, cnt, bunches=[1, 2], reps=1, cache=True)["cached"]
    cphot.autotune_cache_clear()
    assert not cphot.autotune(S, det, bins, None, cnt, bunches=[1, 2], reps=1, cache=True)["cached"]


def test_autotune_fitted_window_on_an_inclined_shower():
    """A grid too large for LDS: the autotuner's pilot launch finds the footprint of a
    60-degree shower (elongated along its azimuth) and its windows are fitted to it;
    whatever shape wins, its bins equal those of global atomics alone, and a window
    fitted to the footprint holds more of the photons than the centred square of the
    same area."""
    sh = W.make_shower(20_000, seed=77, xmax=600.0, zenith_deg=60.0, azimuth_deg=15.0, beta="R", dedx=(0.1, 2.0))
    atm = cphot.Atmosphere(**cases.ATMO_LAYERED)
    run = {**cases.RUN_INCLINED, "seed": 21}
    geom = np.array([[*sh.core, *sh.axis]])
    seg, g, off = cphot.upload(sh.seg, geom)
    S = cphot.make_segments(seg, g, off)
    nb = run["nx"] * run["ny"]
    bins = torch.zeros(nb, dtype=torch.float64, device="cuda")
    cnt = torch.zeros(cphot.NCOUNTERS, dtype=torch.int64, device="cuda")
    cphot.propagate(S, cphot.make_detector(atm, **run, lds_hist=0), bins, None, cnt)
    torch.cuda.synchronize()
    ref = bins.cpu().numpy().reshape(run["ny"], run["nx"])
    best = cphot.autotune(S, cphot.make_detector(atm, **run), bins, None, cnt, reps=1)
    bins.zero_()
    cphot.propagate(S, cphot.make_detector(atm, **run, **cphot.shape_of(best)), bins, None, cnt)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(bins.cpu().numpy().reshape(run["ny"], run["nx"]), ref)
    # the footprint: a 2:1 rectangle along x beats the centred square of the same area
    def held(w, h, dx, dy):
        x0 = min(max((run["nx"] - w) // 2 + dx, 0), run["nx"] - w)
        y0 = min(max((run["ny"] - h) // 2 + dy, 0), run["ny"] - h)
        return ref[y0:y0 + h, x0:x0 + w].sum()
    best_rect = max(held(90, 45, dx, dy) for dx in range(-20, 21, 2) for dy in range(-10, 11, 2))
    assert best_rect > 1.05 * held(64, 64, 0, 0), (best_rect, held(64, 64, 0, 0), ref.sum())
