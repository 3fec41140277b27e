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
    tuned = cphot.make_detector(atm, **run, block_size=best["block_size"], grid_blocks=best["grid_blocks"],
                                lds_hist=best["lds_hist"])
    bins.zero_()
    cphot.propagate(S, tuned, bins, None, cnt)
    torch.cuda.synchronize()
    assert torch.equal(bins, ref)
