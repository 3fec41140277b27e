"""Host-memory chunk streamer (cphot_streamer_*) against one resident launch:
the same global segment ids give the same photons, so bins and counters must be
identical whatever the chunk size."""
import numpy as np
import pytest

from paper_2405_04229_amd import workload as W
from tests import cases

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2405_04229_amd import cphot  # noqa: E402


def _resident(atm, run, sh, dtype, first_id):
    g = np.array([[*sh.core, *sh.axis]])
    seg, gg, off = cphot.upload(sh.seg, g)
    S = cphot.make_segments(seg, gg, off, first_id=first_id)
    det = cphot.make_detector(atm, **run)
    bins = torch.zeros(run["nx"] * run["ny"], dtype=dtype, device="cuda")
    cnt = torch.zeros(cphot.NCOUNTERS, dtype=torch.int64, device="cuda")
    cphot.propagate(S, det, bins, None, cnt)
    torch.cuda.synchronize()
    return bins.cpu().numpy(), cnt.cpu().numpy(), gg


def _streamed(atm, run, sh, dtype, chunk, first_id, gg, repeat=1):
    st = cphot.Streamer(chunk)
    det = cphot.make_detector(atm, **run)
    bins = torch.zeros(run["nx"] * run["ny"], dtype=dtype, device="cuda")
    cnt = torch.zeros(cphot.NCOUNTERS, dtype=torch.int64, device="cuda")
    for _ in range(repeat):
        st.run(sh.seg, gg, det, bins, None, cnt, first_id=first_id)
    torch.cuda.synchronize()
    st.close()
    return bins.cpu().numpy(), cnt.cpu().numpy()


@pytest.mark.parametrize("chunk", [7_000, 25_000, 100_000])
def test_streamed_curved_fluorescence_equals_resident(chunk):
    sh = W.make_shower(25_000, seed=501, xmax=600.0, zenith_deg=60.0, beta="R", dedx=(0.1, 2.0))
    run = {**cases.RUN_INCLINED, "nx": 300, "ny": 300, "cell": 30.0, "seed": 31}
    atm = cphot.Atmosphere(**cases.ATMO_LAYERED)
    rb, rc, gg = _resident(atm, run, sh, torch.float64, 12_345)
    sb, sc = _streamed(atm, run, sh, torch.float64, chunk, 12_345, gg)
    np.testing.assert_array_equal(sb, rb)
    np.testing.assert_array_equal(sc, rc)
    assert rc[10] > 0 and rb.sum() > 1e5


@pytest.mark.parametrize("chunk", [9_000, 400_000])
def test_streamed_from_pinned_and_threaded_staging_equal_resident(chunk):
    """Pinned host columns (copied to the device without staging) and pageable ones
    large enough to be staged by several host threads give the resident launch's
    bins and counters; pinned columns may be reused once run returns."""
    sh = W.make_shower(400_000, seed=504, xmax=600.0, zenith_deg=60.0, beta="R", dedx=(0.1, 2.0))
    run = {**cases.RUN_INCLINED, "nx": 300, "ny": 300, "cell": 30.0, "seed": 33}
    atm = cphot.Atmosphere(**cases.ATMO_LAYERED)
    rb, rc, gg = _resident(atm, run, sh, torch.float64, 777)
    sb, sc = _streamed(atm, run, sh, torch.float64, chunk, 777, gg)
    np.testing.assert_array_equal(sb, rb)
    np.testing.assert_array_equal(sc, rc)
    pinned = {k: torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32)).pin_memory() for k, v in sh.seg.items()}
    assert all(t.is_pinned() for t in pinned.values())
    st = cphot.Streamer(chunk)
    det = cphot.make_detector(atm, **run)
    bins = torch.zeros(run["nx"] * run["ny"], dtype=torch.float64, device="cuda")
    cnt = torch.zeros(cphot.NCOUNTERS, dtype=torch.int64, device="cuda")
    st.run(pinned, gg, det, bins, None, cnt, first_id=777)
    for t in pinned.values():
        t.fill_(float("nan"))  # the copies have completed: overwriting cannot reach the device
    torch.cuda.synchronize()
    st.close()
    np.testing.assert_array_equal(bins.cpu().numpy(), rb)
    np.testing.assert_array_equal(cnt.cpu().numpy(), rc)


def test_streamed_straight_tiny_chunks_and_repeat():
    sh = W.make_shower(3_001, seed=502, beta="R")
    run = {**cases.RUN_TINY, "seed": 32}
    atm = cphot.Atmosphere(**cases.ATMO_STRAIGHT)
    rb, rc, gg = _resident(atm, run, sh, torch.int32, 0)
    sb, sc = _streamed(atm, run, sh, torch.int32, 1_000, 0, gg, repeat=2)  # runs accumulate
    np.testing.assert_array_equal(sb, 2 * rb)
    np.testing.assert_array_equal(sc, 2 * rc)


def test_streamer_empty_and_errors():
    atm = cphot.Atmosphere(**cases.ATMO_STRAIGHT)
    with pytest.raises(cphot.CphotError):
        cphot.Streamer(0)
    sh = W.make_shower(10, seed=503, beta="R")
    empty = {k: v[:0] for k, v in sh.seg.items()}
    g = torch.tensor([[*sh.core, *sh.axis]], dtype=torch.float64, device="cuda")
    st = cphot.Streamer(4)
    det = cphot.make_detector(atm, **{**cases.RUN_TINY, "seed": 1})
    bins = torch.zeros(100 * 100, dtype=torch.int32, device="cuda")
    st.run(empty, g, det, bins)
    torch.cuda.synchronize()
    assert int(bins.sum()) == 0
    small = torch.zeros(10, dtype=torch.int32, device="cuda")
    with pytest.raises(cphot.CphotError, match="bins_capacity"):
        st.run(sh.seg, g, det, small)
    st.close()
