"""Helpers that run the HIP library and the oracle on the same seeded inputs and
compare them. Imported by the GPU tests only."""
import math

import numpy as np

from oracle import oracle as O
from paper_2405_04229_amd import cphot

# Per-photon tolerances (floating point, FP32 kernel vs FP64 oracle):
#  positions |d| <= 1e-4 max(r, 10 m) + DIR_TOL H / u_z^2, with r the distance
#  from the core; the second term is the displacement of the landing point that
#  a direction error of DIR_TOL rad causes over a descent of H metres at
#  vertical direction cosine u_z (the problem's own conditioning: the kernel's
#  FP32 emission direction is asserted to lie within DIR_TOL of the oracle's),
#  times |d| <= 1e-4 |t| + 0.01 ns, optical depth |d| <= 1e-4 tau + 1e-6.
POS_REL, POS_FLOOR = 1e-4, 10.0
DIR_TOL = 4e-7
T_REL, T_ABS = 1e-4, 0.01
TAU_REL, TAU_ABS = 1e-4, 1e-6
# A decision taken by floating point may legitimately differ when the oracle's
# quantity lies this close to the decision boundary (FP32 rounding of the
# kernel's inputs to it): survival |u - exp(-tau)|, bin edges (m), time-bin
# edges (ns), layer boundaries (m), wavelength-bin edges (fraction of a bin).
FLIP_SURV, FLIP_EDGE_REL, FLIP_T, FLIP_LAYER, FLIP_LAMBIN = 2e-5, 1e-4, 0.02, 5e-3, 1e-4
# Every flip must lie inside one of those bands; their number is further
# bounded by this fraction of the photons (a few per 1e4 on grids of 4 m cells).
MAX_FLIP_FRACTION = 3e-4


def device_run(atm_kw, run_kw, seg_np, geom, offsets=None, first_id=0, counters=True, id_stride=1):
    import torch
    atm = cphot.Atmosphere(**atm_kw)
    det = cphot.make_detector(atm, **run_kw)
    seg, g, off = cphot.upload(seg_np, geom, offsets)
    S = cphot.make_segments(seg, g, off, first_id=first_id, id_stride=id_stride)
    ns = g.shape[0]
    if run_kw.get("detector", "grid") == "grid":
        per = run_kw.get("nx", 100) * run_kw.get("ny", 100)
    else:
        per = run_kw.get("snx", 10) * run_kw.get("sny", 10)
    bins = torch.zeros(ns * per, dtype=torch.int64, device="cuda")
    n_t = run_kw.get("n_t", 0)
    th = torch.zeros(ns * per * (n_t + 1), dtype=torch.int32, device="cuda") if (
        run_kw.get("detector") == "spheres" and n_t > 0) else None
    cnt = torch.zeros(cphot.NCOUNTERS, dtype=torch.int64, device="cuda")
    cphot.propagate(S, det, bins, th, cnt)
    torch.cuda.synchronize()
    out = (bins.cpu().numpy().reshape(ns, per), None if th is None else th.cpu().numpy().reshape(ns, per, n_t + 1),
           cnt.cpu().numpy())
    del atm
    return out


def device_counts(atm_kw, run_kw, seg_np, geom, first_id=0, with_mu=False, id_stride=1):
    import torch
    atm = cphot.Atmosphere(**atm_kw)
    det = cphot.make_detector(atm, **run_kw)
    seg, g, off = cphot.upload(seg_np, geom)
    S = cphot.make_segments(seg, g, off, first_id=first_id, id_stride=id_stride)
    counts = torch.zeros(S.n, dtype=torch.int32, device="cuda")
    mu = torch.zeros(S.n, dtype=torch.float64, device="cuda") if with_mu else None
    cphot.segment_counts(S, det, counts, mu)
    torch.cuda.synchronize()
    if with_mu:
        return counts.cpu().numpy(), mu.cpu().numpy()
    return counts.cpu().numpy()


def device_records(atm_kw, run_kw, seg_np, geom, first_id=0, id_stride=1):
    import torch
    atm = cphot.Atmosphere(**atm_kw)
    det = cphot.make_detector(atm, **run_kw)
    seg, g, off = cphot.upload(seg_np, geom)
    S = cphot.make_segments(seg, g, off, first_id=first_id, id_stride=id_stride)
    counts = torch.zeros(S.n, dtype=torch.int32, device="cuda")
    cphot.segment_counts(S, det, counts)
    offs = torch.cumsum(counts.to(torch.int64), 0) - counts.to(torch.int64)
    total = int(counts.sum().item())
    rec = torch.zeros(max(total, 1) * cphot.RECORD_BYTES, dtype=torch.uint8, device="cuda")
    cphot.trace_records(S, det, offs.contiguous(), rec)
    torch.cuda.synchronize()
    return cphot.records_to_numpy(rec.cpu())[:total]


def oracle_atm(atm_kw):
    return O.Atmosphere(**atm_kw)


def near_boundary(orc, core, atm_kw, run_kw, surv_thr=None):
    """Records of the oracle whose decisions (survival, bin, time bin, start
    layer, wavelength bin) lie within rounding distance of their boundary, and
    the per-record position tolerance. `surv_thr`: the survival thresholds where
    they are not exp(-tau) (detector efficiency, pre-emission reduction); under the
    dispersive spectrum the emission decision u < p_emit is one more boundary.
    Returns (near, pos_tol, h_emit, layer_m, lambin_m)."""
    p_emit = orc["p_emit"]  # 1 except under the dispersive spectrum
    thr = np.exp(-orc["tau"]) * p_emit if surv_thr is None else surv_thr
    surv_m = np.minimum(np.abs(orc["u_abs"] - thr), np.abs(orc["u_abs"] - p_emit))
    transport = run_kw.get("transport", "straight")
    if transport == "curved_walk":  # the same shells, walked shell by shell
        transport = "curved"
    h_emit = orc["ez"]
    if transport == "curved":
        re = atm_kw.get("earth_radius", 6.371e6)
        h_emit = np.sqrt(orc["ex"] ** 2 + orc["ey"] ** 2 + (orc["ez"] + re) ** 2) - re
    r = np.hypot(orc["x"] - core[0], orc["y"] - core[1])
    descent = np.maximum(h_emit - run_kw.get("h_obs", 2200.0), 0.0)
    pos_tol = POS_REL * np.maximum(r, POS_FLOOR) + DIR_TOL * descent / np.maximum(orc["dz"] ** 2, 1e-12)
    near = (surv_m < FLIP_SURV) | (orc["margin"] < pos_tol + FLIP_EDGE_REL * 10) | (orc["tmargin"] < FLIP_T)
    lm = lbm = None
    if transport in ("layered", "curved"):
        dh = atm_kw["h_top"] / atm_kw["n_layers"]
        lm = np.abs(h_emit / dh - np.round(h_emit / dh)) * dh
        lam0, lam1 = atm_kw.get("lam_min", 300.0), atm_kw.get("lam_max", 600.0)
        lb = (orc["lambda"] - lam0) / (lam1 - lam0) * atm_kw["n_lam"]
        lbm = np.abs(lb - np.round(lb))
        near |= (lm < FLIP_LAYER) | (lbm < FLIP_LAMBIN)
    return near, pos_tol, h_emit, lm, lbm


def flip_budget(orc, core, atm_kw, run_kw):
    """Most bin-count differences the same photons may legitimately show: each
    record near a decision boundary can move one bunch between two bins."""
    near, *_ = near_boundary(orc, core, atm_kw, run_kw)
    return 2 * run_kw.get("bunch", 1) * int(near.sum())


def compare_records(gpu, orc, core, atm_kw, run_kw, surv_thr=None):
    """Element-by-element comparison. Returns (n_flips, report). Raises on any
    mismatch that is not a legitimate flip."""
    assert len(gpu) == len(orc), (len(gpu), len(orc))
    assert np.array_equal(gpu["seg"].astype(np.int64), orc["seg"])
    assert np.array_equal(gpu["k"].astype(np.int64), orc["k"])
    # the same uniforms on both sides: the survival uniform is exact in FP32
    np.testing.assert_array_equal(gpu["u_abs"].astype(np.float64), orc["u_abs"])
    np.testing.assert_allclose(gpu["lambda"], orc["lambda"], rtol=2e-6)
    # directions of records never emitted (dispersive spectrum, state 4 in the
    # oracle) are not compared: next to the threshold the cone's opening is
    # ill-conditioned and such a record carries no photon
    du = np.stack([gpu["dx"], gpu["dy"], gpu["dz"]], 1) - np.stack([orc["dx"], orc["dy"], orc["dz"]], 1)
    du = du[orc["state"] != 4]
    assert du.size == 0 or np.abs(du).max() <= DIR_TOL, np.abs(du).max()
    transport = run_kw.get("transport", "straight")
    if transport == "curved_walk":
        transport = "curved"
    layered = transport in ("layered", "curved")
    near, pos_tol, h_emit, lm, lbm = near_boundary(orc, core, atm_kw, run_kw, surv_thr)
    r = np.hypot(orc["x"] - core[0], orc["y"] - core[1])
    state_diff = gpu["state"] != orc["state"]
    bin_diff = (gpu["bin"] != orc["bin"]) | (gpu["tbin"] != orc["tbin"])
    bad = (state_diff | bin_diff) & ~near
    assert not bad.any(), f"{bad.sum()} records differ away from any decision boundary: " \
                          f"{gpu[bad][:3]} vs {orc[bad][:3]}"
    flips = (state_diff | bin_diff) & near
    # continuous quantities where both sides reached the observation level
    live = (orc["state"] != 1) & (orc["state"] != 4) & ~((orc["state"] == 3) & (h_emit < run_kw.get("h_obs", 2200.0)))
    if transport == "curved":
        live &= orc["margin"] < 1e29      # left the top of the atmosphere: no arrival point
    live &= ~(near & (lm < FLIP_LAYER) if layered else np.zeros(len(orc), bool))
    # a legitimate hit/miss flip moves the arrival point (sphere entry vs plane crossing)
    live &= ~bin_diff
    live &= gpu["state"] != 4  # an emission flip: one side stopped at the emission point
    dpos = np.hypot(gpu["x"] - orc["x"], gpu["y"] - orc["y"])
    assert np.all(dpos[live] <= pos_tol[live]), f"max position error {np.max(dpos[live] / pos_tol[live])} of tolerance"
    dt = np.abs(gpu["t"] - orc["t"])
    assert np.all(dt[live] <= T_REL * np.abs(orc["t"][live]) + T_ABS), f"max time error {dt[live].max()}"
    dtau = np.abs(gpu["tau"] - orc["tau"])
    lam_edge = np.zeros(len(orc), bool)
    if layered:
        lam_edge = lbm < FLIP_LAMBIN
    ok_tau = live & ~lam_edge
    assert np.all(dtau[ok_tau] <= TAU_REL * orc["tau"][ok_tau] + TAU_ABS), f"max tau error {dtau[ok_tau].max()}"
    def mx(a):
        return float(a.max()) if a.size else 0.0
    report = dict(n=len(orc), flips=int(flips.sum()), compared=int(live.sum()),
                  max_pos_frac=mx(dpos[live] / pos_tol[live]),
                  max_pos_m=mx(dpos[live]), max_pos_rel=mx(dpos[live] / np.maximum(r[live], POS_FLOOR)),
                  max_t_ns=mx(dt[live]), max_t_rel=mx(dt[live] / np.maximum(np.abs(orc["t"][live]), 1e-9)),
                  max_tau=mx(dtau[ok_tau]), max_tau_rel=mx(dtau[ok_tau] / np.maximum(orc["tau"][ok_tau], 1e-12)),
                  max_dir=float(np.abs(du).max()) if du.size else 0.0)
    print("parity errors:", report)
    return int(flips.sum()), report


def chi2_two_sample(a, b, min_count=20):
    """Two-sample chi^2 over bins where both samples are well populated.
    Returns (chi2, dof, p)."""
    from scipy import stats
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    m = (a + b) >= min_count
    A, B = a[m], b[m]
    ka = math.sqrt(B.sum() / A.sum())
    kb = math.sqrt(A.sum() / B.sum())
    chi2 = float(np.sum((ka * A - kb * B) ** 2 / (A + B)))
    dof = int(m.sum()) - 1
    return chi2, dof, float(stats.chi2.sf(chi2, dof))
