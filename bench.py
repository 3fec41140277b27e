"""Benchmark: photons propagated per second on one MI355X.

Headline step = one pass of the whole photon path over one batch: cphot_propagate
over the resident chunk of the large inclined shower (1e7 track segments of a
60-degree shower, curved Earth, Cherenkov emission plus isotropic fluorescence in
three bands, FP64 bins on a 1000 x 1000 ground grid of 10 m), exact transport
(closed-form shell sums, the shell walk where they do not hold), bins and
counters zeroed first. Inputs are resident in HBM before timing starts.

The same JSON line carries:
- roofline: the headline kernel against the VALU issue peak, with the algorithmic
  work of the iterative shell method and, from the kept profile, the instructions
  the kernel actually issues;
- cpu_baseline: the FP64 CPU oracle on the deterministic subset of the same chunk
  (global segment ids = 0 mod 1000), one thread and all host cores, beside the
  GPU's run of that subset and its error per output against the oracle;
- inclined: beside the headline, the plain shell walk (the iterative tracer), the
  transport network trained on the GPU (same photons, bins compared cell by
  cell), the interpolated correction table, and the whole 1e8-segment shower
  streamed from host memory;
- telescope: the refracting telescope workload (1e6 segments, bunches of 5, 100
  bounding spheres with 1 ns time histograms) with its own roofline, the
  data-reduction cuts, detector efficiency with pre-emission reduction, Poisson
  counts, the dispersive spectrum, the planar network and table;
- batched: 256 showers of uneven size in one captured launch per step, launch
  shape picked by the autotuner among the bunch sizes whose bins stay within 1 %
  of bunch 1.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X public figures: 256 CUs at 2.4 GHz and 157.3 TFLOP/s FP32 vector, an FMA
# counted as two flops: 128 FP32 lane-operations per CU per clock (the published
# peak; it needs two wave64 VALU instructions per CU per clock). One wave64 VALU
# instruction per CU per clock is 64 lane-operations: reported beside it.
PEAK_VALU_LANE_OPS = 256 * 128 * 2.4e9
PEAK_WAVE64_ISSUE = 256 * 64 * 2.4e9
PEAK_HBM = 8.0e12

# Algorithmic VALU lane-slots per unit of work, counted from the method's steps
# (32-bit multiplies and transcendentals weighted 4 as quarter-rate operations):
# a segment's FP64 yield, Philox word and rotation bisector; a record's Philox
# block, uniforms, cone, rotation, final leg, detector test and exp(-tau); one
# layer or shell crossing of the iterative refraction (Sec. 3.4.2: chord, Snell
# update, optical depth, delay terms); the FP64 arrival point on the observation
# sphere of the curved geometry (about 20 FP64 operations, weight 2).
SLOTS_PER_SEGMENT = 350.0
SLOTS_PER_RECORD_BASE = 320.0
SLOTS_PER_CROSSING = 24.0
SLOTS_FP64_ARRIVAL = 40.0
SEGMENT_BYTES = 32.0
SEGMENT_BYTES_DEDX = 36.0

METRIC = "photons propagated/s, exact vs MLP surrogate, at <=1% per-bin density error"

# Measured facts of a kernel at one launch shape, from rocprofv3 (VALU instructions
# issued per launch; HBM bytes per launch = FETCH_SIZE and WRITE_SIZE scaled by a
# plain copy's factors), valid only for the sources and shape they were taken on
# (sha256 prefixes of the kernel sources), else reported as null.
KERNEL_SOURCES = ("cphot_kernels.hip", "cphot_device.h", "cphot_internal.h", "cphot_mlp.h")
MEASURED = {
    # profiles/k_propagate_curved_inclined_1e7.md: mean of the six launches of the timed step
    "inclined_curved": {"sha": "66494fdc41f0885c", "shape": [256, 2048, 1, 90, 45, 1, 1],
                        "valu_insts": 8.553303493e9, "hbm_bytes": (176773.29 * 2.0 + 576439.55 * 1.0) * 1024,
                        "profile": "profiles/k_propagate_curved_inclined_1e7.md"},
    # profiles/k_propagate_telescope_1e6.md: mean of the six launches of the timed step
    "telescope_layered": {"sha": "66494fdc41f0885c", "shape": [256, 1024, 1, 0, 0, 0, 0],
                          "valu_insts": 7.3883896e7, "hbm_bytes": (16270.24 * 2.0 + 288.0 * 1.0) * 1024,
                          "profile": "profiles/k_propagate_telescope_1e6.md"},
}


def sources_sha():
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2405_04229_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_if_current(key, tune):
    m = MEASURED.get(key)
    if not m or m["sha"] != sources_sha():
        return None
    # the kernel variant (block size) and the histogram mode fix the instructions issued per launch;
    # the grid size and the window change them by under 1 % (the autotuner trials of one variant)
    if (int(tune["block_size"]), int(tune["lds_hist"])) != (m["shape"][0], m["shape"][2]):
        return None
    return m


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_steps(torch, step, steps, warmup, stream):
    """Wall time per step over `steps` after `warmup`, and the mean launch time
    from HIP events recorded on the launch stream around each launch."""
    for _ in range(warmup):
        step(None)
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        step(events[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0) * 1e3 / steps, float(np.mean([a.elapsed_time(b) for a, b in events]))


def density_error(s, e, min_count=1000):
    """Worst relative error over bins with >= min_count exact photons (and, as the
    statistical resolution of a 1000-photon bin is itself ~3 %, over bins with
    >= 10 x min_count), and the global L1 error sum|s - e| / sum e."""
    s = np.asarray(s, dtype=np.float64).ravel()
    e = np.asarray(e, dtype=np.float64).ravel()
    out = {"l1": float(np.abs(s - e).sum() / max(e.sum(), 1.0))}
    for key, mc in (("", min_count), ("_10x", 10 * min_count)):
        m = e >= mc
        out["worst_bin" + key] = float(np.max(np.abs(s[m] - e[m]) / e[m])) if m.any() else None
        out["bins_compared" + key] = int(m.sum())
    out["min_count"] = min_count
    out["within_1pct"] = bool(out["l1"] <= 0.01 and (out["worst_bin"] is None or out["worst_bin"] <= 0.01))
    return out


def radial_height(x, y, z, R=6.371e6):
    x, y, z = (np.asarray(a, dtype=np.float64) for a in (x, y, z))
    return (x * x + y * y + z * (2 * R + z)) / (np.sqrt(x * x + y * y + (z + R) ** 2) + R)


def traced_records(torch, cphot, seg_np, geom, det, first_id=0, id_stride=1):
    sg, sgg, _ = cphot.upload(seg_np, geom)
    SS = cphot.make_segments(sg, sgg, None, first_id=first_id, id_stride=id_stride)
    counts = torch.zeros(SS.n, dtype=torch.int32, device="cuda")
    cphot.segment_counts(SS, det, counts)
    offs = torch.cumsum(counts.to(torch.int64), 0) - counts.to(torch.int64)
    tot = int(counts.sum().item())
    rec = torch.zeros(max(tot, 1) * cphot.RECORD_BYTES, dtype=torch.uint8, device="cuda")
    cphot.trace_records(SS, det, offs.contiguous(), rec)
    torch.cuda.synchronize()
    return cphot.records_to_numpy(rec.cpu())[:tot]


def crossing_profile(torch, cphot, seg_np, geom, det, h_obs, dh, n_layers, curved, n=20000):
    """Mean number of layer (planar) or shell (curved) boundaries a record's ray
    crosses on its way down to the observation level, over the records of the
    first n segments (upward records and those emitted below h_obs cross none):
    the iterative method's work per record."""
    sample = {k: v[:n] for k, v in seg_np.items()}
    r = traced_records(torch, cphot, sample, geom, det)
    s = r["seg"].astype(np.int64)
    xm = 0.5 * (sample["x0"].astype(np.float64) + sample["x1"])
    ym = 0.5 * (sample["y0"].astype(np.float64) + sample["y1"])
    zm = 0.5 * (sample["z0"].astype(np.float64) + sample["z1"])
    h = radial_height(xm, ym, zm) if curved else zm
    start = np.minimum((h[s] // dh).astype(np.int64), n_layers - 1)
    obs = int(h_obs // dh)
    down = r["state"] != 1
    cross = np.where(down, np.maximum(start - obs, 0), 0)
    return float(cross.mean()) if len(cross) else 0.0, len(r)


def tuned_detector(cphot, S, atm, run, bins, th, cnt, stream, reps=3, **extra):
    """Detector with the autotuner's launch shape for this workload; the bunch
    stays the workload's own (it defines the workload, not the launch)."""
    det0 = cphot.make_detector(atm, **run, **extra)
    t0 = time.perf_counter()
    tune = cphot.autotune(S, det0, bins, th, cnt, bunches=[run["bunch"]], reps=reps, stream=stream)
    tune["tune_s"] = time.perf_counter() - t0
    shape = cphot.shape_of(tune)
    return cphot.make_detector(atm, **run, **shape, **extra), tune


def roofline_entry(kernel, kern_ms, n_seg, seg_bytes, records, crossings, fp64_arrival, tune, key):
    """Achieved algorithmic lane-operations per second of one launch against the
    VALU peak; with a current profile, the issued VALU lane-instructions too."""
    per_record = SLOTS_PER_RECORD_BASE + SLOTS_PER_CROSSING * crossings + (SLOTS_FP64_ARRIVAL if fp64_arrival else 0.0)
    slots = n_seg * SLOTS_PER_SEGMENT + records * per_record
    achieved = slots / (kern_ms * 1e-3)
    m = measured_if_current(key, tune)
    out = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_VALU_LANE_OPS / 1e12, "unit": "Tlane-ops/s",
           "frac": achieved / PEAK_VALU_LANE_OPS, "frac_vs_wave64_issue": achieved / PEAK_WAVE64_ISSUE,
           "traffic": m["hbm_bytes"] if m else None,
           "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's)",
           "kernel": kernel, "kernel_ms": kern_ms, "tuning": tune,
           "algorithmic_slots_per_launch": slots, "slots_per_record": per_record,
           "crossings_per_record": crossings,
           "algorithmic_hbm_bytes": n_seg * seg_bytes,
           "hbm_gbps_algorithmic": n_seg * seg_bytes / (kern_ms * 1e-3) / 1e9,
           "model": "segment 350 slots; record 320 + 24 per layer/shell crossing of the iterative method"
                    + (" + 40 for the FP64 arrival" if fp64_arrival else "")}
    if m:
        issued = m["valu_insts"] * 64.0
        out["isa"] = {"valu_lane_instructions_per_launch": issued,
                      "valu_lane_instructions_per_record": issued / max(records, 1.0),
                      "achieved": issued / (kern_ms * 1e-3) / 1e12,
                      "frac": issued / (kern_ms * 1e-3) / PEAK_VALU_LANE_OPS,
                      "frac_vs_wave64_issue": issued / (kern_ms * 1e-3) / PEAK_WAVE64_ISSUE,
                      "profile": m["profile"]}
    return out


# ------------------------------------------------------------------------------ inclined shower

def run_path(torch, cphot, S, det, nbins, stream, steps, warmup, dtype):
    bins = torch.zeros(nbins, dtype=dtype, device="cuda")
    cnt = torch.zeros(cphot.NCOUNTERS, dtype=torch.int64, device="cuda")

    def step(ev):
        bins.zero_()
        cnt.zero_()
        if ev is not None:
            ev[0].record(stream)
        cphot.propagate(S, det, bins, None, cnt, stream=stream)
        if ev is not None:
            ev[1].record(stream)

    ms, kern = time_steps(torch, step, steps, warmup, stream)
    return ms, kern, bins.cpu().numpy(), cnt.cpu().numpy()


def bench_inclined(torch, cphot, W, args, stream):
    """The resident chunk through the curved shells: the exact step (headline),
    its roofline, then the plain walk, the network, the table and the streamed shower."""
    t0 = time.perf_counter()
    sh = W.workload_inclined_chunk(0, beta=args.beta)
    log(f"inclined chunk generated in {time.perf_counter() - t0:.1f} s")
    geom = np.array([[*sh.core, *sh.axis]])
    seg, g, off = cphot.upload(sh.seg, geom)
    S = cphot.make_segments(seg, g, off, first_id=sh.first_id)
    atm = cphot.Atmosphere(**W.ATMO_LAYERED)
    run = {**W.RUN_INCLINED, "seed": 5}
    nb = run["nx"] * run["ny"]
    bins = torch.zeros(nb, dtype=torch.float64, device="cuda")
    cnt = torch.zeros(cphot.NCOUNTERS, dtype=torch.int64, device="cuda")
    det, tune = tuned_detector(cphot, S, atm, run, bins, None, cnt, stream, reps=2)
    log(f"inclined autotune: {tune}")
    steps = max(5, args.steps // 2)
    ms, kern, exact_bins, c = run_path(torch, cphot, S, det, nb, stream, steps, args.warmup, torch.float64)
    records = float(c[3])
    photons = records * run["bunch"]
    log(f"inclined exact: {ms:.3f} ms/step, kernel {kern:.3f} ms, {records:.4g} records")
    dh = W.ATMO_LAYERED["h_top"] / W.ATMO_LAYERED["n_layers"]
    cross, _ = crossing_profile(torch, cphot, sh.seg, geom, det, run["h_obs"], dh, W.ATMO_LAYERED["n_layers"], True)
    roof = roofline_entry(f"k_propagate<{tune['block_size']},CURVED,GRID,PROPAGATE>", kern, float(sh.n),
                          SEGMENT_BYTES_DEDX, records, cross, True, tune, "inclined_curved")
    head = {"value": photons / (ms * 1e-3), "ms_per_step": ms, "kernel_ms": kern, "records": records,
            "photons": photons, "segments": sh.n, "fluorescence_records": float(c[10]),
            "records_walked": float(c[9]), "photons_binned": float(c[8]), "tuning": tune}
    extra = {}
    paths = [x for x in args.inclined_paths.split(",") if x]
    # the same step with filter level 3 for the grid (an exact bound: identical bins)
    det_c = cphot.make_detector(atm, **run, cuts=("photon",), **cphot.shape_of(tune))
    ms_c, kern_c, b_c, c_c = run_path(torch, cphot, S, det_c, nb, stream, steps, 1, torch.float64)
    extra["exact_photon_cut"] = {
        "value": photons / (ms_c * 1e-3), "unit": "photons/s (uncut records)", "ms_per_step": ms_c,
        "kernel_ms": kern_c, "speedup_vs_exact": ms / ms_c, "bins_identical": bool(np.array_equal(b_c, exact_bins)),
        "records_culled": float(c_c[12]), "records_walked": float(c_c[9]),
        "note": "filter level 3 on the ground grid (Sec. 4.3.4): records whose straight line lands beyond the "
                "Bouguer bound of the grid are outside before transport; same launch shape"}
    log(f"inclined exact with photon cut: {ms_c:.3f} ms/step, identical bins "
        f"{extra['exact_photon_cut']['bins_identical']}")
    ms_w = ms_wc = None
    if "walk" in paths:
        # the plain exact tracer: every ray walked shell by shell (Sec. 3.4.2 over shells)
        det_w, tune_w = tuned_detector(cphot, S, atm, {**run, "transport": "curved_walk"}, bins, None, cnt, stream,
                                       reps=1)
        ms_w, kern_w, b_w, c_w = run_path(torch, cphot, S, det_w, nb, stream, max(3, steps // 2), 1, torch.float64)
        extra["walk"] = {"value": float(c_w[3]) * run["bunch"] / (ms_w * 1e-3), "unit": "photons/s",
                         "ms_per_step": ms_w, "kernel_ms": kern_w, "tuning": tune_w,
                         "bins_identical_to_headline": bool(np.array_equal(b_w, exact_bins)),
                         "bins_diff_l1": float(np.abs(b_w - exact_bins).sum()),
                         "note": "the iterative tracer: every ray walked shell by shell"}
        det_wc = cphot.make_detector(atm, **{**run, "transport": "curved_walk"}, cuts=("photon",),
                                     **cphot.shape_of(tune_w))
        ms_wc, kern_wc, b_wc, c_wc = run_path(torch, cphot, S, det_wc, nb, stream, max(3, steps // 2), 1,
                                              torch.float64)
        extra["walk"]["with_photon_cut"] = {"ms_per_step": ms_wc, "kernel_ms": kern_wc,
                                            "bins_identical_to_walk": bool(np.array_equal(b_wc, b_w))}
        log(f"inclined walk: {ms_w:.3f} ms/step, with the photon cut {ms_wc:.3f}")
    if not args.no_surrogate and "surrogate" in paths:
        sur = cphot.Surrogate(W.SURROGATE_CURVED_LO, W.SURROGATE_CURVED_HI, max_batch=4096, init_seed=2,
                              geometry="curved")
        t0 = time.perf_counter()
        X, Y = sur.make_training_set(atm, args.train_samples, seed=1005)
        sur.fit_normalization(Y)
        loss = sur.train(X, Y, batch=4096, steps=4 * args.train_steps, lr=3e-3)
        torch.cuda.synchronize()
        train_s = time.perf_counter() - t0
        del X, Y
        det_s, tune_s = tuned_detector(cphot, S, atm, {**run, "transport": "surrogate"}, bins, None, cnt, stream,
                                       reps=1, surrogate=sur)
        ms_s, kern_s, b_s, c_s = run_path(torch, cphot, S, det_s, nb, stream, max(3, steps // 2), 1, torch.float64)
        shape_s = cphot.shape_of(tune_s)
        det_sc = cphot.make_detector(atm, **{**run, "transport": "surrogate"}, surrogate=sur, cuts=("photon",),
                                     **shape_s)
        ms_sc, kern_sc, b_sc, c_sc = run_path(torch, cphot, S, det_sc, nb, stream, max(3, steps // 2), 1,
                                              torch.float64)
        extra["surrogate"] = {
            "value": float(c_s[3]) * run["bunch"] / (ms_s * 1e-3), "unit": "photons/s", "ms_per_step": ms_s,
            "kernel_ms": kern_s, "speedup_vs_exact": ms / ms_s,
            "speedup_vs_walk": ms_w / ms_s if ms_w else None,
            "density_error_vs_exact": density_error(b_s, exact_bins),
            "fallback_fraction": float(c_s[9]) / max(float(c_s[3]), 1.0), "tuning": tune_s,
            "with_photon_cut": {
                "value": float(c_sc[3]) * run["bunch"] / (ms_sc * 1e-3), "unit": "photons/s", "ms_per_step": ms_sc,
                "kernel_ms": kern_sc, "speedup_vs_exact_with_cut": ms_c / ms_sc,
                "speedup_vs_walk_with_cut": ms_wc / ms_sc if ms_wc else None,
                "density_error_vs_exact": density_error(b_sc, exact_bins),
                "fallback_fraction": float(c_sc[9]) / max(float(c_sc[3]), 1.0),
                "records_culled": float(c_sc[12])},
            "training": {"samples": args.train_samples, "steps": 4 * args.train_steps, "train_s": train_s,
                         "final_loss": float(loss[-100:].mean().item())},
            "domain": {"lo": list(W.SURROGATE_CURVED_LO), "hi": list(W.SURROGATE_CURVED_HI)}}
        log(f"inclined surrogate: {extra['surrogate']['value']:.3e} photons/s, "
            f"worst bin {extra['surrogate']['density_error_vs_exact']['worst_bin']}")
        sur.close()
    if "table" in paths:
        bench_inclined_table(torch, cphot, S, atm, run, bins, cnt, stream, steps, nb, exact_bins, ms, ms_w, extra)
    return finish_inclined(torch, cphot, W, args, stream, sh, g, geom, det, run, atm, bins, cnt, head, roof, extra)


def bench_inclined_table(torch, cphot, S, atm, run, bins, cnt, stream, steps, nb, exact_bins, ms, ms_w, extra):
    t0 = time.perf_counter()
    tab = cphot.Table(atm, run["h_obs"], "curved", n_c=512, c_lo=0.15)
    tab_build_s = time.perf_counter() - t0
    det_t, tune_t = tuned_detector(cphot, S, atm, {**run, "transport": "table"}, bins, None, cnt, stream, reps=1,
                                   table=tab)
    ms_t, kern_t, b_t, c_t = run_path(torch, cphot, S, det_t, nb, stream, max(3, steps // 2), 1, torch.float64)
    extra["table"] = {"value": float(c_t[3]) * run["bunch"] / (ms_t * 1e-3), "unit": "photons/s", "ms_per_step": ms_t,
                      "kernel_ms": kern_t, "speedup_vs_exact": ms / ms_t,
                      "speedup_vs_walk": ms_w / ms_t if ms_w else None,
                      "density_error_vs_exact": density_error(b_t, exact_bins),
                      "fallback_fraction": float(c_t[9]) / max(float(c_t[3]), 1.0), "build_s": tab_build_s,
                      "tuning": tune_t,
                      "note": "interpolation tracing (Sec. 4.4.1), curved shells: 4 heights per shell x 512 "
                              "tan-zenith nodes up to 81 deg"}
    log(f"inclined table: {extra['table']['value']:.3e} photons/s")
    tab.close()


def finish_inclined(torch, cphot, W, args, stream, sh, g, geom, det, run, atm, bins, cnt, head, roof, extra):
    """The whole shower streamed from host memory with the headline's detector."""
    if args.inclined_chunks > 0:
        chunks = [sh] + [W.workload_inclined_chunk(k, beta=args.beta) for k in range(1, args.inclined_chunks)]
        streamer = cphot.Streamer(sh.n)
        bins.zero_()
        cnt.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for ch in chunks:
            streamer.run(ch.seg, g, det, bins, None, cnt, first_id=ch.first_id, stream=stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        cs = cnt.cpu().numpy()
        streamer.close()
        extra["streamed"] = {"value": float(cs[3]) * run["bunch"] / dt, "unit": "photons/s", "seconds": dt,
                             "segments": int(sum(ch.n for ch in chunks)), "chunks": len(chunks),
                             "records": float(cs[3]), "fluorescence_records": float(cs[10]),
                             "photons_binned": float(cs[8]),
                             "note": "host-resident (pageable) segments, staged by host threads into pinned "
                                     "double buffers, copies overlapped with propagation (PCIe-inclusive)"}
        log(f"inclined streamed: {extra['streamed']['value']:.3e} photons/s over {len(chunks)} chunks")
        # the same shower from page-locked host memory: the copy engine reads it directly
        pinned = [{k: torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32)).pin_memory()
                   for k, v in ch.seg.items()} for ch in chunks]
        ids = [ch.first_id for ch in chunks]
        del chunks
        streamer = cphot.Streamer(sh.n)
        bins.zero_()
        cnt.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for seg_p, fid in zip(pinned, ids):
            streamer.run(seg_p, g, det, bins, None, cnt, first_id=fid)
        torch.cuda.synchronize()
        dt_p = time.perf_counter() - t0
        cp = cnt.cpu().numpy()
        streamer.close()
        extra["streamed"]["pinned_host_memory"] = {
            "value": float(cp[3]) * run["bunch"] / dt_p, "unit": "photons/s", "seconds": dt_p,
            "counters_equal": bool(np.array_equal(cp, cs)),
            "note": "the same chunks in page-locked host memory, copied to the device without staging"}
        log(f"inclined streamed from pinned memory: {extra['streamed']['pinned_host_memory']['value']:.3e} photons/s")
        del pinned
    ctx = {"sh": sh, "geom": geom, "det": det, "run": run, "atm": atm}
    return head, roof, extra, ctx


# ------------------------------------------------------------------------------ CPU baseline

def output_errors(gpu, orc, core, h_obs, dh, curved, lam_range=(300.0, 600.0), n_lam=64):
    """Largest differences of the GPU's records from the oracle's on the outputs
    both sides compute, over records that reached the observation level with the
    same decisions (state, bin) and start away from a layer boundary."""
    assert len(gpu) == len(orc)
    same = (gpu["state"] == orc["state"]) & (gpu["bin"] == orc["bin"])
    arrived = (orc["state"] == 0) | (orc["state"] == 2)
    h_e = radial_height(orc["ex"], orc["ey"], orc["ez"]) if curved else orc["ez"]
    away = np.abs(h_e / dh - np.round(h_e / dh)) * dh > 5e-3
    # a wavelength next to an absorption-bin edge may fall into the neighbouring bin
    lb = (orc["lambda"] - lam_range[0]) / (lam_range[1] - lam_range[0]) * n_lam
    away &= np.abs(lb - np.round(lb)) > 1e-4
    live = same & arrived & away
    r = np.hypot(orc["x"] - core[0], orc["y"] - core[1])
    dpos = np.hypot(gpu["x"] - orc["x"], gpu["y"] - orc["y"])
    dt = np.abs(gpu["t"] - orc["t"])
    dtau = np.abs(gpu["tau"] - orc["tau"])
    ddir = np.max(np.abs(np.stack([gpu["dx"] - orc["dx"], gpu["dy"] - orc["dy"], gpu["dz"] - orc["dz"]], 1)), 1)
    # the position bar: 1e-4 max(r, 10 m) plus a 4e-7 rad direction error carried over the descent
    pos_bar = 1e-4 * np.maximum(r, 10.0) + 4e-7 * np.maximum(h_e - h_obs, 0.0) / np.maximum(orc["dz"] ** 2, 1e-12)
    L = live

    def mx(a):
        return float(a.max()) if a.size else 0.0
    return {"records": int(len(orc)), "records_compared": int(L.sum()),
            "decision_flips": int((~same).sum()),
            "position_abs_m": mx(dpos[L]), "position_rel": mx(dpos[L] / np.maximum(r[L], 10.0)),
            "position_vs_bar": mx(dpos[L] / pos_bar[L]),
            "position_rel_worst_r_m": float(r[L][np.argmax(dpos[L] / np.maximum(r[L], 10.0))]) if L.any() else None,
            "time_abs_ns": mx(dt[L]), "time_rel": mx(dt[L] / np.maximum(np.abs(orc["t"][L]), 1e-9)),
            "tau_abs": mx(dtau[L]), "tau_rel": mx(dtau[L] / np.maximum(orc["tau"][L], 1e-12)),
            "direction_abs": mx(ddir), "wavelength_rel": mx(np.abs(gpu["lambda"] - orc["lambda"]) / orc["lambda"]),
            "survival_uniform_identical": bool(np.array_equal(gpu["u_abs"].astype(np.float64), orc["u_abs"]))}


def cpu_baseline(torch, cphot, W, ctx, target_s=12.0):
    """The FP64 oracle on the deterministic subset of the inclined chunk (segment
    ids = 0 mod 1000): one thread, then all host cores; the GPU runs the same
    subset for parity (bins, counts, expected counts, every record's outputs)."""
    from oracle import oracle as O
    sh, geom, det, run = ctx["sh"], ctx["geom"], ctx["det"], ctx["run"]
    stride = 1000
    sub = {k: np.ascontiguousarray(v[::stride]) for k, v in sh.seg.items()}
    oatm = O.Atmosphere(**W.ATMO_LAYERED)
    orun = O.make_run(**run)
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = max(1, min(threads, 64))
    t0 = time.perf_counter()
    ob, _, oc = O.propagate(oatm, orun, sub, geom, first_id=sh.first_id, threads=1, id_stride=stride)
    t1 = time.perf_counter() - t0
    photons = float(oc[3]) * run["bunch"]
    passes, total = 0, 0.0
    while total < target_s and passes < 200:
        t0 = time.perf_counter()
        O.propagate(oatm, orun, sub, geom, first_id=sh.first_id, threads=threads, id_stride=stride)
        total += time.perf_counter() - t0
        passes += 1
    out = {"value": photons * passes / total, "unit": "photons/s", "cores": threads, "kind": "oracle",
           "per_core": photons / t1, "single_thread_s": t1,
           "sample": f"segments with global id = 0 mod {stride} of the 1e7-segment inclined chunk ({len(sub['x0'])} "
                     f"segments, the same ids and random streams as in the full launch), {int(oc[3])} records per "
                     f"pass; one thread {t1:.2f} s, {threads} threads {passes} passes in {total:.1f} s"}
    # the GPU on the same subset
    seg, g, off = cphot.upload(sub, geom)
    S = cphot.make_segments(seg, g, off, first_id=sh.first_id, id_stride=stride)
    bins = torch.zeros(run["nx"] * run["ny"], dtype=torch.float64, device="cuda")
    cnt = torch.zeros(cphot.NCOUNTERS, dtype=torch.int64, device="cuda")
    cphot.propagate(S, det, bins, None, cnt)
    counts = torch.zeros(S.n, dtype=torch.int32, device="cuda")
    mu = torch.zeros(S.n, dtype=torch.float64, device="cuda")
    cphot.segment_counts(S, det, counts, mu)
    torch.cuda.synchronize()
    gb, gc = bins.cpu().numpy(), cnt.cpu().numpy().astype(np.uint64)
    osc = O.segment_counts(oatm, orun, sub, first_id=sh.first_id, id_stride=stride)
    grec = traced_records(torch, cphot, sub, geom, det, first_id=sh.first_id, id_stride=stride)
    orec = O.trace(oatm, orun, sub, core=sh.core, axis=sh.axis, first_id=sh.first_id, id_stride=stride)
    dh = W.ATMO_LAYERED["h_top"] / W.ATMO_LAYERED["n_layers"]
    errs = output_errors(grec, orec, sh.core, run["h_obs"], dh, True, n_lam=W.ATMO_LAYERED["n_lam"])
    ob0 = ob[0].astype(np.float64)
    errs.update({"records_generated_equal": bool(gc[3] == oc[3]),
                 "fluorescence_records_equal": bool(int(gc[10]) == int(osc["nf"].sum())),
                 "counts_identical": bool(np.array_equal(counts.cpu().numpy(), osc["n"] + osc["nf"].sum(1))),
                 "expected_count_max_abs_diff": float(np.max(np.abs(mu.cpu().numpy() - osc["mu"]))),
                 "bins_l1_diff": float(np.abs(gb - ob0).sum()), "bins_photons": float(ob0.sum()),
                 "bins_cells_differing": int((gb != ob0).sum())})
    out["gpu_subset_parity"] = errs
    return out


# ------------------------------------------------------------------------------ telescope

def bench_telescope(torch, cphot, W, args, stream):
    run = {**W.RUN_TELESCOPE, "seed": 2}
    sh = W.workload_telescope(args.beta)
    geom = np.array([[*sh.core, *sh.axis]])
    atm = cphot.Atmosphere(**W.ATMO_LAYERED)
    seg, g, off = cphot.upload(sh.seg, geom)
    S = cphot.make_segments(seg, g, off)
    nsph = run["snx"] * run["sny"]
    # the step's outputs in one buffer, cleared by one fill per step
    nb, nc, nt = nsph * 8, cphot.NCOUNTERS * 8, nsph * (run["n_t"] + 1) * 4
    out_buf = torch.zeros(nb + nc + nt, dtype=torch.uint8, device="cuda")
    bins = out_buf[:nb].view(torch.int64)
    cnt = out_buf[nb:nb + nc].view(torch.int64)
    th = out_buf[nb + nc:].view(torch.int32)
    if args.telescope_shape != "auto":
        bs_, gb_, lds_ = (int(v) for v in args.telescope_shape.split(","))
        det = cphot.make_detector(atm, **run, block_size=bs_, grid_blocks=gb_, lds_hist=lds_)
        tune = {"block_size": bs_, "grid_blocks": gb_, "lds_hist": lds_, "bunch": run["bunch"], "fixed": True}
    else:
        det, tune = tuned_detector(cphot, S, atm, run, bins, th, cnt, stream)

    def step(ev):
        out_buf.zero_()
        if ev is not None:
            ev[0].record(stream)
        cphot.propagate(S, det, bins, th, cnt, stream=stream)
        if ev is not None:
            ev[1].record(stream)

    ms, kern = time_steps(torch, step, args.steps, args.warmup, stream)
    log(f"exact telescope: {ms:.3f} ms/step, kernel {kern:.3f} ms")
    c = cnt.cpu().numpy()
    exact_bins = bins.cpu().numpy()
    exact_th = th.cpu().numpy()
    records = float(c[3])
    photons = records * run["bunch"]
    dh = W.ATMO_LAYERED["h_top"] / W.ATMO_LAYERED["n_layers"]
    cross, _ = crossing_profile(torch, cphot, sh.seg, geom, det, run["h_obs"], dh, W.ATMO_LAYERED["n_layers"], False)
    res = {"value": photons / (ms * 1e-3), "unit": "photons/s", "ms_per_step": ms, "kernel_ms": kern,
           "records_per_step": records, "photons_per_step": photons, "segments_per_s": sh.n / (ms * 1e-3),
           "workload": f"1e6 segments, zenith 20 deg, Xmax 400, beta variant {args.beta}, 100 layers x 64 "
                       "wavelength bins, bunch 5, 10x10 spheres r=6 m pitch 150 m, 512 x 1 ns time bins",
           "roofline": roofline_entry(f"k_propagate<{tune['block_size']},LAYERED,SPHERES,PROPAGATE>", kern,
                                      float(sh.n), SEGMENT_BYTES, records, cross, False, tune, "telescope_layered")}
    shape = {k: tune[k] for k in ("block_size", "grid_blocks", "lds_hist")}
    if not args.no_cuts:
        res["reduction"] = bench_reduction(torch, cphot, W, S, atm, run, out_buf, bins, th, cnt, stream, args, shape)
        res["emission_options"] = bench_emission_options(torch, cphot, S, atm, run, out_buf, bins, th, cnt, stream,
                                                         args, shape, {"ms_per_step": ms, "binned": float(c[8])})
        res["cuts"] = bench_cuts(torch, cphot, S, atm, run, out_buf, bins, th, cnt, stream, args, exact_bins,
                                 exact_th, photons, ms)
        log(f"telescope with cuts: {res['cuts']['ms_per_step']:.3f} ms/step")
    if not args.no_surrogate:
        res["surrogate"] = bench_surrogate(torch, cphot, W, args, atm, S, run, exact_bins, ms, stream)
        log(f"telescope surrogate: {res['surrogate']['value']:.3e} photons/s")
    if not args.no_cpu_baseline:
        res["cpu_oracle"] = oracle_rate_subset(W, sh, geom, run, stride=100)
        log(f"telescope oracle: {res['cpu_oracle']['value']:.3e} photons/s on {res['cpu_oracle']['cores']} cores")
    return res


def oracle_rate_subset(W, sh, geom, run, stride, target_s=4.0):
    """The FP64 oracle's rate on the segments with id = 0 mod stride of a
    workload: one thread, then all host cores (a context figure beside the
    telescope step; the headline's baseline is the inclined subset's)."""
    from oracle import oracle as O
    sub = {k: np.ascontiguousarray(v[::stride]) for k, v in sh.seg.items()}
    oatm = O.Atmosphere(**W.ATMO_LAYERED)
    orun = O.make_run(**run)
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = max(1, min(threads, 64))
    passes1, t1 = 0, 0.0
    while t1 < 0.25 * target_s and passes1 < 200:
        t0 = time.perf_counter()
        _, _, oc = O.propagate(oatm, orun, sub, geom, threads=1, id_stride=stride)
        t1 += time.perf_counter() - t0
        passes1 += 1
    t1 /= passes1
    photons = float(oc[3]) * run["bunch"]
    passes, total = 0, 0.0
    while total < target_s and passes < 200:
        t0 = time.perf_counter()
        O.propagate(oatm, orun, sub, geom, threads=threads, id_stride=stride)
        total += time.perf_counter() - t0
        passes += 1
    return {"value": photons * passes / total, "unit": "photons/s", "cores": threads, "kind": "oracle",
            "per_core": photons / t1, "single_thread_s": t1,
            "sample": f"segments with id = 0 mod {stride} ({len(sub['x0'])} segments, the full launch's ids and random streams), "
                      f"{int(oc[3])} records of bunch {run['bunch']} per pass; one thread {t1:.3f} s per pass, {threads} "
                      f"threads {passes} passes in {total:.1f} s"}


def bench_cuts(torch, cphot, S, atm, run, out_buf, bins, th, cnt, stream, args, exact_bins, exact_th, photons,
               exact_ms):
    """The telescope step with the data-reduction cuts (filter levels 1 and 3, exact
    bounds): same bins and time histograms, fewer records generated and transported."""
    det, tune = tuned_detector(cphot, S, atm, run, bins, th, cnt, stream, cuts=("track", "photon"))

    def step(ev):
        out_buf.zero_()
        if ev is not None:
            ev[0].record(stream)
        cphot.propagate(S, det, bins, th, cnt, stream=stream)
        if ev is not None:
            ev[1].record(stream)

    ms, kern = time_steps(torch, step, args.steps, args.warmup, stream)
    c = cnt.cpu().numpy()
    same = bool(np.array_equal(bins.cpu().numpy(), exact_bins) and np.array_equal(th.cpu().numpy(), exact_th))
    # the track cut alone: on this kernel the photon cut's test costs about what it saves
    det_t, tune_t = tuned_detector(cphot, S, atm, run, bins, th, cnt, stream, cuts=("track",))

    def step_t(ev):
        out_buf.zero_()
        if ev is not None:
            ev[0].record(stream)
        cphot.propagate(S, det_t, bins, th, cnt, stream=stream)
        if ev is not None:
            ev[1].record(stream)

    ms_t, kern_t = time_steps(torch, step_t, args.steps, args.warmup, stream)
    same_t = bool(np.array_equal(bins.cpu().numpy(), exact_bins) and np.array_equal(th.cpu().numpy(), exact_th))
    track_only = {"ms_per_step": ms_t, "kernel_ms": kern_t, "bins_identical": same_t,
                  "speedup_vs_exact": exact_ms / ms_t, "tuning": tune_t}
    return {"ms_per_step": ms, "kernel_ms": kern, "bins_identical": same, "track_cut_only": track_only,
            "photons_per_s_equivalent": photons / (ms * 1e-3), "speedup_vs_exact": exact_ms / ms,
            "records_generated": float(c[3]), "records_culled_track": float(c[11]),
            "records_culled_photon": float(c[12]), "tuning": tune,
            "note": "filter levels 1 (track cone vs sphere array) and 3 (straight line vs nearest sphere) as "
                    "conservative bounds: bins and time histograms identical to the uncut step; the rate "
                    "counts the uncut step's photons"}


def bench_reduction(torch, cphot, W, S, atm, run, out_buf, bins, th, cnt, stream, args, shape):
    """The telescope step with a detector efficiency (synthetic SiPM-like curve
    times a mirror), without and with the pre-emission reduction (Sec. 4.3.1):
    fewer records generated for the same expected detections."""
    eff = W.efficiency_curve(W.ATMO_LAYERED["n_lam"])
    q = cphot.reduction_table(atm, run["h_obs"], eff)
    eff_d = torch.from_numpy(eff).cuda()
    q_d = torch.from_numpy(q).cuda()
    res = {}
    for name, red in (("efficiency_only", None), ("reduced", q_d)):
        det = cphot.make_detector(atm, **run, **shape, efficiency=eff_d, reduction=red)

        def step(ev, det=det):
            out_buf.zero_()
            if ev is not None:
                ev[0].record(stream)
            cphot.propagate(S, det, bins, th, cnt, stream=stream)
            if ev is not None:
                ev[1].record(stream)

        ms, kern = time_steps(torch, step, args.steps, args.warmup, stream)
        c = cnt.cpu().numpy()
        res[name] = {"ms_per_step": ms, "kernel_ms": kern, "records_generated": float(c[3]),
                     "photons_binned": float(c[8])}
    a, b = res["efficiency_only"], res["reduced"]
    res["speedup"] = a["ms_per_step"] / b["ms_per_step"]
    res["binned_ratio"] = b["photons_binned"] / max(a["photons_binned"], 1.0)
    res["binned_sigma"] = (b["photons_binned"] - a["photons_binned"]) / max(
        np.sqrt(a["photons_binned"] + b["photons_binned"]) * np.sqrt(run["bunch"]), 1.0)
    res["note"] = ("synthetic detector efficiency 0.11-0.40 (SiPM-like x mirror 0.9); the reduced step draws "
                   "each segment's records times the per-layer bound q and keeps them with probability p/q")
    return res


def bench_emission_options(torch, cphot, S, atm, run, out_buf, bins, th, cnt, stream, args, shape, exact):
    """The telescope step with Poisson record counts and with the dispersive
    spectrum (n - 1 stated at 400 nm): the kernels that carry these options,
    their time beside the default step's and the photons they bin."""
    res = {}
    for name, extra in (("poisson_counts", {"counts": "poisson"}),
                        ("dispersive", {"spectrum": "dispersive", "lambda_ref": 400.0})):
        det = cphot.make_detector(atm, **{**run, **extra}, **shape)

        def step(ev, det=det):
            out_buf.zero_()
            if ev is not None:
                ev[0].record(stream)
            cphot.propagate(S, det, bins, th, cnt, stream=stream)
            if ev is not None:
                ev[1].record(stream)

        ms, kern = time_steps(torch, step, args.steps, args.warmup, stream)
        c = cnt.cpu().numpy()
        res[name] = {"ms_per_step": ms, "kernel_ms": kern, "vs_default_step": ms / exact["ms_per_step"],
                     "records_generated": float(c[3]), "records_not_emitted": float(c[13]),
                     "photons_binned": float(c[8]), "binned_vs_default": float(c[8]) / max(exact["binned"], 1.0)}
    res["note"] = ("same workload and launch shape as the default step; Poisson counts keep the expected "
                   "records, the dispersive spectrum draws records for the largest cone and emits each "
                   "with sin^2(theta(lambda)) / sin^2(theta_max)")
    return res


def bench_surrogate(torch, cphot, W, args, atm, S, run, exact_bins, exact_ms, stream):
    """Train the planar transport network on the GPU, then run the telescope
    workload through it; its bins against the exact tracer's (same photons)."""
    sur = cphot.Surrogate(W.SURROGATE_LO, W.SURROGATE_HI, max_batch=4096, init_seed=1)
    t0 = time.perf_counter()
    X, Y = sur.make_training_set(atm, args.train_samples, seed=1004)
    sur.fit_normalization(Y)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss = sur.train(X, Y, batch=4096, steps=args.train_steps, lr=3e-3)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    loss = loss.cpu().numpy()
    del X, Y
    nsph = run["snx"] * run["sny"]

    def run_spheres(det):
        bins = torch.zeros(nsph, dtype=torch.int64, device="cuda")
        th = torch.zeros(nsph * (run["n_t"] + 1), dtype=torch.int32, device="cuda")
        cnt = torch.zeros(cphot.NCOUNTERS, dtype=torch.int64, device="cuda")

        def step(ev):
            bins.zero_()
            th.zero_()
            cnt.zero_()
            if ev is not None:
                ev[0].record(stream)
            cphot.propagate(S, det, bins, th, cnt, stream=stream)
            if ev is not None:
                ev[1].record(stream)

        ms, kern = time_steps(torch, step, args.steps, args.warmup, stream)
        return ms, kern, bins.cpu().numpy(), cnt.cpu().numpy()

    def tuned(transport, **extra):
        b = torch.zeros(nsph, dtype=torch.int64, device="cuda")
        t = torch.zeros(nsph * (run["n_t"] + 1), dtype=torch.int32, device="cuda")
        c = torch.zeros(cphot.NCOUNTERS, dtype=torch.int64, device="cuda")
        return tuned_detector(cphot, S, atm, {**run, "transport": transport}, b, t, c, stream, **extra)

    det_s, tune_s = tuned("surrogate", surrogate=sur)
    ms, kern, b_s, c_s = run_spheres(det_s)
    det_l, _ = tuned("straight")
    ms_l, _, b_l, _ = run_spheres(det_l)
    photons = float(c_s[3]) * run["bunch"]
    tb = time.perf_counter()
    tab = cphot.Table(atm, run["h_obs"], "planar", c_lo=0.4)
    tab_build_s = time.perf_counter() - tb
    det_t, tune_t = tuned("table", table=tab)
    ms_t, kern_t, b_t, c_t = run_spheres(det_t)

    def grid_density(S_, grid_run):
        """Exact vs network vs straight line vs table on a ground grid (same photons)."""
        out = {}
        for name in ("layered", "surrogate", "straight", "table"):
            d = cphot.make_detector(atm, **{**grid_run, "transport": name},
                                    surrogate=sur if name == "surrogate" else None,
                                    table=tab if name == "table" else None)
            b = torch.zeros(grid_run["nx"] * grid_run["ny"], dtype=torch.int64, device="cuda")
            cphot.propagate(S_, d, b, None, None, stream=stream)
            out[name] = b.cpu().numpy()
        return {"surrogate": density_error(out["surrogate"], out["layered"]),
                "table": density_error(out["table"], out["layered"]),
                "straight_line": density_error(out["straight"], out["layered"]),
                "photons": float(out["layered"].sum())}

    # the 10 m grid of the same shower: hundreds of bins above 1000 photons
    tele_grid = grid_density(S, dict(detector="grid", spectrum="frank_tamm", bunch=1, h_obs=2200.0, nx=100, ny=100,
                                     cell=10.0, seed=2))
    tiny = W.workload_tiny_vertical("R")
    tg = np.array([[*tiny.core, *tiny.axis]])
    ts, tgg, toff = cphot.upload(tiny.seg, tg)
    tiny_grid = grid_density(cphot.make_segments(ts, tgg, toff),
                             {**W.RUN_TINY, "spectrum": "frank_tamm", "bunch": 1, "seed": 1})
    res = {
        "value": photons / (ms * 1e-3), "unit": "photons/s", "ms_per_step": ms, "kernel_ms": kern,
        "speedup_vs_exact": exact_ms / ms,
        "density_error_vs_exact_spheres": density_error(b_s, exact_bins),
        "density_error_vs_exact_grid_10m": tele_grid,
        "fallback_fraction": float(c_s[9]) / max(float(c_s[3]), 1.0), "tuning": tune_s,
        "tiny_vertical_shower_grid": tiny_grid,
        "straight_line_without_correction": {"ms_per_step": ms_l,
                                             "density_error_vs_exact": density_error(b_l, exact_bins)},
        "table": {"value": float(c_t[3]) * run["bunch"] / (ms_t * 1e-3), "unit": "photons/s", "ms_per_step": ms_t,
                  "kernel_ms": kern_t, "speedup_vs_exact": exact_ms / ms_t,
                  "density_error_vs_exact": density_error(b_t, exact_bins),
                  "fallback_fraction": float(c_t[9]) / max(float(c_t[3]), 1.0), "build_s": tab_build_s,
                  "tuning": tune_t,
                  "note": "interpolation tracing (Sec. 4.4.1): 4 heights per layer x 256 tan-zenith nodes"},
        "network": "5-64-64-4 ReLU, bf16 weights on MFMA 16x16x32, FP32 accumulate",
        "training": {"samples": args.train_samples, "steps": args.train_steps, "batch": 4096,
                     "set_build_s": t1 - t0, "train_s": t2 - t1,
                     "samples_per_s": args.train_steps * 4096 / max(t2 - t1, 1e-9),
                     "final_loss": float(loss[-100:].mean())},
    }
    sur.close()
    tab.close()
    return res


# ------------------------------------------------------------------------------ batched

def bench_batched(torch, cphot, W, args, stream):
    """256 showers, segment counts log-uniform in [1e3, 1e6], zenith U[0, 60],
    Xmax U[350, 750], each with its own 200 x 200 grid of 5 m cells, straight
    rays; one captured launch per step with the autotuner's shape, the bunch
    chosen among those whose bins stay within 1 % of bunch 1."""
    t0 = time.perf_counter()
    shs = W.make_batch(args.batch_showers, seed=1003, beta=args.beta)
    log(f"batched workload generated in {time.perf_counter() - t0:.1f} s")
    ns = len(shs)
    n = int(sum(s.n for s in shs))
    fields = ("x0", "y0", "z0", "x1", "y1", "z1", "beta", "charge")
    dev = {k: torch.empty(n, dtype=torch.float32, device="cuda") for k in fields}
    o = 0
    for s in shs:  # per-shower copies straight into the device columns
        for k in fields:
            dev[k][o:o + s.n].copy_(torch.from_numpy(s.seg[k]))
        o += s.n
    offs = np.zeros(ns + 1, dtype=np.int64)
    offs[1:] = np.cumsum([s.n for s in shs])
    geom = np.array([[s.core[0], s.core[1], *s.axis] for s in shs], dtype=np.float64)
    del shs
    g = torch.from_numpy(geom).cuda()
    off = torch.from_numpy(offs).cuda()
    S = cphot.make_segments(dev, g, off)
    run = {**W.RUN_BATCH, "seed": 3}
    atm = cphot.Atmosphere(**W.ATMO_STRAIGHT)
    per = run["nx"] * run["ny"]
    bins = torch.zeros(ns * per, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(cphot.NCOUNTERS, dtype=torch.int64, device="cuda")
    det0 = cphot.make_detector(atm, **run)
    t0 = time.perf_counter()
    tune = cphot.autotune_accuracy(S, det0, bins, None, cnt, bunches=[1, 2, 5], reps=2, max_error=0.01,
                                   min_count=1000.0, stream=stream)
    tune_s = time.perf_counter() - t0
    log(f"autotune: {tune} in {tune_s:.1f} s")
    det = cphot.make_detector(atm, **{**run, "bunch": tune["bunch"]}, **cphot.shape_of(tune))
    step_g = cphot.Step(S, det, bins, None, cnt, clear=True)

    def step(ev):
        if ev is not None:
            ev[0].record(stream)
        step_g.launch(stream=stream)
        if ev is not None:
            ev[1].record(stream)

    ms, kern = time_steps(torch, step, args.steps, args.warmup, stream)
    c = cnt.cpu().numpy()
    photons = float(c[3]) * tune["bunch"]
    res = {"value": photons / (ms * 1e-3), "unit": "photons/s", "ms_per_step": ms, "graph_launch_ms": kern,
           "showers": ns, "segments": n, "records_per_step": float(c[3]), "photons_per_step": photons,
           "tuning": {**tune, "tune_s": tune_s, "bunch_candidates": [1, 2, 5]},
           "workload": "256 showers, 10^U[3,6] segments each, zenith U[0,60] deg, Xmax U[350,750], "
                       "200x200 grid of 5 m per shower, straight rays, Rayleigh; one HIP-graph launch per step"}
    if tune["bunch"] == 1:
        # the rate the rejected bunch of 5 would give, with the same shape, labelled as such
        det5 = cphot.make_detector(atm, **{**run, "bunch": 5}, **cphot.shape_of(tune))
        step_5 = cphot.Step(S, det5, bins, None, cnt, clear=True)

        def step5(ev):
            if ev is not None:
                ev[0].record(stream)
            step_5.launch(stream=stream)
            if ev is not None:
                ev[1].record(stream)

        ms5, _ = time_steps(torch, step5, max(3, args.steps // 2), 1, stream)
        c5 = cnt.cpu().numpy()
        res["bunch5_rejected"] = {"value": float(c5[3]) * 5 / (ms5 * 1e-3), "ms_per_step": ms5,
                                  "worst_bin_vs_bunch1": tune["bin_errors"].get(5),
                                  "note": "coarser statistics: per-shower bins beyond 1 % of bunch 1"}
        step_5.close()
    step_g.close()
    res["block_balance"] = block_balance(torch, cphot, S, det, n, tune)
    return res


def block_balance(torch, cphot, S, det, n, tune):
    """Records per block of the persistent grid's static partition (each block
    walks a contiguous range of tiles), from the per-segment record counts."""
    counts = torch.zeros(n, dtype=torch.int32, device="cuda")
    cphot.segment_counts(S, det, counts)
    torch.cuda.synchronize()
    c = counts.cpu().numpy().astype(np.int64)
    bs = int(tune["block_size"])
    tiles = np.add.reduceat(c, np.arange(0, n, bs))
    nt = len(tiles)
    grid = min(int(tune["grid_blocks"]), nt)  # the library clamps the grid to the tile count
    first = (np.arange(grid, dtype=np.int64) * nt) // grid
    per_block = np.add.reduceat(tiles, first)
    mean = float(per_block.mean())
    return {"blocks": grid, "tiles": nt, "records_per_block_mean": mean,
            "records_per_block_max_over_mean": float(per_block.max()) / mean,
            "records_per_block_cv": float(per_block.std()) / mean,
            "note": "static contiguous tile ranges; more blocks than fit on the chip at once, so the "
                    "dispatcher starts the later ones as earlier ones finish"}


# ------------------------------------------------------------------------------ main

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--beta", default="R", choices=["R", "literal"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-telescope", action="store_true")
    ap.add_argument("--no-cuts", action="store_true", help="skip the telescope steps with cuts, reduction and options")
    ap.add_argument("--telescope-shape", default="256,1024,1", metavar="BS,GRID,LDS|auto",
                    help="launch shape of the exact telescope step: a fixed shape (default) or 'auto'")
    ap.add_argument("--inclined-paths", default="walk,surrogate,table",
                    help="paths run beside the headline on the inclined chunk (comma list; empty for none)")
    ap.add_argument("--inclined-chunks", type=int, default=10,
                    help="chunks of 1e7 segments streamed from host memory (0: only the resident chunk)")
    ap.add_argument("--train-samples", type=int, default=10_000_000)
    ap.add_argument("--train-steps", type=int, default=20_000)
    ap.add_argument("--batch-showers", type=int, default=256)
    ap.add_argument("--part", choices=["telescope", "batched"], default=None,
                    help="run only this part and print its figures (for profiling; not the benchmark line)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (scale for the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the photon path needs no collectives and the benchmark "
              "measures one MI355X; multi-GPU figures are not produced.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2405_04229_amd import cphot
    from paper_2405_04229_amd import workload as W

    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each_way": n * 4, "launches": 3}), flush=True)
        return
    stream = torch.cuda.current_stream()
    if args.part:
        part = (bench_telescope if args.part == "telescope" else bench_batched)(torch, cphot, W, args, stream)
        print(json.dumps({"part": args.part, **part}), flush=True)
        return
    head, roof, inclined, ctx = bench_inclined(torch, cphot, W, args, stream)
    out = {
        "metric": METRIC,
        "value": head["value"], "unit": "photons/s", "n_gpus": 1, "steps": max(5, args.steps // 2),
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "large inclined shower, resident chunk: 1e7 segments of a 60-degree shower "
                               f"(Xmax 600, beta variant {args.beta}), curved Earth (100 shells of 250 m), "
                               "Cherenkov + fluorescence (3 bands, dE/dx U[0.1,2] MeV/m), 64 wavelength bins, "
                               "1000x1000 grid of 10 m, FP64 bins",
                   "path": "exact (closed-form shell sums, shell walk beyond them)",
                   "records_per_step": head["records"], "photons_per_step": head["photons"],
                   "segments_per_s": head["segments"] / (head["ms_per_step"] * 1e-3),
                   "kernel_ms": head["kernel_ms"], "tuning": head["tuning"],
                   "records_walked": head["records_walked"], "fluorescence_records": head["fluorescence_records"]},
        "roofline": roof,
        "inclined": inclined,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(torch, cphot, W, ctx)
        log(f"cpu baseline: {out['cpu_baseline']['value']:.3e} photons/s on {out['cpu_baseline']['cores']} cores")
    del ctx
    torch.cuda.empty_cache()
    if not args.no_telescope:
        out["telescope"] = bench_telescope(torch, cphot, W, args, stream)
        torch.cuda.empty_cache()
    if not args.no_batched:
        out["batched"] = bench_batched(torch, cphot, W, args, stream)
        log(f"batched: {out['batched']['value']:.3e} photons/s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
