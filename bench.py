"""Benchmark: photons propagated per second on one MI355X.

One step = one pass of the whole photon path over one batch: cphot_propagate
over the telescope workload (1e6 track segments of a 20-degree gamma-like
shower, refraction through 100 homogeneous layers with Rayleigh + aerosol
absorption on 64 wavelength bins, bunches of 5 photons, 100 bounding spheres of
6 m on a 150 m grid, 1 ns arrival-time histograms), bins and counters zeroed
first. Inputs are resident in HBM before timing starts.

Prints one JSON line. Extra fields: the dominant kernel's roofline position and
the FP64 CPU oracle timed on a bounded sample on the host cores.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X public figures: 256 CUs, 2.4 GHz peak engine clock, 64 VALU lanes per CU per clock.
PEAK_VALU_LANE_OPS = 256 * 64 * 2.4e9
PEAK_HBM = 8.0e12

# Algorithmic VALU lane-slots per unit of work (counted from the method's steps;
# 32-bit multiplies and transcendentals weighted 4 as quarter-rate operations).
SLOTS_PER_SEGMENT = 350.0
SLOTS_PER_RECORD_BASE = 320.0
SLOTS_PER_LAYER_CROSSING = 22.0
SEGMENT_BYTES = 32.0

def atmo_kw():
    from paper_2405_04229_amd import workload as W
    return dict(profile="linsley5", a=W.LINSLEY_A, b=W.LINSLEY_B, c=W.LINSLEY_C, hb=W.LINSLEY_HB_M, kappa=W.KAPPA,
                h_top=25000.0, step=1.0, rayleigh400=2974.0, aer_tau350=0.05, aer_H=1200.0, aer_angstrom=1.0,
                n_layers=100, n_lam=64)


RUN = dict(transport="layered", detector="spheres", spectrum="frank_tamm", bunch=5, h_obs=2200.0, snx=10, sny=10,
           pitch=150.0, radius=6.0, n_t=512, dt=1.0, seed=2)


def cpu_baseline(sh, target_s=12.0):
    """The FP64 oracle on a contiguous sample of the same workload, all host cores."""
    from oracle import oracle as O
    atm = O.Atmosphere(**atmo_kw())
    run = O.make_run(**RUN)
    geom = [[*sh.core, *sh.axis]]
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = max(1, min(threads, 64))
    n = 20_000
    while True:
        seg = {k: v[:n] for k, v in sh.seg.items()}
        t0 = time.perf_counter()
        _, _, cnt = O.propagate(atm, run, seg, geom, threads=threads)
        dt = time.perf_counter() - t0
        if dt >= target_s / 4 or n >= sh.n:
            break
        n = min(sh.n, int(n * max(2.0, target_s / max(dt, 1e-3) * 0.5)))
    photons = float(cnt[3]) * RUN["bunch"]
    return {"value": photons / dt, "unit": "photons/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n} of {sh.n} segments (same ids and random streams), {int(cnt[3])} records, "
                      f"{dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--beta", default="R", choices=["R", "literal"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (scale for the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the photon path needs no collectives and this build "
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
    sh = W.workload_telescope(args.beta)
    geom = np.array([[*sh.core, *sh.axis]])
    atm = cphot.Atmosphere(**atmo_kw())
    det = cphot.make_detector(atm, **RUN)
    seg, g, off = cphot.upload(sh.seg, geom)
    S = cphot.make_segments(seg, g, off)
    nsph = RUN["snx"] * RUN["sny"]
    bins = torch.zeros(nsph, dtype=torch.int64, device="cuda")
    th = torch.zeros(nsph * (RUN["n_t"] + 1), dtype=torch.int32, device="cuda")
    cnt = torch.zeros(cphot.NCOUNTERS, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()

    def step(ev=None):
        bins.zero_()
        th.zero_()
        cnt.zero_()
        if ev is not None:
            ev[0].record(stream)
        cphot.propagate(S, det, bins, th, cnt, stream=stream)
        if ev is not None:
            ev[1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(events[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))
    c = cnt.cpu().numpy()
    records = float(c[3])
    photons = records * RUN["bunch"]
    value = photons / (ms_per_step * 1e-3)

    # mean layer crossings per record from a sample of traced records
    sample = {k: v[:20000] for k, v in sh.seg.items()}
    sg, sgg, _ = cphot.upload(sample, geom)
    SS = cphot.make_segments(sg, sgg, None)
    counts = torch.zeros(SS.n, dtype=torch.int32, device="cuda")
    cphot.segment_counts(SS, det, counts)
    offs = torch.cumsum(counts.to(torch.int64), 0) - counts.to(torch.int64)
    tot = int(counts.sum().item())
    rec = torch.zeros(max(tot, 1) * cphot.RECORD_BYTES, dtype=torch.uint8, device="cuda")
    cphot.trace_records(SS, det, offs.contiguous(), rec)
    torch.cuda.synchronize()
    r = cphot.records_to_numpy(rec.cpu())[:tot]
    # layer crossings of each record: from the layer of its segment's midpoint down to the observation layer
    dh = 250.0
    obs_layer = int(RUN["h_obs"] // dh)
    zmid = 0.5 * (sample["z0"].astype(np.float64) + sample["z1"])
    start_layer = np.minimum((zmid[r["seg"].astype(np.int64)] // dh).astype(np.int64), 99)
    crossings = np.maximum(start_layer - obs_layer, 0)
    mean_cross = float(crossings[r["state"] != 1].mean()) if len(r) else 0.0

    n_seg = float(sh.n)
    slots = n_seg * SLOTS_PER_SEGMENT + records * (SLOTS_PER_RECORD_BASE + SLOTS_PER_LAYER_CROSSING * mean_cross)
    achieved = slots / (kern_ms * 1e-3)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_VALU_LANE_OPS / 1e12,
                "unit": "Tlane-ops/s", "frac": achieved / PEAK_VALU_LANE_OPS, "traffic": None,
                "kernel": "k_propagate<256,LAYERED,SPHERES,PROPAGATE>", "kernel_ms": kern_ms,
                "algorithmic_slots_per_launch": slots, "mean_layer_crossings": mean_cross,
                "hbm_gbps_algorithmic": n_seg * SEGMENT_BYTES / (kern_ms * 1e-3) / 1e9}
    out = {
        "metric": "photons propagated/s, exact vs MLP surrogate, at <=1% per-bin density error",
        "value": value, "unit": "photons/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"telescope: 1e6 segments, zenith 20 deg, Xmax 400, beta variant {args.beta}, "
                               "100 layers x 64 wavelength bins, bunch 5, 10x10 spheres r=6 m pitch 150 m, "
                               "512 x 1 ns time bins",
                   "path": "exact", "records_per_step": records, "photons_per_step": photons,
                   "segments_per_s": n_seg / (ms_per_step * 1e-3)},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sh)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
