#!/usr/bin/env python3
"""Throughput of the MI355X TPC sector tracker on one GPU.

One step = one pass of the whole hot path (grid, CA links, cleaning and
starts, tracklets, selection, three-pass refit, compaction, FP64 totals) over
one batch of synthetic input with the clusters already resident in device
memory. The default workload is the batched central event: eight central
Pb-Pb-like events (36 sectors x 152 pad rows, 8000 primaries + 800
secondaries, 2 % noise each; 288 sector instances, ~10.9 M clusters) tracked
in one batch. The timed form is the batched one (one launch per stage over all
sector instances, replayed as a HIP graph); the plain form (every stage
launched per sector instance) is timed beside it.

Prints one JSON line (rank 0): clusters/s as `value`, tracks/s, the roofline
of the dominant kernel (per-stage HIP events measured in this run over an
algorithmic byte model fed by the kernels' own work counters), the other
workloads, and the oracle timed on the host cores as a CPU baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "TPC clusters/sec + tracks/sec (CA+Kalman, 1 GPU), % HBM roofline; batched vs plain"
HBM_PEAK_GBS = 8000.0       # MI355X HBM3E
FP32_VECTOR_PEAK_TFLOPS = 157.3

WORKLOADS = {
    "C2": "central Pb-Pb-like event: 36 sectors x 152 pad rows, 8000 primary + 800 secondary helices "
          "(pT exp(0.5 GeV) in [0.1,10], |eta|<0.9, 0.5 T), sigma 0.1 cm, 2% noise",
    "C2x8": "batched central event: eight central Pb-Pb-like events (36 sectors x 152 pad rows each, 8000 "
            "primary + 800 secondary helices, 2% noise; 288 sector instances) in one batch",
    "C3": "continuous-readout slice: 100 collisions x Exp(800) tracks, drift shift 0-250 cm, 2% noise",
    "C4": "256 sector instances, log-uniform 50-2000 helices each, 1% noise",
    "C1": "one sector, 200 helices, 1% noise",
    "C5": "twelve central Pb-Pb-like events (432 sector instances) with a smooth synthetic space-charge "
          "displacement (amplitude 0.5 cm) applied before the smear",
}


def byte_model(stage: str, st: dict, n_clusters: int, n_seg: int, hits_per_bin: int) -> int:
    """Algorithmic bytes of one launch of a stage: what the method itself must
    move given its stage barriers, from the kernels' own work counters (caches
    not credited). Per stage:
      grid        16 B read + 12 B written per cluster, 4 B per bin and per row
      links       8 B (y, z) + 8 B (up, dn) per cluster, 4 B per bin
      clean+start 24 B per cluster (own links, partner links, written links), 4 B per start
      tracklets   12 B per chain hit, 12 B per visited pick row (bin range, row
                  table), 8 B per tested candidate, 8 B per picked hit (weight)
      select      4 B x rows per selected tracklet, 4 B per pick, 4 B per owned hit, 16 B per track
      refit       12 B per cluster visit (id, y, z) over the three passes,
                  4 B per accepted cluster, 108 B per output track
      write       8 B per output cluster"""
    N = n_clusters
    nbins = N // max(1, hits_per_bin) + n_seg
    if stage == "grid":
        return 16 * N + 12 * N + 4 * (nbins + n_seg)
    if stage == "links":
        return 8 * N + 4 * nbins + 8 * N
    if stage == "clean_starts":
        return 24 * N + 4 * st["n_starts"]
    if stage == "tracklets":
        return 12 * st["n_chain_hits"] + 12 * st["tl_rows_visited"] + 8 * st["tl_candidates"] + 8 * st["tl_picks"]
    if stage == "select":
        return 4 * 152 * st["n_selected"] + 4 * st["tl_picks"] + 4 * st["n_selected_hits"] + 16 * st["n_selected"]
    if stage == "refit":
        return 12 * st["rf_hit_visits"] + 4 * st["n_track_hits"] + 108 * st["n_tracks"]
    if stage == "write":
        return 8 * st["n_track_hits"]
    return 0


def impl_byte_model(stage: str, st: dict, n_clusters: int, n_seg: int, hits_per_bin: int) -> int:
    """Bytes the implementation's own data layout moves per launch (its 32-byte
    row headers, 80-byte tracklet states, pick tables, refit records): a second
    column beside the algorithmic model, never the roofline numerator."""
    N = n_clusters
    if stage == "grid":
        return 24 * N + 32 * n_seg + 4 * (N // max(1, hits_per_bin) + n_seg)
    if stage == "links":
        return 32 * N
    if stage == "tracklets":
        return (100 * st["n_starts"] + 12 * st["n_chain_hits"] + 64 * st["tl_rows_visited"]
                + 8 * st["tl_candidates"] + 13 * st["tl_picks"])
    if stage == "refit":
        return 192 * st["n_selected"] + 14 * st["rf_hit_visits"]
    if stage == "clean_starts":
        return 24 * N + 12 * st["n_starts"]
    if stage == "select":
        return 2 * (8 * st["n_starts"] + 8 * st["tl_picks"]) + 13 * st["n_selected_hits"] + 12 * st["n_selected"]
    if stage == "write":
        return 2 * 8 * st["n_selected"] + 108 * st["n_tracks"] + 9 * st["n_selected_hits"]
    return 0


def kernel_source_sha256() -> str:
    """Hash of the tracking kernels' sources (the differentiable refit's files
    do not enter: they build no kernel of the tracking path)."""
    import hashlib
    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_1811_11481_amd", "csrc")
    for f in ("internal.h", "kernels.hip", "kf_device.h"):
        h.update(open(os.path.join(src, f), "rb").read())
    return h.hexdigest()


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of a stage's kernels from the committed rocprofv3
    PMC summary (FETCH_SIZE and WRITE_SIZE scaled by a copy of known size), or
    None when there is none for this stage and workload or the kernels have
    changed since."""
    path = os.path.join(ROOT, "profiles", "pmc_%s_%s.json" % (kernel.replace("k_", ""), workload))
    if not os.path.exists(path):
        path = os.path.join(ROOT, "profiles", "pmc_%s_%s.json" % (kernel, workload))
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("source_sha256") != kernel_source_sha256():
        return None
    return int(d["traffic_bytes_per_launch"])


def measured_issue(kernel: str, workload: str, launch_ms: float):
    """VALU issue of the dominant stage's kernels from the committed rocprofv3
    SQ counters (wave-level VALU instructions per launch, fraction of lanes
    enabled) and the live launch time: the fraction of the 1024 SIMDs' issue
    slots (one wave64 instruction per 4 cycles at 2.4 GHz) they kept busy.
    None when there is no summary or the kernels have changed since."""
    path = os.path.join(ROOT, "profiles", "pmc_%s_%s.json" % (kernel.replace("k_", ""), workload))
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("source_sha256") != kernel_source_sha256() or "valu_insts_per_launch" not in d or launch_ms <= 0:
        return None
    n = float(d["valu_insts_per_launch"])
    return {"valu_wave_insts": int(n), "lanes_active": d.get("lanes_active"),
            "busy_frac": round(n * 4 / (1024 * 2.4e9 * launch_ms * 1e-3), 4)}


def copy_bandwidth(torch, mib=1024, reps=5):
    """Device copy bandwidth measured here (read + write of a mib-MiB buffer,
    HIP events around each copy, best of reps): the attainable counterpart of
    the 8 TB/s vendor peak."""
    n = mib * (1 << 18)
    src = torch.empty(n, dtype=torch.float32, device="cuda")
    src.fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del src, dst
    return 2.0 * n * 4 / (best * 1e-3) / 1e9


def stage_kernels(stage, tuning, max_row=0):
    """The kernels one launch of a stage runs (their times add up to the
    stage's event-timed duration); max_row is the largest row of the batch
    (rows next to one of more than 512 clusters go to the neighbour kernel's
    second variant)."""
    if stage == "tracklets":
        if tuning.inward_wgs > 0:
            return ["k_tracklet<1>", "k_tracklet_in"]
        if tuning.inward_sort:
            return ["k_tracklet<1>", "k_tl_order", "k_tracklet_inward"]
        return ["k_tracklet<0>"]
    if stage == "links":
        return ["k_links<8>", "k_links<16>"] if max_row > 512 else ["k_links<8>"]
    return [{"refit": "k_refit", "grid": "k_grid<4096>"}.get(stage, stage)]


def stage_roofline(trk, dc, cs, workload, warmup, steps):
    """Per-stage kernel time (HIP events between the stages, on the launch
    stream), algorithmic bytes from the work counters, and the roofline of the
    dominant kernel."""
    from paper_1811_11481_amd import Tracker, default_params
    from paper_1811_11481_amd.tpcca import FLAG_STATS, FLAG_TIMING

    trk_t = Tracker(params=default_params(flags=FLAG_TIMING), tuning=trk.tuning)
    outt = trk_t.alloc_tracks(dc)
    stage_ms = {}
    for k in range(warmup + steps):
        trk_t.track(dc, outt, batched=True)
        if k >= warmup:
            for name, v in trk_t.stage_times().items():
                stage_ms.setdefault(name, []).append(v)
    stage_avg = {k: statistics.mean(v) for k, v in stage_ms.items()}
    # work counters for the byte model (separate pass: the counters use atomics)
    trk_s = Tracker(params=default_params(flags=FLAG_STATS), tuning=trk.tuning)
    trk_s.track(dc, trk_s.alloc_tracks(dc), batched=True)
    st = trk_s.stats()
    nseg = cs.n_inst * 152
    hpb = trk.tuning.hits_per_bin
    stages = {}
    for name, t in stage_avg.items():
        b = byte_model(name, st, cs.n_clusters, nseg, hpb)
        bi = impl_byte_model(name, st, cs.n_clusters, nseg, hpb)
        stages[name] = {"ms": round(t, 4), "alg_bytes": b, "impl_bytes": bi,
                        "GBps": round(b / (t * 1e-3) / 1e9, 2) if t > 0 and b else None}
    dom = max((k for k in stages if k != "finish"), key=lambda k: stages[k]["ms"])
    dom_bytes = stages[dom]["alg_bytes"]
    achieved = dom_bytes / (stages[dom]["ms"] * 1e-3) / 1e9
    kname = {"tracklets": "k_tracklet", "refit": "k_refit", "links": "k_links", "grid": "k_grid"}.get(dom, dom)
    import numpy as np
    kernels = stage_kernels(dom, trk.tuning, int(np.diff(np.asarray(cs.row_start)).max()) if cs.n_clusters else 0)
    roofline = {"bound": "hbm", "kernel": " + ".join(kernels), "stage": dom, "achieved": round(achieved, 2),
                "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                "traffic": measured_traffic(kname, workload),
                "alg_bytes_per_launch": dom_bytes, "impl_bytes_per_launch": stages[dom]["impl_bytes"],
                "avg_launch_ms": stages[dom]["ms"], "valu_issue": measured_issue(kname, workload, stages[dom]["ms"]),
                "work_counters": st}
    return stages, roofline


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads() -> int:
    """Worker threads for the oracle baseline: the cores this process may run
    on, at most 16 (a one-GPU share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def diff_leg(args, torch, np, synth):
    """Differentiable refit: chi2 of the frozen-mask three-pass refit of the
    first tracks found in C5, as a function of the start states and a
    correction map, forward and reverse sweep (binary32 and binary64 adjoint)."""
    from paper_1811_11481_amd import FLAG_ADJOINT_F64, DeviceClusters, RefitSet, Tracker, default_params

    cs = synth.generate("C5")
    dc = DeviceClusters.from_host(cs)
    trk = Tracker()
    out = trk.track(dc, batched=True)
    rs = RefitSet.from_tracker(trk).head(args.diff_tracks)
    coef = (0.1 * torch.randn((3, 16, 16, 32), generator=torch.Generator().manual_seed(5))).float().cuda()
    w = torch.ones(rs.n_tracks, dtype=torch.float32, device="cuda")
    res = {"workload": "C5: " + WORKLOADS["C5"], "n_clusters": cs.n_clusters, "n_tracks_found": out.n_tracks,
           "n_tracks": rs.n_tracks, "n_hits": rs.n_hits, "map": "random smooth B-spline map, sigma 0.1 cm"}
    for name, flags in (("f32", 0), ("f64", FLAG_ADJOINT_F64)):
        t = Tracker(params=default_params(flags=flags)) if flags else trk
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        fw, bw = [], []
        for k in range(args.warmup + max(3, args.steps // 2)):
            ev[0].record()
            t.refit_forward(dc, rs, coef=coef)
            ev[1].record()
            t.refit_backward(w)
            ev[2].record()
            torch.cuda.synchronize()
            if k >= args.warmup:
                fw.append(ev[0].elapsed_time(ev[1]))
                bw.append(ev[1].elapsed_time(ev[2]))
        f, b = statistics.median(fw), statistics.median(bw)
        res[name] = {"fwd_ms": round(f, 4), "bwd_ms": round(b, 4),
                     "tracks_per_s_fwd_bwd": round(rs.n_tracks / ((f + b) * 1e-3), 1)}
        print("[bench] differentiable refit %s: fwd %.3f ms, bwd %.3f ms (%d tracks)" % (name, f, b, rs.n_tracks),
              file=sys.stderr, flush=True)
    return res


def next_leg(torch, np, synth, cs, dc, warmup, steps):
    """The steps that follow the sector tracking, each timed on the headline
    workload (device time around the call, inputs resident): the cross-sector
    merge after a track call (its one count read-back included), the batched
    track call on native (pad, time) clusters, the corrected final fit of a
    track call's tracks, and the batched track call that also writes the
    compression residuals (every call writes z0)."""
    from paper_1811_11481_amd import FLAG_MERGE, DeviceNativeClusters, Tracker, default_params

    def timed(fn):
        for _ in range(max(1, warmup)):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps * 1e3

    res = {}
    # merge: events of 36 sector instances each (mode-1 generator layout)
    mp = default_params(flags=FLAG_MERGE)
    trk = Tracker(params=mp)
    out = trk.alloc_tracks(dc)
    trk.track(dc, out, batched=True)
    ev = torch.as_tensor((np.arange(cs.n_inst) // 36).astype(np.int32), device="cuda")
    state = {}

    def do_merge():
        state["m"] = trk.merge(ev)

    mms = timed(do_merge)
    M, nseg, _ = state["m"]
    res["merge"] = {"ms": round(mms, 4), "sector_tracks": out.n_tracks, "merged_tracks": M.n_tracks,
                    "tracks_with_2plus_segments": int((nseg > 1).sum().item())}
    del state, M, nseg, trk, out
    # native (pad, time) input, transformed by the grid kernel
    p = default_params()
    pad, tm = synth.to_native(cs, np.array(p.pad_width[:152]), np.array(p.pad_center[:152]), p.z_per_bin,
                              p.z_readout)
    dn = DeviceNativeClusters.from_host(cs.n_inst, cs.inst_sector, cs.row_start, pad, tm)
    trk = Tracker()
    out = trk.alloc_tracks(dn)
    nms = timed(lambda: trk.track_native(dn, out))
    res["native_input"] = {"ms_per_step": round(nms, 4), "clusters_per_s": round(cs.n_clusters / (nms * 1e-3), 1),
                           "n_tracks": out.n_tracks}
    del dn, out
    # corrected final fit: clusters moved to each track's absolute frame and
    # corrected by a random smooth map, three passes again (the track call's
    # outputs stay alive for it)
    rng = np.random.default_rng(11)
    coef = torch.as_tensor((0.1 * rng.standard_normal(3 * 16 * 16 * 32)).astype(np.float32), device="cuda")
    out = trk.alloc_tracks(dc)
    trk.track(dc, out, batched=True)
    cst = {}

    def do_corr():
        cst["g"] = trk.fit_corrected(coef=coef)

    cms = timed(do_corr)
    res["corrected_fit"] = {"ms": round(cms, 4), "n_tracks": out.n_tracks,
                            "n_fitted": int((cst["g"]["ndf"] >= 0).sum().item())}
    del cst, out
    # compression residuals (int16 per cluster and coordinate, step 2^-7 cm)
    out = trk.alloc_tracks(dc).want_residuals(-7)
    rms = timed(lambda: trk.track(dc, out, batched=True))
    res["residuals"] = {"ms_per_step": round(rms, 4), "n_tracks": out.n_tracks, "n_hits": out.n_hits}
    print("[bench] next steps: merge %.3f ms, native %.3f ms/step, corrected fit %.3f ms, residuals %.3f ms/step"
          % (mms, nms, cms, rms), file=sys.stderr, flush=True)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="C2x8", choices=sorted(WORKLOADS))
    ap.add_argument("--plain-steps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--autotune", action="store_true", help="pick tiling with tpcca_autotune before timing")
    ap.add_argument("--extra", default="C2,C4,C3", help="comma-separated extra workloads timed in the batched form")
    ap.add_argument("--no-diff", action="store_true", help="skip the differentiable-refit leg (C5)")
    ap.add_argument("--no-next", action="store_true",
                    help="skip the merge / native-input / residuals timings on the headline workload")
    ap.add_argument("--diff-tracks", type=int, default=100000)
    ap.add_argument("--diff-only", action="store_true",
                    help="run only the differentiable-refit leg and print its JSON object")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one device copy of MIB MiB (reference for PMC byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU (--gpus 1): the tracker shards by sector instance with no "
              "communication, so several GPUs run independent instance sets; multi-GPU runs are not measured.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1811_11481_amd import DeviceClusters, Tracker

    if not torch.cuda.is_available():
        print("no HIP device", file=sys.stderr)
        sys.exit(1)
    if args.diff_only:
        print(json.dumps({"differentiable_refit": diff_leg(args, torch, np, synth)}))
        return
    if args.copy_calibration:
        src = torch.empty(args.copy_calibration * (1 << 18), dtype=torch.float32, device="cuda")
        src.fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    t_gen = time.perf_counter()
    cs = synth.generate(args.workload)
    print("[bench] workload %s: %d clusters, %d instances (generated in %.1fs)"
          % (args.workload, cs.n_clusters, cs.n_inst, time.perf_counter() - t_gen), file=sys.stderr, flush=True)
    dc = DeviceClusters.from_host(cs)
    trk = Tracker()
    tuning_note = "default"
    if args.autotune:
        t = trk.autotune(dc, repeats=3)
        tuning_note = "autotuned %s" % t.as_dict()
    out = trk.alloc_tracks(dc)
    for _ in range(args.warmup):
        trk.track(dc, out, batched=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        trk.track(dc, out, batched=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) / args.steps * 1e3
    n_tracks = out.n_tracks
    print("[bench] batched: %.3f ms/step, %d tracks" % (ms, n_tracks), file=sys.stderr, flush=True)

    plain_ms = None
    if not args.no_plain and args.plain_steps > 0:
        trk.track(dc, out, batched=False)
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        for _ in range(args.plain_steps):
            trk.track(dc, out, batched=False)
        torch.cuda.synchronize()
        plain_ms = (time.perf_counter() - p0) / args.plain_steps * 1e3
        assert out.n_tracks == n_tracks
        print("[bench] plain: %.3f ms/step" % plain_ms, file=sys.stderr, flush=True)

    stages, roofline = stage_roofline(trk, dc, cs, args.workload, args.warmup, args.steps)
    copy_gbs = copy_bandwidth(torch)
    roofline["copy_measured_GBps"] = round(copy_gbs, 1)
    roofline["frac_of_copy"] = round(roofline["achieved"] / copy_gbs, 5)
    print("[bench] stages (ms): %s" % {k: v["ms"] for k, v in stages.items()}, file=sys.stderr, flush=True)

    extra = {}
    for wl in [w for w in args.extra.split(",") if w and w != args.workload]:
        ecs = synth.generate(wl)
        edc = DeviceClusters.from_host(ecs)
        eout = trk.alloc_tracks(edc)
        for _ in range(max(1, args.warmup)):
            trk.track(edc, eout, batched=True)
        torch.cuda.synchronize()
        e0 = time.perf_counter()
        ek = max(3, args.steps // 2)
        for _ in range(ek):
            trk.track(edc, eout, batched=True)
        torch.cuda.synchronize()
        ems = (time.perf_counter() - e0) / ek * 1e3
        est, eroof = stage_roofline(trk, edc, ecs, wl, max(1, args.warmup), ek)
        extra[wl] = {"workload": WORKLOADS[wl], "n_clusters": ecs.n_clusters, "n_instances": ecs.n_inst,
                     "ms_per_step": round(ems, 4), "clusters_per_s": round(ecs.n_clusters / (ems * 1e-3), 1),
                     "tracks_per_s": round(eout.n_tracks / (ems * 1e-3), 1), "n_tracks": eout.n_tracks,
                     "steps": ek, "stages": est, "roofline": eroof}
        print("[bench] %s batched: %.3f ms/step" % (wl, ems), file=sys.stderr, flush=True)
        del edc, eout

    nxt = None
    if not args.no_next:
        nxt = next_leg(torch, np, synth, cs, dc, args.warmup, max(3, args.steps // 2))

    diff = None
    if not args.no_diff:
        diff = diff_leg(args, torch, np, synth)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle  # CPU baseline leg only
        nthr = host_threads()
        # bounded sample: about 1.5 M clusters per worker thread (~10-20 s)
        sample, note = cs, "full %s workload" % args.workload
        budget = 1_500_000 * nthr
        if cs.n_clusters > budget:
            k = max(1, int(cs.n_inst * budget / cs.n_clusters))
            sample = cs.subset(list(range(k)))
            note = "first %d of %d sector instances of %s" % (k, cs.n_inst, args.workload)
        c0 = time.perf_counter()
        r = oracle.run(sample, 32, threads=nthr)
        dt = time.perf_counter() - c0
        print("[bench] cpu oracle (%d threads): %.2fs" % (nthr, dt), file=sys.stderr, flush=True)
        # one thread on one central event, for the per-core rate
        one = sample.subset(list(range(min(36, sample.n_inst))))
        c1 = time.perf_counter()
        oracle.run(one, 32, threads=1)
        dt1 = time.perf_counter() - c1
        print("[bench] cpu oracle (1 thread, %d instances): %.2fs" % (one.n_inst, dt1), file=sys.stderr, flush=True)
        # the binary64 oracle on the same one-event sample, one thread (context)
        c2 = time.perf_counter()
        oracle.run(one, 64, threads=1)
        dt2 = time.perf_counter() - c2
        print("[bench] cpu oracle binary64 (1 thread, %d instances): %.2fs" % (one.n_inst, dt2), file=sys.stderr,
              flush=True)
        cpu = {"value": round(sample.n_clusters / dt, 1), "unit": "clusters/s", "cores": nthr, "kind": "oracle",
               "sample": "%s (%d clusters), binary32 oracle, %d worker threads over sector instances"
                         % (note, sample.n_clusters, nthr),
               "seconds": round(dt, 3), "tracks_per_s": round(r.n_tracks / dt, 1),
               "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
               "single_thread": {"clusters_per_s": round(one.n_clusters / dt1, 1), "seconds": round(dt1, 3),
                                 "sample": "first %d instances (%d clusters)" % (one.n_inst, one.n_clusters)},
               "single_thread_binary64": {"clusters_per_s": round(one.n_clusters / dt2, 1),
                                          "seconds": round(dt2, 3)}}

    line = {
        "metric": METRIC,
        "value": round(cs.n_clusters / (ms * 1e-3), 1),
        "unit": "clusters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%s: %s" % (args.workload, WORKLOADS[args.workload]), "n_clusters": cs.n_clusters,
                   "n_instances": cs.n_inst, "form": "batched, HIP graph", "tuning": tuning_note},
        "tracks_per_s": round(n_tracks / (ms * 1e-3), 1),
        "n_tracks": n_tracks,
        "plain_ms_per_step": round(plain_ms, 4) if plain_ms else None,
        "batched_speedup_vs_plain": round(plain_ms / ms, 3) if plain_ms else None,
        "stages": stages,
        "extra_workloads": extra,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "differentiable_refit": diff,
        "next_steps": nxt,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
