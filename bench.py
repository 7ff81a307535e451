"""Benchmark: photon histories per second of one MC forward projection on one GPU.

Workload (default, the largest one-GPU configuration): 512^3 voxel phantom at
0.25 mm with 20 random ellipsoids of water / aluminium / bone-like calcium mix
(densities 0.9 - 2.7 g/cm^3) and an iron cylinder insert in air, 150 kVp
Kramers spectrum behind 2 mm Al in 1 keV bins, source 500 mm from the axis,
2048 x 2048 panel of 0.2 mm at 1000 mm with scatter tallied on 256 x 256,
0.25 mm march step, 1e9 photons per projection; fp32 transport, int64
fixed-point tallies.  `--workload ellipsoids256_poly` (256^3, 512^2 panel,
1e8 photons) and `--workload batch360_uneven16` (the batched launch) are the
other modes.  Inputs are resident in GPU memory before the timed region.  A
"step" is one whole projection: clearing both images and the transport kernel
over all photons.

Output: one JSON line (metric, value, roofline of the transport kernel, CPU
oracle baseline).  `python bench.py --gpus N` with N > 1 exits: the benchmark
measures one GPU.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, published
# 32-bit VALU issue peak (non-packed): 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9
# arithmetic of one fixed-step march step as the transport specifies it:
# advance of the step centre (3 adds), clamp (3) and truncation (3) of the
# voxel coordinates, linear voxel index (2 multiplies, 2 adds), end-of-chord
# test and last-step length selection (2), optical depth (multiply, add) and
# its test against tau* (1)
ALU_OPS_PER_STEP = 18
TALLY_BYTES = 8                  # one int64 atomic add per detected photon
PHANTOMS = {
    "ellipsoids512_hires": "512^3 voxels at 0.25 mm, 20 random ellipsoids (water, Al, bone-Ca; "
                           "0.9-2.7 g/cm^3) and an iron cylinder insert (r 5 mm) in air",
    "ellipsoids256_poly": "256^3 voxels at 0.5 mm, 20 random ellipsoids (water, Al, bone-Ca; "
                          "0.9-2.7 g/cm^3) in air",
    "cylinder64": "64^3 voxels at 1 mm, water cylinder r 25 mm in air",
}

KERNEL_SOURCES = [os.path.join(ROOT, "paper_2201_13191_amd", "csrc", f)
                  for f in ("transport.hip", "kernel_params.hpp")]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def counters_path(workload):
    return os.path.join(ROOT, "profiles", f"transport_{workload}_counters.json")


def measured_traffic(workload):
    """HBM bytes per launch from the committed rocprofv3 counter record, if it
    was taken on this exact kernel source and workload; else None."""
    try:
        rec = json.load(open(counters_path(workload)))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != kernel_source_hash() or rec.get("workload") != workload:
        return None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads():
    """Threads the oracle may use: the CPUs this process may run on, capped by
    OMP_NUM_THREADS where the host sets it (the CPU share given to one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    cap = os.environ.get("OMP_NUM_THREADS", "")
    if cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return max(1, n)


def _time_oracle(o, w, n, threads):
    t = time.perf_counter()
    o.project(w["angle"], n, w["seed"], threads=threads)
    return time.perf_counter() - t


def cpu_baseline(w, seconds):
    """The oracle, unchanged, on the host cores over a bounded photon sample
    (photons 0 .. n-1 of the same projection), and on one thread."""
    import oracle
    threads = host_threads()
    o = oracle.Oracle()
    o.load_phantom(w["ids"], w["rho"], w["voxel_mm"])
    o.set_geometry(**w["geometry"])
    o.set_spectrum(*w["spectrum"])
    n0 = 20_000 * threads
    dt = _time_oracle(o, w, n0, threads)
    n = int(min(max(n0, n0 * seconds / max(dt, 1e-6)), 1e8))
    dt = _time_oracle(o, w, n, threads)
    n1 = 20_000
    dt1 = _time_oracle(o, w, n1, 1)
    n1 = int(min(max(n1, n1 * (seconds / 4) / max(dt1, 1e-6)), 1e7))
    dt1 = _time_oracle(o, w, n1, 1)
    return dict(value=n / dt, unit="photon histories/s", cores=threads, kind="oracle",
                sample=f"photons 0..{n - 1} of the same projection ({n / w['n_photons']:.2%} of "
                       f"one step), {dt:.1f} s wall on {threads} host threads; one thread: "
                       f"photons 0..{n1 - 1} in {dt1:.1f} s",
                single_thread=n1 / dt1, cpu_model=cpu_model(), host_cpus=os.cpu_count())


def roofline(st, gather_bytes, launch_s, workload, kernel):
    """The transport kernel against the gather roofline: algorithmic bytes per
    launch = one voxel lookup of the stored representation per march step
    (1 B palette code, or 5 B material id + density) plus one 8 B int64 add per
    detected photon, over the launch's measured duration, against HBM peak.
    The VALU-issue view (counted march arithmetic per step) is kept beside it."""
    tallies = st["primary_hits"] + st["scatter_hits"]
    alg_bytes = st["steps"] * gather_bytes + tallies * TALLY_BYTES
    gbs = alg_bytes / launch_s / 1e9
    alg_ops = st["steps"] * ALU_OPS_PER_STEP
    tops = alg_ops / launch_s / 1e12
    traffic = measured_traffic(workload)
    return {
        "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": gbs / HBM_PEAK_GBS, "traffic": traffic, "kernel": kernel,
        "algorithmic_bytes_per_launch": alg_bytes, "bytes_per_step": gather_bytes,
        "tally_bytes": TALLY_BYTES, "steps_per_launch": st["steps"],
        "tallies_per_launch": tallies, "launch_ms": launch_s * 1e3,
        "steps_per_history": st["steps"] / max(st["histories"], 1),
        "skipped_fraction": st.get("skipped_steps", 0) / max(st["steps"], 1),
        "traffic_over_algorithmic": (traffic / alg_bytes) if traffic else None,
        "alu": {"achieved": tops, "peak": VALU_PEAK_OPS / 1e12, "unit": "T op/s",
                "frac": tops / (VALU_PEAK_OPS / 1e12), "ops_per_step": ALU_OPS_PER_STEP,
                "algorithmic_ops_per_launch": alg_ops},
    }


def bench_batch(args):
    """Batched persistent launch (hipGraph replay) over the batch workload:
    360 angles of the 256^3 object plus 16 objects of uneven size."""
    import torch
    from paper_2201_13191_amd import inputs, mcx
    log("generating batch workload")
    w = inputs.batch_workload()
    g = mcx.Projector(0)
    g.load_phantom(*w["phantoms"][0])
    handles = [0] + [mcx.mc_phantom_add(g.ctx, ids, rho, h) for ids, rho, h in w["phantoms"][1:]]
    g.set_geometry(**w["geometry"])
    g.set_spectrum(*w["spectrum"])
    geo = w["geometry"]
    per = geo["nu"] * geo["nv"] + geo["snu"] * geo["snv"]
    jobs = [dict(j, phantom=handles[j["phantom"]], primary_offset=i * per,
                 scatter_offset=i * per + geo["nu"] * geo["nv"]) for i, j in enumerate(w["jobs"])]
    out_buf = torch.empty(len(jobs) * per, dtype=torch.int64, device="cuda:0")
    stream = torch.cuda.current_stream()
    n = sum(j["n_photons"] for j in jobs)

    def step():
        mcx.mc_project_batch(g.ctx, jobs, out_buf, out_buf.numel(), flags=mcx.MC_BATCH_GRAPH,
                             stream=stream)

    log("counting pass")
    g.stats(True)
    mcx.mc_project_batch(g.ctx, jobs, out_buf, out_buf.numel(), flags=0, stream=stream)
    torch.cuda.synchronize()
    st = g.stats()
    g.stats(False)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        step()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_s = float(np.mean([a.elapsed_time(b) for a, b in ev])) * 1e-3
    out = {
        "metric": "photon histories/s on 1 GPU (batched persistent launch, hipGraph)",
        "value": n * args.steps / wall, "unit": "photon histories/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w["name"], "jobs": len(jobs), "photons_per_step": n,
                   "objects": "256^3 (360 angles x 1e7) + 16 objects 64^3..384^3 at 0.5 mm",
                   "detector": f"{geo['nu']}x{geo['nv']} at {geo['pu_mm']} mm"},
        "roofline": roofline(st, 1, launch_s, w["name"], "transport_kernel (batch)"),
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    g.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="ellipsoids512_hires")
    ap.add_argument("--photons", type=int, default=0, help="override photons per step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-probe", action="store_true", help="skip the march-ceiling probe")
    ap.add_argument("--no-autotune", action="store_true", help="default launch shape")
    ap.add_argument("--layout", choices=["lane", "shared", "generic"], default="",
                    help="voxel layout instead of the automatic choice")
    ap.add_argument("--launch", default="", metavar="BLOCK,BPC,EVENT_BATCH",
                    help="this launch shape instead of the autotuner's")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--pd-split", type=int, default=20,
                    help="point-detector pseudo-particles per scattering (0: skip that part)")
    ap.add_argument("--pd-rr", type=float, default=1.0,
                    help="roulette threshold, keV (0: no roulette)")
    ap.add_argument("--pd-point-only", dest="pd_mixed", action="store_false",
                    help="the point detector also for Rayleigh events (default: mixed, Rayleigh "
                         "pseudo-particles along their own law)")
    ap.add_argument("--pd-launch", default="", metavar="BLOCK,BPC,EVENT_BATCH",
                    help="launch shape for the point-detector runs (default: the analog one)")
    ap.add_argument("--pd-fraction", type=float, default=0.1,
                    help="point-detector photons as a fraction of the step's")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (three times), "
                         "to scale HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (projections "
              "and photon-id ranges would shard across GPUs without communication, the images "
              "summed once at the end)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2201_13191_amd import inputs, mcx, metrics
    if not torch.cuda.is_available():
        sys.exit("bench.py needs a GPU")
    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes}), flush=True)
        return

    if args.workload == "batch360_uneven16":
        bench_batch(args)
        return
    log("generating workload", args.workload)
    w = inputs.workload(args.workload)
    n = args.photons or w["n_photons"]
    g = mcx.Projector(0)
    if args.layout:
        g.set_layout({"lane": mcx.MC_LAYOUT_PALETTE_LANE, "shared": mcx.MC_LAYOUT_PALETTE_SHARED,
                      "generic": mcx.MC_LAYOUT_GENERIC}[args.layout])
    # set-up, outside the timed region and reported on its own: the object's
    # upload (with its layout and uniform-cell map) and the geometry and tables
    t_s = time.perf_counter()
    g.load_phantom(w["ids"], w["rho"], w["voxel_mm"])
    t_p = time.perf_counter()
    g.set_geometry(**w["geometry"])
    g.set_spectrum(*w["spectrum"])
    t_t = time.perf_counter()
    geo = w["geometry"]
    dev = torch.device("cuda:0")
    prim = torch.empty((geo["nv"], geo["nu"]), dtype=torch.int64, device=dev)
    scat = torch.empty((geo["snv"], geo["snu"]), dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()
    setup = {"load_phantom_s": t_p - t_s, "geometry_and_tables_s": t_t - t_p}
    log(f"set-up: phantom {setup['load_phantom_s']:.2f} s, geometry and tables "
        f"{setup['geometry_and_tables_s']:.3f} s")

    def step():
        mcx.mc_project_async(g.ctx, w["angle"], n, w["seed"], prim, scat, stream)

    # launch shape from the autotuner (untimed; every candidate is checked
    # bitwise against the first, the choice cached in the temp directory)
    tuning = None
    if args.launch:
        blk, bpc, eb = (int(x) for x in args.launch.split(","))
        g.set_launch(blk, bpc, eb)
        log(f"launch shape set: block {blk}, blocks/CU {bpc}, event batch {eb}")
    elif not args.no_autotune:
        import tempfile
        log("autotune")
        # tuned on the step itself: the photon count sets how much of a launch
        # is its tail, so a shorter run can prefer another shape
        tuning = mcx.mc_autotune(g.ctx, w["angle"], n, w["seed"] + 7,
                                 os.path.join(tempfile.gettempdir(), "mcx_tune.jsonl"))
        log(f"autotune: block {tuning['block']}, blocks/CU {tuning['blocks_per_cu']}, event batch "
            f"{tuning['event_batch']}, table layout {tuning['table_layout']}, "
            f"{tuning['candidates']} candidates, {tuning['rejected']} rejected")

    launch_shape = ((blk, bpc, eb) if args.launch else
                    (tuning["block"], tuning["blocks_per_cu"], tuning["event_batch"]) if tuning
                    else (0, 0, 0))

    # exact algorithmic work of one step (untimed counting pass)
    log("counting pass")
    g.stats(True)
    step()
    torch.cuda.synchronize()
    st = g.stats()
    g.stats(False)
    layout, n_pal = g.layout()
    gather_bytes = 1 if layout != mcx.MC_LAYOUT_GENERIC else 5   # bytes per voxel lookup

    log("warmup", args.warmup)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    log("timed", args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        step()
        b.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    step_ms = [a.elapsed_time(b) for a, b in ev]
    launch_s = float(np.mean(step_ms)) * 1e-3
    log(f"{n * args.steps / wall:.4g} histories/s, {launch_s * 1e3:.2f} ms per step (events), "
        f"steps/history {st['steps'] / max(st['histories'], 1):.1f}")

    # end to end through the blocking entry point: host images (clear, launch,
    # copy back over PCIe); reported beside the value, never as it
    pg, sg = g.images()
    mcx.mc_project(g.ctx, w["angle"], n, w["seed"], pg, sg)
    t_e = time.perf_counter()
    for _ in range(2):
        mcx.mc_project(g.ctx, w["angle"], n, w["seed"], pg, sg)
    end_to_end_ms = (time.perf_counter() - t_e) / 2 * 1e3
    log(f"mc_project with host images: {end_to_end_ms:.2f} ms")

    # plain MC's own noise: a second projection with another seed gives the
    # scatter map's rel-RMS r(n) at n photons (the two maps are independent with
    # the same mean), so plain MC reaches 2 % at n (r / 0.02)^2 photons
    p1, s1 = prim.clone(), scat.clone()
    mcx.mc_project_async(g.ctx, w["angle"], n, w["seed"] + 1, prim, scat, stream)
    torch.cuda.synchronize()
    r = metrics.pair_rel_rms(s1.cpu().numpy(), scat.cpu().numpy())
    n2 = n * (r / 0.02) ** 2
    plain_2pct = {"scatter_rel_rms_at_step": r, "photons_for_2pct": n2,
                  "seconds_for_2pct": n2 / (n * args.steps / wall),
                  "method": "two independent projections (seeds s, s+1) of the step's photon "
                            "count; r^2 = (|a-b|^2 / 2) / ((|a|^2 + |b|^2) / 2 - |a-b|^2 / 2)"}
    log(f"plain MC scatter rel-RMS {r:.4f} at {n:.3g} photons: 2 % needs {n2:.3g} photons, "
        f"{plain_2pct['seconds_for_2pct']:.2f} s")
    del p1

    # the paper's scorer: point-detector scatter estimates (eq. (3)-(5)) with
    # splitting and roulette, two seeds of a smaller photon count, timed on the
    # launch stream; its time to a 2 % scatter map against plain MC's
    pd = None
    if args.pd_split > 0:
        n_pd = max(1, int(n * args.pd_fraction))
        g.set_estimator(mcx.MC_SCORE_POINT_MIXED if args.pd_mixed else mcx.MC_SCORE_POINT,
                        args.pd_split, args.pd_rr)
        pd_tuning = None
        if args.pd_launch:
            g.set_launch(*[int(v) for v in args.pd_launch.split(",")])
        elif tuning is not None:
            # the analog shape came from the autotuner: tune the point-detector
            # kernel too (its own candidates, checked bitwise; not cached, the
            # cache key does not tell the estimators apart)
            log("autotune (point detector)")
            pd_tuning = mcx.mc_autotune(g.ctx, w["angle"], n_pd, w["seed"] + 9, None)
            log(f"autotune (point detector): block {pd_tuning['block']}, blocks/CU "
                f"{pd_tuning['blocks_per_cu']}, event batch {pd_tuning['event_batch']}, "
                f"table layout {pd_tuning['table_layout']}")
        mcx.mc_project_async(g.ctx, w["angle"], n_pd, w["seed"], prim, scat, stream)
        torch.cuda.synchronize()
        imgs, times = [], []
        for sd in (w["seed"] + 2, w["seed"] + 3):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            mcx.mc_project_async(g.ctx, w["angle"], n_pd, sd, prim, scat, stream)
            b.record(stream)
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b) * 1e-3)
            imgs.append(scat.cpu().numpy())
        g.set_estimator(mcx.MC_SCORE_ANALOG)
        if args.pd_launch or pd_tuning:
            g.set_launch(*launch_shape)
            if tuning is not None:
                tl = tuning["table_layout"]
                g.set_layout(mcx.MC_LAYOUT_AUTO if tl == mcx.MC_LAYOUT_PALETTE_LANE else tl)
        t_pd = float(np.mean(times))
        r_pd = metrics.pair_rel_rms(*imgs)
        n2_pd = n_pd * (r_pd / 0.02) ** 2
        pd = {"estimator": "mixed" if args.pd_mixed else "point", "split": args.pd_split,
              "roulette_kev": args.pd_rr, "photons": n_pd,
              "launch": ({k: pd_tuning[k] for k in ("block", "blocks_per_cu", "event_batch",
                                                     "table_layout")} if pd_tuning else
                         args.pd_launch or "as the analog step"),
              "ms_per_projection": t_pd * 1e3, "histories_per_s": n_pd / t_pd,
              "scatter_rel_rms": r_pd, "photons_for_2pct": n2_pd,
              "seconds_for_2pct": n2_pd * t_pd / n_pd,
              "speedup_vs_plain_mc": plain_2pct["seconds_for_2pct"] / (n2_pd * t_pd / n_pd)}
        log(f"point detector (split {args.pd_split}): {t_pd * 1e3:.1f} ms per {n_pd:.3g} photons, "
            f"scatter rel-RMS {r_pd:.4f}; 2 % in {pd['seconds_for_2pct']:.3f} s "
            f"({pd['speedup_vs_plain_mc']:.1f}x plain MC)")

    # march probe: the fixed-step march of straight rays alone (no physics)
    probe = None
    if not args.no_probe:
        log("march probe")
        best = None
        n_rays = 30_000_000
        d = torch.zeros(2, dtype=torch.int64, device=dev)
        for bpc, refill in ((0, 8), (0, 16), (0, 40), (8, 16), (8, 40)):
            g.set_launch(0, bpc, 0)
            mcx.mc_march_probe_async(g.ctx, w["angle"], n_rays, w["seed"], refill, d, stream)
            torch.cuda.synchronize()
            d.zero_()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(3):
                mcx.mc_march_probe_async(g.ctx, w["angle"], n_rays, w["seed"], refill, d, stream)
            b.record(stream)
            torch.cuda.synchronize()
            rate = int(d[1].item()) / (a.elapsed_time(b) * 1e-3)
            if best is None or rate > best[0]:
                best = (rate, refill, bpc)
        g.set_launch(0, 0, 0)
        # the probe gathers every step; compare the transport's executed lookups
        t_rate = (st["steps"] - st.get("skipped_steps", 0)) / launch_s
        # and, beside it, the march steps the transport advances its photons by
        # (uniform runs included) against the probe's
        s_rate = st["steps"] / launch_s
        probe = {"steps_per_s": best[0], "refill_batch": best[1],
                 "blocks_per_cu": best[2] or "occupancy", "rays": n_rays,
                 "gather_GBs": best[0] * gather_bytes / 1e9,
                 "transport_lookups_per_s": t_rate, "frac": t_rate / best[0],
                 "transport_steps_per_s": s_rate, "steps_frac": s_rate / best[0]}
        log(f"march probe {best[0]:.4g} steps/s (refill {best[1]}), transport "
            f"{t_rate:.4g} voxel lookups/s = {t_rate / best[0]:.1%}")

    # tally probe: int64 atomic adds alone, spread over an image of the primary's size
    tally = None
    if not args.no_probe:
        log("tally probe")
        n_pix = geo["nu"] * geo["nv"]
        n_adds = 200_000_000
        img = torch.zeros(n_pix, dtype=torch.int64, device=dev)
        mcx.mc_atomic_probe_async(g.ctx, n_adds, 1, img, n_pix, stream)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(3):
            mcx.mc_atomic_probe_async(g.ctx, n_adds, 1, img, n_pix, stream)
        b.record(stream)
        torch.cuda.synchronize()
        rate = 3 * n_adds / (a.elapsed_time(b) * 1e-3)
        t_adds = (st["primary_hits"] + st["scatter_hits"]) / launch_s
        tally = {"adds_per_s": rate, "pixels": n_pix, "transport_adds_per_s": t_adds,
                 "frac": t_adds / rate}
        log(f"tally probe {rate:.4g} int64 adds/s, transport {t_adds:.4g} = {t_adds / rate:.2%}")

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline")
        cpu = cpu_baseline(w, args.cpu_seconds)

    out = {
        "metric": "photon histories/s on 1 GPU; time to scatter map at \u22642% rel-RMS vs plain MC",
        "value": n * args.steps / wall,
        "unit": "photon histories/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "phantom": PHANTOMS.get(args.workload, args.workload),
            "spectrum": f"{len(w['spectrum'][0])} bins",
            "detector": f"{geo['nu']}x{geo['nv']} at {geo['pu_mm']} mm, scatter "
                        f"{geo['snu']}x{geo['snv']}",
            "photons_per_step": n,
            "step_mm": geo["step_mm"],
            "tallies": "int64 fixed point",
            "launch": ({k: tuning[k] for k in ("block", "blocks_per_cu", "event_batch",
                                                "table_layout", "from_cache")} if tuning else
                       args.launch or "default"),
        },
        "roofline": dict(roofline(st, gather_bytes, launch_s, args.workload, "transport_kernel"),
                         layout={0: "auto", 1: "palette-lane", 2: "palette-shared",
                                 3: "generic"}[layout],
                         march_probe=probe, tally_probe=tally),
        "time_to_2pct_plain_mc": plain_2pct,
        "time_to_2pct_point_detector": pd,
        "cpu_baseline": cpu,
        "setup": setup,
        "end_to_end": {"entry": "mc_project (host images)", "ms": end_to_end_ms,
                       "histories_per_s": n / (end_to_end_ms * 1e-3)},
    }
    print(json.dumps(out), flush=True)
    g.close()


if __name__ == "__main__":
    main()
