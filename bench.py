"""Benchmark of the per-frame hybrid-ocean hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c5]

A step is one frame: FFT background (evolve + two LDS FFT passes), particle
update (subdivide / survive / inject / emit, bin count, scan, scatter) and the
per-bucket splat with the blend epilogue, for every patch of the scene.

The default workload is the stress scene, the largest one that runs on one
GPU: FFT 4096^2 over 8 km, 64 patches of 128^2 to 1024^2 cells at 0.25 m
following their own moving sources, 16 buckets (wavelengths 0.25-64 m),
about 15.5M live particles.  The scene is first pre-rolled (untimed) to
frame 900 of its 1000-frame run so the timed frames see the steady particle
population; then W warm-up frames, then exactly K timed frames.

Printed: one JSON line.  `value` is ms per frame of the production form
(16-byte records, all patches per launch, frame replayed as a hipGraph);
the plain form (32-byte records, launches per patch, no graph) is timed on
the same frames and reported beside it.  `roofline` is for the kernel with
the largest share of the frame, timed with HIP events on the library stream;
`error` is the height error of both forms at the last timed frame against
the FP64 oracle (background, raw and blended maps of every patch);
`cpu_baseline` is the FP64 oracle on a bounded sample of the same frames.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ms/frame & particle splats/s (batched FP16-attr vs plain FP32); FFT GB/s"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
PREROLL = {"c1": 0, "c2": 540, "c3": 900, "c4": 540, "c5": 900, "p0": 3540}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def spin(ocean, n, chunk=100):
    done = 0
    while done < n:
        k = min(chunk, n - done)
        ocean.step(k)
        done += k
    ocean.sync()


def time_frames(ocean, steps):
    import torch
    torch.cuda.synchronize()
    ocean.sync()
    t0 = time.perf_counter()
    ocean.step(steps)
    ocean.sync()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def live_total(ocean, scene):
    tot = 0
    for p in range(len(scene.patches)):
        tot += int(ocean.counts(p, allow_overflow=True)[:, 0].sum())
    return tot


def algorithmic(scene, rec_bytes, n_live):
    """Minimum HBM bytes per launch of each kernel (see the design notes)."""
    N = scene.fft_n
    cells = sum(p.nx * p.ny for p in scene.patches)
    half = (N // 2 + 1) * N
    return {
        "fft_a": N * N * 8 + half * 8,            # h0 read once, half-plane write
        "fft_b": half * 8 + N * N * 4,            # half-plane read, H write
        "count": 0,                               # new particles only: no records read or written
        "scatter": 2 * n_live * rec_bytes,        # read once, written once
        "splat": n_live * rec_bytes + cells * 8,  # records once, two maps written
    }


def splat_flops(ocean, scene):
    """FP32 flops of the splat as a contraction: every crest and trough adds
    A w(d_x) w(d_y) to the cells of its (2 r / dx)^2 square footprint (on
    average), one multiply-add per cell; the radial kernel reaches only the
    disc of radius r, pi/4 of that square.  Radii come from the library's
    bucket table."""
    r = ocean.buckets()[:, 2]
    area = math.pi / 4.0 if getattr(scene, "kernel", 0) == 1 else 1.0
    flops = 0.0
    for p, P in enumerate(scene.patches):
        live = ocean.counts(p, allow_overflow=True)[:, 0]
        for i in range(len(r)):
            rc = r[i] / P.dx
            flops += float(live[i]) * 2.0 * (2.0 * rc) ** 2 * 2.0 * area
    return flops


def layer_work(ocean, scene, rec_bytes, n_live):
    """Algorithmic flops and bytes of the texel-layer stages.  Per (patch,
    bucket) the layer spans the patch plus R = ceil(r / dx) - 1 cells each
    side; the x pass makes (ny + 2R) nx outputs and the y pass ny nx, each a
    (2R + 1)-tap multiply-add.  deposit_x reads every record once and writes
    the x-filtered layers; filter_y reads them and writes one plane per
    bucket; layer_sum reads the planes and writes the two maps."""
    r = ocean.buckets()[:, 2]
    fx = fy = bx = by = bs = 0.0
    for P in scene.patches:
        for ri in r:
            R = max(0, math.ceil(ri / P.dx) - 1)
            rows = P.ny + 2 * R
            fx += 2.0 * rows * P.nx * (2 * R + 1)
            fy += 2.0 * P.ny * P.nx * (2 * R + 1)
            bx += 4.0 * rows * P.nx
            by += 4.0 * rows * P.nx + 4.0 * P.nx * P.ny
            bs += 4.0 * P.nx * P.ny
        bs += 8.0 * P.nx * P.ny
    bx += n_live * rec_bytes
    return {"deposit_x": (fx, bx), "filter_y": (fy, by), "layer_sum": (0.0, bs)}


DOM_KERNEL = {"splat": "k_splat<RecCompact, false, false>", "fft_a": "k_fft_a", "fft_b": "k_fft_b",
              "count": "k_update<RecCompact, 0>", "scatter": "k_update<RecCompact, 1>",
              "deposit_x": "k_deposit_x<RecCompact>", "filter_y": "k_filter_y", "layer_sum": "k_layer_sum"}


def measured_traffic(config, dom, radial=False, tuned=None, bins=None):
    """HBM bytes per launch of the dominant kernel from profiles/traffic.json
    (rocprofv3 FETCH_SIZE and WRITE_SIZE, each scaled by what the counter
    reads for a device copy of known size), or None when there is no entry
    for this workload, kernel, bin edges and splat partition, or the kernel
    sources changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    e = json.load(open(path)).get(config)
    splat_kernel = tuned["plan"].get("splat_kernel", 2) if tuned else 2
    name = DOM_KERNEL.get(dom)
    if dom == "splat":   # the schedule and the crest/trough kernel are template instances
        name = ("k_splat", "k_splat_q", "k_splat_h")[splat_kernel] + \
            ("<RecCompact, true, false>" if radial else "<RecCompact, false, false>")
    if not e or e.get("kernel") != name:
        return None
    if e.get("plan") != (tuned["plan"] if tuned else None) or e.get("bins") != bins:
        return None   # measured with other bin edges or another partition
    h = hashlib.sha256(b"".join(open(os.path.join(ROOT, p), "rb").read() for p in e["sources"])).hexdigest()
    return int(e["bytes_per_launch"]) if h == e["sources_sha256"] else None


def copy_bandwidth(mib=512, reps=10):
    """Achieved device-to-device copy bandwidth (read + write bytes / time),
    the practical ceiling the HBM fractions can also be read against."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    return 2.0 * mib * (1 << 20) / (ms * 1e-3) / 1e9


def splat_bucket_report(prof, splat_ms, ocean, scene, rec_bytes, launches):
    """Per-bucket time of the splat from its in-kernel profile and the
    binding roof of each bucket.  A bucket's time is its share of the
    wavefront ticks (its footprints plus its share of record decoding, by
    points visited) times the splat's time per launch; its algorithmic work
    is its records read once (bytes) and two flops per cell of every crest
    and trough footprint (2 r / dx)^2 (FP32 matrix flops); the binding roof
    is the one whose floor time is larger, and frac = floor / time.  The
    profile holds `launches` launches; points visited are two per record
    entry a tile reads (records near a tile's edge are read by every tile
    their footprints reach)."""
    nb = scene.spectrum.n_buckets
    r = ocean.buckets()[:, 2]
    live = np.zeros(nb)
    area = np.zeros(nb)
    for p, P in enumerate(scene.patches):
        c = ocean.counts(p, allow_overflow=True)[:, 0]
        live += c
        area += c * (2.0 * r / P.dx) ** 2
    bt, pts = prof["bucket"], prof["points"]
    over = prof["setup"] + prof["wait"] + prof["epilogue"]
    tot = over + prof["decode"] + bt.sum()
    rows = []
    for b in range(nb):
        share = (bt[b] + prof["decode"] * pts[b] / max(pts.sum(), 1.0)) / tot
        t = share * splat_ms * 1e-3
        byts = live[b] * rec_bytes
        flops = 2.0 * 2.0 * area[b]
        t_hbm, t_mfma = byts / (HBM_PEAK_GBS * 1e9), flops / (FP32_PEAK_TFLOPS * 1e12)
        bound = "mfma" if t_mfma > t_hbm else "hbm"
        rows.append({"bucket": b, "r_cells": round(float(r[b] / min(P.dx for P in scene.patches)), 2),
                     "live": int(live[b]), "points_visited_per_launch": int(pts[b] / launches),
                     "record_reads_per_particle": round(float(pts[b] / launches / 2.0 / max(live[b], 1.0)), 3),
                     "share": round(float(share), 4), "ms": round(t * 1e3, 5), "bound": bound,
                     "frac": round(max(t_hbm, t_mfma) / t, 5) if t > 0 else None})
    return {"buckets": rows,
            "overhead_share": {k: round(float(prof[k] / tot), 4) for k in ("setup", "wait", "epilogue")},
            "decode_share": round(float(prof["decode"] / tot), 4)}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def cpu_baseline(scene, preroll, nframes):
    """Time the FP64 oracle (one thread) on nframes full frames after the pre-roll."""
    import oracle
    o = oracle.Oracle(scene)
    o.step(preroll)
    t0 = time.perf_counter()
    for _ in range(nframes):
        o.step(1)
        H = o.background()
        for p in range(len(scene.patches)):
            o.patch_maps(p, H)
    dt = time.perf_counter() - t0
    o.close()
    return dt * 1e3 / nframes, dt


def oracle_frame(scene, n, P):
    """One full frame of the FP64 oracle (one thread) on a large scene,
    started from the particle state after step n given as records P (the
    library's state, whose integer part equals the oracle's own bit for bit
    in the full-length parity tests): the background and both maps of every
    patch at step n, then the bookkeeping of step n + 1.  Returns the time,
    the background and the (raw, blended) maps of step n."""
    import oracle
    o = oracle.Oracle(scene)
    o.load(n, P)
    t0 = time.perf_counter()
    H = o.background()
    maps = [o.patch_maps(p, H) for p in range(len(scene.patches))]
    o.step(1)
    dt = time.perf_counter() - t0
    o.close()
    return dt, H, maps


def rel_rms(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.sqrt(np.mean((a - b) ** 2)) / max(np.sqrt(np.mean(b ** 2)), 1e-300))


def height_errors(ocean, scene, H, maps):
    """Height error of a GPU frame against the FP64 oracle, per result:
    background, raw wave-particle map and blended map; relative RMS (the
    largest over patches for the maps) and the largest absolute error (m)."""
    gh = ocean.background()
    out = {"background": {"rel_rms": rel_rms(gh, H), "max_abs": float(np.max(np.abs(gh - H)))}}
    for name, layer, k in (("raw", 1, 0), ("blended", 0, 1)):
        rr = ma = 0.0
        for p in range(len(scene.patches)):
            gm = ocean.patch_map(p, layer)
            rr = max(rr, rel_rms(gm, maps[p][k]))
            ma = max(ma, float(np.max(np.abs(gm - maps[p][k]))))
        out[name] = {"rel_rms": rr, "max_abs": ma}
    return {k: {kk: float(f"{vv:.3e}") for kk, vv in v.items()} for k, v in out.items()}


def bins_for(ocean, scene):
    """Bin edge (cells) per bucket from the library's bucket radii: at least 8
    cells, doubled while below the wavelength (up to 32 cells), and further
    while a 64-cell tile would need more than 32 bin rows."""
    r = ocean.buckets()[:, 2]
    dx = min(p.dx for p in scene.patches)
    out = []
    for ri in r:
        cells = 2.0 * ri / dx
        b = 8
        while (b < cells and b < 32) or (64 + 8.0 * ri / dx) / b + 1 > 32:
            b *= 2
        out.append(b)
    return out


def trends(K, W, synth=0):
    """The paper's default scene (U10 = 5, N_omega = N_theta = 16) over wind
    speed and sampling density, each run to the steady state of its slowest
    waves: the cost trends of the paper's parameter table."""
    import dataclasses
    import torch
    from paper_2511_02852_amd import hwo, scenes
    base = scenes.p0().replace(synth=synth)
    runs = [(u, 16) for u in (3.0, 5.0, 10.0, 15.0)] + [(5.0, 8), (5.0, 12)]
    rows = []
    for u10, ns in runs:
        sp = dataclasses.replace(base.spectrum, U10=u10, n_buckets=ns, eta=float(ns))
        sc = base.replace(spectrum=sp, bins=[32] * ns)
        probe = hwo.Ocean(sc, compact=True, batched=True)
        bins = bins_for(probe, sc)
        c_min = float(probe.buckets()[:, 3].min())
        probe.close()
        sc = sc.replace(bins=bins)
        size = max(p.nx * p.dx for p in sc.patches)
        pre = int(math.ceil(size / (c_min * sc.dt))) + 60
        g = hwo.Ocean(sc, compact=True, batched=True)
        spin(g, pre)
        plan = None
        if synth == 0:
            # the library's own search of the splat partition and schedule
            # on the steady-state frame (the bin edges stay as chosen above)
            plan = g.autotune(4)[0]
        spin(g, W)
        ms = time_frames(g, K)
        live = live_total(g, sc)
        g.close()
        rows.append({"U10": u10, "n_omega": ns, "n_theta": ns, "ms_per_frame": round(ms, 5),
                     "live_particles": live, "preroll_frames": pre, "plan": plan})
        log(f"[trends] U10={u10} N={ns}: {ms:.4f} ms/frame, {live} live particles")
    torch.cuda.synchronize()
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", default="c5")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-error", action="store_true",
                    help="skip the height error against the FP64 oracle")
    ap.add_argument("--no-tune", action="store_true",
                    help="production form with the default bin edges and splat partition (no autotuner)")
    ap.add_argument("--cpu-frames", type=int, default=0)
    ap.add_argument("--trends", action="store_true",
                    help="paper-default scene over wind speeds and sampling densities (Table 2 trends)")
    ap.add_argument("--synth", type=int, default=0,
                    help="height synthesis: 0 exact-position splat, 1 the paper's texel layers")
    ap.add_argument("--kernel", type=int, default=0,
                    help="crest/trough kernel: 0 separable w(dx) w(dy), 1 radial W(|d|) (exact splat only)")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="also run a plain device-to-device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is described in the design notes, not implemented).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2511_02852_amd import hwo, scenes

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.trends:
        rows = trends(args.steps, args.warmup, args.synth)
        print(json.dumps({"metric": "ms/frame of the paper-default scene over U10 and (N_omega, N_theta)",
                          "synthesis": "texel layers + separable passes" if args.synth else "exact-position splat",
                          "unit": "ms/frame", "higher_is_better": False, "n_gpus": 1, "steps": args.steps,
                          "warmup": args.warmup, "data": "synthetic", "trends": rows}), flush=True)
        return
    scene = scenes.get(args.config).replace(synth=args.synth, kernel=args.kernel)
    layers = args.synth == 1
    radial = args.kernel == 1
    preroll = PREROLL.get(args.config, 0)
    K, W = args.steps, args.warmup

    # ---- autotuner: bin edges and splat partition of the production form
    tuned = None
    scene_p = scene
    if not args.no_tune and not layers:
        from paper_2511_02852_amd import autotune
        tuned = autotune.tune(scene, preroll, cache=autotune.TUNED_PATH, log=log)
        scene_p = scene.replace(bins=tuned["bins"])
        log(f"[bench] autotuned: bins {tuned['bins']}, plan {tuned['plan']} "
            f"({tuned['frame_ms']:.4f} vs default {tuned['default_frame_ms']:.4f} ms/frame in the search)")

    # ---- production form: compact records, batched launches, hipGraph replay
    g = hwo.Ocean(scene_p, compact=True, batched=True)
    if tuned:
        autotune.apply(g, tuned)
    spin(g, preroll)
    spin(g, W)
    ms = time_frames(g, K)
    live = live_total(g, scene)
    log(f"[bench] {scene.name}: production form {ms:.4f} ms/frame, {live} live particles")

    # ---- plain form on the same frames
    plain_ms = None
    if not args.no_plain:
        gp = hwo.Ocean(scene, compact=False, batched=False)
        spin(gp, preroll)
        spin(gp, W)
        plain_ms = time_frames(gp, K)
        log(f"[bench] plain form {plain_ms:.4f} ms/frame")

    # ---- the FP64 oracle on the last timed frame: height error of both
    #      forms, and (large scenes) the oracle's time for one full frame
    n_end = preroll + W + K
    big = len(scene.patches) > 1 or preroll > 1000
    error = frame_sec = None
    if not (args.no_error and (args.no_cpu or not big)):
        P = g.particles()
        frame_sec, H_o, maps_o = oracle_frame(scene, n_end, P)
        del P
        if not args.no_error:
            error = {"frame": n_end, "patches": len(scene.patches), "tolerance_rel_rms": 1e-4,
                     "oracle": "FP64 background and maps of every patch at that frame, from the library's "
                               "particle state (integer state equal to the oracle's, full-length parity tests)",
                     "production": height_errors(g, scene, H_o, maps_o)}
            if plain_ms is not None:
                error["plain_fp32"] = height_errors(gp, scene, H_o, maps_o)
            log(f"[bench] height error vs FP64 oracle at frame {n_end}: {error['production']}")
        del H_o, maps_o
    if plain_ms is not None:
        gp.close()

    # ---- per-kernel times with HIP events on the library stream (same frames)
    gt = hwo.Ocean(scene_p, compact=True, batched=True)
    if tuned:
        autotune.apply(gt, tuned)
    spin(gt, preroll)
    spin(gt, W)
    gt.set_timing(True)
    gt.step(K)
    gt.sync()
    st = gt.stage_times()
    gt.set_timing(False)
    live_t = live_total(gt, scene)
    flops = splat_flops(gt, scene)
    lw = layer_work(gt, scene, g.record_bytes, live_t) if layers else None
    # kernels that can be re-launched on the finished frame: mean time per
    # launch over back-to-back launches (no per-launch event overhead)
    rep = ("fft_a", "fft_b", "deposit_x", "filter_y", "layer_sum") if layers else \
        ("fft_a", "fft_b", "splat", "splat_plan", "splat_reduce")
    rep_ms = {k: gt.time_stage(k, 20) for k in rep}
    prof = None
    if not layers:
        # in-kernel per-bucket profile of the splat over K more frames
        gt.set_splat_profile(True)
        gt.step(K)
        gt.sync()
        prof = gt.splat_profile()
        gt.set_splat_profile(False)
        prof_live = gt
    else:
        gt.close()
    per_launch = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in st.items()}
    per_launch.update(rep_ms)
    per_frame = {k: v[0] / K for k, v in st.items()}
    log("[bench] per-kernel ms/frame: " + ", ".join(f"{k}={v:.4f}" for k, v in per_frame.items()))
    log("[bench] back-to-back ms/launch: " + ", ".join(f"{k}={v:.4f}" for k, v in rep_ms.items()))
    rec = g.record_bytes
    alg = algorithmic(scene, rec, live_t)
    N = scene.fft_n
    fft_ms = per_launch["fft_a"] + per_launch["fft_b"]
    fft_bytes = alg["fft_a"] + alg["fft_b"]
    fft_gbs = fft_bytes / (fft_ms * 1e-3) / 1e9 if fft_ms > 0 else None
    splat_ms = (per_launch["deposit_x"] + per_launch["filter_y"] + per_launch["layer_sum"]) if layers \
        else per_launch["splat"]
    splats_per_s = live_t / (splat_ms * 1e-3) if splat_ms > 0 else None
    splat_buckets = None
    if prof is not None:
        splat_buckets = splat_bucket_report(prof, per_launch["splat"], prof_live, scene, g.record_bytes, K)
        prof_live.close()
        log("[bench] splat per bucket (share, frac of binding roof): " +
            ", ".join(f"b{r['bucket']}={r['share']:.3f}/{r['frac']}" for r in splat_buckets["buckets"]))

    # dominant kernel (largest time share) and its roofline: the roof whose
    # floor time (algorithmic bytes / 8 TB/s or flops / FP32 matrix peak) is
    # larger binds the kernel
    cands = ("fft_a", "fft_b", "count", "scatter") + (("deposit_x", "filter_y", "layer_sum") if layers else ("splat",))
    dom = max(cands, key=lambda k: per_frame[k])
    t = per_launch[dom] * 1e-3
    if layers and dom in lw:
        flops_dom, alg[dom] = lw[dom]
    else:
        flops_dom = flops if dom == "splat" else 0.0
    t_hbm = alg[dom] / (HBM_PEAK_GBS * 1e9)
    t_mfma = flops_dom / (FP32_PEAK_TFLOPS * 1e12)
    traffic = measured_traffic(args.config + ("-layers" if layers else "") + ("-radial" if radial else ""), dom,
                               radial, tuned, tuned["bins"] if tuned else None)
    if (layers or radial) and t_mfma > t_hbm:
        # the layer passes and the radial kernel are FP32 vector work (no
        # matrix cores): bound by the vector ALUs, FP32 vector peak 157.3 TFLOP/s
        achieved = flops_dom / t / 1e12 if t > 0 else 0.0
        roofline = {"kernel": dom, "bound": "alu", "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(achieved / FP32_PEAK_TFLOPS, 5), "traffic": traffic,
                    "avg_launch_ms": round(per_launch[dom], 5), "algorithmic_flops_per_launch": int(flops_dom),
                    "algorithmic_bytes_per_launch": int(alg[dom]),
                    "hbm_frac": round(t_hbm / t, 5) if t > 0 else None}
    elif t_mfma > t_hbm:
        achieved = flops / t / 1e12 if t > 0 else 0.0
        roofline = {"kernel": dom, "bound": "mfma", "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(achieved / FP32_PEAK_TFLOPS, 5), "traffic": traffic,
                    "avg_launch_ms": round(per_launch[dom], 5), "algorithmic_flops_per_launch": int(flops),
                    "algorithmic_bytes_per_launch": int(alg[dom]),
                    "hbm_frac": round(t_hbm / t, 5) if t > 0 else None}
    else:
        achieved = alg[dom] / t / 1e9 if t > 0 else 0.0
        roofline = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                    "avg_launch_ms": round(per_launch[dom], 5),
                    "algorithmic_bytes_per_launch": int(alg[dom])}

    # achieved algorithmic bandwidth of the bandwidth-bound kernels, and the
    # copy bandwidth of this device as a second reference
    kernel_gbps = {k: round(alg[k] / (per_launch[k] * 1e-3) / 1e9, 1)
                   for k in ("fft_a", "fft_b", "scatter") if per_launch.get(k, 0.0) > 0}
    copy_gbs = copy_bandwidth()

    if args.copy_mb > 0:
        # reference kernel of known traffic for hardware byte counters:
        # reads and writes exactly copy_mb MiB
        n = args.copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {args.copy_mb} MiB done")
        del src, dst

    cpu = None
    if not args.no_cpu:
        if big and frame_sec is not None:
            cpu = {"value": round(frame_sec * 1e3, 3), "unit": "ms/frame", "cores": 1, "kind": "oracle",
                   "sample": f"one full frame (FP64 FFT background, splat and blend of all "
                             f"{len(scene.patches)} patches at frame {n_end}, then the bookkeeping of frame "
                             f"{n_end + 1}), started from the particle state of frame {n_end}; "
                             f"{frame_sec:.1f} s; one thread of {os.cpu_count()} ({cpu_model()})"}
            log(f"[bench] oracle {frame_sec * 1e3:.1f} ms/frame (one frame)")
        else:
            nf = args.cpu_frames or 200
            cms, csec = cpu_baseline(scene, preroll + W, nf)
            cpu = {"value": round(cms, 3), "unit": "ms/frame", "cores": 1, "kind": "oracle",
                   "sample": f"{nf} full frames (bookkeeping, FP64 FFT background, splat and blend of every "
                             f"patch) after frame {preroll + W}; {csec:.1f} s; one thread of {os.cpu_count()} "
                             f"({cpu_model()})"}
            log(f"[bench] oracle {cms:.1f} ms/frame over {nf} frames")

    out = {
        "metric": METRIC,
        "value": round(ms, 5),
        "unit": "ms/frame",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(ms, 5),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{scene.name}: FFT {N}^2 over {scene.fft_L:g} m, "
                               f"{len(scene.patches)} patch(es), {scene.spectrum.n_buckets} buckets, "
                               f"frames {preroll + W + 1}..{preroll + W + K}",
                   "form": "16-byte records, batched launches, hipGraph"
                           + (", autotuned bin edges and splat partition" if tuned else ""),
                   "synthesis": "texel layers + separable passes" if layers else "exact-position splat",
                   "kernel": "radial" if radial else "separable",
                   "live_particles": live, "preroll_frames": preroll},
        "splats_per_s": round(splats_per_s, 1) if splats_per_s else None,
        "fft_gbps": round(fft_gbs, 2) if fft_gbs else None,
        "plain_fp32_ms_per_frame": round(plain_ms, 5) if plain_ms else None,
        "speedup_vs_plain": round(plain_ms / ms, 3) if plain_ms else None,
        "kernel_ms_per_frame": {k: round(v, 5) for k, v in per_frame.items()},
        "kernel_gbps": kernel_gbps,
        "copy_gbps": round(copy_gbs, 1),
        "kernel_ms_per_launch": {k: round(v, 5) for k, v in per_launch.items()},
        "roofline": roofline,
        "splat_per_bucket": splat_buckets,
        "autotune": None if tuned is None else {
            "bins": tuned["bins"], "plan": tuned["plan"], "cached": tuned["cached"],
            "search_frame_ms": {"tuned": round(tuned["frame_ms"], 5),
                                "default": round(tuned["default_frame_ms"], 5)
                                if tuned["default_frame_ms"] else None}},
        "cpu_baseline": cpu,
        "error": error,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
