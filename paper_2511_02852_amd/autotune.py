"""Autotuner of the splat's work partition and the per-bucket bin edges.

Two kinds of parameters decide how the per-bucket splat is cut into work:

* the bin edge of each bucket (cells), fixed when an ocean is built: the
  counting sort groups particles by bin, and a tile visits the bins within
  reach of its footprints, so the edge trades sort granularity against the
  particles a tile reads without using them;
* the work partition of the batched splat (least cost of a work item, item
  budget per frame, persistent grid size) and which of its three schedules
  runs (batches per wavefront, a quadrant per wavefront, or the hybrid of
  the two), searched on a finished frame by the library itself
  (``hwo_autotune``).

``tune`` builds one ocean per candidate set of bin edges, runs it to the
pre-roll frame, lets the library tune the partition, times whole frames,
and keeps the fastest.  Results are cached as JSON, keyed by the device and
a signature of the scene's inputs, so a later run on the same device and
scene reuses them.  Neither choice changes any integer result other than
the bin histogram itself, nor any height beyond FP32 summation order.
"""
from __future__ import annotations

import dataclasses
import hashlib
import json
import math
import os
import time
from typing import Callable, List, Optional

TILE = 64         # output tile edge (cells)
MAX_ROWS = 32     # bin rows a tile may read per bucket
MIN_BIN, MAX_BIN = 4, 64


def scene_signature(scene) -> str:
    """SHA-256 of the scene's inputs that shape the work: spectrum, patches,
    sources, grid, time step, seed and the synthesis options (not its name,
    run length or bin edges, which are what is tuned)."""
    d = dataclasses.asdict(scene)
    for k in ("name", "steps", "bins"):
        d.pop(k, None)
    return hashlib.sha256(json.dumps(d, sort_keys=True).encode()).hexdigest()


def device_name() -> str:
    """Architecture and compute-unit count of the current device (the
    marketing name and the target-feature suffix of the architecture can
    differ between runtimes on the same part)."""
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(p, "gcnArchName", "") or p.name
    return f"{arch.split(':')[0]}|{p.multi_processor_count}"


def bins_fit(edge: int, r_cells: float) -> bool:
    """A bin edge is usable for a bucket of radius r_cells when the bins a
    tile reads (its crests lie up to 2 r outside the tile, and the survival
    margin adds 2 r to the binned span) fit in MAX_ROWS bin rows, the
    library's limit."""
    return MIN_BIN <= edge <= MAX_BIN and (TILE + 4.0 * r_cells) / edge + 2 <= MAX_ROWS


def bin_candidates(base: List[int], r_cells: List[float]) -> List[List[int]]:
    """The scene's bin edges, all halved and all doubled, each edge pushed up
    to the least usable power of two where needed; duplicates removed."""
    out = []
    for scale in (1.0, 0.5, 2.0):
        cand = []
        for e, r in zip(base, r_cells):
            v = max(MIN_BIN, min(MAX_BIN, int(round(e * scale))))
            while not bins_fit(v, r) and v < MAX_BIN:
                v *= 2
            cand.append(v)
        if cand not in out:
            out.append(cand)
    return out


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def default_cache_path() -> str:
    return os.path.join(os.path.expanduser("~"), ".cache", "hwo_autotune.json")


# Settings tuned on the target device for the benchmark scenes, shipped with
# the package so that timed runs and their hardware-counter profiles use the
# same bin edges and partition (the search itself varies by a few percent
# from run to run); a scene or device without an entry is tuned and added.
TUNED_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")


def _time_frames(ocean, frames: int) -> float:
    import torch
    torch.cuda.synchronize()
    ocean.sync()
    t0 = time.perf_counter()
    ocean.step(frames)
    ocean.sync()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / frames


def _spin(ocean, n: int):
    done = 0
    while done < n:
        k = min(100, n - done)
        ocean.step(k)
        done += k
    ocean.sync()


def tune(scene, preroll: int, cache: Optional[str] = None, reps: int = 8, frames: int = 30,
         search_bins: bool = True, log: Callable[[str], None] = lambda s: None, margin: float = 0.02) -> dict:
    """Bin edges and splat partition for the production form of a scene
    (16-byte records, batched launches, graph replay), from the cache when
    present.  Another set of bin edges, or the partition the library's search
    finds, replaces the scene's own only when its frames are faster by more
    than `margin` (timing noise of a few tens of frames is about that size).  Returns {"bins", "plan", "frame_ms",
    "default_frame_ms", "candidates", "cached"}."""
    from . import hwo
    path = cache or default_cache_path()
    key = f"{device_name()}|{scene_signature(scene)}|{preroll}"
    store = _load(path)
    if key in store:
        out = dict(store[key])
        out["cached"] = True
        return out
    probe = hwo.Ocean(scene, compact=True, batched=True)
    r = probe.buckets()[:, 2]
    probe.close()
    dx = min(p.dx for p in scene.patches)
    base = list(scene.bins) if scene.bins is not None else [16] * len(r)
    cands = bin_candidates(base, [float(ri / dx) for ri in r]) if search_bins else [base]
    results = []
    default_ms = None
    for bins in cands:
        g = hwo.Ocean(scene.replace(bins=bins), compact=True, batched=True)
        _spin(g, preroll)
        # frames with the starting partition, then with the searched one: the
        # search times the splat alone, so its pick is kept only when whole
        # frames are faster with it by more than the margin too (a partition
        # with more parts writes more partial tiles, so a tie keeps the
        # starting one)
        plan0 = g.get_plan()
        ms0 = _time_frames(g, frames)
        if bins == base:
            default_ms = ms0
        plan, best, start = g.autotune(reps)
        ms = _time_frames(g, frames)
        if ms >= ms0 * (1.0 - margin):
            plan, ms = plan0, ms0
        g.close()
        results.append({"bins": bins, "plan": plan, "frame_ms": ms, "splat_ms": best, "splat_ms_start": start})
        log(f"[autotune] bins {bins}: plan {plan}, {ms:.4f} ms/frame")
    best = results[0]   # the scene's own bin edges, with the tuned partition
    for e in results[1:]:
        if e["frame_ms"] < best["frame_ms"] * (1.0 - margin):
            best = e
    out = {"bins": best["bins"], "plan": best["plan"], "frame_ms": best["frame_ms"],
           "default_frame_ms": default_ms, "candidates": results}
    store = _load(path)
    store[key] = out
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(store, f, indent=1)
    os.replace(tmp, path)
    out = dict(out)
    out["cached"] = False
    return out


def apply(ocean, tuned: dict):
    """Set the tuned splat partition on an ocean built with tuned["bins"]."""
    p = tuned["plan"]
    ocean.set_plan(p["chunk_load"], p["items_target"], p["splat_grid"], p.get("splat_kernel", 2))
