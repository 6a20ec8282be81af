"""Autotuner of the volume kernels' launch shapes.

Results never depend on the tile shape (the tests check it bitwise); only
the time does.  The tuner times candidates on the device with HIP events and
caches the winner per GPU architecture and workload class in a JSON file
next to this module (``tuning_cache.json``):

* plain path: bins per thread, pixels per workgroup and per wavefront row of
  the fusion and the band width of its tile order for a (K, D, width, height)
  class: a launch shape the caller
  passes with each call (``tuning=`` of the volume calls, the C ABI's
  ``gg_volume_tuning``); nothing is set process-wide;
* batched path: (pixels per fusion workgroup, resident workgroups per
  compute unit of the persistent splat binning, bins per thread, graph
  branches) for a batch signature.
"""
from __future__ import annotations

import json
import os
import time

import torch

from . import ops

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning_cache.json")

# (pixels per workgroup, pixels per wavefront row, bins per thread, band width of the tile
# order in pixels); 0 = default
PLAIN_CANDIDATES = [(0, 0, 4, 0), (8, 8, 4, 0), (16, 8, 4, 0), (16, 16, 4, 0), (32, 8, 4, 0),
                    (32, 16, 4, 0), (0, 0, 8, 0), (16, 16, 8, 0), (32, 16, 8, 0), (32, 32, 8, 0),
                    (64, 16, 8, 0), (64, 32, 8, 0), (16, 16, 8, 128), (16, 16, 8, 192),
                    (16, 16, 8, 512), (16, 16, 8, 65536), (32, 16, 8, 128)]
# (target pixels per fusion workgroup, resident workgroups per compute unit of
# the persistent splat binning phases, bins per thread, graph branches);
# 0 = default
BATCH_CANDIDATES = [(16, 0, 8, 2), (16, 0, 8, 1), (32, 0, 8, 2), (16, 1, 8, 2), (16, 2, 8, 2),
                    (16, 0, 4, 2), (32, 0, 4, 2)]


def arch(device=None) -> str:
    p = torch.cuda.get_device_properties(device or torch.device("cuda:0"))
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def _load():
    if os.path.exists(CACHE):
        with open(CACHE) as f:
            return json.load(f)
    return {}


def _save(c):
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def _time(fn, reps=5, warm=2):
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(reps):
        s.record()
        fn()
        e.record()
        e.synchronize()
        best = min(best, s.elapsed_time(e))
    return best


def plain_key(K, D, width, height):
    return f"plain-b/K{K}/D{D}/{width}x{height}"


def tune_plain(src, depth, tgt, params, reps=5, use_cache=True):
    """Best (pixels per workgroup, pixels per row, bins per thread, band width) of
    tsdf_integrate for this class; returns (best, {candidate: ms}), best to
    be passed as ``tuning=`` to the volume calls."""
    tg, tp = ops.camera(tgt), ops.tsdf_params(params)
    key = plain_key(len(src), tp.num_bins, tg.width, tg.height)
    cache = _load()
    a = arch(depth.device)
    if use_cache and key in cache.get(a, {}):
        return tuple(cache[a][key]["best"]), cache[a][key]["times"]
    F, W, _, _ = ops.tsdf_integrate(src, depth, tgt, params)
    times = {}
    for cand in PLAIN_CANDIDATES:
        times[",".join(map(str, cand))] = _time(lambda: ops.tsdf_integrate(
            src, depth, tgt, params, F_prev=F, W_prev=W, F=F, W=W, tuning=cand), reps)
    best = tuple(int(v) for v in min(times, key=times.get).split(","))
    cache.setdefault(a, {})[key] = {"best": list(best), "times": times, "when": time.time()}
    _save(cache)
    return best, times


def tune_plain_step(step, first, reps=8, warm=2):
    """Best launch shape of the fusion for a whole step of the caller's
    pipeline (``step(i, tuning)`` runs frame i with that launch shape,
    perhaps on several streams, where the fusion shares the device with
    other work): each candidate is timed over ``reps`` steps after ``warm``
    untimed ones.  Returns (best, {candidate: ms per step}, next frame
    index)."""
    times = {}
    i = first
    for cand in PLAIN_CANDIDATES:
        for _ in range(warm):
            step(i, tuning=cand)
            i += 1
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            step(i, tuning=cand)
            i += 1
        torch.cuda.synchronize()
        times[",".join(map(str, cand))] = (time.perf_counter() - t0) * 1e3 / reps
    best = tuple(int(v) for v in min(times, key=times.get).split(","))
    return best, times, i


def batch_signature(items):
    """The batch's items by view count, bins, target size, splat and their own fusion launch
    shapes (an item's ``volume``, if any)."""
    def own(it):
        v = ops.volume_tuning(it.get("volume"))
        return "" if v is None else "/v%d,%d,%d,%d" % (v.pixels_per_block, v.pixels_per_row,
                                                        v.bins_per_thread, v.band_width)
    sig = sorted((len(it["src"]), ops.tsdf_params(it["tsdf"]).num_bins,
                  ops.camera(it["tgt"]).width, ops.camera(it["tgt"]).height,
                  it.get("rgb") is not None, own(it)) for it in items)
    return "batch-v/" + ";".join("K%dD%d/%dx%d/%d%s" % s for s in sig)


def tune_batch(items, reps=3, use_cache=True):
    """Best (pixels_per_block, blocks_per_cu, bins_per_thread, branches) for this batch (one plan per
    candidate over the same buffers, each closed before the next).
    Returns (tuning, {candidate: ms})."""
    key = batch_signature(items)
    cache = _load()
    a = arch(items[0]["depth"].device)
    if use_cache and key in cache.get(a, {}):
        return tuple(cache[a][key]["best"]), cache[a][key]["times"]
    times = {}
    for cand in BATCH_CANDIDATES:
        plan = ops.BatchPlan(items, *cand)
        times[",".join(map(str, cand))] = _time(plan.launch, reps)
        plan.close()
    best = min(times, key=times.get)
    tun = tuple(int(v) for v in best.split(","))
    cache.setdefault(a, {})[key] = {"best": list(tun), "times": times, "when": time.time()}
    _save(cache)
    return tun, times
