"""Throughput of the geometry stage on one MI355X.

Workload (the metric's configuration): a 16-camera ring (radius 1 m, aimed
inward), K = 4 input views of 1280x720 FP32 depth + uint8 RGB, target view
between two ring cameras, D = 128 inverse-depth bins over 0.5-5 m, truncation
4 bins, decay 0.9, weight cap 32; a 30-frame sequence of 5 moving spheres over
a textured floor, 1% depth noise, 2% holes.  All 30 frames are resident in HBM
before timing starts.  One step = one frame of the whole hot path:
splat_views (K views into the target) + tsdf_integrate (fusion weight map,
fusion into the carried 1280x720x128 volume, fused zero-crossing extraction).

Prints one JSON line: target-view Mpix/s, the roofline of the dominant kernel
(the fusion) measured with HIP events inside the timed region, the
backward/forward time ratio on the differentiation workload, and the CPU
oracle's throughput on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import multiprocessing as mp
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import scenes  # noqa: E402

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
VALU_PEAK_TLANE = 256 * 64 * 2.4e9 / 1e12  # T lane-instructions/s: 256 CUs x 64 lanes x 2.4 GHz
WORKLOAD = "video ring K=4 1280x720 D=128 (30 frames, carried volume)"


def _frame(t):
    c = scenes.config2(seed=0)
    return c["seq"].frame(t)


def make_frames(n, procs):
    if procs > 1:
        with mp.get_context("fork").Pool(procs) as pool:
            out = pool.map(_frame, range(n))
    else:
        out = [_frame(t) for t in range(n)]
    return np.stack([o[0] for o in out]), np.stack([o[1] for o in out])


def measure_copy_gbs(torch, dev, mib=1024, reps=10):
    """Device-to-device copy bandwidth (bytes read + written per second, GB/s) of a
    `mib` MiB tensor, timed with HIP events on the current stream."""
    n = mib * (1 << 20) // 4
    a = torch.ones(n, device=dev)
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * n * 4 / (ms * 1e-3) / 1e9


def kernel_sha():
    h = hashlib.sha256()
    for name in ("tsdf.hip", "tsdf_device.h", "ggeom_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2505_18932_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def recorded_traffic():
    """Per-launch HBM bytes of the fusion kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "integrate_video_1280x720_K4_D128_counters.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"kernel_sha:\s*([0-9a-f]+)", txt)
    b = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m or not b or m.group(1) != kernel_sha():
        return None
    return float(b.group(1))


def recorded_valu_instructions():
    """Wavefront VALU instructions per launch of the fusion kernel
    (SQ_INSTS_VALU) from the committed counter summary, if it was taken on
    the current kernel source."""
    path = os.path.join(ROOT, "profiles", "integrate_video_1280x720_K4_D128_counters.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"kernel_sha:\s*([0-9a-f]+)", txt)
    v = re.search(r"valu_instructions_per_launch:\s*([0-9.eE+]+)", txt)
    if not m or not v or m.group(1) != kernel_sha():
        return None
    return float(v.group(1))


# The fusion launch shape the main leg tuned (or --tile), passed with every later fusion call of
# this script (the library keeps no launch shape of its own).
TILE = [None]


def _oracle_frames(oracle, c, frames, carry):
    """Wall seconds of the oracle's forward (splat, fusion with the volume
    carried from frame to frame when ``carry``, extraction) over ``frames``
    ((depth, rgb) pairs, generated beforehand)."""
    t0 = time.perf_counter()
    F = W = None
    for d, r in frames:
        oracle.splat(c["src"], d, r, c["tgt"], c["splat"])
        if carry:
            F, W = oracle.integrate(c["src"], d, c["tgt"], c["tsdf"], F_prev=F, W_prev=W)
        else:
            F, W = oracle.integrate(c["src"], d, c["tgt"], c["tsdf"])
        oracle.extract(F, W, c["tsdf"])
    return time.perf_counter() - t0


def cpu_plan(procs):
    """The CPU oracle's timing plan, whole frames of the forward (splat +
    fusion + extraction) on all host cores, scene generation excluded:
    the two parallel-rig scenes in full, the video sequence's 30 frames with
    the volume carried, the 24 batching items in sequence, and 3 frames of
    the streaming sequence extrapolated to its 300 (labelled as such).  No
    GPU work.  Returns one record per workload."""
    import oracle

    cores = oracle.num_threads()
    out = {"cores": cores, "cpu": _cpu_model(), "kind": "oracle", "unit": "Mpix/s"}

    def rec(name, c, frames, carry, note, extrapolate_to=None):
        el = _oracle_frames(oracle, c, frames, carry)
        npix = c["tgt"].width * c["tgt"].height * len(frames)
        r = {"frames": len(frames), "seconds": round(el, 2),
             "mpix_s": round(npix / el / 1e6, 4), "ms_per_frame": round(el * 1e3 / len(frames), 1),
             "workload": note}
        if extrapolate_to:
            r["extrapolated_seconds_%d_frames" % extrapolate_to] = round(
                el / len(frames) * extrapolate_to, 1)
        out[name] = r
        print("# cpu plan: %s %s" % (name, r), file=sys.stderr, flush=True)

    for name, cfg in (("tiny_320x240_K2_D64", scenes.config1()),
                      ("differentiation_640x360_K4_D96", scenes.config3())):
        rec(name, cfg, [(cfg["depth"], cfg["rgb"])], False, "one frame, in full")
    c2 = scenes.config2(seed=0)
    f2 = make_frames(30, procs)
    rec("video_1280x720_K4_D128", c2, list(zip(f2[0], f2[1])), True,
        "all 30 frames of the video sequence, volume carried")
    descs = scenes.config4_items()
    if procs > 1:
        with mp.get_context("fork").Pool(procs) as pool:
            items = pool.map(scenes.config4_item, descs)
    else:
        items = [scenes.config4_item(d) for d in descs]
    t0 = time.perf_counter()
    px = 0
    for it in items:
        _oracle_frames(oracle, it, [(it["depth"], it["rgb"])], False)
        px += it["tgt"].width * it["tgt"].height
    el = time.perf_counter() - t0
    out["batch_24_items"] = {"frames": len(items), "seconds": round(el, 2),
                             "mpix_s": round(px / el / 1e6, 4),
                             "workload": "the 24 batching items in sequence, each one frame"}
    print("# cpu plan: batch %s" % out["batch_24_items"], file=sys.stderr, flush=True)
    c5, d5, r5 = streaming_sequence(procs, 3)
    rec("streaming_1920x1080_K8_D256", c5, list(zip(d5, r5)), True,
        "3 consecutive frames of the streaming sequence, volume carried; seconds for its 300 "
        "frames extrapolated from them", extrapolate_to=300)
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def fusion_stream_probe_ms(gg, torch, dev, tgt, tp, F, W, reps=10):
    """Mean duration of the fusion kernel launched with no views on the
    volume (F, W) in place (gg_fusion_stream_probe), HIP events on the
    current stream."""
    H, Wd = F.shape[0], F.shape[1]
    od = torch.empty((H, Wd), device=dev)
    ob = torch.empty((H, Wd), dtype=torch.int32, device=dev)
    ws = torch.empty(gg.workspace_size(3, 1, 1, 1, Wd, H, tp.num_bins), dtype=torch.uint8,
                     device=dev)
    for _ in range(2):
        gg.ops.fusion_stream_probe(tgt, tp, F, W, F, W, od, ob, ws=ws, tuning=TILE[0])
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        gg.ops.fusion_stream_probe(tgt, tp, F, W, F, W, od, ob, ws=ws, tuning=TILE[0])
    e.record()
    e.synchronize()
    return s.elapsed_time(e) / reps


def cpu_baseline(c, depth, rgb, budget_s=12.0, max_frames=30):
    """The CPU oracle (plain C, OpenMP) on the same workload: whole frames
    (splat + fusion with carry + extraction) in sequence until the time
    budget is used (a bounded sample of the sequence)."""
    import oracle

    t0 = time.perf_counter()
    F = W = None
    frames = 0
    while frames < min(max_frames, len(depth)):
        oracle.splat(c["src"], depth[frames], rgb[frames], c["tgt"], c["splat"])
        F, W = oracle.integrate(c["src"], depth[frames], c["tgt"], c["tsdf"], F_prev=F, W_prev=W)
        oracle.extract(F, W, c["tsdf"])
        frames += 1
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    npix = c["tgt"].width * c["tgt"].height
    cores = oracle.num_threads()
    # one frame on one thread (the oracle's serial speed)
    oracle.set_threads(1)
    t1 = time.perf_counter()
    oracle.splat(c["src"], depth[0], rgb[0], c["tgt"], c["splat"])
    F1, W1 = oracle.integrate(c["src"], depth[0], c["tgt"], c["tsdf"])
    oracle.extract(F1, W1, c["tsdf"])
    el1 = time.perf_counter() - t1
    oracle.set_threads(cores)
    return {"value": round(frames * npix / el / 1e6, 4), "unit": "Mpix/s",
            "cores": cores, "kind": "oracle",
            "sample": f"{frames} full frame(s) of the same sequence (splat + fusion + "
                      f"extraction), {el:.1f} s",
            "single_thread": {"value": round(npix / el1 / 1e6, 4), "unit": "Mpix/s",
                              "sample": f"frame 0 without carry, {el1:.1f} s"}}


STREAM_FRAMES = 30


def streaming_sequence(procs, frames=STREAM_FRAMES):
    """Frames 0 .. frames-1 of the streaming workload (1920x1080, K=8, D=256,
    20 moving spheres and 2 rotating boxes): each view ray-cast at half
    resolution and repeated to the full maps, noise and holes per full pixel
    (scenes.coarse_frame: 30 x 8 full-resolution ray casts would take the
    host minutes)."""
    c = scenes.config5()
    fr = [scenes.coarse_frame(c["seq"], t, 2, procs) for t in range(frames)]
    return c, np.stack([d for d, _ in fr]), np.stack([r for _, r in fr])


def streaming_leg(gg, torch, dev, c, depth_h, rgb_h, warm=3, tile=None):
    """The streaming workload as a sequence: every frame runs the forward
    (splat, fusion with the volume carried in place, fused extraction) and
    the backward (the three adjoints for fixed random upstream gradients),
    on one stream, HIP events around each half.  The fusion takes ``tile``,
    else the launch shape the autotuner picks for this workload.  Returns
    per-frame means."""
    src, tgt, sp, tp = c["src"], c["tgt"], c["splat"], c["tsdf"]
    nf = depth_h.shape[0]
    depth = torch.from_numpy(depth_h).to(dev)
    rgb = torch.from_numpy(rgb_h).to(dev)
    K, Hs, Ws = depth.shape[1], depth.shape[2], depth.shape[3]
    H, Wd, D = tgt.height, tgt.width, tp["num_bins"]
    F = torch.zeros((H, Wd, D), device=dev)
    Wv = torch.zeros_like(F)
    ws_t = torch.empty(gg.workspace_size(3, K, Ws, Hs, Wd, H, D), dtype=torch.uint8, device=dev)
    ws_b = torch.empty(gg.workspace_size(4, K, Ws, Hs, Wd, H, D), dtype=torch.uint8, device=dev)
    ws_s = torch.empty(gg.workspace_size(1, K, Ws, Hs, Wd, H, 2, gg.splat_params(sp)),
                       dtype=torch.uint8, device=dev)
    if tile is None:
        from paper_2505_18932_amd import autotune
        tile = autotune.tune_plain(src, depth[0], tgt, tp, reps=3, use_cache=False)[0]
    so = gg.splat_views(src, depth[0], rgb[0], tgt, sp, ws=ws_s)
    g_rgb, g_z, g_a = (torch.randn_like(so["rgb"]), torch.randn_like(so["depth"]),
                       torch.randn_like(so["alpha"]))
    gdep = torch.randn((H, Wd), device=dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    fwd_ms, bwd_ms = [], []

    def frame(t, carry, timed):
        ev[0].record()
        gg.splat_views(src, depth[t], rgb[t], tgt, sp, out=so, ws=ws_s)
        kw = dict(F_prev=F, W_prev=Wv) if carry else {}
        _, _, d, b = gg.tsdf_integrate(src, depth[t], tgt, tp, F=F, W=Wv, ws=ws_t,
                                       tuning=tile, **kw)
        ev[1].record()
        gg.splat_views_backward(src, depth[t], rgb[t], tgt, sp, so, g_rgb, g_z, g_a)
        g2 = gg.tsdf_extract_depth_backward(tgt, tp, F, Wv, b, gdep)
        gg.tsdf_integrate_backward(src, depth[t], tgt, tp, F, Wv, b, g2, ws=ws_b)
        ev[2].record()
        if timed:
            ev[2].synchronize()
            fwd_ms.append(ev[0].elapsed_time(ev[1]))
            bwd_ms.append(ev[1].elapsed_time(ev[2]))

    for t in range(min(warm, nf)):
        frame(t, t > 0, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(nf):
        frame(t, t > 0, True)
    wall = (time.perf_counter() - t0) * 1e3 / nf
    del depth, rgb, F, Wv, ws_t, ws_b, ws_s
    tf, tb = float(np.mean(fwd_ms)), float(np.mean(bwd_ms))
    return {"ratio": round(tb / tf, 3), "fwd_ms": round(tf, 3), "bwd_ms": round(tb, 3),
            "ms_per_frame": round(tf + tb, 3), "wall_ms_per_frame": round(wall, 3),
            "frames": nf, "fwd_ms_range": [round(min(fwd_ms), 3), round(max(fwd_ms), 3)],
            "bwd_ms_range": [round(min(bwd_ms), 3), round(max(bwd_ms), 3)],
            "fusion_tile": list(tile),
            "workload": "streaming 1920x1080 K=8 D=256, %d consecutive frames, volume carried, "
                        "forward + backward every frame (views rendered at half resolution and "
                        "repeated to full size)" % nf}


def paper_shape_leg(gg, torch, dev, c, frames, steps=20):
    """Context beside the paper's Table 4 (1352x1014, K=4): per frame the
    volume path (splat + fusion + extraction, pipelined on two streams as
    in the main measurement), the EWA compositing (the renderer the paper's
    10 ms splatting uses) and the volume-free raymarch (the paper's own 6 ms
    per-ray TSDF form); frames resident, cycled."""
    src, tgt = gg.cameras(c["src"]), gg.camera(c["tgt"])
    sp, tp = gg.splat_params(c["splat"]), gg.tsdf_params(c["tsdf"])
    depth = torch.from_numpy(np.stack([f[0] for f in frames])).to(dev)
    rgb = torch.from_numpy(np.stack([f[1] for f in frames])).to(dev)
    nf, K, H, Wd = depth.shape
    D = tp.num_bins
    F = torch.zeros((H, Wd, D), device=dev)
    Wv = torch.zeros_like(F)
    wss = [torch.empty(gg.workspace_size(3, K, Wd, H, Wd, H, D), dtype=torch.uint8, device=dev)
           for _ in range(2)]
    ws_s = torch.empty(gg.workspace_size(1, K, Wd, H, Wd, H, 2, sp), dtype=torch.uint8, device=dev)
    sout = gg.splat_views(src, depth[0], rgb[0], tgt, sp, ws=ws_s)
    torch.cuda.synchronize()  # the side stream reuses these buffers
    side = torch.cuda.Stream(device=dev)
    ev_t = [torch.cuda.Event(), torch.cuda.Event()]
    ev_f = [torch.cuda.Event(), torch.cuda.Event()]

    def step(i):
        f, b = i % nf, i % 2
        main = torch.cuda.current_stream(dev)
        side.wait_event(ev_f[b])
        gg.tsdf_view_table(src, depth[f], tp, ws=wss[b], stream=side)
        ev_t[b].record(side)
        gg.splat_views(src, depth[f], rgb[f], tgt, sp, out=sout, ws=ws_s, stream=side)
        main.wait_event(ev_t[b])
        gg.tsdf_integrate(src, depth[f], tgt, tp, F_prev=F, W_prev=Wv, F=F, W=Wv, ws=wss[b],
                          table_ready=True, tuning=TILE[0])
        ev_f[b].record(main)

    def per_frame(fn):
        for i in range(3):
            fn(i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            fn(3 + i)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    vol = per_frame(step)
    ws_e = torch.empty(gg.workspace_size(6, K, Wd, H, Wd, H, 2, sp), dtype=torch.uint8,
                       device=dev)
    torch.cuda.synchronize()
    eo = gg.splat_views_ewa(src, depth[0], rgb[0], tgt, sp, ws=ws_e)
    ewa = per_frame(lambda i: gg.splat_views_ewa(src, depth[i % nf], rgb[i % nf], tgt, sp,
                                                 ws=ws_e, out=eo))
    dbuf = [torch.zeros((H, Wd), device=dev) for _ in range(2)]
    abuf = [torch.zeros((H, Wd), device=dev) for _ in range(2)]
    ws_r = wss[0]
    rm = per_frame(lambda i: gg.tsdf_raymarch(src, depth[i % nf], tgt, tp, depth_prev=dbuf[i % 2],
                                              acc_prev=abuf[i % 2], out_depth=dbuf[(i + 1) % 2],
                                              out_acc=abuf[(i + 1) % 2], ws=ws_r))
    px = H * Wd
    return {"workload": "video scene and rig at 1352x1014, K=4, D=128 (the paper's test shape)",
            "volume_path_ms": round(vol, 4), "volume_path_mpix_s": round(px / vol / 1e3, 2),
            "ewa_compositing_ms": round(ewa, 4), "raymarch_ms": round(rm, 4),
            "paper_table4_ms": {"forward_splatting": 10.0, "image_based_tsdf": 6.0},
            "note": "context only: the paper's hardware is not stated"}


def bwd_fwd_ratio(gg, torch, dev, c=None, reps=10):
    """Backward / forward time (default: the differentiation workload,
    640x360, K=4, D=96): forward = splat + fusion + extraction, backward =
    the three adjoints for random upstream gradients."""
    c = scenes.config3() if c is None else c
    depth = torch.from_numpy(c["depth"]).to(dev)
    rgb = torch.from_numpy(c["rgb"]).to(dev)

    def fwd():
        o = gg.splat_views(c["src"], depth, rgb, c["tgt"], c["splat"])
        F, W, d, b = gg.tsdf_integrate(c["src"], depth, c["tgt"], c["tsdf"], tuning=TILE[0])
        return o, F, W, d, b

    o, F, W, d, b = fwd()
    g_rgb, g_z, g_a = (torch.randn_like(o["rgb"]), torch.randn_like(o["depth"]),
                       torch.randn_like(o["alpha"]))
    gdep = torch.randn_like(d)

    def bwd():
        gg.splat_views_backward(c["src"], depth, rgb, c["tgt"], c["splat"], o, g_rgb, g_z, g_a)
        g2 = gg.tsdf_extract_depth_backward(c["tgt"], c["tsdf"], F, W, b, gdep)
        gg.tsdf_integrate_backward(c["src"], depth, c["tgt"], c["tsdf"], F, W, b, g2)

    for _ in range(3):
        fwd()
        bwd()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fwd()
    torch.cuda.synchronize()
    tf = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        bwd()
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / reps
    return tb / tf, tf * 1e3, tb * 1e3


def _batch_item(desc):
    c = scenes.config4_item(desc)
    return c["depth"], c["rgb"]


def batched_speedup(gg, torch, dev, procs, tune=True, tuning=None):
    """Batching workload: 24 target views of uneven resolution, view count and
    bin count.  One hipGraph launch of the batched plan against the 24 plain
    sequences (splat_views + tsdf_integrate per item), same outputs."""
    from paper_2505_18932_amd import autotune

    descs = scenes.config4_items()
    if procs > 1:
        with mp.get_context("fork").Pool(procs) as pool:
            frames = pool.map(_batch_item, descs)
    else:
        frames = [_batch_item(d) for d in descs]
    items = []
    for desc, (d, r) in zip(descs, frames):
        seq = scenes.RingSequence(4, desc["seed"], 16, 1.0, desc["width"], desc["height"],
                                  desc["k"], scenes.MovingSpheres(desc["seed"], 4),
                                  target_angle=desc["angle"])
        items.append(dict(src=gg.cameras(seq.src), tgt=gg.camera(seq.tgt),
                          depth=torch.from_numpy(d).to(dev), rgb=torch.from_numpy(r).to(dev),
                          splat=gg.splat_params(scenes.splat_params()),
                          tsdf=gg.tsdf_params(scenes.tsdf_params(num_bins=desc["d"], trunc=4.0))))
    voxels = sum(it["tgt"].width * it["tgt"].height * it["tsdf"].num_bins for it in items)
    pixels = sum(it["tgt"].width * it["tgt"].height for it in items)
    ttimes = {}
    if tuning is None:
        tuning, ttimes = autotune.tune_batch(items) if tune else ((0, 0, 0), {})
    plan = gg.BatchPlan(items, *tuning)
    outs = [dict(F=it["F"], W=it["W"]) for it in items]
    # the plain calls each at the best launch shape of its item's class (K, D, size), tuned as
    # the main leg's is: the strongest sequence of plain calls to compare with
    ptiles = [autotune.tune_plain(it["src"], it["depth"], it["tgt"], it["tsdf"], reps=3)[0]
              if tune else TILE[0] for it in items]

    def plain():
        for it, o, tl in zip(items, outs, ptiles):
            gg.splat_views(it["src"], it["depth"], it["rgb"], it["tgt"], it["splat"])
            gg.tsdf_integrate(it["src"], it["depth"], it["tgt"], it["tsdf"], F=o["F"], W=o["W"],
                              tuning=tl)

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps * 1e3

    tb = timed(plan.launch)
    tp = timed(plain)
    plan.close()
    return {"items": len(items), "target_mpix": round(pixels / 1e6, 3),
            "voxels_g": round(voxels / 1e9, 3), "graph_ms": round(tb, 3), "plain_ms": round(tp, 3),
            "speedup": round(tp / tb, 3), "tuning": list(tuning),
            "plain_tunings": sorted(set(",".join(map(str, t)) for t in ptiles if t)),
            "tuning_ms": {k: round(v, 3) for k, v in ttimes.items()},
            "batched_mpix_s": round(pixels / tb / 1e3, 1)}


def temporal_path(gg, torch, dev, src, tgt, sp, tp, depth, rgb, steps, warmup):
    """The paper's full temporal path on the video workload (§3.2, Suppl.
    A.2): per frame the colour-difference masks of the K views and their
    filtered depths, the splat carrying the masks (maximum over views), and
    the fusion of the filtered depths with that maximum weighting the carried
    volume; all inputs resident, state carried in place.

    Pipelined on two streams: the second stream runs a frame's masks and
    filter, its view table and its masked splat, then signals; the main
    stream fuses that frame while the second stream moves on to the next.
    The view tables and splat outputs alternate between two buffers (the
    second stream waits until the fusion two frames back is done with one)."""
    nf, K, H, Wd = depth.shape[0], depth.shape[1], depth.shape[2], depth.shape[3]
    D = tp.num_bins
    F = torch.zeros((H, Wd, D), dtype=torch.float32, device=dev)
    Wv = torch.zeros_like(F)
    filt = depth[0].clone()
    mask = torch.empty((K, H, Wd), device=dev)
    wsm = torch.empty(gg.workspace_size(5, K, Wd, H, Wd, H, 4), dtype=torch.uint8, device=dev)
    ws_s = torch.empty(gg.workspace_size(1, K, Wd, H, Wd, H, 2, sp), dtype=torch.uint8, device=dev)
    wst = [torch.empty(gg.workspace_size(3, K, Wd, H, Wd, H, D), dtype=torch.uint8, device=dev)
           for _ in range(2)]

    def outs():
        return dict(win_idx=torch.empty((K, H, Wd), dtype=torch.int32, device=dev),
                    depth=torch.empty((K, H, Wd), device=dev),
                    rgb=torch.empty((K, 3, H, Wd), device=dev),
                    alpha=torch.empty((K, H, Wd), device=dev),
                    tape=torch.empty((K, 3, H, Wd), device=dev),
                    mask=torch.empty((K, H, Wd), device=dev),
                    mask_max=torch.empty((H, Wd), device=dev))

    so = [outs(), outs()]
    side = torch.cuda.Stream(device=dev)
    ready = [torch.cuda.Event(), torch.cuda.Event()]
    done = [torch.cuda.Event(), torch.cuda.Event()]
    pipelined = [True]

    def step(i):
        f, g = (i + 1) % nf, i % nf  # frame t and t - 1 (the sequence wraps)
        if not pipelined[0]:
            gg.difference_masks(rgb[f], rgb[g], depth=depth[f], depth_prev=filt, mask=mask,
                                filtered=filt, ws=wsm)
            gg.splat_views(src, filt, rgb[f], tgt, sp, mask=mask, out=so[0], ws=ws_s)
            gg.tsdf_integrate(src, filt, tgt, tp, F_prev=F, W_prev=Wv, F=F, W=Wv,
                              mask=so[0]["mask_max"], ws=wst[0], tuning=TILE[0])
            return
        b = i % 2
        main = torch.cuda.current_stream(dev)
        side.wait_event(done[b])
        gg.difference_masks(rgb[f], rgb[g], depth=depth[f], depth_prev=filt, mask=mask,
                            filtered=filt, ws=wsm, stream=side)
        gg.tsdf_view_table(src, filt, tp, ws=wst[b], stream=side)
        gg.splat_views(src, filt, rgb[f], tgt, sp, mask=mask, out=so[b], ws=ws_s, stream=side)
        ready[b].record(side)
        main.wait_event(ready[b])
        gg.tsdf_integrate(src, filt, tgt, tp, F_prev=F, W_prev=Wv, F=F, W=Wv,
                          mask=so[b]["mask_max"], ws=wst[b], table_ready=True, tuning=TILE[0])
        done[b].record(main)

    def timed(first):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            step(first + i)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    for i in range(warmup):
        step(i)
    ms = timed(warmup)
    # per-kernel breakdown (every launch bracketed) and the one-stream comparison
    gg.timing_reset()
    gg.timing_enable(True)
    for i in range(min(steps, 10)):
        step(warmup + steps + i)
    torch.cuda.synchronize()
    gg.timing_enable(False)
    nb = min(steps, 10)
    kt = {}
    for name in ("difference_masks", "conf", "splat_raster", "integrate"):
        t, n = gg.timing_read(name)
        kt[name] = round(t / max(nb, 1), 4)
    pipelined[0] = False
    ms1 = timed(warmup + steps + nb)
    # algorithmic bytes of the mask pass: two colour frames and the depth
    # read, the mask and filtered depth written, the previous filtered depth
    # read (per source pixel and view)
    mb = K * H * Wd * (3 + 3 + 4 + 4 + 4 + 4)
    return {"workload": "video ring K=4 1280x720 D=128, masks + filter + mask splat + fusion",
            "ms_per_frame": round(ms, 4), "mpix_s": round(H * Wd / ms / 1e3, 2),
            "one_stream_ms_per_frame": round(ms1, 4),
            "kernel_ms_per_frame": kt,
            "difference_masks_gb_s": round(mb / (kt["difference_masks"] * 1e-3) / 1e9, 1)
            if kt["difference_masks"] > 0 else None}


def raymarch_path(gg, torch, dev, src, tgt, tp, depth, steps, warmup):
    """The paper's own volume-free fusion (Suppl. A.1 march, Suppl. A.2
    temporal input) on the video workload: per frame one march of every
    target ray, the previous output depth and its accumulated weight carried
    (ping-pong buffers); inputs resident."""
    nf, K, H, Wd = depth.shape[0], depth.shape[1], depth.shape[2], depth.shape[3]
    ws = torch.empty(gg.workspace_size(3, K, Wd, H, Wd, H, tp.num_bins), dtype=torch.uint8,
                     device=dev)
    dbuf = [torch.zeros((H, Wd), device=dev) for _ in range(2)]
    abuf = [torch.zeros((H, Wd), device=dev) for _ in range(2)]

    def step(i):
        a, b = i % 2, (i + 1) % 2
        gg.tsdf_raymarch(src, depth[i % nf], tgt, tp, depth_prev=dbuf[a], acc_prev=abuf[a],
                         out_depth=dbuf[b], out_acc=abuf[b], ws=ws)

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    gg.timing_reset()
    gg.timing_enable(True)
    t0 = time.perf_counter()
    for i in range(steps):
        step(warmup + i)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    gg.timing_enable(False)
    rm, n = gg.timing_read("raymarch")
    cf, _ = gg.timing_read("conf")
    _, _, st = gg.tsdf_raymarch(src, depth[0], tgt, tp, steps=True, ws=ws)
    ms = el * 1e3 / steps
    return {"workload": "video ring K=4 1280x720, march bounds as D=128, temporal input carried",
            "ms_per_frame": round(ms, 4), "mpix_s": round(H * Wd / ms / 1e3, 2),
            "kernel_ms_per_frame": {"raymarch": round(rm / max(n, 1), 4),
                                    "conf": round(cf / max(n, 1), 4)},
            "samples_per_ray_mean": round(float(st.float().mean()), 2)}


def ewa_path(gg, torch, dev, src, tgt, sp, depth, rgb, steps, warmup):
    """EWA-projected pixel Gaussians composited front to back (the 3D
    Gaussian splatting renderer of §3.1) on the video workload: one call per
    frame renders the K views into the target; inputs resident."""
    nf, K, H, Wd = depth.shape[0], depth.shape[1], depth.shape[2], depth.shape[3]
    need = gg.workspace_size(6, K, Wd, H, Wd, H, 2, sp)
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    out = gg.splat_views_ewa(src, depth[0], rgb[0], tgt, sp, ws=ws)
    for i in range(warmup):
        gg.splat_views_ewa(src, depth[i % nf], rgb[i % nf], tgt, sp, ws=ws, out=out)
    torch.cuda.synchronize()
    gg.timing_reset()
    gg.timing_enable(True)
    t0 = time.perf_counter()
    for i in range(steps):
        gg.splat_views_ewa(src, depth[(warmup + i) % nf], rgb[(warmup + i) % nf], tgt, sp, ws=ws,
                           out=out)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    gg.timing_enable(False)
    kt = {}
    for name in ("ewa_zero", "ewa_count", "ewa_alloc", "ewa_fill", "ewa_raster"):
        t, n = gg.timing_read(name)
        kt[name] = round(t / max(n, 1), 4)
    # list statistics from the workspace's per-tile counts (the first array
    # of the EWA workspace, followed by the total): entries of the last frame
    # and the longest tile list
    ntiles = ((Wd + 7) // 8) * ((H + 7) // 8)
    n = K * ntiles
    cnt = ws[:4 * (n + 1)].view(torch.int32).cpu().numpy().astype("int64")
    ms = el * 1e3 / steps
    return {"workload": "video ring K=4 1280x720, per-view EWA compositing, lowpass 0.3",
            "ms_per_frame": round(ms, 4), "mpix_s": round(H * Wd / ms / 1e3, 2),
            "kernel_ms_per_frame": kt,
            "list_entries": int(cnt[n]), "entries_per_gaussian":
                round(float(cnt[n]) / float((depth[0] > 0).sum()), 3),
            "tile_list_mean": round(float(cnt[n]) / n, 1),
            "tile_list_max": int(cnt[:n].max())}


def network_path(gg, torch, dev, src, tgt, sp, tp, depth, rgb, steps):
    """The blending network's input stack and the Eq. 4-5 blend (with
    synthetic weights) on one frame of the video workload; algorithmic HBM
    bytes per launch over the kernels' mean times."""
    K, H, Wd = depth.shape[1], depth.shape[2], depth.shape[3]
    so = gg.splat_views(src, depth[0], rgb[0], tgt, sp)
    _, _, dep, _ = gg.tsdf_integrate(src, depth[0], tgt, tp)
    w = torch.rand((K, H, Wd), device=dev)
    wb = torch.rand((H, Wd), device=dev)
    bg = torch.rand((3, H, Wd), device=dev)
    out = torch.empty((9 * K + 1, H, Wd), device=dev)
    for _ in range(3):
        gg.network_inputs(src, tgt, dep, so, out=out)
        gg.blend_views(so["rgb"], so["depth"], so["alpha"], w, wb, bg)
    torch.cuda.synchronize()
    gg.timing_reset()
    gg.timing_enable(True)
    for _ in range(steps):
        gg.network_inputs(src, tgt, dep, so, out=out)
        gg.blend_views(so["rgb"], so["depth"], so["alpha"], w, wb, bg)
    torch.cuda.synchronize()
    gg.timing_enable(False)
    ni, n = gg.timing_read("network_inputs")
    bl, _ = gg.timing_read("blend")
    ni, bl = ni / max(n, 1), bl / max(n, 1)
    px = H * Wd
    # network inputs: read 5K planes + the TSDF depth (5 taps, cached), write 9K + 1 planes
    b_ni = px * 4 * (5 * K + 1 + 9 * K + 1)
    # blend: read 6K + 4 planes, write 4
    b_bl = px * 4 * (6 * K + 4 + 4)
    return {"workload": "video ring K=4 1280x720, one frame",
            "network_inputs_ms": round(ni, 4), "network_inputs_gb_s": round(b_ni / ni / 1e6, 1),
            "blend_ms": round(bl, 4), "blend_gb_s": round(b_bl / bl / 1e6, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--frames", type=int, default=30)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bwd", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--cpu-plan", action="store_true",
                    help="run only the CPU oracle's timing plan (no GPU work) and print it")
    ap.add_argument("--stream-frames", type=int, default=STREAM_FRAMES,
                    help="frames of the streaming leg (1920x1080, K=8, D=256); the leg warms up "
                         "on min(3, frames) of them first")
    ap.add_argument("--no-temporal", action="store_true")
    ap.add_argument("--no-raymarch", action="store_true")
    ap.add_argument("--no-network", action="store_true")
    ap.add_argument("--no-ewa", action="store_true")
    ap.add_argument("--no-paper-shape", action="store_true")
    ap.add_argument("--batch-tuning", default="",
                    help="batched plan 'threads_per_workgroup,blocks_per_cu' instead of autotuning "
                         "(profiling runs pin what the timed runs pick)")
    ap.add_argument("--streams", type=int, default=2, choices=(1, 2),
                    help="2: the splat on its own stream, overlapping the fusion; 1: one stream")
    ap.add_argument("--tile", default="",
                    help="fusion launch shape 'pixels_per_block,pixels_per_row,bins_per_thread' "
                         "instead of autotuning (profiling runs pin the shape the timed runs pick)")
    ap.add_argument("--procs", type=int, default=0,
                    help="input-generation worker processes (0: min(16, cores))")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="also run a device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.cpu_plan:
        procs = args.procs or max(1, min(16, os.cpu_count() or 1))
        print(json.dumps({"cpu_plan": cpu_plan(procs)}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs the geometry stage on a single "
              "MI355X (no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    procs = args.procs or max(1, min(16, os.cpu_count() or 1))
    depth_h, rgb_h = make_frames(args.frames, procs)
    print(f"# frames generated: {depth_h.shape}", file=sys.stderr, flush=True)
    # the large workload's first frame for its backward/forward ratio, generated (like the
    # frames above) before anything touches the GPU
    large = None if args.no_bwd else streaming_sequence(procs, args.stream_frames)
    paper = None
    if not args.no_paper_shape:
        pc = scenes.paper_shape()
        paper = (pc, [pc["seq"].frame(t, procs=procs) for t in range(4)])

    import torch

    import paper_2505_18932_amd as gg

    dev = torch.device("cuda:0")
    c = scenes.config2(seed=0)
    src, tgt = gg.cameras(c["src"]), gg.camera(c["tgt"])
    sp, tp = gg.splat_params(c["splat"]), gg.tsdf_params(c["tsdf"])
    K, H, Wd, D = 4, tgt.height, tgt.width, tp.num_bins
    depth = torch.from_numpy(depth_h).to(dev)
    rgb = torch.from_numpy(rgb_h).to(dev)
    F = torch.zeros((H, Wd, D), dtype=torch.float32, device=dev)
    Wv = torch.zeros((H, Wd, D), dtype=torch.float32, device=dev)
    ws_s = torch.empty(gg.workspace_size(1, K, Wd, H, Wd, H, 2, sp), dtype=torch.uint8, device=dev)
    ws_t = torch.empty(gg.workspace_size(3, K, Wd, H, Wd, H, D), dtype=torch.uint8, device=dev)
    ws_t2 = torch.empty_like(ws_t)  # the second buffer of the pipelined view tables
    sout = dict(win_idx=torch.empty((K, H, Wd), dtype=torch.int32, device=dev),
                depth=torch.empty((K, H, Wd), device=dev), rgb=torch.empty((K, 3, H, Wd), device=dev),
                alpha=torch.empty((K, H, Wd), device=dev), tape=torch.empty((K, 3, H, Wd), device=dev))
    nf = args.frames
    # A frame's splat and its fusion weights (the view table) depend on that frame's inputs
    # only, so with two streams they run on a second stream (default priority) while the main
    # stream fuses: per frame the second stream builds the view table into one of two
    # workspaces (after the fusion two frames back has released it), records an event and
    # splats; the main stream waits for the event and fuses from that table.  Each stream
    # keeps its own order (the splat outputs and the carried volume are reused frame after
    # frame).
    s_splat = torch.cuda.Stream(device=dev) if args.streams == 2 else None
    wss = [ws_t, ws_t2]
    ev_table = [torch.cuda.Event(), torch.cuda.Event()]
    ev_fused = [torch.cuda.Event(), torch.cuda.Event()]

    def step(i, carry=True, tuning=None):
        f = i % nf
        tun = tuning if tuning is not None else TILE[0]
        prev = dict(F_prev=F if carry else None, W_prev=Wv if carry else None, F=F, W=Wv,
                    tuning=tun)
        if s_splat is None:
            gg.splat_views(src, depth[f], rgb[f], tgt, sp, out=sout, ws=ws_s)
            return gg.tsdf_integrate(src, depth[f], tgt, tp, ws=ws_t, **prev)
        b = i % 2
        main = torch.cuda.current_stream(dev)
        s_splat.wait_event(ev_fused[b])
        gg.tsdf_view_table(src, depth[f], tp, ws=wss[b], stream=s_splat)
        ev_table[b].record(s_splat)
        gg.splat_views(src, depth[f], rgb[f], tgt, sp, out=sout, ws=ws_s, stream=s_splat)
        main.wait_event(ev_table[b])
        r = gg.tsdf_integrate(src, depth[f], tgt, tp, ws=wss[b], table_ready=True, **prev)
        ev_fused[b].record(main)
        return r

    # launch shape of the fusion for this class (autotuned, results unchanged)
    from paper_2505_18932_amd import autotune
    step(0, carry=False)
    if args.tile:
        tile = tuple(int(v) for v in args.tile.split(","))
    elif s_splat is not None:
        # timed inside the two-stream step, where the fusion shares the device
        tile, tile_times, _ = autotune.tune_plain_step(step, 1)
    else:
        tile, tile_times = autotune.tune_plain(src, depth[0], tgt, tp, use_cache=False)
    TILE[0] = tile
    for i in range(1, args.warmup):
        step(i)
    torch.cuda.synchronize()
    gg.timing_reset()
    # the timed region brackets only the fusion kernel (the roofline's) with events
    gg.timing_enable(True, only="integrate")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(args.warmup + i)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    gg.timing_enable(False)
    int_total, int_n = gg.timing_read("integrate")
    ms_per_step = el * 1e3 / args.steps
    value = args.steps * H * Wd / el / 1e6
    # per-kernel breakdown from a separate, untimed pass with every launch bracketed
    nb = min(args.steps, 20)
    gg.timing_reset()
    gg.timing_enable(True)
    for i in range(nb):
        step(args.warmup + args.steps + i)
    torch.cuda.synchronize()
    gg.timing_enable(False)
    kt = {}
    for name in ("integrate", "conf", "bins", "splat_count", "splat_fill", "splat_raster",
                 "splat_scan", "splat_zero"):
        ms, n = gg.timing_read(name)
        kt[name] = (ms, n)
    serial_ms = serial_int_ms = None
    if s_splat is not None:
        # the same steps with both stages on one stream, for comparison (not the metric)
        s_keep, s_splat = s_splat, None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gg.timing_reset()
        gg.timing_enable(True, only="integrate")
        for i in range(args.steps):
            step(args.warmup + args.steps + nb + i)
        torch.cuda.synchronize()
        serial_ms = (time.perf_counter() - t0) * 1e3 / args.steps
        gg.timing_enable(False)
        st, sn = gg.timing_read("integrate")
        serial_int_ms = st / max(sn, 1)
        s_splat = s_keep

    # roofline of the fusion kernel: algorithmic bytes per launch
    ns = H * Wd
    vox = H * Wd * D
    alg = vox * 16 + K * ns * 8 + ns * 8  # F, W read+write; view-table gather; extraction out
    int_ms_timed = int_total / max(int_n, 1)
    # The roofline is the fusion kernel's own: with two streams its launches share the device
    # with the splat, so its duration there is not the kernel's; the one-stream pass over the
    # same frames times it alone (what rocprofv3 sees as well).
    int_ms = serial_int_ms if serial_int_ms is not None else int_ms_timed
    achieved = alg / (int_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": recorded_traffic(),
            "kernel": "integrate_kernel<V=%d, K=%d>" % (tile[2], K), "kernel_ms": round(int_ms, 4),
            "algorithmic_bytes_per_launch": alg,
            "timed_on": "one-stream pass" if serial_int_ms is not None else "timed region",
            "kernel_ms_overlapped": round(int_ms_timed, 4)}

    # the fusion's second bound: VALU issue.  Peak = 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz =
    # 39.3 T lane-instructions/s (FP32 without packed math, which the build disables)
    vi = recorded_valu_instructions()
    roof_valu = None
    if vi is not None:
        lane_ops = vi * 64
        ach = lane_ops / (int_ms * 1e-3) / 1e12
        roof_valu = {"bound": "alu", "achieved": round(ach, 2), "peak": VALU_PEAK_TLANE,
                     "unit": "T lane-instructions/s", "frac": round(ach / VALU_PEAK_TLANE, 4),
                     "lane_instructions_per_launch": lane_ops,
                     "source": "SQ_INSTS_VALU of the committed counter summary"}

    # the same GPU's copy bandwidth (1 GiB device-to-device, read + write), for comparison
    cb = measure_copy_gbs(torch, dev)
    roof["copy_gb_s"] = round(cb, 1)
    roof["frac_of_copy"] = round(achieved / cb, 4)
    # the fusion kernel's own volume stream alone (same kernel and launch shape, no views): the
    # ceiling of its access pattern on this GPU, on the carried volume in place
    pr_ms = fusion_stream_probe_ms(gg, torch, dev, tgt, tp, F, Wv)
    pr_bytes = vox * 16 + ns * 8
    roof["stream_probe"] = {"kernel_ms": round(pr_ms, 4),
                            "gb_s": round(pr_bytes / (pr_ms * 1e-3) / 1e9, 1),
                            "bytes_per_launch": pr_bytes}
    roof["frac_of_stream_probe"] = round(achieved / roof["stream_probe"]["gb_s"], 4)
    tr = roof["traffic"]
    if tr is not None:
        # counted HBM-side bytes (read + write of the committed counter summary) over the same time
        roof["traffic_gb_s"] = round(tr / (int_ms * 1e-3) / 1e9, 1)
        roof["traffic_frac"] = round(roof["traffic_gb_s"] / HBM_PEAK_GBS, 4)

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()

    out = {
        "metric": "target-view Mpix/s (splat+TSDF+extract, K=4, 1280x720, D=128)",
        "value": round(value, 2), "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOAD, "K": K, "width": Wd, "height": H, "bins": D,
                   "frames_resident": nf, "fusion_tile": list(tile), "streams": args.streams},
        "roofline": roof,
        "roofline_valu": roof_valu,
        "kernel_ms_per_step": {k: round(v[0] / max(nb, 1), 4) for k, v in kt.items()},
    }
    if args.streams > 1:
        out["kernel_ms_note"] = ("HIP events around each launch, in an untimed pass of the same "
                                 "two-stream pipeline: a second-stream kernel's time includes "
                                 "waiting for compute units that the fusion holds")
    if serial_ms is not None:
        out["one_stream_ms_per_step"] = round(serial_ms, 4)
    if not args.no_bwd:
        r, tf, tb = bwd_fwd_ratio(gg, torch, dev)
        out["bwd_fwd"] = {"ratio": round(r, 3), "fwd_ms": round(tf, 3), "bwd_ms": round(tb, 3),
                          "workload": "differentiation 640x360 K=4 D=96"}
        # the streaming workload's own tuned launch shape, unless the command pins one
        out["bwd_fwd_large"] = streaming_leg(gg, torch, dev, *large,
                                             tile=TILE[0] if args.tile else None)
        del large
        torch.cuda.empty_cache()
    del F, Wv, sout
    torch.cuda.empty_cache()
    if not args.no_temporal:
        out["temporal_path"] = temporal_path(gg, torch, dev, src, tgt, sp, tp, depth, rgb,
                                             min(args.steps, 30), 3)
    if not args.no_raymarch:
        out["raymarch"] = raymarch_path(gg, torch, dev, src, tgt, tp, depth, min(args.steps, 30), 3)
    if not args.no_network:
        out["network_inputs"] = network_path(gg, torch, dev, src, tgt, sp, tp, depth, rgb, 20)
    if not args.no_ewa:
        out["ewa_compositing"] = ewa_path(gg, torch, dev, src, tgt, sp, depth, rgb,
                                          min(args.steps, 30), 3)
    if paper is not None:
        out["paper_shape"] = paper_shape_leg(gg, torch, dev, paper[0], paper[1])
        del paper
        torch.cuda.empty_cache()
    if not args.no_batch:
        del depth, rgb, ws_s, ws_t, ws_t2, wss
        torch.cuda.empty_cache()
        bt = tuple(int(v) for v in args.batch_tuning.split(",")) if args.batch_tuning else None
        out["batched"] = batched_speedup(gg, torch, dev, procs, tuning=bt)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(c, depth_h, rgb_h)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
