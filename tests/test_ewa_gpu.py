"""EWA front-to-back compositing on the GPU against the oracle, bitwise:
colour, opacity and depth per view, on the small parallel-rig scene and
ring-rig scenes (several tiles, ragged tails), a zoomed-out target whose
tile lists outgrow the LDS sort (the global merge path), the sort-limit
invariance of both paths, sampled pixels of the full 1280x720 K=4 video
frame, and the degenerate cases."""
import numpy as np
import pytest
import torch

import oracle
import paper_2505_18932_amd as gg
import scenes

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def bits(a):
    return np.ascontiguousarray(a, np.float32).view(np.uint32)


def run(c, lowpass=0.3, sort_limit=0):
    o = gg.splat_views_ewa(c["src"], torch.from_numpy(np.ascontiguousarray(c["depth"])).to(DEV),
                           torch.from_numpy(np.ascontiguousarray(c["rgb"])).to(DEV), c["tgt"],
                           c["splat"], lowpass=lowpass, sort_limit=sort_limit)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in o.items()}


def check(c, lowpass=0.3):
    g = run(c, lowpass)
    r = oracle.splat_ewa(c["src"], c["depth"], c["rgb"], c["tgt"], c["splat"], lowpass=lowpass)
    for key in ("rgb", "alpha", "depth"):
        assert np.array_equal(bits(g[key]), bits(r[key])), key
    return r


def test_tiny_config_bitwise():
    r = check(scenes.config1())
    assert (r["alpha"] > 0.9).mean() > 0.9


@pytest.mark.parametrize("lowpass", [0.0, 1.0])
def test_lowpass(lowpass):
    check(scenes.config1(), lowpass)


@pytest.mark.parametrize("k,w,h", [(1, 37, 29), (3, 96, 64), (5, 61, 43), (8, 40, 24)])
def test_ring_scenes_ragged(k, w, h):
    c = scenes.small_ring(seed=k, width=w, height=h, k=k, noise=0.01, holes=0.02)
    check(c)


def _zoomed_out(scale=6, seed=0):
    """Sources at 240x160, the target at the same pose with fx / scale and
    its principal point scaled: about scale^2 source pixels per target
    pixel, so 8 x 8 tiles collect hundreds to thousands of Gaussians (lists
    on both sides of every sort threshold)."""
    c = scenes.small_ring(seed=seed, width=240, height=160, k=2, noise=0.01)
    t = c["tgt"]
    w, h = 240 // scale + 3, 160 // scale + 2
    c["tgt"] = scenes.Camera(float(np.float32(t.fx / scale)), float(np.float32(t.fy / scale)),
                             float(np.float32(w / 2)), float(np.float32(h / 2)), t.R, t.t, w, h)
    return c


def test_long_lists_take_the_merge_path():
    c = _zoomed_out()
    r = check(c)
    assert (r["alpha"] > 0.5).mean() > 0.5


@pytest.mark.parametrize("limit", [64, 100, 256, 300])
def test_sort_limit_invariance(limit):
    cs = [scenes.config1(), _zoomed_out(4, seed=1)]
    ref = [run(c) for c in cs]
    got = [run(c, sort_limit=limit) for c in cs]
    for a, b in zip(ref, got):
        for key in ("rgb", "alpha", "depth"):
            assert np.array_equal(bits(a[key]), bits(b[key])), key


def test_repeatable():
    c = scenes.small_ring(seed=3, width=64, height=48, k=3)
    a, b = run(c), run(c)
    for key in a:
        assert np.array_equal(bits(a[key]), bits(b[key]))


def test_full_video_frame_sampled():
    """1280x720, K=4 ring video frame: 600 sampled pixels against the
    oracle's per-pixel rendering, bitwise."""
    c = scenes.config2()
    depth, rgb = c["seq"].frame(0)
    c = dict(src=c["src"], tgt=c["tgt"], depth=depth, rgb=rgb, splat=c["splat"])
    g = run(c)
    rng = np.random.default_rng(11)
    n = c["tgt"].width * c["tgt"].height
    pix = rng.choice(n, 600, replace=False)
    r = oracle.splat_ewa(c["src"], depth, rgb, c["tgt"], c["splat"], pixels=pix)
    for key in ("rgb", "alpha", "depth"):
        a = g[key].reshape(*g[key].shape[:-2], -1)[..., pix]
        b = r[key].reshape(*r[key].shape[:-2], -1)[..., pix]
        assert np.array_equal(bits(a), bits(b)), key
    assert (g["alpha"].max(0) > 0.9).mean() > 0.9  # the union of the views covers the target


def test_nothing_drawn():
    c = scenes.config1()
    c = dict(c, depth=np.zeros_like(c["depth"]))
    g = run(c)
    assert all(np.all(v == 0) for v in g.values())
    c = scenes.config1()
    c = dict(c, splat=scenes.splat_params(z_min=50.0))
    g = run(c)
    assert all(np.all(v == 0) for v in g.values())


def test_one_pixel_target():
    c = scenes.small_ring(seed=2, width=40, height=30, k=2)
    t = c["tgt"]
    c["tgt"] = scenes.Camera(t.fx, t.fy, float(np.float32(t.cx - 20)), float(np.float32(t.cy - 15)),
                             t.R, t.t, 1, 1)
    check(c)


def test_streaming_frame_sampled(streaming_frame):
    """1920x1080, K=8 (the large streaming shape): 400 sampled pixels of
    every view against the oracle's per-pixel rendering, bitwise."""
    c, (depth, rgb) = streaming_frame
    c = dict(src=c["src"], tgt=c["tgt"], depth=depth, rgb=rgb, splat=c["splat"])
    g = run(c)
    n = c["tgt"].width * c["tgt"].height
    pix = np.random.default_rng(5).choice(n, 400, replace=False)
    r = oracle.splat_ewa(c["src"], depth, rgb, c["tgt"], c["splat"], pixels=pix)
    for key in ("rgb", "alpha", "depth"):
        a = g[key].reshape(*g[key].shape[:-2], -1)[..., pix]
        b = r[key].reshape(*r[key].shape[:-2], -1)[..., pix]
        assert np.array_equal(bits(a), bits(b)), key
