"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compare the oracle with itself: each checks a closed form, an
invariant, a special case with a known answer, or an independent FP64 brute
force (``tests/bruteforce.py``) that works through world space literally.
"""
import math
import os

import numpy as np
import pytest

import oracle
import scenes
from tests import bruteforce as bf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_golden(name):
    out = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, v = line.split()
        out[k] = float(v)
    return out


def fronto_rig(offsets, W=48, H=36, f=40.0):
    """Cameras sharing one rotation, translated in the image plane."""
    return [scenes.make_camera(W, H, f, (x, y, 0.0), (x, y, 1.0)).quantized() for x, y in offsets]


# ---------------------------------------------------------------------------
# relative projection: pinned against the literal K (R p + t) of Suppl. A.1


def test_relproj_matches_world_projection():
    ring = scenes.ring_rig(8, 1.0, 64, 48)
    a, b = ring[1].quantized(), ring[3].quantized()
    H, c = oracle.relproj64(a, b)
    rng = np.random.default_rng(0)
    for _ in range(50):
        i, j = rng.uniform(0, 64), rng.uniform(0, 48)
        z = rng.uniform(0.5, 5.0)
        P = bf.backproject(a, np.array(i - 0.5), np.array(j - 0.5), np.array(z))
        X = bf.project(b, P)
        got = z * (H @ np.array([i, j, 1.0])) + c
        np.testing.assert_allclose(got, X, rtol=1e-12, atol=1e-9)
    # identity pair: H = I, c = 0 up to the FP32 quantisation of R (R R^T = I
    # only to ~1e-7, scaled by the principal point in the last column)
    H, c = oracle.relproj64(a, a)
    np.testing.assert_allclose(H, np.eye(3), atol=5e-6)
    np.testing.assert_allclose(c, 0, atol=1e-5)


def test_bins_closed_form():
    prm = scenes.tsdf_params(num_bins=64, trunc=3.0)
    z, tau = oracle.bins(prm)
    u = 1.0 / z.astype(np.float64)
    assert abs(z[0] - 0.5) <= 1e-7
    assert abs(z[-1] - 5.0) <= 5e-6
    du = np.diff(u)
    np.testing.assert_allclose(du, du.mean(), rtol=1e-5)  # uniform in inverse depth
    # truncation of 3 bins = 3 * du * z^2 (metric width of a bin at depth z)
    np.testing.assert_allclose(tau, 3 * (2.0 - 0.2) / 63 * z.astype(np.float64) ** 2, rtol=1e-5)


# ---------------------------------------------------------------------------
# P6: the fusion weight's closed forms (Suppl. A.1)


def _conf_at(depth, prm):
    return oracle.confidence(depth, prm)[10, 10]


def test_confidence_closed_forms():
    gold = load_golden("confidence_closed_forms.txt")
    prm = scenes.tsdf_params()
    d = np.ones((21, 21), np.float32)
    assert _conf_at(d, prm) == 1.0
    for n, key in ((7, "step7"), (14, "step14"), (21, "step21")):
        d = np.ones((21, 21), np.float32)
        d[:, 14 - n // 7:] = 2.0  # n far pixels inside the 7x7 window of (10, 10)
        got = _conf_at(d, prm)
        assert abs(got - gold[key]) <= 2e-6 * gold[key], (n, got)
    g = 2.0 ** -10
    d = (1.0 + g * np.arange(21, dtype=np.float64))[None, :].repeat(21, 0).astype(np.float32)
    got = _conf_at(d, prm)
    assert abs(got - gold["ramp"]) <= 1e-6, got
    # a hole pixel has zero weight; a hole neighbour counts as tau^2
    d = np.ones((21, 21), np.float32)
    d[10, 10] = 0
    assert oracle.confidence(d, prm)[10, 10] == 0
    d = np.ones((21, 21), np.float32)
    d[10, 11] = 0
    np.testing.assert_allclose(_conf_at(d, prm), 0.35 / math.sqrt(1), rtol=1e-6)


def test_confidence_matches_bruteforce_fp64():
    c = scenes.small_ring(width=24, height=16, noise=0.01, holes=0.05)
    prm = c["tsdf"]
    for k in range(2):
        got = oracle.confidence(c["depth"][k], prm, prec=64)
        # the parameters cross the interface as FP32 values
        ref = bf.confidence(c["depth"][k], float(np.float32(prm["conf_tau"])),
                            float(np.float32(prm["conf_scale"])), prm["conf_window"])
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-15)


# ---------------------------------------------------------------------------
# P1: fronto-parallel plane, P8: temporal weight sequence, P9: static scene


@pytest.mark.parametrize("K", [1, 2, 4])
def test_plane_fuses_to_exact_depth(K):
    offs = [(0.0, 0.0), (0.04, 0.0), (-0.03, 0.02), (0.02, -0.03)][:K]
    src = fronto_rig(offs)
    tgt = fronto_rig([(0.01, 0.01)])[0]
    prm = scenes.tsdf_params(num_bins=64, trunc=3.0)
    d0 = 2.0
    depth = np.full((K, tgt.height, tgt.width), d0, np.float32)
    F, W = oracle.integrate(src, depth, tgt, prm)
    dep, b = oracle.extract(F, W, prm)
    assert (b >= 0).mean() > 0.9
    assert np.abs(dep[b >= 0] - d0).max() <= 2e-5 * d0
    # carried over a second identical frame: unchanged surface
    F2, W2 = oracle.integrate(src, depth, tgt, prm, F_prev=F, W_prev=W)
    dep2, b2 = oracle.extract(F2, W2, prm)
    assert np.array_equal(b2, b)
    assert np.abs(dep2[b2 >= 0] - d0).max() <= 2e-5 * d0


def test_temporal_weight_sequence():
    gold = load_golden("temporal_weights.txt")
    src = fronto_rig([(0.0, 0.0), (0.01, 0.0), (0.0, 0.01), (0.01, 0.01)])
    tgt = fronto_rig([(0.005, 0.005)])[0]
    prm = scenes.tsdf_params(num_bins=64, trunc=3.0, decay=0.9, weight_cap=32.0)
    depth = np.full((4, tgt.height, tgt.width), 2.0, np.float32)
    pix = np.array([18 * tgt.width + 24], np.int32)
    F = W = None
    z, _ = oracle.bins(prm)
    d = int(np.searchsorted(z, 2.0)) - 3  # a voxel in front of the surface
    F0 = None
    for t in range(1, 31):
        F, W = oracle.integrate(src, depth, tgt, prm, F_prev=F, W_prev=W, pixels=pix)
        assert abs(W[0, d] - gold[str(t)]) <= 1e-5 * gold[str(t)], (t, W[0, d])
        if F0 is None:
            F0 = F[0, d]
        assert abs(F[0, d] - F0) <= 1e-6 * abs(F0) + 1e-7


def test_static_scene_invariance():
    c = scenes.config1()
    prm = c["tsdf"]
    rng = np.random.default_rng(5)
    pix = rng.choice(c["tgt"].width * c["tgt"].height, 600, replace=False).astype(np.int32)
    F1, W1 = oracle.integrate(c["src"], c["depth"], c["tgt"], prm, pixels=pix)
    F, W = F1, W1
    for _ in range(5):
        F, W = oracle.integrate(c["src"], c["depth"], c["tgt"], prm, F_prev=F, W_prev=W, pixels=pix)
    obs = W1 > 0
    assert obs.mean() > 0.5
    assert np.all(np.abs(F[obs] - F1[obs]) <= 1e-5 * np.abs(F1[obs]) + 1e-6)
    assert np.all(W[obs] > W1[obs])


def test_mask_stops_carry():
    """A temporal mask of 1 (dynamic everywhere) makes max(1 - M, 0) = 0,
    so nothing is carried (Suppl. A.2)."""
    c = scenes.config1()
    prm = c["tsdf"]
    pix = np.arange(0, 76800, 97, dtype=np.int32)
    F1, W1 = oracle.integrate(c["src"], c["depth"], c["tgt"], prm, pixels=pix)
    mask = np.ones((240, 320), np.float32)
    F2, W2 = oracle.integrate(c["src"], c["depth"], c["tgt"], prm, mask=mask, F_prev=F1 + 1,
                              W_prev=W1, pixels=pix)
    assert np.array_equal(F2, F1) and np.array_equal(W2, W1)


# ---------------------------------------------------------------------------
# P2: analytic sphere; P3: identity warp


def _sphere_scene():
    return [scenes.Backdrop(3.0, 1, (0.6, 0.7, 0.8)), scenes.Floor(-0.5, 2, (0.7, 0.7, 0.5)),
            scenes.Sphere((0.1, 0.0, 0.05), 0.3, 3, (0.9, 0.3, 0.3))]


def test_sphere_identity_views_fuse_exactly():
    ring = scenes.ring_rig(16, 1.0, 96, 72)
    cam = ring[2].quantized()
    true, _ = scenes.render(cam, _sphere_scene())
    depth = true.astype(np.float32)[None]
    prm = scenes.tsdf_params(num_bins=128, trunc=3.0)
    for K in (1, 2):
        F, W = oracle.integrate([cam] * K, np.repeat(depth, K, 0), cam, prm)
        dep, b = oracle.extract(F, W, prm)
        inside = (true.ravel() > 0.55) & (true.ravel() < 4.9)
        assert (b[inside] >= 0).all()
        np.testing.assert_allclose(dep[inside], true.ravel()[inside], rtol=1e-5)


def test_sphere_two_views_error_shrinks_with_resolution():
    errs = []
    for W, H in ((80, 60), (160, 120)):
        ring = scenes.ring_rig(16, 1.0, W, H)
        tgt = scenes.ring_target(2 * math.pi * 2.5 / 16, 1.0, W, H).quantized()
        src = [ring[2].quantized(), ring[3].quantized()]
        scene = _sphere_scene()
        depth = np.stack([scenes.render(c, scene)[0] for c in src]).astype(np.float32)
        true, _ = scenes.render(tgt, scene)
        prm = scenes.tsdf_params(num_bins=256, trunc=3.0)
        F, W_ = oracle.integrate(src, depth, tgt, prm)
        dep, b = oracle.extract(F, W_, prm)
        sph = scene[2]
        o, d = scenes.rays(tgt)
        lam, _, _ = sph.hit(o, d)
        on = (np.abs(lam - true) < 1e-9).ravel() & (b >= 0)
        e = np.abs(dep - true.ravel())[on]
        errs.append(np.median(e))
    # nearest sampling: error ~ half a pixel of depth change, halving with resolution
    assert errs[0] < 5e-3
    assert errs[1] < 0.75 * errs[0]


def test_identity_warp_splat():
    c = scenes.config1()
    cam = c["src"][0]
    depth = c["depth"][:1].copy()
    rng = np.random.default_rng(1)
    holes = rng.random(depth.shape) < 0.05
    depth[holes] = 0
    out = oracle.splat([cam], depth, c["rgb"][:1], cam, c["splat"])
    Hh, Ww = depth.shape[1:]
    idx = np.arange(Hh * Ww).reshape(Hh, Ww)
    valid = ~holes[0]
    assert np.array_equal(out["win_idx"][0][valid], idx[valid])
    assert (out["win_idx"][0][~valid] == -1).all()
    np.testing.assert_allclose(out["depth"][0][valid], depth[0][valid], rtol=1e-6)
    ref = c["rgb"][0].astype(np.float64) / 255.0
    for ch in range(3):
        np.testing.assert_allclose(out["rgb"][0, ch][valid], ref[..., ch][valid], atol=1e-6)
    assert (out["alpha"][0][valid] == 1.0).all()
    assert (out["alpha"][0][~valid] == 0).all()


def test_surface_exactly_on_a_bin():
    """F_{d+1} = 0 counts as the crossing: a surface lying exactly on bin d
    (an axis-aligned camera, so the sampled depth difference is exactly 0)
    extracts bin d - 1 with depth z_d."""
    cam = fronto_rig([(0.0, 0.0)], W=16, H=12)[0]
    prm = scenes.tsdf_params(num_bins=32, trunc=3.0)
    z, _ = oracle.bins(prm)
    d = 17
    depth = np.full((1, 12, 16), z[d], np.float32)
    F, W = oracle.integrate([cam], depth, cam, prm)
    assert (F[:, d] == 0).all()
    dep, b = oracle.extract(F, W, prm)
    assert (b == d - 1).all()
    assert np.array_equal(dep, np.full_like(dep, z[d]))


def test_identity_warp_tsdf():
    c = scenes.config1()
    cam = c["src"][0]
    depth = c["depth"][:1]
    prm = c["tsdf"]
    F, W = oracle.integrate([cam], depth, cam, prm)
    dep, b = oracle.extract(F, W, prm)
    z, _ = oracle.bins(prm)
    inside = (depth[0].ravel() > z[1]) & (depth[0].ravel() < z[-2])
    assert (b[inside] >= 0).all()
    np.testing.assert_allclose(dep[inside], depth[0].ravel()[inside], rtol=1e-5)


# ---------------------------------------------------------------------------
# P5: integer-disparity shift


def test_integer_disparity_shift():
    W, H, f = 64, 24, 300.0
    d0 = 3.0
    src = [scenes.make_camera(W, H, f, (0.05, 0, 0), (0.05, 0, 1)).quantized()]
    tgt = scenes.make_camera(W, H, f, (0.0, 0, 0), (0.0, 0, 1)).quantized()
    depth = np.full((1, H, W), d0, np.float32)
    rng = np.random.default_rng(2)
    rgb = rng.integers(0, 256, (1, H, W, 3), dtype=np.uint8)
    out = oracle.splat(src, depth, rgb, tgt, scenes.splat_params())
    # f * b / d0 = 5 px: target pixel a sees source pixel a + 5
    for b in range(H):
        for a in range(W - 5):
            assert out["win_idx"][0, b, a] == b * W + a + 5
            np.testing.assert_allclose(out["rgb"][0, :, b, a], rgb[0, b, a + 5] / 255.0, atol=1e-6)
        assert (out["win_idx"][0, b, W - 5:] == -1).all()


# ---------------------------------------------------------------------------
# P4: brute-force per-ray TSDF (8x8); P7: brute-force z-buffer (16x16)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tsdf_matches_bruteforce(seed):
    c = scenes.small_ring(seed=seed, width=8, height=8, k=2, noise=0.01, holes=0.05, f=7.5)
    prm = c["tsdf"]
    F, W = oracle.integrate(c["src"], c["depth"], c["tgt"], prm)
    Fb, Wb, amb = bf.tsdf(c["src"], c["depth"], c["tgt"], prm)
    ok = ~amb
    assert ok.mean() > 0.97
    assert (Wb[ok] > 0).mean() > 0.3
    np.testing.assert_allclose(W[ok], Wb[ok], rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(F[ok], Fb[ok], rtol=1e-5, atol=2e-6)
    dep, b = oracle.extract(F, W, prm)
    depb, bb = bf.extract(Fb, Wb, prm)
    clean = ~amb.any(1)
    assert np.array_equal(b[clean], bb[clean])
    np.testing.assert_allclose(dep[clean], depb[clean], rtol=1e-5)


@pytest.mark.parametrize("seed,tgt_f", [(0, 15.0), (3, 15.0), (1, 27.0), (2, 9.0)])
def test_splat_matches_bruteforce_zbuffer(seed, tgt_f):
    c = scenes.small_ring(seed=seed, width=16, height=16, k=2, noise=0.01, holes=0.03, f=15.0)
    c["tgt"].fx = c["tgt"].fy = tgt_f  # zoomed target: splat size scales with f_T / f_k
    out = oracle.splat(c["src"], c["depth"], c["rgb"], c["tgt"], c["splat"])
    win, zw, col, alpha, amb = bf.zbuffer(c["src"], c["depth"], c["rgb"], c["tgt"], c["splat"])
    ok = ~amb
    assert ok.mean() > 0.95
    assert (win[ok] >= 0).mean() > (0.5 if tgt_f >= 15 else 0.25)  # zoomed out: sparse splats
    assert np.array_equal(out["win_idx"][ok], win[ok])
    np.testing.assert_allclose(out["depth"][ok], zw[ok], rtol=1e-6)
    np.testing.assert_allclose(out["alpha"][ok], alpha[ok], rtol=1e-5, atol=1e-6)
    okc = np.broadcast_to(ok[:, None], col.shape)
    np.testing.assert_allclose(out["rgb"][okc], col[okc], rtol=1e-5, atol=1e-6)


# ---------------------------------------------------------------------------
# FP32 oracle within rounding of the FP64 build


def test_fp32_within_rounding_of_fp64():
    c = scenes.config1()
    prm = c["tsdf"]
    pix = np.arange(0, 76800, 53, dtype=np.int32)
    F32, W32 = oracle.integrate(c["src"], c["depth"], c["tgt"], prm, pixels=pix)
    F64, W64 = oracle.integrate(c["src"], c["depth"], c["tgt"], prm, pixels=pix, prec=64)
    same = (W32 > 0) == (W64 > 0)
    assert same.mean() > 0.999
    np.testing.assert_allclose(F32[same], F64[same], rtol=1e-4, atol=1e-5)
