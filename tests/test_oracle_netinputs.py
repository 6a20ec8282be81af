"""Pins of the oracle's network-input maps and blend (§3.3, the supplement's
network inputs, Eq. 4-5): closed forms on planes, an FP64 numpy brute force
through world space, an analytic sphere, and the blend's special cases."""
import numpy as np
import pytest

import oracle
import scenes


def centre(c):
    R = np.asarray(c.R, np.float64).reshape(3, 3)
    return -R.T @ np.asarray(c.t, np.float64)


def world_points(tgt, D):
    """FP64 back-projection of every target pixel at depth D, world space."""
    H, W = D.shape
    j, i = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    x = (i + 0.5 - tgt.cx) / tgt.fx
    y = (j + 0.5 - tgt.cy) / tgt.fy
    cam = np.stack([x * D, y * D, D], -1)
    R = np.asarray(tgt.R, np.float64).reshape(3, 3)
    return (cam - np.asarray(tgt.t, np.float64)) @ R  # R^T (X_c - t)


def bruteforce(src, tgt, D):
    """FP64 normal (central / one-sided differences) and ray dot products."""
    P = world_points(tgt, D.astype(np.float64))
    H, W = D.shape
    ok = D > 0
    pad = np.pad(P, ((1, 1), (1, 1), (0, 0)))
    okp = np.pad(ok, 1)
    L, Rr, U, Dn = pad[1:-1, :-2], pad[1:-1, 2:], pad[:-2, 1:-1], pad[2:, 1:-1]
    oL, oR, oU, oD = okp[1:-1, :-2], okp[1:-1, 2:], okp[:-2, 1:-1], okp[2:, 1:-1]
    tx = np.where((oL & oR)[..., None], Rr - L, np.where(oR[..., None], Rr - P,
                  np.where(oL[..., None], P - L, 0)))
    ty = np.where((oU & oD)[..., None], Dn - U, np.where(oD[..., None], Dn - P,
                  np.where(oU[..., None], P - U, 0)))
    n = np.cross(tx, ty)
    ln = np.linalg.norm(n, axis=-1, keepdims=True)
    n = np.where(ln > 0, n / np.where(ln > 0, ln, 1), 0)
    Ct = centre(tgt)
    flip = ((Ct - P) * n).sum(-1) < 0
    n[flip] *= -1
    hasn = ok & (oL | oR) & (oU | oD) & (ln[..., 0] > 0)
    dt = P - Ct
    dt /= np.linalg.norm(dt, axis=-1, keepdims=True)
    dn, dd = [], []
    for c in src:
        r = P - centre(c)
        r /= np.linalg.norm(r, axis=-1, keepdims=True)
        dn.append(np.where(hasn, (r * n).sum(-1), 0))
        dd.append(np.where(ok, (r * dt).sum(-1), 0))
    return np.array(dn), np.array(dd), n, hasn


def _inputs(K=3, W=40, H=30):
    ring = scenes.ring_rig(16, 1.0, W, H)
    tgt = scenes.ring_target(2 * np.pi * 2.5 / 16, 1.0, W, H).quantized()
    src = [ring[i].quantized() for i in (1, 2, 3, 4)[:K]]
    rng = np.random.default_rng(0)
    rgb = rng.uniform(0, 1, (K, 3, H, W)).astype(np.float32)
    dk = rng.uniform(0.5, 5, (K, H, W)).astype(np.float32)
    al = rng.uniform(0, 1, (K, H, W)).astype(np.float32)
    return src, tgt, rgb, dk, al


def test_layout_and_constant_planes():
    src, tgt, rgb, dk, al = _inputs()
    K = len(src)
    D = np.full((tgt.height, tgt.width), 2.0, np.float32)
    out = oracle.network_inputs(src, tgt, D, rgb, dk, al, prec=64)
    assert out.shape == (9 * K + 1, tgt.height, tgt.width)
    np.testing.assert_array_equal(out[:3 * K], rgb.reshape(3 * K, tgt.height, tgt.width))
    np.testing.assert_array_equal(out[3 * K:4 * K], dk)
    np.testing.assert_array_equal(out[4 * K:5 * K], al)
    np.testing.assert_array_equal(out[5 * K], D)
    Ct = centre(tgt)
    for k, c in enumerate(src):
        np.testing.assert_allclose(out[7 * K + 1 + k], np.linalg.norm(centre(c) - Ct), rtol=1e-12)
        ax = np.dot(np.asarray(c.R, np.float64).ravel()[6:], np.asarray(tgt.R, np.float64).ravel()[6:])
        np.testing.assert_allclose(out[8 * K + 1 + k], ax, rtol=1e-12)


@pytest.mark.parametrize("shape", ["plane", "tilted", "holes"])
def test_maps_match_world_space_bruteforce(shape):
    src, tgt, rgb, dk, al = _inputs()
    K = len(src)
    H, W = tgt.height, tgt.width
    j, i = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    if shape == "plane":
        D = np.full((H, W), 2.3)
    else:
        # a plane tilted in the target frame: 1/D affine in pixel coordinates
        D = 1.0 / (0.45 + 0.004 * (i - W / 2) - 0.003 * (j - H / 2))
    D = D.astype(np.float32)
    if shape == "holes":
        D[np.random.default_rng(3).random(D.shape) < 0.1] = 0
    out = oracle.network_inputs(src, tgt, D, rgb, dk, al, prec=64)
    dn, dd, n, hasn = bruteforce(src, tgt, D)
    np.testing.assert_allclose(out[5 * K + 1:6 * K + 1], dn, atol=1e-9)
    np.testing.assert_allclose(out[6 * K + 1:7 * K + 1], dd, atol=1e-9)
    out32 = oracle.network_inputs(src, tgt, D, rgb, dk, al)
    np.testing.assert_allclose(out32[5 * K + 1:7 * K + 1], out[5 * K + 1:7 * K + 1], atol=2e-4)
    if shape != "holes":
        # a plane: every normal is the plane's, facing the target
        assert hasn.all()
        Ct = centre(tgt)
        P = world_points(tgt, D.astype(np.float64))
        assert (((Ct - P) * n).sum(-1) > 0).all()
        # (the FP32 depths are coplanar to ~1e-7 relative)
        assert np.abs(n - n[H // 2, W // 2]).max() < 2e-5


def test_sphere_normals_are_radial():
    """A sphere fills the target: the map's normal dot each input ray equals
    the analytic one (radial normal) to the chord error of neighbouring
    pixels."""
    W, H = 96, 72
    ring = scenes.ring_rig(16, 1.0, W, H)
    tgt = ring[2].quantized()
    src = [ring[1].quantized(), ring[3].quantized()]
    sph = scenes.Sphere(np.zeros(3), 0.45, 0, np.array([0.5, 0.5, 0.5]))
    o, d = scenes.rays(tgt)
    lam, _, _ = sph.hit(o, d)
    hit = np.isfinite(lam) & (lam > 0)
    # ray length -> camera z depth
    fwd = np.asarray(tgt.R, np.float64).ravel()[6:]
    zc = np.where(hit, lam * (d @ fwd), 0).astype(np.float32)
    K = 2
    out = oracle.network_inputs(src, tgt, zc, np.zeros((K, 3, H, W), np.float32),
                                np.zeros((K, H, W), np.float32), np.zeros((K, H, W), np.float32),
                                prec=64)
    P = world_points(tgt, zc.astype(np.float64))
    nrm = P / np.linalg.norm(P, axis=-1, keepdims=True)
    inner = hit.copy()
    for s in ((0, 1), (0, -1), (1, 0), (-1, 0)):
        inner &= np.roll(hit, s, axis=(0, 1))
    for k, c in enumerate(src):
        r = P - centre(c)
        r /= np.linalg.norm(r, axis=-1, keepdims=True)
        ref = (r * nrm).sum(-1)
        err = np.abs(out[5 * K + 1 + k] - ref)[inner]
        # chords grow towards the silhouette (grazing view)
        assert np.median(err) < 2e-3 and np.percentile(err, 95) < 1e-2 and err.max() < 0.1


def test_blend_special_cases():
    rng = np.random.default_rng(5)
    K, H, W = 3, 7, 9
    rgb = rng.uniform(0, 1, (K, 3, H, W)).astype(np.float32)
    dep = rng.uniform(0.5, 5, (K, H, W)).astype(np.float32)
    one = np.ones((K, H, W), np.float32)
    zero_bg = np.zeros((H, W), np.float32)
    bg = rng.uniform(0, 1, (3, H, W)).astype(np.float32)
    # a single view with weight and alpha 1 is reproduced exactly
    w = np.zeros((K, H, W), np.float32)
    w[1] = 1
    o, d = oracle.blend(rgb, dep, one, w, zero_bg, bg)
    np.testing.assert_array_equal(o, rgb[1])
    np.testing.assert_array_equal(d, dep[1])
    # w_BG = 1 gives the background
    o, _ = oracle.blend(rgb, dep, one, one, np.ones((H, W), np.float32), bg)
    np.testing.assert_array_equal(o, bg)
    # no weight anywhere: the foreground is 0
    o, d = oracle.blend(rgb, dep, one, np.zeros_like(one), np.full((H, W), 0.25, np.float32), bg)
    np.testing.assert_allclose(o, 0.25 * bg, rtol=1e-6)
    assert (d == 0).all()
    # equal weights: the alpha-weighted mean, FP64
    al = rng.uniform(0.1, 1, (K, H, W)).astype(np.float32)
    o, d = oracle.blend(rgb, dep, al, one, zero_bg, bg, prec=64)
    r64, a64, d64 = rgb.astype(np.float64), al.astype(np.float64), dep.astype(np.float64)
    ref = (r64 * a64[:, None]).sum(0) / a64.sum(0)
    np.testing.assert_allclose(o, ref, rtol=1e-12)
    np.testing.assert_allclose(d, (d64 * a64).sum(0) / a64.sum(0), rtol=1e-12)
