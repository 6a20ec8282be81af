"""Pins of the oracle's EWA front-to-back compositing (§3.1, the per-pixel
Gaussians rendered as by the 3D Gaussian splatting rasteriser): the exp
routine against numpy, closed forms for a single Gaussian under an identity
warp, the EWA covariance against a numerically differentiated projection
through world space, an FP64 numpy brute force of the sorted compositing on
tiny scenes, and invariants (termination bound, colour and depth of
uniform planes, per-pixel sampling)."""
import numpy as np
import pytest

import oracle
import scenes

LP = 0.3


def _sp(**kw):
    p = dict(sigma_px=0.5, band_rel=0.01, z_min=0.05, r_max_px=8.0)
    p.update(kw)
    return p


def test_exp_accuracy_and_shape():
    x = np.linspace(-86.0, 0.0, 400001).astype(np.float32)
    y = oracle.exp_cw(x).astype(np.float64)
    e = np.exp(x.astype(np.float64))
    ulp = np.abs(y - e) / np.spacing(e.astype(np.float32)).astype(np.float64)
    assert ulp.max() <= 3.0
    assert np.all(np.diff(y) >= 0)  # monotone, so thresholds cut one interval
    assert oracle.exp_cw([0.0])[0] == 1.0
    assert np.all(oracle.exp_cw([-86.5, -100.0, -np.inf]) == 0.0)
    # around the switch points of the reduction, (n + 1/2) ln 2, where the
    # reduced argument jumps from +ln2/2 to -ln2/2
    n = np.arange(-120, 0, dtype=np.float64)
    c = ((n + 0.5) * np.log(2.0)).astype(np.float32)
    x = np.concatenate([np.nextafter(c, np.float32(-np.inf)), c,
                        np.nextafter(c, np.float32(np.inf))]).astype(np.float32)
    y = oracle.exp_cw(x).astype(np.float64)
    e = np.exp(x.astype(np.float64))
    assert np.all(np.abs(y - e) <= 3 * np.spacing(e.astype(np.float32)))


def _identity(W=9, H=7, f=12.0, z0=2.0, rgb=(200, 100, 50), valid=None):
    cam = scenes.make_camera(W, H, f, (0.0, 0.0, 0.0), (0.0, 0.0, 1.0)).quantized()
    depth = np.full((1, H, W), z0, np.float32)
    if valid is not None:
        depth[0][~valid] = 0.0
    col = np.zeros((1, H, W, 3), np.uint8)
    col[...] = np.array(rgb, np.uint8)
    return cam, depth, col


@pytest.mark.parametrize("lp", [0.3, 0.0, 1.0])
def test_single_gaussian_closed_form(lp):
    """One valid source pixel, the target equal to the source camera, at the
    principal point: S = (sigma_px^2 + lp) I, so alpha at offset (dx, dy) is
    min(0.99, exp(-(dx^2 + dy^2) / (2 (0.25 + lp))))."""
    W, H = 9, 7
    valid = np.zeros((H, W), bool)
    valid[3, 4] = True
    cam, depth, col = _identity(W, H, valid=valid)
    # principal point at the centre of pixel (4, 3)
    cam = scenes.Camera(cam.fx, cam.fy, 4.5, 3.5, cam.R, cam.t, W, H)
    o = oracle.splat_ewa([cam], depth, col, cam, _sp(), lowpass=lp, prec=64)
    j, i = np.mgrid[0:H, 0:W]
    d2 = (i - 4.0) ** 2 + (j - 3.0) ** 2
    a = np.minimum(0.99, np.exp(-d2 / (2 * (0.25 + lp))))
    a = np.where(a >= 1 / 255, a, 0.0)
    np.testing.assert_allclose(o["alpha"][0], a, rtol=1e-6, atol=1e-12)
    c = np.array([200, 100, 50]) / 255.0
    np.testing.assert_allclose(o["rgb"][0], c[:, None, None] * a[None], rtol=1e-6, atol=1e-12)
    np.testing.assert_allclose(o["depth"][0], np.where(a > 0, 2.0, 0.0), rtol=1e-9)


def _world_to_cam(c, X):
    return X @ np.asarray(c.R, np.float64).T + np.asarray(c.t, np.float64)


def _project(c, Xc):
    return np.stack([c.fx * Xc[..., 0] / Xc[..., 2] + c.cx,
                     c.fy * Xc[..., 1] / Xc[..., 2] + c.cy], -1)


def _gaussians(src_cams, depth, rgb, tgt, sp, lp):
    """FP64 Gaussians of every valid source pixel, built through world space:
    mean = projection of the back-projected point, covariance =
    sigma3^2 J J^T + lp I with J the numerically differentiated projection
    (central differences) and sigma3 = sigma_px D / f_k."""
    out = []
    for k, c in enumerate(src_cams):
        Hs, Ws = depth[k].shape
        Rk = np.asarray(c.R, np.float64)
        for j in range(Hs):
            for i in range(Ws):
                D = float(depth[k, j, i])
                if not (D > 0 and np.isfinite(D)):
                    continue
                xc = np.array([(i + 0.5 - c.cx) / c.fx * D, (j + 0.5 - c.cy) / c.fy * D, D])
                X = Rk.T @ (xc - np.asarray(c.t, np.float64))
                Xt = _world_to_cam(tgt, X[None])[0]
                if not Xt[2] > sp["z_min"]:
                    continue
                mu = _project(tgt, Xt[None])[0]
                h = 1e-5 * max(1.0, abs(Xt[2]))
                J = np.zeros((2, 3))
                for e in range(3):
                    dp = np.zeros(3)
                    dp[e] = h
                    J[:, e] = (_project(tgt, (Xt + dp)[None])[0]
                               - _project(tgt, (Xt - dp)[None])[0]) / (2 * h)
                s3 = sp["sigma_px"] * D / c.fx
                S = s3 * s3 * (J @ J.T) + lp * np.eye(2)
                out.append(dict(k=k, q=j * Ws + i, z=Xt[2], mu=mu, Si=np.linalg.inv(S),
                                S=S, c=rgb[k, j, i].astype(np.float64) / 255.0))
    return out


def _bruteforce(src_cams, depth, rgb, tgt, sp, lp):
    g = _gaussians(src_cams, depth, rgb, tgt, sp, lp)
    K = len(src_cams)
    Ht, Wt = tgt.height, tgt.width
    rgb_o = np.zeros((K, 3, Ht, Wt))
    a_o = np.zeros((K, Ht, Wt))
    d_o = np.zeros((K, Ht, Wt))
    r = sp["r_max_px"]
    for k in range(K):
        gk = sorted([e for e in g if e["k"] == k],
                    key=lambda e: (np.float32(e["z"]), e["q"]))
        for y in range(Ht):
            for x in range(Wt):
                T, col, zs = 1.0, np.zeros(3), 0.0
                for e in gk:
                    d = np.array([x + 0.5, y + 0.5]) - e["mu"]
                    if abs(d[0]) > r or abs(d[1]) > r:
                        continue
                    al = min(0.99, np.exp(-0.5 * d @ e["Si"] @ d))
                    if al < 1 / 255:
                        continue
                    if T * (1 - al) < 1e-4:
                        break
                    col += e["c"] * al * T
                    zs += e["z"] * al * T
                    T *= 1 - al
                rgb_o[k, :, y, x] = col
                a_o[k, y, x] = 1 - T
                d_o[k, y, x] = zs / (1 - T) if T < 1 else 0.0
    return dict(rgb=rgb_o, alpha=a_o, depth=d_o), g


def _tiny(seed, K=2, Ws=10, Hs=8, Wt=12, Ht=9, holes=0.15):
    rng = np.random.default_rng(seed)
    ring = scenes.ring_rig(12, 1.0, Ws, Hs, f=0.9 * Ws)
    tgt = scenes.ring_target(2 * np.pi * 1.4 / 12, 1.0, Wt, Ht, f=0.9 * Wt).quantized()
    src = [ring[i].quantized() for i in range(1, 1 + K)]
    # a lumpy surface: depths vary smoothly plus an occluding step
    depth = np.empty((K, Hs, Ws), np.float32)
    for k in range(K):
        jj, ii = np.mgrid[0:Hs, 0:Ws]
        d = 0.9 + 0.08 * np.sin(ii * 0.7 + k) + 0.05 * np.cos(jj * 0.9)
        d[:, Ws // 2:] -= 0.15  # a step: the right half is nearer
        d[rng.random((Hs, Ws)) < holes] = 0.0
        depth[k] = d
    rgb = rng.integers(0, 256, (K, Hs, Ws, 3), dtype=np.uint8)
    return src, depth, rgb, tgt


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bruteforce_world_space(seed):
    """The FP64 oracle equals an FP64 brute force that projects through
    world space, differentiates the projection numerically, sorts with
    Python's sort and composites with numpy's exp."""
    src, depth, rgb, tgt = _tiny(seed)
    sp = _sp(sigma_px=0.5 + 0.4 * seed)
    o = oracle.splat_ewa(src, depth, rgb, tgt, sp, lowpass=LP, prec=64)
    b, g = _bruteforce(src, depth, rgb, tgt, sp, LP)
    assert len(g) > 50
    assert (b["alpha"] > 0.5).mean() > 0.2  # the scene covers the target
    for key in ("rgb", "alpha", "depth"):
        np.testing.assert_allclose(o[key], b[key], rtol=2e-6, atol=2e-7, err_msg=key)


def test_bruteforce_clip_binds():
    """A target much nearer than the sources magnifies the Gaussians beyond
    the r_max clip: the clipped square edges must match the brute force."""
    src, depth, rgb, tgt = _tiny(5, K=1, Wt=14, Ht=10)
    sp = _sp(sigma_px=2.5, r_max_px=2.0)
    o = oracle.splat_ewa(src, depth, rgb, tgt, sp, lowpass=LP, prec=64)
    b, _ = _bruteforce(src, depth, rgb, tgt, sp, LP)
    for key in ("rgb", "alpha", "depth"):
        np.testing.assert_allclose(o[key], b[key], rtol=2e-6, atol=2e-7, err_msg=key)
    o2 = oracle.splat_ewa(src, depth, rgb, tgt, _sp(sigma_px=2.5, r_max_px=8.0), lowpass=LP,
                          prec=64)
    assert np.abs(o2["alpha"] - o["alpha"]).max() > 1e-3  # the clip is active


def test_fp32_build_tracks_fp64():
    src, depth, rgb, tgt = _tiny(3, Wt=16, Ht=12)
    sp = _sp()
    o32 = oracle.splat_ewa(src, depth, rgb, tgt, sp, prec=32)
    o64 = oracle.splat_ewa(src, depth, rgb, tgt, sp, prec=64)
    for key in ("rgb", "alpha", "depth"):
        d = np.abs(o32[key].astype(np.float64) - o64[key])
        assert np.median(d) < 1e-6 and np.quantile(d, 0.99) < 1e-5, key


def _plane_scene(W=24, H=18, seed=0, rgb_const=None):
    rng = np.random.default_rng(seed)
    cam = scenes.make_camera(W, H, 20.0, (0.0, 0.0, 0.0), (0.0, 0.0, 1.0)).quantized()
    tgt = scenes.make_camera(W, H, 20.0, (0.02, -0.01, 0.0), (0.02, -0.01, 1.0)).quantized()
    depth = np.full((1, H, W), 1.5, np.float32)
    if rgb_const is None:
        col = rng.integers(0, 256, (1, H, W, 3), dtype=np.uint8)
    else:
        col = np.zeros((1, H, W, 3), np.uint8)
        col[...] = np.array(rgb_const, np.uint8)
    return [cam], depth, col, tgt


@pytest.mark.parametrize("prec", [32, 64])
def test_plane_invariants(prec):
    """A fronto-parallel plane seen by a translated camera: every drawn pixel
    has depth 1.5 (all terms share z), opacity below 1 - 1e-4 (the stopping
    rule), interior pixels saturate, and a constant colour c gives rgb =
    c alpha."""
    src, depth, col, tgt = _plane_scene(rgb_const=(255, 128, 3))
    o = oracle.splat_ewa(src, depth, col, tgt, _sp(), prec=prec)
    a, d = o["alpha"][0], o["depth"][0]
    tol = 1e-6 if prec == 32 else 1e-12
    drawn = a > 0
    np.testing.assert_allclose(d[drawn], 1.5, rtol=tol)
    assert np.all(d[~drawn] == 0)
    assert a.max() <= 1 - 1e-4 + tol
    assert a[3:-3, 3:-3].min() > 0.99  # the stopping rule leaves T of a few 1e-3
    c = np.array([255, 128, 3]) / 255.0
    np.testing.assert_allclose(o["rgb"][0], c[:, None, None] * a[None], rtol=4 * tol,
                               atol=tol)


def test_equal_depth_ties_follow_source_index():
    """On a fronto-parallel plane all depths tie, so the order is the source
    index: swapping the colours of two overlapping pixels changes the
    result, and the brute force with (z, q) order agrees."""
    src, depth, col, tgt = _plane_scene(W=8, H=6, seed=4)
    sp = _sp()
    o = oracle.splat_ewa(src, depth, col, tgt, sp, lowpass=LP, prec=64)
    b, _ = _bruteforce(src, depth, col, tgt, sp, LP)
    np.testing.assert_allclose(o["rgb"], b["rgb"], rtol=2e-6, atol=2e-7)


def test_pixel_selection():
    src, depth, rgb, tgt = _tiny(7, Wt=20, Ht=15)
    full = oracle.splat_ewa(src, depth, rgb, tgt, _sp())
    pix = np.random.default_rng(0).choice(20 * 15, 40, replace=False)
    part = oracle.splat_ewa(src, depth, rgb, tgt, _sp(), pixels=pix)
    for key in ("rgb", "alpha", "depth"):
        f = full[key].reshape(*full[key].shape[:-2], -1)
        p = part[key].reshape(*part[key].shape[:-2], -1)
        assert np.array_equal(f[..., pix], p[..., pix])
        rest = np.setdiff1d(np.arange(300), pix)
        assert np.all(p[..., rest] == 0)


def test_nothing_valid():
    src, depth, rgb, tgt = _tiny(0)
    o = oracle.splat_ewa(src, np.zeros_like(depth), rgb, tgt, _sp())
    assert all(np.all(v == 0) for v in o.values())
    # everything behind the near plane
    o = oracle.splat_ewa(src, depth, rgb, tgt, _sp(z_min=100.0))
    assert all(np.all(v == 0) for v in o.values())


def test_exp_below_alpha_floor_for_every_float_under_minus_5_6():
    """Every FP32 x in [-86, -5.6] gives exp_cw(x) < 1/255 (exhaustive), so a
    term whose exponent is below -5.6 is always skipped: the GPU raster may
    skip such terms for a whole wavefront without evaluating them."""
    hi = np.array([-5.6], np.float32).view(np.uint32)[0]
    lo = np.array([-86.0], np.float32).view(np.uint32)[0]
    x = np.arange(hi, lo + 1, dtype=np.uint32).view(np.float32)
    amin = np.float32(1) / np.float32(255)
    for i in range(0, x.size, 1 << 23):
        assert oracle.exp_cw(x[i:i + (1 << 23)]).max() < amin
