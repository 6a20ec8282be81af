"""The oracle's adjoints against central finite differences (FP64 build).

The losses are L = <g, depth_tsdf> for fusion + extraction and
L = <g_rgb, rgb> + <g_z, depth> + <g_a, alpha> for the splat, with seeded
random upstream gradients.  Finite differences use h = 1e-3 m on the input
depth (the perturbed inputs are FP32, so the quotient divides by the actual
representable step).  The extracted depth is a rational function of F on the
scale of the truncation (centimetres), so a 1 mm step carries an O(h^2) error
of ~1e-4: the quotients at h, h/2 and h/4 are Richardson-extrapolated.  The
method is piecewise smooth: coverage, band and winner sets, clamps, the
zero-crossing bin and the min of the fusion weight switch at kinks.  A sample
whose two extrapolations (h, h/2) and (h/2, h/4) disagree straddles such a
kink and is skipped.  With 1 cm noise against a 2 cm window threshold, a
millimetre step meets a kink of the fusion weight for a large share of the
samples, so the 1 mm check bounds the skip rate loosely and a second check at
h = 1e-5 m, where kinks are rare, bounds it tightly.
"""
import numpy as np

import oracle
import scenes


def _small_parallel(W=64, H=36, D=48):
    f = 0.9375 * W
    src = scenes._quantize_all(scenes.parallel_rig([-0.15, -0.05, 0.05, 0.15], W, H, f))
    tgt = scenes.parallel_rig([0.0], W, H, f)[0].quantized()
    rng = np.random.default_rng(11)
    depth, rgb = scenes.make_frame(src, tgt, scenes._cfg1_scene(0), rng, 0.01, 0.01)
    return dict(src=src, tgt=tgt, depth=depth, rgb=rgb, splat=scenes.splat_params(),
                tsdf=scenes.tsdf_params(num_bins=D, trunc=3.0))


def _fd(loss, depth, k, j, i, h):
    dp = depth.copy()
    dm = depth.copy()
    dp[k, j, i] = np.float32(depth[k, j, i] + h)
    dm[k, j, i] = np.float32(depth[k, j, i] - h)
    step = float(dp[k, j, i]) - float(dm[k, j, i])
    return (loss(dp) - loss(dm)) / step


def _check(loss, grad, depth, rng, n=256, h=1e-3):
    K, H, W = depth.shape
    cand = np.argwhere((grad != 0) & (depth > 0))
    assert len(cand) > n
    pick = cand[rng.choice(len(cand), n, replace=False)]
    skipped = 0
    errs = []
    scale = np.abs(grad).max()
    for k, j, i in pick:
        f1, f2, f4 = (_fd(loss, depth, k, j, i, h / m) for m in (1, 2, 4))
        a = (4 * f2 - f1) / 3
        b = (4 * f4 - f2) / 3
        if abs(a - b) > 1e-3 * max(abs(b), 1e-3 * scale):
            skipped += 1
            continue
        g = grad[k, j, i]
        errs.append(abs(b - g) / max(abs(g), 1e-3 * scale))
    return skipped / n, np.array(errs)


def test_tsdf_backward_matches_finite_differences():
    c = _small_parallel()
    prm = c["tsdf"]
    rng = np.random.default_rng(3)
    g = rng.standard_normal(c["tgt"].width * c["tgt"].height)

    def loss(depth):
        F, W = oracle.integrate(c["src"], depth, c["tgt"], prm, prec=64)
        dep, b = oracle.extract(F, W, prm, prec=64)
        return float((g * dep).sum())

    grad = oracle.tsdf_backward(c["src"], c["depth"], c["tgt"], prm, g, prec=64)
    skip, worst = _check(loss, grad, c["depth"], rng)
    assert skip < 0.6, skip
    # a kink can hide inside the 1 mm bracket: bound the bulk, not the tail
    assert np.median(worst) < 1e-5 and np.percentile(worst, 90) < 1e-3, worst
    skip, worst = _check(loss, grad, c["depth"], rng, n=128, h=1e-5)
    assert skip < 0.1, skip
    assert worst.max() < 1e-4, worst


def test_tsdf_backward_with_carry():
    c = _small_parallel(W=48, H=27, D=32)
    prm = c["tsdf"]
    rng = np.random.default_rng(4)
    F0, W0 = oracle.integrate(c["src"], c["depth"], c["tgt"], prm, prec=64)
    depth2 = (c["depth"] * np.float32(1.002)).astype(np.float32)
    g = rng.standard_normal(c["tgt"].width * c["tgt"].height)

    def loss(depth):
        F, W = oracle.integrate(c["src"], depth, c["tgt"], prm, F_prev=F0, W_prev=W0, prec=64)
        dep, b = oracle.extract(F, W, prm, prec=64)
        return float((g * dep).sum())

    grad = oracle.tsdf_backward(c["src"], depth2, c["tgt"], prm, g, F_prev=F0, W_prev=W0, prec=64)
    skip, worst = _check(loss, grad, depth2, rng, n=128)
    assert skip < 0.6, skip
    # a kink can hide inside the 1 mm bracket: bound the bulk, not the tail
    assert np.median(worst) < 1e-5 and np.percentile(worst, 90) < 1e-3, worst
    skip, worst = _check(loss, grad, depth2, rng, n=128, h=1e-5)
    assert skip < 0.1, skip
    assert worst.max() < 1e-4, worst


def test_splat_backward_depth_matches_finite_differences():
    c = _small_parallel(W=48, H=27)
    sp = c["splat"]
    K, H, W = c["depth"].shape
    rng = np.random.default_rng(5)
    g_rgb = rng.standard_normal((K, 3, H, W))
    g_z = rng.standard_normal((K, H, W))
    g_a = rng.standard_normal((K, H, W))

    def loss(depth):
        o = oracle.splat(c["src"], depth, c["rgb"], c["tgt"], sp, prec=64)
        return float((g_rgb * o["rgb"]).sum() + (g_z * o["depth"]).sum() + (g_a * o["alpha"]).sum())

    gd, gc = oracle.splat_backward(c["src"], c["depth"], c["rgb"], c["tgt"], sp, g_rgb, g_z, g_a,
                                   prec=64)
    skip, worst = _check(loss, gd, c["depth"], rng)
    assert skip < 0.6, skip
    # a kink can hide inside the 1 mm bracket: bound the bulk, not the tail
    assert np.median(worst) < 1e-5 and np.percentile(worst, 90) < 1e-3, worst
    skip, worst = _check(loss, gd, c["depth"], rng, n=128, h=1e-5)
    assert skip < 0.1, skip
    assert worst.max() < 1e-4, worst


def test_splat_backward_depth_ring_rig():
    """Rotated views with depth-direction baselines, so the footprint's
    dependence on depth (sigma = s_k D / z_T) enters the gradient."""
    c = scenes.small_ring(seed=4, width=40, height=30, k=2, noise=0.01, holes=0.02)
    c["tgt"].fx = c["tgt"].fy = float(np.float32(c["tgt"].fx * 1.7))
    sp = c["splat"]
    K, H, W = c["depth"].shape
    Ht, Wt = c["tgt"].height, c["tgt"].width
    rng = np.random.default_rng(8)
    g_rgb = rng.standard_normal((K, 3, Ht, Wt))
    g_z = rng.standard_normal((K, Ht, Wt))
    g_a = rng.standard_normal((K, Ht, Wt))

    def loss(depth):
        o = oracle.splat(c["src"], depth, c["rgb"], c["tgt"], sp, prec=64)
        return float((g_rgb * o["rgb"]).sum() + (g_z * o["depth"]).sum() + (g_a * o["alpha"]).sum())

    gd, gc = oracle.splat_backward(c["src"], c["depth"], c["rgb"], c["tgt"], sp, g_rgb, g_z, g_a,
                                   prec=64)
    skip, worst = _check(loss, gd, c["depth"], rng, n=128, h=1e-5)
    assert skip < 0.1, skip
    assert worst.max() < 1e-4, worst


def test_splat_backward_colour_is_exact_linear():
    """Colour enters linearly: L(c) - L(0) = <dL/dc, c> exactly, and one
    8-bit step of one input pixel moves L by dL/dc / 255."""
    c = _small_parallel(W=48, H=27)
    sp = c["splat"]
    K, H, W = c["depth"].shape
    rng = np.random.default_rng(6)
    g_rgb = rng.standard_normal((K, 3, H, W))
    zeros = np.zeros((K, H, W))

    def loss(rgb):
        o = oracle.splat(c["src"], c["depth"], rgb, c["tgt"], sp, prec=64)
        return float((g_rgb * o["rgb"]).sum())

    gd, gc = oracle.splat_backward(c["src"], c["depth"], c["rgb"], c["tgt"], sp, g_rgb, zeros,
                                   zeros, prec=64)
    cf = c["rgb"].astype(np.float64) / 255.0
    lhs = loss(c["rgb"]) - loss(np.zeros_like(c["rgb"]))
    np.testing.assert_allclose(lhs, (gc * cf).sum(), rtol=1e-10)
    for _ in range(20):
        k, j, i, ch = (rng.integers(K), rng.integers(H), rng.integers(W), rng.integers(3))
        rgb2 = c["rgb"].copy()
        up = rgb2[k, j, i, ch] < 255
        rgb2[k, j, i, ch] = rgb2[k, j, i, ch] + (1 if up else -1)
        dl = loss(rgb2) - loss(c["rgb"])
        np.testing.assert_allclose(dl, (1 if up else -1) * gc[k, j, i, ch] / 255.0,
                                   rtol=1e-9, atol=1e-12)
