"""Pins of the oracle's temporal path: the difference masks of Eq. 1, the
filtered depth of Eq. 2 and the splat of the masks with their maximum over
the views (§3.2, Suppl. A.2).  Closed forms, an independent FP64 brute force
and special cases that reduce to the identity."""
import numpy as np
import pytest

import oracle
import scenes
from tests import bruteforce as bf

BETA, LAM = 0.6, 0.7
# the parameters reach the oracle as FP32 (both builds)
B32, L32 = float(np.float32(BETA)), float(np.float32(LAM))


def _frames(seed, H, W, K=1, lo=0, hi=256):
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi, (K, H, W, 3), dtype=np.uint8)


@pytest.mark.parametrize("H,W", [(23, 41), (16, 16), (1, 1), (5, 130)])
def test_identical_frames_give_beta(H, W):
    a = _frames(0, H, W, K=2)
    m = oracle.difference_mask(a, a)
    assert (m == np.float32(BETA)).all()


@pytest.mark.parametrize("k", [1, 10, 60, 200])
def test_uniform_colour_change_closed_form(k):
    a = _frames(1, 21, 35, lo=0, hi=256 - k)
    b = (a.astype(np.int32) + k).astype(np.uint8)
    m = oracle.difference_mask(b, a, prec=64)
    ref = min(k / 255.0 / L32 + B32, 1.0)
    np.testing.assert_allclose(m, ref, rtol=1e-14)
    m32 = oracle.difference_mask(b, a)
    np.testing.assert_allclose(m32, ref, rtol=3e-7)
    assert (m32 <= 1.0).all()


@pytest.mark.parametrize("seed,H,W,factor", [(0, 37, 53, 4), (1, 16, 16, 4), (2, 30, 9, 4),
                                             (3, 20, 28, 2), (4, 13, 17, 3)])
def test_difference_mask_matches_bruteforce(seed, H, W, factor):
    a = _frames(seed, H, W)[0]
    b = a.copy()
    rng = np.random.default_rng(seed + 10)
    # a few changed patches of different strength, the rest static
    for _ in range(4):
        y, x = rng.integers(0, H), rng.integers(0, W)
        h, w = rng.integers(1, 9), rng.integers(1, 9)
        b[y:y + h, x:x + w] = rng.integers(0, 256, (min(h, H - y), min(w, W - x), 3))
    ref = bf.difference_mask(b, a, factor, B32, L32)
    m64 = oracle.difference_mask(b, a, factor=factor, prec=64)
    np.testing.assert_allclose(m64, ref, rtol=0, atol=1e-13)
    m32 = oracle.difference_mask(b, a, factor=factor)
    np.testing.assert_allclose(m32, ref, rtol=0, atol=1e-6)
    assert (ref > B32 + 1e-3).any()


def test_single_changed_block_spreads_over_its_pooled_neighbourhood():
    """One fully changed 4x4 block (low-res pixel (3, 5)) saturates the mask
    at 1 there; the max-pool spreads it to low-res pixels 2..4 x 4..6, and a
    full-resolution pixel reads only those where both bilinear samples lie in
    that range: rows 4*3-2 .. 4*3+1 and columns 4*5-2 .. 4*5+1 and beyond
    into the pooled neighbourhood."""
    H, W = 40, 48
    a = np.zeros((H, W, 3), np.uint8)
    b = a.copy()
    b[12:16, 20:24] = 255
    m = oracle.difference_mask(b, a, prec=64)
    # low-res 1 on rows 2..4 (full-res sample window [8, 20)), cols 4..6
    # x in [a-1, a+1] needs both taps inside: i + 0.5 in [4 * 4 + 2, 4 * 6 + 2]
    ones = m == 1.0
    assert ones[10:18, 18:26].all()
    assert not ones[:9].any() and not ones[19:].any()
    assert not ones[:, :17].any() and not ones[:, 27:].any()
    far = m[30:, 40:]
    assert (far == B32).all()


def test_temporal_filter_closed_forms():
    rng = np.random.default_rng(3)
    D = rng.uniform(0.5, 5.0, (6, 9)).astype(np.float32)
    prev = rng.uniform(0.5, 5.0, (6, 9)).astype(np.float64)
    one = np.ones_like(D, np.float64)
    np.testing.assert_array_equal(oracle.temporal_filter(D, one, prev, prec=64), D)
    # static pixel, mask beta: Dd_t = D + (Dd_0 - D) (1 - beta)^t
    m = np.full(D.shape, BETA)
    cur = prev.copy()
    for t in range(1, 9):
        cur = oracle.temporal_filter(D, m, cur, prec=64)
        np.testing.assert_allclose(cur, D + (prev - D) * (1 - BETA) ** t, rtol=1e-13)
    # first frame and holes
    np.testing.assert_array_equal(oracle.temporal_filter(D, m, None, prec=64), D)
    Dh = D.copy()
    Dh[0, :3] = 0
    Dh[1, 0] = np.inf
    ph = prev.copy()
    ph[2, :4] = 0
    out = oracle.temporal_filter(Dh, m, ph, prec=64)
    assert (out[0, :3] == 0).all() and out[1, 0] == 0
    np.testing.assert_array_equal(out[2, :4], Dh[2, :4])
    inner = np.ones(D.shape, bool)
    inner[0, :3] = inner[1, 0] = False
    inner[2, :4] = False
    ref = BETA * Dh.astype(np.float64) + (1 - BETA) * ph
    np.testing.assert_allclose(out[inner], ref[inner], rtol=1e-14)


def test_temporal_filter_fp32_order():
    """FP32: fma(M, D, (1 - M) Dd_prev), one rounding per step."""
    rng = np.random.default_rng(4)
    D = rng.uniform(0.5, 5.0, 500).astype(np.float32)
    m = rng.uniform(0.6, 1.0, 500).astype(np.float32)
    p = rng.uniform(0.5, 5.0, 500).astype(np.float32)
    out = oracle.temporal_filter(D, m, p)
    a = (np.float32(1) - m).astype(np.float32)
    b = (a * p).astype(np.float32)
    ref = (m.astype(np.float64) * D.astype(np.float64) + b.astype(np.float64)).astype(np.float32)
    np.testing.assert_array_equal(out, ref)


def test_identity_warp_mask_splat():
    """Views that coincide with the target: each target pixel is covered by
    its own source pixel alone (G = 1), so the splatted mask is the input
    mask and the maximum is the maximum over the views; holes stay 0."""
    c = scenes.config1()
    cam = c["src"][0]
    depth = np.repeat(c["depth"][:1], 3, axis=0).copy()
    rng = np.random.default_rng(5)
    holes = rng.random(depth.shape) < 0.05
    depth[holes] = 0
    masks = rng.uniform(0.6, 1.0, depth.shape).astype(np.float32)
    rgb = np.repeat(c["rgb"][:1], 3, axis=0)
    out = oracle.splat([cam] * 3, depth, rgb, cam, c["splat"], mask=masks)
    valid = ~holes
    np.testing.assert_array_equal(out["mask"][valid], masks[valid])
    assert (out["mask"][~valid] == 0).all()
    ref = np.where(valid, masks, 0).max(0)
    np.testing.assert_array_equal(out["mask_max"], ref)


@pytest.mark.parametrize("seed,tgt_f", [(0, 15.0), (1, 27.0), (2, 9.0)])
def test_mask_splat_matches_bruteforce(seed, tgt_f):
    c = scenes.small_ring(seed=seed, width=16, height=16, k=2, noise=0.01, holes=0.03, f=15.0)
    c["tgt"].fx = c["tgt"].fy = tgt_f
    rng = np.random.default_rng(seed)
    masks = rng.uniform(0.6, 1.0, c["depth"].shape).astype(np.float32)
    out = oracle.splat(c["src"], c["depth"], c["rgb"], c["tgt"], c["splat"], mask=masks, prec=64)
    *_, amb, msk = bf.zbuffer(c["src"], c["depth"], c["rgb"], c["tgt"], c["splat"], mask=masks)
    ok = ~amb
    assert ok.mean() > 0.95
    np.testing.assert_allclose(out["mask"][ok], msk[ok], rtol=1e-9, atol=1e-12)
    okall = ok.all(0)
    np.testing.assert_allclose(out["mask_max"][okall], msk.max(0)[okall], rtol=1e-9, atol=1e-12)
    # the mask splat changes none of the other outputs
    plain = oracle.splat(c["src"], c["depth"], c["rgb"], c["tgt"], c["splat"], prec=64)
    for key in ("win_idx", "depth", "rgb", "alpha", "tape"):
        np.testing.assert_array_equal(out[key], plain[key])
