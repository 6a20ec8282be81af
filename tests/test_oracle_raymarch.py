"""Pins of the oracle's volume-free raymarch (Suppl. A.1 step 0.8 s and
three bisections; Suppl. A.2 temporal input): closed forms on planes, the
temporal input alone, special cases that switch the temporal term off, a
cross-check against the volume algorithm, and an FP64 brute force of the
fused signed distance on a fine depth grid."""
import math

import numpy as np
import pytest

import oracle
import scenes


def fronto(W=40, H=30, f=35.0, offsets=((0.0, 0.0),)):
    return [scenes.make_camera(W, H, f, (x, y, 0.0), (x, y, 1.0)).quantized() for x, y in offsets]


def step_min(prm, z):
    un, uf = 1.0 / prm["z_near"], 1.0 / prm["z_far"]
    return (un - uf) / (prm["num_bins"] - 1) * z * z


@pytest.mark.parametrize("d", [0.71, 1.3, 2.77, 4.4])
def test_plane_seen_by_the_target_itself(d):
    """Views that coincide with the target and see a plane at depth d:
    s(z) = min(d - z, tau) exactly (omega = 1 on a constant depth), so the
    march brackets d with one minimal step and three bisections leave it
    within step_min / 16 of the bracket's midpoint."""
    cam = fronto()[0]
    prm = scenes.tsdf_params(num_bins=64, trunc=3.0)
    depth = np.full((2, 30, 40), d, np.float32)
    dep, acc, st = oracle.raymarch([cam, cam], depth, cam, prm, prec=64)
    assert (np.abs(dep - d) <= step_min(prm, d) / 16 * (1 + 1e-9)).all()
    assert (np.abs(dep - d) > 0).any()  # a bisection estimate, not a lookup
    np.testing.assert_allclose(acc, 2.0)  # two views, omega = 1 each, no temporal weight
    # the march takes fewer samples than the dense bins it replaces
    assert st.max() < prm["num_bins"]


def test_temporal_input_alone():
    """No view observes anything (all holes): only the previous depth Dp
    with weight omega_tmp = min(decay acc, cap) > 0, so the march finds Dp
    within the same bound, and passes on acc_next = omega_tmp."""
    cam = fronto()[0]
    prm = scenes.tsdf_params(num_bins=64, trunc=3.0)
    depth = np.zeros((1, 30, 40), np.float32)
    rng = np.random.default_rng(0)
    Dp = rng.uniform(0.8, 4.0, (30, 40))
    acc = np.where(np.arange(40)[None, :] < 20, 10.0, 100.0) * np.ones((30, 1))
    dep, an, _ = oracle.raymarch([cam], depth, cam, prm, dprev=Dp, acc=acc, prec=64)
    assert (np.abs(dep - Dp) <= step_min(prm, Dp) / 16 * (1 + 1e-9)).all()
    # below and above the cap (decay 0.9, cap 32): 9 and 32
    np.testing.assert_allclose(an, np.minimum(prm["decay"] * acc, prm["weight_cap"]))
    dep0, _, _ = oracle.raymarch([cam], depth, cam, prm, prec=64)
    assert (dep0 == 0).all()  # nothing observed: no surface


def test_full_mask_switches_the_temporal_term_off():
    c = scenes.config1()
    rng = np.random.default_rng(1)
    Dp = rng.uniform(0.5, 5.0, (c["tgt"].height, c["tgt"].width))
    acc = np.full_like(Dp, 20.0)
    ref = oracle.raymarch(c["src"], c["depth"], c["tgt"], c["tsdf"])
    out = oracle.raymarch(c["src"], c["depth"], c["tgt"], c["tsdf"], dprev=Dp, acc=acc,
                          mask=np.ones_like(Dp, np.float32))
    for a, b in zip(out, ref):
        assert np.array_equal(a, b)


def test_temporal_weight_pulls_towards_the_previous_depth():
    """A strong temporal weight (mask 0) on a previous depth 2 cm behind the
    observed plane moves the surface towards it, by the weighted mean."""
    cam = fronto()[0]
    prm = scenes.tsdf_params(num_bins=128, trunc=6.0)
    d = 2.0
    depth = np.full((1, 30, 40), d, np.float32)
    Dp = np.full((30, 40), d + 0.02)
    free, _, _ = oracle.raymarch([cam], depth, cam, prm, prec=64)
    pulled, _, _ = oracle.raymarch([cam], depth, cam, prm, dprev=Dp, acc=np.full((30, 40), 100.0),
                                   mask=np.zeros((30, 40), np.float32), prec=64)
    # omega_tmp = cap = 32 against omega = 1: s(z) = (1 (d - z) + 32 (Dp - z)) / 33
    target = (d + 32 * (d + 0.02)) / 33
    assert (np.abs(pulled - target) <= step_min(prm, target) / 16 * 1.01).all()
    assert (np.abs(free - d) <= step_min(prm, d) / 16 * 1.01).all()


@pytest.mark.parametrize("make", ["config1", "small"])
def test_agrees_with_the_volume_algorithm(make):
    """The march and the dense-bin extraction estimate the same first sign
    change of the same fused signed distance: where both find it they agree
    to about a bin width, and they find it on the same pixels."""
    if make == "config1":
        c = scenes.config1()
    else:
        c = scenes.small_ring(seed=4, width=64, height=48, k=3, bins=96)
    prm = c["tsdf"]
    dep, _, st = oracle.raymarch(c["src"], c["depth"], c["tgt"], prm)
    F, W = oracle.integrate(c["src"], c["depth"], c["tgt"], prm)
    dv, bv = oracle.extract(F, W, prm)
    dv = dv.reshape(dep.shape)
    both = (dep > 0) & (dv > 0)
    assert ((dep > 0) == (dv > 0)).mean() > 0.98
    width = step_min(prm, dv[both])
    err = np.abs(dep[both] - dv[both])
    assert np.median(err / width) < 0.25
    assert (err < 2 * width).mean() > 0.98
    assert st.mean() < prm["num_bins"]


def _fused_fp64(src, depth, tgt, prm, x, y, z):
    """FP64 fused s at target depth z on pixel (x, y), through world space."""
    tK = np.array([[tgt.fx, 0, tgt.cx], [0, tgt.fy, tgt.cy], [0, 0, 1.0]])
    ray = np.linalg.solve(tK, [x + 0.5, y + 0.5, 1.0])
    Rt = np.asarray(tgt.R, np.float64).reshape(3, 3)
    p_world = Rt.T @ (ray * z - np.asarray(tgt.t, np.float64))
    un, uf = 1.0 / prm["z_near"], 1.0 / prm["z_far"]
    du = (un - uf) / (prm["num_bins"] - 1)
    tau = prm["trunc"] * du * z * z if prm["trunc_in_bins"] else prm["trunc"]
    conf = oracle.confidence(depth, prm, prec=64)
    S = Wt = 0.0
    for k, cam in enumerate(src):
        K = np.array([[cam.fx, 0, cam.cx], [0, cam.fy, cam.cy], [0, 0, 1.0]])
        X = K @ (np.asarray(cam.R, np.float64).reshape(3, 3) @ p_world + np.asarray(cam.t, np.float64))
        if X[2] <= 0:
            continue
        u, v = X[0] / X[2], X[1] / X[2]
        if not (0 <= u < cam.width and 0 <= v < cam.height):
            continue
        Dk = float(depth[k, int(v), int(u)])
        if not (Dk > 0 and math.isfinite(Dk)):
            continue
        s = Dk - X[2]
        if s < -tau:
            continue
        w = float(conf[k, int(v), int(u)])
        S += w * min(s, tau)
        Wt += w
    return (S / Wt) if Wt > 0 else None


def test_march_matches_a_fine_grid_bruteforce():
    """On an 8x8 rotated-ring scene, every depth the march returns lies on a
    + -> - change of the FP64 fused s on a fine grid (1/64 of a bin), within
    the march's resolution (step_min / 16 plus the grid step); nearly always
    on the first one.  A step of 0.8 s may pass over a negative interval
    shorter than the step (a jump of the sampled depth at an object edge),
    which dense sampling would report first: that is the march's own rule."""
    c = scenes.small_ring(seed=2, width=8, height=8, k=2, noise=0.01, holes=0.0, f=7.5)
    prm = c["tsdf"]
    dep, _, _ = oracle.raymarch(c["src"], c["depth"], c["tgt"], prm, prec=64)
    grid = np.linspace(prm["z_near"], prm["z_far"], 64 * prm["num_bins"])
    first = later = 0
    for y in range(8):
        for x in range(8):
            if dep[y, x] == 0:
                continue
            crossings = []
            prev = None
            for z in grid:
                s = _fused_fp64(c["src"], c["depth"], c["tgt"], prm, x, y, z)
                if s is not None and prev is not None and prev > 0 and s <= 0:
                    crossings.append(z)
                prev = s
            near = [abs(dep[y, x] - z) <= step_min(prm, z) / 16 + 2 * (grid[1] - grid[0])
                    for z in crossings]
            assert any(near), (x, y, dep[y, x], crossings)
            if near[0]:
                first += 1
            else:
                later += 1
    assert first >= 40 and later <= first // 10
