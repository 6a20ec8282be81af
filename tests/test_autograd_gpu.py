"""The autograd Functions against the oracle's adjoints and central finite
differences, on the differentiation workload's geometry (scaled down)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2505_18932_amd as gg
import scenes
from tests.test_parity_gpu import grad_close, splat_ref, tsdf_ref

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _case(W=160, H=90):
    f = 0.9375 * W
    src = scenes._quantize_all(scenes.parallel_rig([-0.15, -0.05, 0.05, 0.15], W, H, f))
    tgt = scenes.parallel_rig([0.0], W, H, f)[0].quantized()
    rng = np.random.default_rng(21)
    depth, rgb = scenes.make_frame(src, tgt, scenes._cfg1_scene(0), rng, 0.01, 0.01)
    return dict(src=src, tgt=tgt, depth=depth, rgb=rgb, splat=scenes.splat_params(),
                tsdf=scenes.tsdf_params(num_bins=96, trunc=3.0))


def test_autograd_matches_oracle_adjoints():
    c = _case()
    depth = torch.from_numpy(c["depth"]).to(DEV).requires_grad_(True)
    rgb = torch.from_numpy(c["rgb"]).to(DEV)
    colour = (rgb.float() / 255.0).requires_grad_(True)
    rgb_o, dep_o, alpha_o, win = gg.autograd.splat(c["src"], depth, rgb, c["tgt"], c["splat"],
                                                   colour=colour)
    dep_t, b, F, W = gg.autograd.tsdf(c["src"], depth, c["tgt"], c["tsdf"])
    rng = np.random.default_rng(5)
    g_rgb = rng.standard_normal(rgb_o.shape).astype(np.float32)
    g_z = rng.standard_normal(dep_o.shape).astype(np.float32)
    g_a = rng.standard_normal(alpha_o.shape).astype(np.float32)
    g_t = rng.standard_normal(dep_t.shape).astype(np.float32)
    loss = (rgb_o * torch.from_numpy(g_rgb).to(DEV)).sum() + \
        (dep_o * torch.from_numpy(g_z).to(DEV)).sum() + \
        (alpha_o * torch.from_numpy(g_a).to(DEV)).sum() + \
        (dep_t * torch.from_numpy(g_t).to(DEV)).sum()
    loss.backward()
    torch.cuda.synchronize()
    (rd, (md, nd)), (rc, bc) = splat_ref(c, g_rgb, g_z, g_a)
    rt, (mt, nt, qt) = tsdf_ref(c, g_t.ravel())
    grad_close(colour.grad.cpu().numpy(), rc, bc, "colour gradient")
    # the two adjoints add: so do their magnitudes, term counts and allowances
    grad_close(depth.grad.cpu().numpy(), rd + rt, (md + mt, nd + nt, qt),
               "depth gradient (splat + fusion)")


def test_fusion_gradient_matches_finite_differences():
    """Central differences of the GPU forward itself (h = 4, 2, 1 mm, 64
    sampled input pixels, Richardson-extrapolated; kinks skipped).  The
    forward is FP32: an output depth carries ~3e-7 m of rounding, ~3e-4 of a
    unit gradient after the 2 mm quotient and the extrapolation.  This is a
    sanity check of sign and scale (a dropped term or a wrong sign is off by
    O(1)); the tight checks are the FP64 oracle's differences and the
    GPU-oracle gradient parity at 1e-5."""
    c = _case(W=96, H=54)
    depth = torch.from_numpy(c["depth"]).to(DEV).requires_grad_(True)
    rng = np.random.default_rng(8)
    g = torch.from_numpy(rng.standard_normal((54, 96)).astype(np.float32)).to(DEV)
    dep_t, _, _, _ = gg.autograd.tsdf(c["src"], depth, c["tgt"], c["tsdf"])
    (dep_t * g).sum().backward()
    grad = depth.grad.cpu().numpy()

    def loss(d):
        with torch.no_grad():
            F, W, dp, _ = gg.tsdf_integrate(c["src"], torch.from_numpy(d).to(DEV), c["tgt"],
                                            c["tsdf"])
            return float((dp.double() * g.double()).sum())

    cand = np.argwhere(grad != 0)
    pick = cand[rng.choice(len(cand), 64, replace=False)]
    errs = []
    scale = np.abs(grad).max()
    for k, j, i in pick:
        fd = []
        for h in (4e-3, 2e-3, 1e-3):
            dp, dm = c["depth"].copy(), c["depth"].copy()
            dp[k, j, i] = np.float32(dp[k, j, i] + h)
            dm[k, j, i] = np.float32(dm[k, j, i] - h)
            fd.append((loss(dp) - loss(dm)) / (float(dp[k, j, i]) - float(dm[k, j, i])))
        a, b = (4 * fd[1] - fd[0]) / 3, (4 * fd[2] - fd[1]) / 3
        if abs(a - b) > 1e-2 * max(abs(b), 1e-2 * scale):
            continue  # a kink inside the bracket
        errs.append(abs(b - grad[k, j, i]) / max(abs(grad[k, j, i]), 1e-2 * scale))
    errs = np.array(errs)
    assert len(errs) >= 24
    # FP32 quotients: bound the bulk (a kink can hide inside the bracket)
    assert np.median(errs) < 5e-3 and np.percentile(errs, 90) < 3e-2, np.sort(errs)[-5:]
