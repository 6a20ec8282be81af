"""Resume: the state carried from frame to frame -- the volume F, W of the
running weight (Suppl. A.2) and, on the temporal path, the filtered depth of
Eq. 2 -- is all a run needs to continue.  Frames 1-30 run straight equal
frames 1-15, the state copied to host memory and back into fresh device
buffers, then frames 16-30: bitwise, on every output of every frame.  The
volume-free raymarch carries its previous depth and accumulated weight the
same way."""
import numpy as np
import pytest
import torch

import paper_2505_18932_amd as gg
import scenes

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
FRAMES = 30
CUT = 15


@pytest.fixture(scope="module")
def video():
    c = scenes.small_video(seed=4, width=160, height=96, k=4, bins=64)
    frames = [c["seq"].frame(t) for t in range(FRAMES)]
    depth = torch.from_numpy(np.stack([d for d, _ in frames])).to(DEV)
    rgb = torch.from_numpy(np.stack([r for _, r in frames])).to(DEV)
    return c, depth, rgb


def _bitwise(a, b, what):
    assert a.dtype == b.dtype and a.shape == b.shape, what
    x = a.contiguous().view(torch.int32) if a.dtype == torch.float32 else a
    y = b.contiguous().view(torch.int32) if b.dtype == torch.float32 else b
    assert torch.equal(x, y), what


def _to_host_and_back(state):
    """The carried state through host memory into new device buffers."""
    host = {k: v.cpu().numpy().copy() for k, v in state.items()}
    torch.cuda.synchronize()
    return {k: torch.from_numpy(v).to(DEV) for k, v in host.items()}


def _run_plain(c, depth, rgb, frames, state):
    """Splat + fusion with the volume carried in place; per-frame outputs."""
    outs = []
    for t in frames:
        so = gg.splat_views(c["src"], depth[t], rgb[t], c["tgt"], c["splat"])
        kw = dict(F_prev=state["F"], W_prev=state["W"], F=state["F"], W=state["W"]) \
            if state else {}
        F, W, d, b = gg.tsdf_integrate(c["src"], depth[t], c["tgt"], c["tsdf"], **kw)
        state = dict(F=F, W=W)
        outs.append([so[k].clone() for k in ("win_idx", "depth", "rgb", "alpha", "tape")] +
                    [d.clone(), b.clone()])
    return outs, state


def _run_temporal(c, depth, rgb, frames, state):
    """Difference masks + filtered depth (state), the masked splat, and the
    fusion of the filtered depth weighted by the splatted masks' maximum."""
    outs = []
    for t in frames:
        prev = rgb[t - 1] if t > 0 else rgb[t]
        m, filt = gg.difference_masks(rgb[t], prev, depth=depth[t],
                                      depth_prev=state.get("filt"))
        so = gg.splat_views(c["src"], filt, rgb[t], c["tgt"], c["splat"], mask=m)
        kw = dict(F_prev=state["F"], W_prev=state["W"], F=state["F"], W=state["W"]) \
            if "F" in state else {}
        F, W, d, b = gg.tsdf_integrate(c["src"], filt, c["tgt"], c["tsdf"], mask=so["mask_max"],
                                       **kw)
        state = dict(F=F, W=W, filt=filt)
        outs.append([m.clone(), filt.clone()] +
                    [so[k].clone() for k in ("win_idx", "depth", "rgb", "alpha", "mask_max")] +
                    [d.clone(), b.clone()])
    return outs, state


def _run_raymarch(c, depth, rgb, frames, state):
    outs = []
    for t in frames:
        d, acc, n = gg.tsdf_raymarch(c["src"], depth[t], c["tgt"], c["tsdf"],
                                     depth_prev=state.get("d"), acc_prev=state.get("acc"),
                                     steps=True)
        state = dict(d=d, acc=acc)
        outs.append([d.clone(), acc.clone(), n.clone()])
    return outs, state


@pytest.mark.parametrize("run", [_run_plain, _run_temporal, _run_raymarch],
                         ids=["plain", "temporal", "raymarch"])
def test_resume_equals_straight_run(video, run):
    c, depth, rgb = video
    straight, end_a = run(c, depth, rgb, range(FRAMES), {})
    first, mid = run(c, depth, rgb, range(CUT), {})
    second, end_b = run(c, depth, rgb, range(CUT, FRAMES), _to_host_and_back(mid))
    torch.cuda.synchronize()
    resumed = first + second
    assert len(resumed) == len(straight) == FRAMES
    for t, (a, b) in enumerate(zip(straight, resumed)):
        for n, (x, y) in enumerate(zip(a, b)):
            _bitwise(x, y, f"frame {t + 1}, output {n}")
    for k in end_a:
        _bitwise(end_a[k], end_b[k], f"final state {k}")
    # the carried state matters: the last frame differs from a cold start
    cold, _ = run(c, depth, rgb, range(FRAMES - 1, FRAMES), {})
    torch.cuda.synchronize()
    assert any(not torch.equal(x, y) for x, y in zip(cold[0], straight[-1]))
