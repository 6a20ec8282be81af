"""Python binding of the C ABI: the same entry points, taking torch tensors.

Argument marshalling only (shape / dtype / device checks, output and workspace
allocation through PyTorch's caching allocator, the current stream).  Every
step of the geometry stage runs in the HIP kernels of libggeom.so.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import torch

from . import _lib as L


# ---------------------------------------------------------------------------
# cameras and parameters


def camera(c) -> L.GGCamera:
    """A GGCamera from any object with fx, fy, cx, cy, R (3x3), t (3),
    width, height."""
    if isinstance(c, L.GGCamera):
        return c
    o = L.GGCamera()
    o.fx, o.fy, o.cx, o.cy = float(c.fx), float(c.fy), float(c.cx), float(c.cy)
    R = [float(v) for row in c.R for v in row] if hasattr(c.R[0], "__len__") else \
        [float(v) for v in c.R]
    o.R[:] = R
    o.t[:] = [float(v) for v in c.t]
    o.width, o.height = int(c.width), int(c.height)
    return o


def cameras(cs: Sequence) -> C.Array:
    if isinstance(cs, C.Array):
        return cs
    arr = (L.GGCamera * len(cs))()
    for i, c in enumerate(cs):
        arr[i] = camera(c)
    return arr


def splat_params(p) -> L.GGSplatParams:
    if isinstance(p, L.GGSplatParams):
        return p
    return L.GGSplatParams(p["sigma_px"], p["band_rel"], p["z_min"], p["r_max_px"])


def mask_params(p=None) -> L.GGMaskParams:
    """Difference-mask parameters; defaults are the paper's (Eq. 1, §3.2)."""
    if isinstance(p, L.GGMaskParams):
        return p
    p = p or {}
    return L.GGMaskParams(p.get("beta", 0.6), p.get("lambda_t", 0.7), int(p.get("factor", 4)))


def tsdf_params(p) -> L.GGTsdfParams:
    if isinstance(p, L.GGTsdfParams):
        return p
    return L.GGTsdfParams(p["z_near"], p["z_far"], int(p["num_bins"]), p["trunc"],
                          int(p["trunc_in_bins"]), p["conf_tau"], p["conf_scale"],
                          int(p["conf_window"]), p["decay"], p["weight_cap"])


# ---------------------------------------------------------------------------
# tensor checks


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _need(t, dtype, shape, name, device):
    if t is None:
        raise ValueError(f"{name} is required")
    if t.dtype != dtype:
        raise TypeError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if t.device != device:
        raise ValueError(f"{name}: on {t.device}, expected {device}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _device(t: torch.Tensor) -> torch.device:
    if t.device.type != "cuda":
        raise ValueError("inputs must be GPU tensors (the geometry stage runs in HIP kernels)")
    return t.device


def _stream(device, stream):
    s = torch.cuda.current_stream(device) if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _ws(nbytes, device, ws):
    if nbytes == 0:
        return None, 0
    if ws is not None:
        if ws.device != device or ws.numel() * ws.element_size() < nbytes:
            raise ValueError("workspace too small or on the wrong device")
        return ws, ws.numel() * ws.element_size()
    # torch allocations are 256-byte aligned
    return torch.empty(nbytes, dtype=torch.uint8, device=device), nbytes


def workspace_size(op, K, src_w, src_h, tgt_w, tgt_h, num_bins=2, sp=None) -> int:
    spp = None if sp is None else C.byref(splat_params(sp))
    return int(L.lib().gg_workspace_size(op, K, src_w, src_h, tgt_w, tgt_h, num_bins, spp))


def _wh(cams_arr):
    return int(cams_arr[0].width), int(cams_arr[0].height)


# ---------------------------------------------------------------------------
# entry points


def splat_views(src, depth: torch.Tensor, rgb: torch.Tensor, tgt, params, *, tape=True,
                mask=None, out=None, ws=None, stream=None):
    """Forward splat of K views into the target (see include/ggeom.h).
    Returns dict(win_idx, depth, rgb, alpha, tape); with ``mask`` (K, H, W)
    float32 (difference masks) also mask (K, Ht, Wt) and mask_max (Ht, Wt)
    through splat_views_masked."""
    dev = _device(depth)
    sa, tg, sp = cameras(src), camera(tgt), splat_params(params)
    K = len(sa)
    sw, sh = _wh(sa)
    tw, th = tg.width, tg.height
    _need(depth, torch.float32, (K, sh, sw), "depth", dev)
    _need(rgb, torch.uint8, (K, sh, sw, 3), "rgb", dev)
    o = out or {}

    def buf(key, shape, dtype):
        t = o.get(key)
        return torch.empty(shape, dtype=dtype, device=dev) if t is None else \
            _need(t, dtype, shape, key, dev)

    win = buf("win_idx", (K, th, tw), torch.int32)
    od = buf("depth", (K, th, tw), torch.float32)
    orgb = buf("rgb", (K, 3, th, tw), torch.float32)
    oa = buf("alpha", (K, th, tw), torch.float32)
    ot = buf("tape", (K, 3, th, tw), torch.float32) if (tape or o.get("tape") is not None) \
        else None
    need = workspace_size(L.GG_OP_SPLAT, K, sw, sh, tw, th, 2, sp)
    wsb, wsn = _ws(need, dev, ws)
    if mask is None:
        L.check(L.lib().splat_views(sa, K, _ptr(depth), _ptr(rgb), C.byref(tg), C.byref(sp),
                                    _ptr(win), _ptr(od), _ptr(orgb), _ptr(oa), _ptr(ot),
                                    _ptr(wsb), wsn, _stream(dev, stream)))
        return dict(win_idx=win, depth=od, rgb=orgb, alpha=oa, tape=ot)
    _need(mask, torch.float32, (K, sh, sw), "mask", dev)
    om = buf("mask", (K, th, tw), torch.float32)
    omax = buf("mask_max", (th, tw), torch.float32)
    L.check(L.lib().splat_views_masked(sa, K, _ptr(depth), _ptr(rgb), C.byref(tg), C.byref(sp),
                                       _ptr(mask), _ptr(win), _ptr(od), _ptr(orgb), _ptr(oa),
                                       _ptr(ot), _ptr(om), _ptr(omax), _ptr(wsb), wsn,
                                       _stream(dev, stream)))
    return dict(win_idx=win, depth=od, rgb=orgb, alpha=oa, tape=ot, mask=om, mask_max=omax)


def splat_views_ewa(src, depth: torch.Tensor, rgb: torch.Tensor, tgt, params, *,
                    lowpass=0.3, sort_limit=0, out=None, ws=None, stream=None):
    """Front-to-back compositing of the EWA-projected per-pixel Gaussians of
    K views into the target (see include/ggeom.h; ``sort_limit`` the longest
    tile list sorted in LDS at once, 64..512, 0 = 512).  Returns dict(rgb
    (K, 3, Ht, Wt), alpha, depth (K, Ht, Wt))."""
    dev = _device(depth)
    sa, tg, sp = cameras(src), camera(tgt), splat_params(params)
    K = len(sa)
    sw, sh = _wh(sa)
    tw, th = tg.width, tg.height
    _need(depth, torch.float32, (K, sh, sw), "depth", dev)
    _need(rgb, torch.uint8, (K, sh, sw, 3), "rgb", dev)
    o = out or {}

    def buf(key, shape):
        t = o.get(key)
        return torch.empty(shape, dtype=torch.float32, device=dev) if t is None else \
            _need(t, torch.float32, shape, key, dev)

    orgb = buf("rgb", (K, 3, th, tw))
    oa = buf("alpha", (K, th, tw))
    od = buf("depth", (K, th, tw))
    need = workspace_size(L.GG_OP_SPLAT_EWA, K, sw, sh, tw, th, 2, sp)
    wsb, wsn = _ws(need, dev, ws)
    L.check(L.lib().splat_views_ewa(sa, K, _ptr(depth), _ptr(rgb), C.byref(tg), C.byref(sp),
                                    float(lowpass), int(sort_limit), _ptr(orgb), _ptr(oa), _ptr(od),
                                    _ptr(wsb), wsn, _stream(dev, stream)))
    return dict(rgb=orgb, alpha=oa, depth=od)


def volume_tuning(t):
    """A launch shape of the volume kernels, (pixels per workgroup, pixels per
    wavefront row, bins per thread[, band width in pixels of the fusion's
    tile order]) with 0 for a default, as the C record (or None: the
    defaults)."""
    if t is None:
        return None
    if isinstance(t, L.GGVolumeTuning):
        return t
    v = [int(x) for x in t]
    if len(v) not in (3, 4):
        raise ValueError("volume tuning: 3 or 4 integers, got %r" % (t,))
    return L.GGVolumeTuning(*(v + [0] * (4 - len(v))))


def _tref(t):
    v = volume_tuning(t)
    return None if v is None else C.byref(v)


def difference_masks(rgb: torch.Tensor, rgb_prev: torch.Tensor, params=None, *, depth=None,
                     depth_prev=None, mask=None, filtered=None, ws=None, stream=None):
    """Soft colour-difference masks (K, H, W) between frames t and t - 1
    (Eq. 1) and, with ``depth``, the temporally filtered depth (Eq. 2;
    ``depth_prev`` None on the first frame; ``filtered`` may be
    ``depth_prev`` for an in-place update).  Returns (mask, filtered)."""
    dev = _device(rgb)
    mp = mask_params(params)
    if rgb.dim() != 4 or rgb.shape[-1] != 3:
        raise ValueError("rgb must be (K, H, W, 3)")
    K, H, W = (int(v) for v in rgb.shape[:3])
    _need(rgb, torch.uint8, (K, H, W, 3), "rgb", dev)
    _need(rgb_prev, torch.uint8, (K, H, W, 3), "rgb_prev", dev)
    om = torch.empty((K, H, W), dtype=torch.float32, device=dev) if mask is None else \
        _need(mask, torch.float32, (K, H, W), "mask", dev)
    of = None
    if depth is not None:
        _need(depth, torch.float32, (K, H, W), "depth", dev)
        if depth_prev is not None:
            _need(depth_prev, torch.float32, (K, H, W), "depth_prev", dev)
        of = torch.empty((K, H, W), dtype=torch.float32, device=dev) if filtered is None else \
            _need(filtered, torch.float32, (K, H, W), "filtered", dev)
    need = workspace_size(L.GG_OP_DIFFERENCE_MASKS, K, W, H, W, H, mp.factor)
    wsb, wsn = _ws(need, dev, ws)
    L.check(L.lib().difference_masks(K, W, H, _ptr(rgb), _ptr(rgb_prev), C.byref(mp), _ptr(om),
                                     _ptr(depth), _ptr(depth_prev), _ptr(of), _ptr(wsb), wsn,
                                     _stream(dev, stream)))
    return om, of


def splat_views_backward(src, depth, rgb, tgt, params, fwd, g_rgb=None, g_depth=None,
                         g_alpha=None, *, stream=None):
    """Adjoint of splat_views; returns (g_depth_in, g_rgb_in) with g_rgb_in
    the gradient with respect to c = rgb / 255, shape (K, H, W, 3)."""
    dev = _device(depth)
    sa, tg, sp = cameras(src), camera(tgt), splat_params(params)
    K = len(sa)
    sw, sh = _wh(sa)
    tw, th = tg.width, tg.height
    _need(depth, torch.float32, (K, sh, sw), "depth", dev)
    _need(rgb, torch.uint8, (K, sh, sw, 3), "rgb", dev)
    for name, t, shp in (("g_rgb", g_rgb, (K, 3, th, tw)), ("g_depth", g_depth, (K, th, tw)),
                         ("g_alpha", g_alpha, (K, th, tw))):
        if t is not None:
            _need(t, torch.float32, shp, name, dev)
    if fwd.get("tape") is None:
        raise ValueError("the forward must have been run with tape=True")
    gd = torch.empty((K, sh, sw), dtype=torch.float32, device=dev)
    gc = torch.empty((K, sh, sw, 3), dtype=torch.float32, device=dev)
    L.check(L.lib().splat_views_backward(
        sa, K, _ptr(depth), _ptr(rgb), C.byref(tg), C.byref(sp), _ptr(fwd["win_idx"]),
        _ptr(fwd["depth"]), _ptr(fwd["rgb"]), _ptr(fwd["tape"]), _ptr(g_rgb), _ptr(g_depth),
        _ptr(g_alpha), _ptr(gd), _ptr(gc), None, 0, _stream(dev, stream)))
    return gd, gc


def tsdf_view_table(src, depth, params, *, ws, stream=None):
    """Build the view table and bin depths of ``depth`` into ``ws`` (the first
    part of tsdf_integrate), for tsdf_integrate(..., table_ready=True)."""
    dev = _device(depth)
    sa, tp = cameras(src), tsdf_params(params)
    K = len(sa)
    sw, sh = _wh(sa)
    _need(depth, torch.float32, (K, sh, sw), "depth", dev)
    need = workspace_size(L.GG_OP_TSDF_INTEGRATE, K, sw, sh, sw, sh, tp.num_bins)
    wsb, wsn = _ws(need, dev, ws)
    L.check(L.lib().tsdf_view_table(sa, K, _ptr(depth), C.byref(tp), _ptr(wsb), wsn,
                                    _stream(dev, stream)))


def tsdf_integrate(src, depth, tgt, params, *, F_prev=None, W_prev=None, F=None, W=None,
                   mask=None, extract=True, ws=None, stream=None, table_ready=False,
                   tuning=None):
    """Fuse K depth maps into the target volume (in place when F is F_prev).
    Returns (F, W, depth, bin) (depth, bin None when extract=False).  With
    ``table_ready`` the view table is the one tsdf_view_table built into
    ``ws`` (``depth`` then only fixes the shapes).  ``tuning``: the launch
    shape (volume_tuning), results unchanged."""
    dev = _device(depth)
    sa, tg, tp = cameras(src), camera(tgt), tsdf_params(params)
    K = len(sa)
    sw, sh = _wh(sa)
    tw, th, D = tg.width, tg.height, tp.num_bins
    _need(depth, torch.float32, (K, sh, sw), "depth", dev)
    vol = (th, tw, D)
    if (F_prev is None) != (W_prev is None):
        raise ValueError("F_prev and W_prev go together")
    if F_prev is not None:
        _need(F_prev, torch.float32, vol, "F_prev", dev)
        _need(W_prev, torch.float32, vol, "W_prev", dev)
    if mask is not None:
        _need(mask, torch.float32, (th, tw), "mask", dev)
    F = torch.empty(vol, dtype=torch.float32, device=dev) if F is None else \
        _need(F, torch.float32, vol, "F", dev)
    W = torch.empty(vol, dtype=torch.float32, device=dev) if W is None else \
        _need(W, torch.float32, vol, "W", dev)
    od = ob = None
    if extract:
        od = torch.empty((th, tw), dtype=torch.float32, device=dev)
        ob = torch.empty((th, tw), dtype=torch.int32, device=dev)
    need = workspace_size(L.GG_OP_TSDF_INTEGRATE, K, sw, sh, tw, th, D)
    if table_ready and ws is None:
        raise ValueError("table_ready needs the workspace tsdf_view_table filled")
    wsb, wsn = _ws(need, dev, ws)
    if table_ready:
        L.check(L.lib().tsdf_integrate_tabled(sa, K, C.byref(tg), C.byref(tp), _ptr(mask),
                                              _ptr(F_prev), _ptr(W_prev), _ptr(F), _ptr(W),
                                              _ptr(od), _ptr(ob), _tref(tuning), _ptr(wsb), wsn,
                                              _stream(dev, stream)))
    else:
        L.check(L.lib().tsdf_integrate(sa, K, _ptr(depth), C.byref(tg), C.byref(tp), _ptr(mask),
                                       _ptr(F_prev), _ptr(W_prev), _ptr(F), _ptr(W), _ptr(od),
                                       _ptr(ob), _tref(tuning), _ptr(wsb), wsn,
                                       _stream(dev, stream)))
    return F, W, od, ob


def fusion_stream_probe(tgt, params, F_prev, W_prev, F, W, out_depth, out_bin, *, ws=None,
                        stream=None, tuning=None):
    """The fusion kernel's volume stream alone (no views, no gathers): the
    ceiling of its memory access pattern (see include/ggeom.h)."""
    dev = _device(F_prev)
    tg, tp = camera(tgt), tsdf_params(params)
    vol = (tg.height, tg.width, tp.num_bins)
    for t, n in ((F_prev, "F_prev"), (W_prev, "W_prev"), (F, "F"), (W, "W")):
        _need(t, torch.float32, vol, n, dev)
    _need(out_depth, torch.float32, vol[:2], "out_depth", dev)
    _need(out_bin, torch.int32, vol[:2], "out_bin", dev)
    need = workspace_size(L.GG_OP_TSDF_INTEGRATE, 1, 1, 1, tg.width, tg.height, tp.num_bins)
    wsb, wsn = _ws(need, dev, ws)
    L.check(L.lib().gg_fusion_stream_probe(C.byref(tg), C.byref(tp), _ptr(F_prev), _ptr(W_prev),
                                           _ptr(F), _ptr(W), _ptr(out_depth), _ptr(out_bin),
                                           _tref(tuning), _ptr(wsb), wsn, _stream(dev, stream)))


def tsdf_integrate_noalloc(src, depth, tgt, params, *, F_prev=None, W_prev=None, F=None, W=None,
                           mask=None, extract=True, stream=None, tuning=None):
    """tsdf_integrate through the entry point that takes no workspace and
    allocates nothing (its scratch is the library's static device array).
    Outputs not passed in are created here; the C call itself allocates
    nothing.  Returns (F, W, depth, bin)."""
    dev = _device(depth)
    sa, tg, tp = cameras(src), camera(tgt), tsdf_params(params)
    K = len(sa)
    sw, sh = _wh(sa)
    tw, th, D = tg.width, tg.height, tp.num_bins
    _need(depth, torch.float32, (K, sh, sw), "depth", dev)
    vol = (th, tw, D)
    if (F_prev is None) != (W_prev is None):
        raise ValueError("F_prev and W_prev go together")
    if F_prev is not None:
        _need(F_prev, torch.float32, vol, "F_prev", dev)
        _need(W_prev, torch.float32, vol, "W_prev", dev)
    if mask is not None:
        _need(mask, torch.float32, (th, tw), "mask", dev)
    F = torch.empty(vol, dtype=torch.float32, device=dev) if F is None else \
        _need(F, torch.float32, vol, "F", dev)
    W = torch.empty(vol, dtype=torch.float32, device=dev) if W is None else \
        _need(W, torch.float32, vol, "W", dev)
    od = ob = None
    if extract:
        od = torch.empty((th, tw), dtype=torch.float32, device=dev)
        ob = torch.empty((th, tw), dtype=torch.int32, device=dev)
    L.check(L.lib().tsdf_integrate_noalloc(sa, K, _ptr(depth), C.byref(tg), C.byref(tp),
                                           _ptr(mask), _ptr(F_prev), _ptr(W_prev), _ptr(F),
                                           _ptr(W), _ptr(od), _ptr(ob), _tref(tuning),
                                           _stream(dev, stream)))
    return F, W, od, ob


def tsdf_raymarch(src, depth, tgt, params, *, depth_prev=None, acc_prev=None, mask=None,
                  steps=False, out_depth=None, out_acc=None, ws=None, stream=None):
    """Volume-free march of every target ray (see include/ggeom.h).
    Returns (depth, acc_next, steps or None); ``depth_prev`` / ``acc_prev``
    (both or neither) switch on the temporal input, ``mask`` weights it."""
    dev = _device(depth)
    sa, tg, tp = cameras(src), camera(tgt), tsdf_params(params)
    K = len(sa)
    sw, sh = _wh(sa)
    th, tw = tg.height, tg.width
    _need(depth, torch.float32, (K, sh, sw), "depth", dev)
    for name, t in (("depth_prev", depth_prev), ("acc_prev", acc_prev), ("mask", mask)):
        if t is not None:
            _need(t, torch.float32, (th, tw), name, dev)
    od = torch.empty((th, tw), dtype=torch.float32, device=dev) if out_depth is None else \
        _need(out_depth, torch.float32, (th, tw), "out_depth", dev)
    oa = torch.empty((th, tw), dtype=torch.float32, device=dev) if out_acc is None else \
        _need(out_acc, torch.float32, (th, tw), "out_acc", dev)
    st = torch.empty((th, tw), dtype=torch.int32, device=dev) if steps else None
    need = workspace_size(L.GG_OP_TSDF_INTEGRATE, K, sw, sh, tw, th, tp.num_bins)
    wsb, wsn = _ws(need, dev, ws)
    L.check(L.lib().tsdf_raymarch(sa, K, _ptr(depth), C.byref(tg), C.byref(tp), _ptr(depth_prev),
                                  _ptr(acc_prev), _ptr(mask), _ptr(od), _ptr(oa), _ptr(st),
                                  _ptr(wsb), wsn, _stream(dev, stream)))
    return od, oa, st


def network_inputs(src, tgt, tsdf_depth, splat, *, out=None, stream=None):
    """(9K+1, Ht, Wt) input stack of the blending network from the TSDF depth
    and the splat outputs ``splat`` (dict with rgb, depth, alpha)."""
    dev = _device(tsdf_depth)
    sa, tg = cameras(src), camera(tgt)
    K = len(sa)
    th, tw = tg.height, tg.width
    _need(tsdf_depth, torch.float32, (th, tw), "tsdf_depth", dev)
    _need(splat["rgb"], torch.float32, (K, 3, th, tw), "rgb", dev)
    _need(splat["depth"], torch.float32, (K, th, tw), "depth", dev)
    _need(splat["alpha"], torch.float32, (K, th, tw), "alpha", dev)
    o = torch.empty((9 * K + 1, th, tw), dtype=torch.float32, device=dev) if out is None else \
        _need(out, torch.float32, (9 * K + 1, th, tw), "out", dev)
    L.check(L.lib().network_inputs(sa, K, C.byref(tg), _ptr(tsdf_depth), _ptr(splat["rgb"]),
                                   _ptr(splat["depth"]), _ptr(splat["alpha"]), _ptr(o),
                                   _stream(dev, stream)))
    return o


def blend_views(rgb, depth, alpha, weights, w_bg, rgb_bg, *, stream=None):
    """Eq. 4-5 with given weights: (image (3, H, W), blended depth (H, W))."""
    dev = _device(rgb)
    K, _, H, W = (int(v) for v in rgb.shape)
    _need(rgb, torch.float32, (K, 3, H, W), "rgb", dev)
    for name, t in (("depth", depth), ("alpha", alpha), ("weights", weights)):
        _need(t, torch.float32, (K, H, W), name, dev)
    _need(w_bg, torch.float32, (H, W), "w_bg", dev)
    _need(rgb_bg, torch.float32, (3, H, W), "rgb_bg", dev)
    orgb = torch.empty((3, H, W), dtype=torch.float32, device=dev)
    od = torch.empty((H, W), dtype=torch.float32, device=dev)
    L.check(L.lib().blend_views(K, W, H, _ptr(rgb), _ptr(depth), _ptr(alpha), _ptr(weights),
                                _ptr(w_bg), _ptr(rgb_bg), _ptr(orgb), _ptr(od),
                                _stream(dev, stream)))
    return orgb, od


def tsdf_extract_depth(tgt, params, F, W, *, stream=None, tuning=None):
    dev = _device(F)
    tg, tp = camera(tgt), tsdf_params(params)
    vol = (tg.height, tg.width, tp.num_bins)
    _need(F, torch.float32, vol, "F", dev)
    _need(W, torch.float32, vol, "W", dev)
    od = torch.empty(vol[:2], dtype=torch.float32, device=dev)
    ob = torch.empty(vol[:2], dtype=torch.int32, device=dev)
    L.check(L.lib().tsdf_extract_depth(C.byref(tg), C.byref(tp), _ptr(F), _ptr(W), _ptr(od),
                                       _ptr(ob), _tref(tuning), _stream(dev, stream)))
    return od, ob


def tsdf_extract_depth_backward(tgt, params, F, W, bin, g_depth, *, stream=None):
    dev = _device(F)
    tg, tp = camera(tgt), tsdf_params(params)
    vol = (tg.height, tg.width, tp.num_bins)
    _need(F, torch.float32, vol, "F", dev)
    _need(W, torch.float32, vol, "W", dev)
    _need(bin, torch.int32, vol[:2], "bin", dev)
    _need(g_depth, torch.float32, vol[:2], "g_depth", dev)
    g2 = torch.empty(vol[:2] + (2,), dtype=torch.float32, device=dev)
    L.check(L.lib().tsdf_extract_depth_backward(C.byref(tg), C.byref(tp), _ptr(F), _ptr(W),
                                                _ptr(bin), _ptr(g_depth), _ptr(g2),
                                                _stream(dev, stream)))
    return g2


def tsdf_integrate_backward(src, depth, tgt, params, F, W, bin, g_F2, *, ws=None, stream=None):
    dev = _device(depth)
    sa, tg, tp = cameras(src), camera(tgt), tsdf_params(params)
    K = len(sa)
    sw, sh = _wh(sa)
    tw, th, D = tg.width, tg.height, tp.num_bins
    _need(depth, torch.float32, (K, sh, sw), "depth", dev)
    _need(F, torch.float32, (th, tw, D), "F", dev)
    _need(W, torch.float32, (th, tw, D), "W", dev)
    _need(bin, torch.int32, (th, tw), "bin", dev)
    _need(g_F2, torch.float32, (th, tw, 2), "g_F2", dev)
    gd = torch.empty((K, sh, sw), dtype=torch.float32, device=dev)
    need = workspace_size(L.GG_OP_TSDF_INTEGRATE_BACKWARD, K, sw, sh, tw, th, D)
    wsb, wsn = _ws(need, dev, ws)
    L.check(L.lib().tsdf_integrate_backward(sa, K, _ptr(depth), C.byref(tg), C.byref(tp),
                                            _ptr(F), _ptr(W), _ptr(bin), _ptr(g_F2), _ptr(gd),
                                            _ptr(wsb), wsn, _stream(dev, stream)))
    return gd


def relative_projection(a, b):
    """FP32 (H (3x3), c (3)) of the relative projection a -> b (host only)."""
    H = (C.c_float * 9)()
    c = (C.c_float * 3)()
    ca, cb = camera(a), camera(b)
    L.check(L.lib().gg_relative_projection(C.byref(ca), C.byref(cb), H, c))
    return [list(H[0:3]), list(H[3:6]), list(H[6:9])], list(c)


# ---------------------------------------------------------------------------
# kernel timing (profiling)


def timing_enable(on=True, only=None):
    """Bracket kernel launches with HIP events; ``only`` restricts it to the
    kernels whose name contains that string."""
    L.check(L.lib().gg_timing_filter(None if only is None else only.encode()))
    L.check(L.lib().gg_timing_enable(1 if on else 0))


def timing_reset():
    L.check(L.lib().gg_timing_reset())


def timing_read(name=None):
    ms = C.c_double()
    n = C.c_int64()
    L.check(L.lib().gg_timing_read(None if name is None else name.encode(), C.byref(ms),
                                   C.byref(n)))
    return ms.value, n.value


# ---------------------------------------------------------------------------
# batched path


class BatchPlan:
    """Many target views fused by one graph launch (see include/ggeom.h).

    ``items``: dicts with keys src, depth, tgt, tsdf and optionally rgb,
    splat, mask, F_prev, W_prev, F, W (allocated if absent), extract (True),
    volume (the item's own fusion launch shape, as ``volume_tuning`` takes it;
    absent: the plan's).
    Outputs live in each item dict after creation: F, W, depth_out, bin_out
    and, with rgb, splat = dict(win_idx, depth, rgb, alpha, tape).  The plan
    binds these buffers; write new inputs into the same tensors between
    launches."""

    def __init__(self, items, pixels_per_block=0, blocks_per_cu=0, bins_per_thread=0,
                 branches=0):
        self.items = items
        self._keep = []
        arr = (L.GGBatchItem * len(items))()
        for i, it in enumerate(items):
            depth = it["depth"]
            dev = _device(depth)
            sa, tg, tp = cameras(it["src"]), camera(it["tgt"]), tsdf_params(it["tsdf"])
            K = len(sa)
            sw, sh = _wh(sa)
            th, tw, D = tg.height, tg.width, tp.num_bins
            _need(depth, torch.float32, (K, sh, sw), "depth", dev)
            vol = (th, tw, D)
            if it.get("F") is None:
                it["F"] = torch.empty(vol, dtype=torch.float32, device=dev)
            if it.get("W") is None:
                it["W"] = torch.empty(vol, dtype=torch.float32, device=dev)
            _need(it["F"], torch.float32, vol, "F", dev)
            _need(it["W"], torch.float32, vol, "W", dev)
            b = arr[i]
            b.src = sa
            b.K = K
            b.depth = depth.data_ptr()
            b.tgt = tg
            b.tsdf = tp
            for key in ("F_prev", "W_prev", "mask"):
                if it.get(key) is not None:
                    _need(it[key], torch.float32, vol if key != "mask" else (th, tw), key, dev)
            b.temporal_mask = _ptr(it.get("mask"))
            b.F_prev = _ptr(it.get("F_prev"))
            b.W_prev = _ptr(it.get("W_prev"))
            b.F = it["F"].data_ptr()
            b.W = it["W"].data_ptr()
            if it.get("extract", True):
                it["depth_out"] = torch.empty((th, tw), dtype=torch.float32, device=dev)
                it["bin_out"] = torch.empty((th, tw), dtype=torch.int32, device=dev)
                b.out_depth = it["depth_out"].data_ptr()
                b.out_bin = it["bin_out"].data_ptr()
            if it.get("rgb") is not None:
                _need(it["rgb"], torch.uint8, (K, sh, sw, 3), "rgb", dev)
                b.rgb = it["rgb"].data_ptr()
                b.splat = splat_params(it["splat"])
                o = dict(win_idx=torch.empty((K, th, tw), dtype=torch.int32, device=dev),
                         depth=torch.empty((K, th, tw), dtype=torch.float32, device=dev),
                         rgb=torch.empty((K, 3, th, tw), dtype=torch.float32, device=dev),
                         alpha=torch.empty((K, th, tw), dtype=torch.float32, device=dev),
                         tape=torch.empty((K, 3, th, tw), dtype=torch.float32, device=dev))
                it["splat_out"] = o
                b.win_idx = o["win_idx"].data_ptr()
                b.sp_depth = o["depth"].data_ptr()
                b.sp_rgb = o["rgb"].data_ptr()
                b.sp_alpha = o["alpha"].data_ptr()
                b.sp_tape = o["tape"].data_ptr()
            if it.get("volume") is not None:
                b.volume = volume_tuning(it["volume"])
            self._keep.append(sa)
        self._arr = arr
        tune = L.GGBatchTuning(int(pixels_per_block), int(blocks_per_cu), int(bins_per_thread),
                               int(branches))
        h = C.c_void_p()
        L.check(L.lib().gg_batch_plan(arr, len(items), C.byref(tune), C.byref(h)))
        self._h = h
        self.device_bytes = int(L.lib().gg_batch_device_bytes(h))

    def launch(self, stream=None):
        dev = self.items[0]["depth"].device
        L.check(L.lib().gg_batch_launch(self._h, _stream(dev, stream)))

    def close(self):
        if self._h:
            torch.cuda.synchronize()
            L.lib().gg_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
