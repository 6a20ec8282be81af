"""ctypes front-end of the plain C oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke``
and the CPU-baseline leg of ``bench.py``; never by the product package.

Every function takes numpy arrays and the camera / parameter records produced
by the ``scenes`` input generators and returns numpy arrays.  ``prec`` selects
the FP32 build (the parity reference) or the FP64 build (finite differences,
rounding bounds).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

HERE = os.path.dirname(os.path.abspath(__file__))


class OrcCamera(C.Structure):
    _fields_ = [("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("R", C.c_float * 9), ("t", C.c_float * 3),
                ("width", C.c_int32), ("height", C.c_int32)]


class OrcSplatParams(C.Structure):
    _fields_ = [("sigma_px", C.c_float), ("band_rel", C.c_float), ("z_min", C.c_float),
                ("r_max_px", C.c_float)]


class OrcTsdfParams(C.Structure):
    _fields_ = [("z_near", C.c_float), ("z_far", C.c_float), ("num_bins", C.c_int32),
                ("trunc", C.c_float), ("trunc_in_bins", C.c_int32),
                ("conf_tau", C.c_float), ("conf_scale", C.c_float), ("conf_window", C.c_int32),
                ("decay", C.c_float), ("weight_cap", C.c_float)]


_libs = {}


def lib(prec=32):
    if prec not in _libs:
        _build.ensure_built()
        L = C.CDLL(os.path.join(HERE, f"liboracle{prec}.so"))
        _libs[prec] = L
    return _libs[prec]


def cam(c) -> OrcCamera:
    p = c.packed()
    o = OrcCamera()
    o.fx, o.fy, o.cx, o.cy = (float(v) for v in p[:4])
    o.R[:] = [float(v) for v in p[4:13]]
    o.t[:] = [float(v) for v in p[13:16]]
    o.width, o.height = int(c.width), int(c.height)
    return o


def cams(cs):
    arr = (OrcCamera * len(cs))()
    for i, c in enumerate(cs):
        arr[i] = cam(c)
    return arr


def splat_params(d) -> OrcSplatParams:
    return OrcSplatParams(d["sigma_px"], d["band_rel"], d["z_min"], d["r_max_px"])


def tsdf_params(d) -> OrcTsdfParams:
    return OrcTsdfParams(d["z_near"], d["z_far"], int(d["num_bins"]), d["trunc"],
                         int(d["trunc_in_bins"]), d["conf_tau"], d["conf_scale"],
                         int(d["conf_window"]), d["decay"], d["weight_cap"])


def _rt(prec):
    return np.float32 if prec == 32 else np.float64


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def relproj(a, b):
    """FP32 (H, c) of the relative projection a -> b."""
    H = np.zeros(9, np.float32)
    c = np.zeros(3, np.float32)
    ca, cb = cam(a), cam(b)
    lib(32).orc_relproj(C.byref(ca), C.byref(cb), _p(H), _p(c))
    return H.reshape(3, 3), c


def relproj64(a, b):
    H = np.zeros(9, np.float64)
    c = np.zeros(3, np.float64)
    ca, cb = cam(a), cam(b)
    lib(32).orc_relproj_d(C.byref(ca), C.byref(cb), _p(H), _p(c))
    return H.reshape(3, 3), c


def confidence(depth, tsdf, prec=32):
    """Per-pixel fusion weight omega of one (H, W) or a stack (K, H, W)."""
    d = _f32(depth)
    out = np.zeros(d.shape, _rt(prec))
    prm = tsdf_params(tsdf)
    flat = d.reshape(-1, d.shape[-2], d.shape[-1])
    o = out.reshape(flat.shape)
    for k in range(flat.shape[0]):
        lib(prec).orc_confidence(_p(flat[k]), flat.shape[2], flat.shape[1], C.byref(prm), _p(o[k]))
    return out


def bins(tsdf, prec=32):
    D = int(tsdf["num_bins"])
    z = np.zeros(D, _rt(prec))
    tau = np.zeros(D, _rt(prec))
    lib(prec).orc_bins(C.byref(tsdf_params(tsdf)), _p(z), _p(tau))
    return z, tau


def integrate(src, depth, tgt, tsdf, mask=None, F_prev=None, W_prev=None, pixels=None,
              conf=None, prec=32):
    """Fused volume (F, W), shape (npix, D) (all target pixels row-major when
    ``pixels`` is None)."""
    rt = _rt(prec)
    K = len(src)
    D = int(tsdf["num_bins"])
    npix = tgt.width * tgt.height if pixels is None else len(pixels)
    F = np.zeros((npix, D), rt)
    W = np.zeros((npix, D), rt)
    d = _f32(depth)
    pix = None if pixels is None else np.ascontiguousarray(pixels, np.int32)
    Fp = None if F_prev is None else np.ascontiguousarray(F_prev, rt).reshape(npix, D)
    Wp = None if W_prev is None else np.ascontiguousarray(W_prev, rt).reshape(npix, D)
    if (Fp is None) != (Wp is None):
        raise ValueError("F_prev and W_prev go together")
    cf = None if conf is None else np.ascontiguousarray(conf, rt)
    m = None if mask is None else _f32(mask)
    tc = cam(tgt)
    rc = lib(prec).orc_integrate(cams(src), K, _p(d), _p(cf), C.byref(tc),
                                 C.byref(tsdf_params(tsdf)), _p(m), _p(Fp), _p(Wp), _p(F), _p(W),
                                 _p(pix), 0 if pix is None else len(pix))
    if rc != 0:
        raise RuntimeError(f"orc_integrate failed: {rc}")
    return F, W


def raymarch(src, depth, tgt, tsdf, dprev=None, acc=None, mask=None, prec=32):
    """Volume-free march of every target ray: (depth, acc_next, samples),
    each (Ht, Wt); ``dprev`` / ``acc`` (the previous output depth and its
    accumulated weight) switch on the temporal term, ``mask`` weights it."""
    rt = _rt(prec)
    K = len(src)
    Ht, Wt = tgt.height, tgt.width
    d = _f32(depth)
    od = np.zeros((Ht, Wt), rt)
    oa = np.zeros((Ht, Wt), rt)
    st = np.zeros((Ht, Wt), np.int32)
    dp = None if dprev is None else np.ascontiguousarray(dprev, rt)
    ac = None if acc is None else np.ascontiguousarray(acc, rt)
    m = None if mask is None else _f32(mask)
    tc = cam(tgt)
    rc = lib(prec).orc_raymarch(cams(src), K, _p(d), C.byref(tc), C.byref(tsdf_params(tsdf)),
                                _p(dp), _p(ac), _p(m), _p(od), _p(oa), _p(st))
    if rc != 0:
        raise RuntimeError(f"orc_raymarch failed: {rc}")
    return od, oa, st


def network_inputs(src, tgt, tsdf_depth, rgb, depth, alpha, prec=32):
    """(9K+1, Ht, Wt) input stack of the blending network."""
    rt = _rt(prec)
    K = len(src)
    Ht, Wt = tgt.height, tgt.width
    out = np.zeros((9 * K + 1, Ht, Wt), rt)
    tc = cam(tgt)
    rc = lib(prec).orc_network_inputs(cams(src), K, C.byref(tc), _p(_f32(tsdf_depth)), _p(_f32(rgb)),
                                      _p(_f32(depth)), _p(_f32(alpha)), _p(out))
    if rc != 0:
        raise RuntimeError(f"orc_network_inputs failed: {rc}")
    return out


def blend(rgb, depth, alpha, w, w_bg, rgb_bg, prec=32):
    """Eq. 4-5: blended (3, H, W) image and (H, W) depth."""
    rt = _rt(prec)
    K, _, H, W = rgb.shape
    orgb = np.zeros((3, H, W), rt)
    od = np.zeros((H, W), rt)
    lib(prec).orc_blend(K, W, H, _p(_f32(rgb)), _p(_f32(depth)), _p(_f32(alpha)), _p(_f32(w)),
                        _p(_f32(w_bg)), _p(_f32(rgb_bg)), _p(orgb), _p(od))
    return orgb, od


def extract(F, W, tsdf, prec=32):
    rt = _rt(prec)
    D = int(tsdf["num_bins"])
    F = np.ascontiguousarray(F, rt).reshape(-1, D)
    W = np.ascontiguousarray(W, rt).reshape(-1, D)
    n = F.shape[0]
    depth = np.zeros(n, rt)
    b = np.zeros(n, np.int32)
    lib(prec).orc_extract(C.byref(tsdf_params(tsdf)), _p(F), _p(W), n, _p(depth), _p(b))
    return depth, b


def splat(src, depth, rgb, tgt, sp, mask=None, prec=32):
    """Per-view splat outputs: win_idx (K,Ht,Wt) int32, depth, rgb (K,3,Ht,Wt),
    alpha, tape (K,3,Ht,Wt); with ``mask`` (K,Hs,Ws) also the splatted masks
    (K,Ht,Wt) and their maximum over the views (Ht,Wt)."""
    rt = _rt(prec)
    K = len(src)
    Ht, Wt = tgt.height, tgt.width
    win = np.zeros((K, Ht, Wt), np.int32)
    od = np.zeros((K, Ht, Wt), rt)
    orgb = np.zeros((K, 3, Ht, Wt), rt)
    oa = np.zeros((K, Ht, Wt), rt)
    tape = np.zeros((K, 3, Ht, Wt), rt)
    d = _f32(depth)
    c = np.ascontiguousarray(rgb, np.uint8)
    m = None if mask is None else _f32(mask)
    om = None if mask is None else np.zeros((K, Ht, Wt), rt)
    omax = None if mask is None else np.zeros((Ht, Wt), rt)
    tc = cam(tgt)
    rc = lib(prec).orc_splat_masked(cams(src), K, _p(d), _p(c), C.byref(tc),
                                    C.byref(splat_params(sp)), _p(win), _p(od), _p(orgb), _p(oa),
                                    _p(tape), _p(m), _p(om), _p(omax))
    if rc != 0:
        raise RuntimeError(f"orc_splat failed: {rc}")
    out = dict(win_idx=win, depth=od, rgb=orgb, alpha=oa, tape=tape)
    if mask is not None:
        out["mask"] = om
        out["mask_max"] = omax
    return out


def exp_cw(x):
    """The FP32 exp of the EWA renderer (Cody-Waite reduction, degree-6
    Taylor polynomial) elementwise."""
    x = np.ascontiguousarray(x, np.float32).ravel()
    y = np.zeros_like(x)
    lib(32).orc_exp_cw_n(_p(x), _p(y), C.c_size_t(x.size))
    return y


def splat_ewa(src, depth, rgb, tgt, sp, lowpass=0.3, pixels=None, prec=32):
    """EWA pixel Gaussians composited front to back per view: rgb
    (K,3,Ht,Wt), alpha and depth (K,Ht,Wt).  ``pixels`` (flat target indices)
    restricts the rendering to those pixels (the rest read as not drawn)."""
    rt = _rt(prec)
    K = len(src)
    Ht, Wt = tgt.height, tgt.width
    orgb = np.zeros((K, 3, Ht, Wt), rt)
    oa = np.zeros((K, Ht, Wt), rt)
    od = np.zeros((K, Ht, Wt), rt)
    d = _f32(depth)
    c = np.ascontiguousarray(rgb, np.uint8)
    pm = None
    if pixels is not None:
        pm = np.zeros(Ht * Wt, np.uint8)
        pm[np.asarray(pixels, np.int64)] = 1
    tc = cam(tgt)
    rc = lib(prec).orc_splat_ewa(cams(src), K, _p(d), _p(c), C.byref(tc),
                                 C.byref(splat_params(sp)), C.c_float(lowpass), _p(pm),
                                 _p(orgb), _p(oa), _p(od))
    if rc != 0:
        raise RuntimeError(f"orc_splat_ewa failed: {rc}")
    return dict(rgb=orgb, alpha=oa, depth=od)


def difference_mask(rgb, rgb_prev, factor=4, beta=0.6, lambda_t=0.7, prec=32):
    """Soft difference masks (Eq. 1) of (H,W,3) or (K,H,W,3) uint8 frames."""
    a = np.ascontiguousarray(rgb, np.uint8)
    b = np.ascontiguousarray(rgb_prev, np.uint8)
    if a.shape != b.shape or a.shape[-1] != 3:
        raise ValueError("rgb and rgb_prev must be (..., H, W, 3) of one shape")
    H, W = a.shape[-3], a.shape[-2]
    fa = a.reshape(-1, H, W, 3)
    fb = b.reshape(-1, H, W, 3)
    out = np.zeros((fa.shape[0], H, W), _rt(prec))
    for k in range(fa.shape[0]):
        rc = lib(prec).orc_difference_mask(_p(fa[k]), _p(fb[k]), W, H, int(factor),
                                           C.c_float(beta), C.c_float(lambda_t), _p(out[k]))
        if rc != 0:
            raise RuntimeError(f"orc_difference_mask failed: {rc}")
    return out.reshape(a.shape[:-1])


def temporal_filter(depth, mask, prev=None, prec=32):
    """Temporally filtered depth (Eq. 2); ``prev`` None on the first frame."""
    rt = _rt(prec)
    d = _f32(depth)
    m = np.ascontiguousarray(mask, rt)
    if m.shape != d.shape:
        raise ValueError("mask and depth must have one shape")
    pv = None if prev is None else np.ascontiguousarray(prev, rt)
    out = np.zeros(d.shape, rt)
    lib(prec).orc_temporal_filter(_p(d), _p(m), _p(pv), C.c_size_t(d.size), _p(out))
    return out


def splat_backward(src, depth, rgb, tgt, sp, g_rgb, g_depth, g_alpha, prec=32, bound=False):
    """Adjoint of the splat: (d depth, d colour); with ``bound`` also the
    terms' magnitude sums of each (same shapes) and the term count of each
    depth entry (the tests' per-entry error bound)."""
    rt = _rt(prec)
    K = len(src)
    d = _f32(depth)
    c = np.ascontiguousarray(rgb, np.uint8)
    gd = np.zeros(d.shape, rt)
    gc = np.zeros(d.shape + (3,), rt)
    md = np.zeros(d.shape, rt) if bound else None
    mc = np.zeros(d.shape + (3,), rt) if bound else None
    nd = np.zeros(d.shape, np.int32) if bound else None
    tc = cam(tgt)
    rc = lib(prec).orc_splat_backward_mag(
        cams(src), K, _p(d), _p(c), C.byref(tc), C.byref(splat_params(sp)),
        _p(np.ascontiguousarray(g_rgb, rt)), _p(np.ascontiguousarray(g_depth, rt)),
        _p(np.ascontiguousarray(g_alpha, rt)), _p(gd), _p(gc), _p(md), _p(mc), _p(nd))
    if rc != 0:
        raise RuntimeError(f"orc_splat_backward failed: {rc}")
    if bound:
        return gd, gc, (md, mc, nd)
    return gd, gc


def tsdf_backward(src, depth, tgt, tsdf, g_out, mask=None, F_prev=None, W_prev=None, prec=32,
                  pixels=None, bound=False):
    """Adjoint of fusion + extraction with respect to the input depths, for
    the upstream gradient ``g_out`` on the extracted depth (all target pixels
    row-major, or one per entry of ``pixels``: every other pixel's gradient
    is zero; F_prev / W_prev then follow the list too).  With ``bound`` also
    the terms' magnitude sum and term count of each entry, the largest term
    count of the fusion-weight adjoint, each entry's error in quanta of a
    fixed-point sum, and the largest |term| (the tests' error bound)."""
    rt = _rt(prec)
    K = len(src)
    d = _f32(depth)
    gd = np.zeros(d.shape, rt)
    D = int(tsdf["num_bins"])
    npix = tgt.width * tgt.height if pixels is None else len(pixels)
    pix = None if pixels is None else np.ascontiguousarray(pixels, np.int32)
    Fp = None if F_prev is None else np.ascontiguousarray(F_prev, rt).reshape(npix, D)
    Wp = None if W_prev is None else np.ascontiguousarray(W_prev, rt).reshape(npix, D)
    m = None if mask is None else _f32(mask)
    md = np.zeros(d.shape, rt) if bound else None
    nd = np.zeros(d.shape, np.int32) if bound else None
    qs = np.zeros(d.shape, rt) if bound else None
    ncmax = C.c_int32(0)
    tbound = C.c_double(0.0)
    tc = cam(tgt)
    g = np.ascontiguousarray(g_out, rt).ravel()
    if g.size != npix:
        raise ValueError("g_out needs one value per (listed) target pixel")
    rc = lib(prec).orc_tsdf_backward_px(
        cams(src), K, _p(d), C.byref(tc), C.byref(tsdf_params(tsdf)), _p(m), _p(Fp), _p(Wp),
        _p(g), _p(pix), 0 if pix is None else len(pix), _p(gd), _p(md), _p(nd),
        C.byref(ncmax) if bound else None, _p(qs), C.byref(tbound) if bound else None)
    if rc != 0:
        raise RuntimeError(f"orc_tsdf_backward failed: {rc}")
    if bound:
        return gd, (md, nd, int(ncmax.value), qs, float(tbound.value))
    return gd


def set_threads(n):
    """Threads of the oracle's OpenMP loops from now on (both builds)."""
    for prec in (32, 64):
        lib(prec).orc_set_threads(int(n))


def num_threads():
    """Threads the oracle's OpenMP loops use in this process."""
    import multiprocessing
    env = os.environ.get("OMP_NUM_THREADS")
    return int(env) if env else multiprocessing.cpu_count()
