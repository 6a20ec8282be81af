"""The C-ABI library on the CPU: it loads, exports every symbol the header
declares, computes the relative projection bitwise like the oracle, and
rejects invalid arguments before enqueuing any GPU work (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
import scenes
from paper_2505_18932_amd import _lib as L
from paper_2505_18932_amd import ops

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "ggeom.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    names = header_functions()
    assert len(names) >= 13
    lib = L.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.SIGNATURES), set(names) ^ set(L.SIGNATURES)


@pytest.mark.parametrize("pair", [(0, 1), (2, 7), (5, 5)])
def test_relative_projection_bitwise_equals_oracle(pair):
    ring = scenes.ring_rig(8, 1.3, 640, 360)
    tgt = scenes.ring_target(0.77, 1.3, 640, 360).quantized()
    a = ring[pair[0]].quantized()
    b = ring[pair[1]].quantized() if pair[0] != pair[1] else tgt
    H, c = ops.relative_projection(a, b)
    Ho, co = oracle.relproj(a, b)
    assert np.array(H, np.float32).tobytes() == Ho.astype(np.float32).tobytes()
    assert np.array(c, np.float32).tobytes() == co.astype(np.float32).tobytes()


def _cams(K=2, w=32, h=24):
    src = scenes._quantize_all(scenes.parallel_rig([0.01 * k for k in range(K)], w, h, 30.0))
    return ops.cameras(src), ops.camera(src[0])


FAKE = C.c_void_p(1 << 20)  # never dereferenced: every call below fails validation


def _err(rc):
    return rc, L.lib().gg_last_error().decode()


def test_splat_rejects_invalid_arguments():
    lib = L.lib()
    src, tgt = _cams()
    sp = ops.splat_params(scenes.splat_params())
    args = lambda K, d=FAKE, prm=sp, ws=FAKE, nws=1 << 40: (
        src, K, d, FAKE, C.byref(tgt), C.byref(prm), FAKE, FAKE, FAKE, FAKE, None, ws, nws, None)
    assert _err(lib.splat_views(*args(0)))[0] == L.GG_ERR_INVALID
    big = ops.cameras([scenes.parallel_rig([0.0], 32, 24, 30.0)[0]] * 17)
    rc = lib.splat_views(big, 17, FAKE, FAKE, C.byref(tgt), C.byref(sp), FAKE, FAKE, FAKE, FAKE,
                         None, FAKE, 1 << 40, None)
    assert rc == L.GG_ERR_UNSUPPORTED
    rc, msg = _err(lib.splat_views(*args(2, d=None)))
    assert rc == L.GG_ERR_INVALID and "NULL" in msg
    bad = ops.splat_params(scenes.splat_params(sigma_px=0.0))
    assert lib.splat_views(*args(2, prm=bad)) == L.GG_ERR_INVALID
    bad = ops.splat_params(scenes.splat_params(band_rel=-0.1))
    assert lib.splat_views(*args(2, prm=bad)) == L.GG_ERR_INVALID
    rc, msg = _err(lib.splat_views(*args(2, nws=16)))
    assert rc == L.GG_ERR_WORKSPACE and "need" in msg
    assert lib.splat_views(*args(2, ws=None)) == L.GG_ERR_WORKSPACE
    # a camera with a non-finite parameter
    bad_src = ops.cameras([scenes.parallel_rig([0.0], 32, 24, 30.0)[0]] * 2)
    bad_src[1].fx = float("nan")
    rc = lib.splat_views(bad_src, 2, FAKE, FAKE, C.byref(tgt), C.byref(sp), FAKE, FAKE, FAKE,
                         FAKE, None, FAKE, 1 << 40, None)
    assert rc == L.GG_ERR_INVALID
    # sources of different sizes
    mixed = ops.cameras([scenes.parallel_rig([0.0], 32, 24, 30.0)[0],
                         scenes.parallel_rig([0.0], 30, 24, 30.0)[0]])
    rc = lib.splat_views(mixed, 2, FAKE, FAKE, C.byref(tgt), C.byref(sp), FAKE, FAKE, FAKE,
                         FAKE, None, FAKE, 1 << 40, None)
    assert rc == L.GG_ERR_INVALID


def test_masked_splat_rejects_invalid_arguments():
    lib = L.lib()
    src, tgt = _cams()
    sp = ops.splat_params(scenes.splat_params())

    def call(mask=FAKE, om=FAKE, omax=FAKE, nws=1 << 40):
        return lib.splat_views_masked(src, 2, FAKE, FAKE, C.byref(tgt), C.byref(sp), mask, FAKE,
                                      FAKE, FAKE, FAKE, None, om, omax, FAKE, nws, None)
    rc, msg = _err(call(mask=None))
    assert rc == L.GG_ERR_INVALID and "NULL" in msg
    rc, msg = _err(call(om=None, omax=None))
    assert rc == L.GG_ERR_INVALID and "out_mask" in msg
    assert call(nws=16) == L.GG_ERR_WORKSPACE


def test_difference_masks_reject_invalid_arguments():
    lib = L.lib()
    good = ops.mask_params()

    def call(K=2, w=64, h=48, prm=good, rgb=FAKE, prev=FAKE, m=FAKE, d=None, dp=None, f=None,
             ws=FAKE, nws=1 << 40):
        return lib.difference_masks(K, w, h, rgb, prev, C.byref(prm) if prm is not None else None,
                                    m, d, dp, f, ws, nws, None)
    assert call(K=0) == L.GG_ERR_INVALID
    assert call(K=17) == L.GG_ERR_INVALID
    assert call(w=0) == L.GG_ERR_INVALID
    assert call(h=20000) == L.GG_ERR_INVALID
    assert call(prm=None) == L.GG_ERR_INVALID
    assert call(prm=ops.mask_params(dict(lambda_t=0.0))) == L.GG_ERR_INVALID
    assert call(prm=ops.mask_params(dict(beta=1.5))) == L.GG_ERR_INVALID
    assert call(prm=ops.mask_params(dict(factor=0))) == L.GG_ERR_INVALID
    assert call(prm=ops.mask_params(dict(factor=17))) == L.GG_ERR_INVALID
    assert call(rgb=None) == L.GG_ERR_INVALID
    assert call(m=None) == L.GG_ERR_INVALID
    assert call(d=FAKE) == L.GG_ERR_INVALID  # depth without an output
    assert call(dp=FAKE) == L.GG_ERR_INVALID  # previous filtered depth without depth
    rc, msg = _err(call(nws=16))
    assert rc == L.GG_ERR_WORKSPACE and "need" in msg
    assert call(ws=None) == L.GG_ERR_WORKSPACE
    # workspace size: two K x ceil(H/f) x ceil(W/f) float planes, 256-aligned
    n = ops.workspace_size(L.GG_OP_DIFFERENCE_MASKS, 2, 65, 47, 65, 47, 4)
    per = 4 * 2 * 17 * 12
    assert n == 2 * ((per + 255) // 256 * 256)
    assert ops.workspace_size(L.GG_OP_DIFFERENCE_MASKS, 2, 65, 47, 65, 47, 0) == 0


def test_raymarch_rejects_invalid_arguments():
    lib = L.lib()
    src, tgt = _cams()
    tp = ops.tsdf_params(scenes.tsdf_params(num_bins=32))

    def call(d=FAKE, dp=None, ac=None, m=None, od=FAKE, nws=1 << 40, prm=tp):
        return lib.tsdf_raymarch(src, 2, d, C.byref(tgt), C.byref(prm), dp, ac, m, od, None, None,
                                 FAKE, nws, None)
    assert call(d=None) == L.GG_ERR_INVALID
    assert call(od=None) == L.GG_ERR_INVALID
    assert call(dp=FAKE) == L.GG_ERR_INVALID  # depth_prev without acc_prev
    assert call(m=FAKE) == L.GG_ERR_INVALID   # mask without the temporal input
    assert call(prm=ops.tsdf_params(scenes.tsdf_params(num_bins=1))) == L.GG_ERR_INVALID
    assert call(nws=8) == L.GG_ERR_WORKSPACE


def test_network_inputs_and_blend_reject_invalid_arguments():
    lib = L.lib()
    src, tgt = _cams()
    assert lib.network_inputs(src, 0, C.byref(tgt), FAKE, FAKE, FAKE, FAKE, FAKE, None) == \
        L.GG_ERR_INVALID
    assert lib.network_inputs(src, 2, C.byref(tgt), None, FAKE, FAKE, FAKE, FAKE, None) == \
        L.GG_ERR_INVALID
    assert lib.network_inputs(src, 2, C.byref(tgt), FAKE, FAKE, FAKE, FAKE, None, None) == \
        L.GG_ERR_INVALID
    args = [FAKE] * 8
    assert lib.blend_views(0, 8, 8, *args, None) == L.GG_ERR_INVALID
    assert lib.blend_views(2, 0, 8, *args, None) == L.GG_ERR_INVALID
    assert lib.blend_views(2, 8, 8, *([None] + args[1:]), None) == L.GG_ERR_INVALID
    assert lib.blend_views(2, 8, 8, *(args[:7] + [None]), None) == L.GG_ERR_INVALID


def test_tsdf_rejects_invalid_arguments():
    lib = L.lib()
    src, tgt = _cams()

    def call(prm, Fp=None, Wp=None, od=None, ob=None, ws=FAKE, nws=1 << 40, F=FAKE, tun=None):
        tp = ops.tsdf_params(prm)
        return lib.tsdf_integrate(src, 2, FAKE, C.byref(tgt), C.byref(tp), None, Fp, Wp, F, FAKE,
                                  od, ob, None if tun is None else C.byref(tun), ws, nws, None)

    good = scenes.tsdf_params(num_bins=64)
    assert call(scenes.tsdf_params(num_bins=1)) == L.GG_ERR_INVALID
    assert call(scenes.tsdf_params(num_bins=5000)) == L.GG_ERR_UNSUPPORTED
    assert call(scenes.tsdf_params(z_near=0.0)) == L.GG_ERR_INVALID
    assert call(scenes.tsdf_params(z_far=0.4)) == L.GG_ERR_INVALID
    assert call(scenes.tsdf_params(trunc=0.0)) == L.GG_ERR_INVALID
    assert call(scenes.tsdf_params(conf_window=6)) == L.GG_ERR_INVALID
    assert call(scenes.tsdf_params(conf_window=17)) == L.GG_ERR_INVALID
    assert call(scenes.tsdf_params(decay=1.5)) == L.GG_ERR_INVALID
    assert call(good, Fp=FAKE) == L.GG_ERR_INVALID
    assert call(good, od=FAKE) == L.GG_ERR_INVALID
    assert call(good, F=None) == L.GG_ERR_INVALID
    assert call(good, F=C.c_void_p((1 << 20) + 4)) == L.GG_ERR_INVALID  # misaligned volume
    assert call(good, nws=100) == L.GG_ERR_WORKSPACE
    assert call(good, ws=C.c_void_p((1 << 20) + 8)) == L.GG_ERR_WORKSPACE  # misaligned ws
    tp = ops.tsdf_params(scenes.tsdf_params(num_bins=1))
    assert lib.tsdf_extract_depth(C.byref(tgt), C.byref(tp), FAKE, FAKE, FAKE, FAKE, None,
                                  None) == L.GG_ERR_INVALID


def test_volume_tuning_is_per_call_and_validated():
    """The launch shape travels with each call (gg_volume_tuning); the
    library has no process-wide setter for it, and rejects invalid shapes
    before touching the device."""
    lib = L.lib()
    for name in ("gg_set_volume_tile", "gg_set_volume_vector", "gg_set_ewa_sort_limit"):
        assert not hasattr(lib, name), name
    src, tgt = _cams()
    tp = ops.tsdf_params(scenes.tsdf_params(num_bins=64))
    ws_small = 100  # fails the workspace check after a valid tuning
    for bad in ((-1, 0, 0), (1025, 0, 0), (8, 65, 0), (0, -1, 0), (0, 0, 3), (0, 0, 16),
                (0, 0, -1), (0, 0, 0, -1), (16, 16, 8, 65537)):
        t = ops.volume_tuning(bad)
        rc = lib.tsdf_integrate(src, 2, FAKE, C.byref(tgt), C.byref(tp), None, None, None, FAKE,
                                FAKE, None, None, C.byref(t), FAKE, 1 << 40, None)
        assert rc == L.GG_ERR_INVALID, bad
        assert lib.tsdf_extract_depth(C.byref(tgt), C.byref(tp), FAKE, FAKE, FAKE, FAKE,
                                      C.byref(t), None) == L.GG_ERR_INVALID, bad
    for ok in ((0, 0, 0), (16, 16, 8), (32, 8, 4), (1024, 64, 1), (3, 1, 2), (16, 16, 8, 128),
               (16, 16, 8, 65536), (8, 8, 4, 1)):
        t = ops.volume_tuning(ok)
        rc = lib.tsdf_integrate(src, 2, FAKE, C.byref(tgt), C.byref(tp), None, None, None, FAKE,
                                FAKE, None, None, C.byref(t), FAKE, ws_small, None)
        assert rc == L.GG_ERR_WORKSPACE, ok


def test_batch_entry_points_carry_the_survey_names():
    lib = L.lib()
    for name in ("gg_batch_plan", "gg_batch_launch", "gg_batch_free", "gg_batch_device_bytes"):
        assert hasattr(lib, name), name
    for name in ("gg_batch_create", "gg_batch_destroy"):
        assert not hasattr(lib, name), name
    tune = L.GGBatchTuning(256, 4, 3)  # bins_per_thread 3: invalid
    h = C.c_void_p()
    assert lib.gg_batch_plan(None, 0, C.byref(tune), C.byref(h)) == L.GG_ERR_INVALID


def test_two_call_fusion_rejects_invalid_arguments():
    lib = L.lib()
    src, tgt = _cams()
    good = ops.tsdf_params(scenes.tsdf_params(num_bins=64))
    bad = ops.tsdf_params(scenes.tsdf_params(num_bins=1))
    assert lib.tsdf_view_table(src, 2, None, C.byref(good), FAKE, 1 << 40, None) == \
        L.GG_ERR_INVALID
    assert lib.tsdf_view_table(src, 2, FAKE, C.byref(bad), FAKE, 1 << 40, None) == L.GG_ERR_INVALID
    assert lib.tsdf_view_table(src, 0, FAKE, C.byref(good), FAKE, 1 << 40, None) == \
        L.GG_ERR_INVALID
    assert lib.tsdf_view_table(src, 2, FAKE, C.byref(good), FAKE, 100, None) == L.GG_ERR_WORKSPACE
    call = lambda F=FAKE, Fp=None, nws=1 << 40: lib.tsdf_integrate_tabled(
        src, 2, C.byref(tgt), C.byref(good), None, Fp, None, F, FAKE, None, None, None, FAKE, nws,
        None)
    assert call(F=None) == L.GG_ERR_INVALID
    assert call(Fp=FAKE) == L.GG_ERR_INVALID
    assert call(nws=100) == L.GG_ERR_WORKSPACE


def test_ewa_splat_rejects_invalid_arguments():
    lib = L.lib()
    src, tgt = _cams()
    sp = ops.splat_params(scenes.splat_params())
    args = lambda K, d=FAKE, prm=sp, lp=0.3, ws=FAKE, nws=1 << 40, o=FAKE: (
        src, K, d, FAKE, C.byref(tgt), C.byref(prm), lp, 0, o, FAKE, FAKE, ws, nws, None)
    assert lib.splat_views_ewa(*args(0)) == L.GG_ERR_INVALID
    rc, msg = _err(lib.splat_views_ewa(*args(2, d=None)))
    assert rc == L.GG_ERR_INVALID and "NULL" in msg
    assert lib.splat_views_ewa(*args(2, o=None)) == L.GG_ERR_INVALID
    for lp in (-0.1, float("nan"), float("inf")):
        rc, msg = _err(lib.splat_views_ewa(*args(2, lp=lp)))
        assert rc == L.GG_ERR_INVALID and "lowpass" in msg
    bad = ops.splat_params(scenes.splat_params(r_max_px=0.0))
    assert lib.splat_views_ewa(*args(2, prm=bad)) == L.GG_ERR_INVALID
    rc, msg = _err(lib.splat_views_ewa(*args(2, nws=16)))
    assert rc == L.GG_ERR_WORKSPACE and "need" in msg
    assert lib.splat_views_ewa(*args(2, ws=None)) == L.GG_ERR_WORKSPACE
    rc = lib.splat_views_ewa(*args(2, ws=C.c_void_p((1 << 20) + 8)))
    assert rc == L.GG_ERR_WORKSPACE


def test_ewa_sort_limit_is_validated():
    lib = L.lib()
    src, tgt = _cams()
    sp = ops.splat_params(scenes.splat_params())
    for bad in (-1, 1, 63, 513, 1024):
        rc = lib.splat_views_ewa(src, 2, FAKE, FAKE, C.byref(tgt), C.byref(sp), 0.3, bad, FAKE, FAKE,
                                 FAKE, FAKE, 1 << 40, None)
        assert rc == L.GG_ERR_INVALID, bad
    for ok in (64, 100, 512, 0):
        rc = lib.splat_views_ewa(src, 2, FAKE, FAKE, C.byref(tgt), C.byref(sp), 0.3, ok, FAKE, FAKE,
                                 FAKE, FAKE, 16, None)
        assert rc == L.GG_ERR_WORKSPACE, ok


def test_workspace_sizes():
    sp = scenes.splat_params()
    n = ops.workspace_size(L.GG_OP_SPLAT, 4, 1280, 720, 1280, 720, 2, sp)
    assert n >= 4 * 1280 * 720 * 4  # at least one list entry per source pixel
    assert ops.workspace_size(L.GG_OP_TSDF_INTEGRATE, 4, 1280, 720, 1280, 720, 128) >= \
        4 * 1280 * 720 * 8
    assert ops.workspace_size(L.GG_OP_TSDF_INTEGRATE_BACKWARD, 4, 1280, 720, 1280, 720, 128) > \
        ops.workspace_size(L.GG_OP_TSDF_INTEGRATE, 4, 1280, 720, 1280, 720, 128)
    e = ops.workspace_size(L.GG_OP_SPLAT_EWA, 4, 1280, 720, 1280, 720, 2, sp)
    # two 8-byte keys per list entry, up to 16 tiles per Gaussian at r_max 8, plus
    # 32-byte records
    assert e >= 4 * 1280 * 720 * (2 * 8 * 16 + 32)
    assert ops.workspace_size(L.GG_OP_SPLAT_EWA, 4, 1280, 720, 1280, 720, 2, None) == 0
    assert ops.workspace_size(L.GG_OP_SPLAT, 0, 1280, 720, 1280, 720, 2, sp) == 0
    assert ops.workspace_size(99, 4, 1280, 720, 1280, 720, 2, sp) == 0


def test_product_path_refuses_cpu_tensors():
    import torch
    c = scenes.config1()
    with pytest.raises(ValueError, match="GPU"):
        ops.tsdf_integrate(c["src"], torch.from_numpy(c["depth"]), c["tgt"], c["tsdf"])


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus above 1 exits with status 2 and says
    so, before it touches a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_missing_library_fails_loudly(monkeypatch):
    """Without the built HIP library every entry point raises at once: there
    is no fallback path."""
    monkeypatch.setattr(L, "LIB_PATH", "/nonexistent/libggeom.so")
    monkeypatch.setattr(L, "_lib", None)
    with pytest.raises(RuntimeError, match="is not built"):
        ops.workspace_size(3, 2, 8, 8, 8, 8, 16)


def test_relative_projection_random_pairs_bitwise_equal_oracle():
    """Library and oracle form H and c independently (a factored evaluation
    and the plain product of the four 3 x 3 factors), both in binary128,
    rounded once, with cancellation residues below 2^-50 of their monomials'
    magnitudes taken as 0: their FP32 constants agree bitwise for random
    rigs, including identical cameras (H near the identity, c near 0)."""
    rng = np.random.default_rng(11)
    for _ in range(600):
        w, h = int(rng.integers(8, 2000)), int(rng.integers(8, 2000))
        ring = scenes.ring_rig(int(rng.integers(3, 24)), float(rng.uniform(0.3, 3.0)), w, h,
                               f=float(rng.uniform(50.0, 3000.0)))
        i, j = rng.integers(0, len(ring), 2)
        if rng.uniform() < 0.25:
            j = i
        a, b = ring[i].quantized(), ring[j].quantized()
        H, c = ops.relative_projection(a, b)
        Ho, co = oracle.relproj(a, b)
        assert np.array(H, np.float32).tobytes() == Ho.astype(np.float32).tobytes(), (i, j)
        assert np.array(c, np.float32).tobytes() == co.astype(np.float32).tobytes(), (i, j)


def test_noalloc_rejects_a_workspace_beyond_its_static_scratch():
    """tsdf_integrate_noalloc checks the size its scratch would need against
    the 64 MiB static array before touching the device."""
    lib = L.lib()
    src = ops.cameras(scenes._quantize_all(scenes.parallel_rig([0.01 * k for k in range(8)],
                                                               1920, 1080, 1000.0)))
    tgt = ops.camera(scenes.parallel_rig([0.0], 1920, 1080, 1000.0)[0])
    tp = ops.tsdf_params(scenes.tsdf_params(num_bins=64, trunc=4.0))
    need = ops.workspace_size(3, 8, 1920, 1080, 1920, 1080, 64)
    assert need > 64 << 20
    rc = lib.tsdf_integrate_noalloc(src, 8, FAKE, C.byref(tgt), C.byref(tp), None, None, None,
                                    FAKE, FAKE, FAKE, FAKE, None, None)
    assert rc == L.GG_ERR_UNSUPPORTED
    assert "static scratch" in lib.gg_last_error().decode()


def test_batch_rejects_an_invalid_item_launch_shape():
    """An item's own fusion launch shape is validated with the item, before any GPU call."""
    lib = L.lib()
    src, tgt = _cams()
    arr = (L.GGBatchItem * 1)()
    b = arr[0]
    b.src, b.K, b.depth, b.tgt = src, 2, FAKE.value, tgt
    b.tsdf = ops.tsdf_params(scenes.tsdf_params(num_bins=64))
    b.F = b.W = FAKE.value
    tune = L.GGBatchTuning(0, 0, 0, 0)
    h = C.c_void_p()
    for bad in [(-1, 0, 0, 0), (0, 65, 0, 0), (0, 0, 3, 0), (0, 0, 8, -1), (0, 0, 8, 65537)]:
        b.volume = ops.volume_tuning(bad)
        rc, msg = _err(lib.gg_batch_plan(arr, 1, C.byref(tune), C.byref(h)))
        assert rc == L.GG_ERR_INVALID and "item 0" in msg, (bad, msg)


def test_binding_structs_match_the_header():
    """Every record the binding marshals has the size and field offsets the C compiler gives
    the header's struct (a small C program built with the host compiler prints them)."""
    import shutil
    import subprocess
    import tempfile
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"gg_camera": L.GGCamera, "gg_splat_params": L.GGSplatParams,
               "gg_tsdf_params": L.GGTsdfParams, "gg_mask_params": L.GGMaskParams,
               "gg_volume_tuning": L.GGVolumeTuning,
               "gg_batch_item": L.GGBatchItem, "gg_batch_tuning": L.GGBatchTuning}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "ggeom.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} %zu\\n", sizeof({cname}));')
        for f in cls._fields_:
            lines.append(f'  printf("{cname}.{f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines += ["  return 0;", "}"]
    with tempfile.TemporaryDirectory() as d:
        src_c, exe = os.path.join(d, "layout.c"), os.path.join(d, "layout")
        open(src_c, "w").write("\n".join(lines) + "\n")
        subprocess.run([cc, "-I", os.path.join(ROOT, "include"), src_c, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    got = dict(l.rsplit(" ", 1) for l in out.strip().splitlines())
    for cname, cls in structs.items():
        assert int(got[cname]) == C.sizeof(cls), cname
        for f in cls._fields_:
            assert int(got[f"{cname}.{f[0]}"]) == getattr(cls, f[0]).offset, f"{cname}.{f[0]}"
