"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Integer outputs (winner indices, zero-crossing bins) and the fused volume
F / W are compared bitwise; colour, opacity and depth within 1e-5 relative
with a floor of 1e-3 of the largest reference magnitude (the FP32
tolerance of the problem statement, floored for values near zero).  Sizes span several tiles with ragged tails; full-size workloads
are compared on sampled target pixels the oracle computes one by one.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2505_18932_amd as gg
import scenes

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def close(got, ref, rtol=1e-5, what=""):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    floor = 1e-3 * max(np.abs(ref).max(), 1e-30)
    bad = np.abs(got - ref) > rtol * np.maximum(np.abs(ref), floor)
    assert not bad.any(), f"{what}: {bad.sum()} of {bad.size} beyond tolerance; " \
                          f"worst {np.abs(got - ref)[bad].max():.3g}"


def bits(a):
    return np.ascontiguousarray(a, np.float32).view(np.uint32)


def to_dev(c):
    return torch.from_numpy(c["depth"]).to(DEV), torch.from_numpy(c["rgb"]).to(DEV)


def check_splat(c, depth, rgb):
    out = gg.splat_views(c["src"], depth, rgb, c["tgt"], c["splat"])
    torch.cuda.synchronize()
    ref = oracle.splat(c["src"], c["depth"], c["rgb"], c["tgt"], c["splat"])
    win = out["win_idx"].cpu().numpy()
    assert np.array_equal(win, ref["win_idx"]), f"winners differ at {(win != ref['win_idx']).sum()}"
    assert np.array_equal(bits(out["depth"].cpu().numpy()), bits(ref["depth"])), "winner depth"
    close(out["rgb"].cpu().numpy(), ref["rgb"], what="rgb")
    close(out["alpha"].cpu().numpy(), ref["alpha"], what="alpha")
    tape = out["tape"].cpu().numpy()
    check_tape(tape, ref["tape"])
    return out, ref


def check_tape(tape, ref):
    """Every plane of the splat tape: sum G, the sum of log(1 - G) over members with G < 1 (fixed
    point here, FP32 in the oracle) and the count of members with G == 1.  The device's and the
    host's expf may differ by an ulp; the paper fixes no exponential, so both are correct.  Near
    G = 1 that ulp moves a member between the count and the log sum, and it changes log(1 - G) by
    up to 2^-23 / (1 - G): the log sum is ill-conditioned there.  So the test checks what is
    well-conditioned -- the transmittance prod(1 - G) = exp(log sum) (0 with a member at G = 1),
    to n ulps absolute -- and the log sum where the counts agree, to its conditioning: at most
    2^-23 / (1 - G) per member, which the pixel's transmittance bounds (each 1 - G is at least the
    product) for up to 24 members."""
    close(tape[:, 0], ref[:, 0], what="tape sum G")
    t_gpu = np.where(tape[:, 2] == 0, np.exp(tape[:, 1].astype(np.float64)), 0.0)
    t_ref = np.where(ref[:, 2] == 0, np.exp(ref[:, 1].astype(np.float64)), 0.0)
    dt = np.abs(t_gpu - t_ref)
    assert dt.max() <= 24 * 2.0 ** -24, f"transmittance differs by {dt.max():.3g}"
    dc = ref[:, 2].astype(np.int64) - tape[:, 2].astype(np.int64)
    covered = int((ref[:, 0] > 0).sum())
    assert (dc != 0).sum() <= max(8, covered // 200), \
        f"tape count of G == 1 differs at {(dc != 0).sum()} of {covered} covered pixels"
    m = (dc == 0) & (t_ref > 1e-6)
    g1 = tape[:, 1].astype(np.float64)[m]
    r1 = ref[:, 1].astype(np.float64)[m]
    bound = 1e-5 * np.abs(r1) + 24 * 2.0 ** -23 / t_ref[m]
    bad = np.abs(g1 - r1) > bound
    assert not bad.any(), f"tape sum log(1 - G): {bad.sum()} of {m.sum()} beyond their conditioning"


def check_tsdf(c, depth, F_prev=None, W_prev=None, mask=None, pixels=None, ref_prev=None):
    """Run the GPU fusion; compare (all or sampled pixels) with the oracle.
    Returns GPU (F, W, dep, bin) and the oracle's sampled (F, W)."""
    p = c["tsdf"]
    D = p["num_bins"]
    m = None if mask is None else torch.from_numpy(mask).to(DEV)
    F, W, dep, b = gg.tsdf_integrate(c["src"], depth, c["tgt"], p, F_prev=F_prev, W_prev=W_prev,
                                     mask=m)
    torch.cuda.synchronize()
    Fr_prev, Wr_prev = ref_prev if ref_prev is not None else (None, None)
    Fr, Wr = oracle.integrate(c["src"], c["depth"], c["tgt"], p, mask=mask, F_prev=Fr_prev,
                              W_prev=Wr_prev, pixels=pixels)
    dr, br = oracle.extract(Fr, Wr, p)
    Fg = F.reshape(-1, D).cpu().numpy()
    Wg = W.reshape(-1, D).cpu().numpy()
    dg = dep.reshape(-1).cpu().numpy()
    bg = b.reshape(-1).cpu().numpy()
    if pixels is not None:
        Fg, Wg, dg, bg = Fg[pixels], Wg[pixels], dg[pixels], bg[pixels]
    nF = (bits(Fg) != bits(Fr)).sum()
    nW = (bits(Wg) != bits(Wr)).sum()
    assert nF == 0 and nW == 0, f"volume differs bitwise: F {nF}, W {nW} of {Fr.size}"
    assert np.array_equal(bg, br), f"bins differ at {(bg != br).sum()}"
    close(dg, dr, what="extracted depth")
    return (F, W, dep, b), (Fr, Wr)


def test_config1_full():
    c = scenes.config1()
    depth, rgb = to_dev(c)
    check_splat(c, depth, rgb)
    check_tsdf(c, depth)


def test_config3_full():
    c = scenes.config3()
    depth, rgb = to_dev(c)
    check_splat(c, depth, rgb)
    check_tsdf(c, depth)


def test_config2_sequence_sampled():
    """Full 1280x720, K=4, D=128 ring video: three frames with the volume
    carried in place; the oracle follows 3000 sampled pixel columns."""
    c = scenes.config2()
    seq = c["seq"]
    rng = np.random.default_rng(0)
    npix = c["tgt"].width * c["tgt"].height
    pix = np.sort(rng.choice(npix, 3000, replace=False)).astype(np.int32)
    F = W = None
    ref = None
    for t in range(3):
        d, r = seq.frame(t)
        ct = dict(c, depth=d, rgb=r)
        depth, rgb = to_dev(ct)
        if t == 0:
            check_splat(ct, depth, rgb)
        (F, W, dep, b), ref = check_tsdf(ct, depth, F_prev=F, W_prev=W, pixels=pix,
                                         ref_prev=ref)


def test_config5_frame_sampled():
    """K=8, 1920x1080, D=256 (the large streaming shape), one frame."""
    c = scenes.config5()
    d, r = c["seq"].frame(0)
    ct = dict(c, depth=d, rgb=r)
    depth, rgb = to_dev(ct)
    rng = np.random.default_rng(1)
    pix = np.sort(rng.choice(1920 * 1080, 1500, replace=False)).astype(np.int32)
    check_tsdf(ct, depth, pixels=pix)


@pytest.mark.parametrize("idx", [0, 5, 11])
def test_batch_items_plain(idx):
    desc = scenes.config4_items()[idx]
    c = scenes.config4_item(desc, scale=2)
    depth, rgb = to_dev(c)
    check_splat(c, depth, rgb)
    check_tsdf(c, depth)


# ---------------------------------------------------------------------------
# edge cases


def small(seed=0, w=37, h=29, k=3, bins=24, noise=0.01, holes=0.05):
    return scenes.small_ring(seed=seed, width=w, height=h, k=k, bins=bins, noise=noise,
                             holes=holes)


@pytest.mark.parametrize("bins", [2, 3, 5, 63, 96, 130])
def test_odd_and_tiny_bin_counts(bins):
    c = small(bins=bins)
    depth, rgb = to_dev(c)
    check_tsdf(c, depth)


@pytest.mark.parametrize("wh", [(1, 1), (3, 2), (17, 1), (1, 33), (16, 16), (33, 17)])
def test_tiny_and_ragged_images(wh):
    c = small(w=wh[0], h=wh[1], k=2, bins=16)
    depth, rgb = to_dev(c)
    check_splat(c, depth, rgb)
    check_tsdf(c, depth)


@pytest.mark.parametrize("window", [1, 3, 5, 7, 9, 11, 13, 15])
def test_every_confidence_window(window):
    """Each odd window side 1 .. 15 has its own unrolled interior form in the
    confidence kernel and in both window kernels of the fusion backward; at
    80 x 40 every one of them meets interior and border tiles.  Volume
    bitwise, depth gradient to the gradient tolerance."""
    c = small(w=80, h=40, k=3, bins=24)
    c["tsdf"] = dict(c["tsdf"], conf_window=window)
    depth, _ = to_dev(c)
    (F, W, dep, b), _ = check_tsdf(c, depth)
    rng = np.random.default_rng(window)
    g = rng.standard_normal(dep.shape).astype(np.float32)
    g2 = gg.tsdf_extract_depth_backward(c["tgt"], c["tsdf"], F, W, b, torch.from_numpy(g).to(DEV))
    gd = gg.tsdf_integrate_backward(c["src"], depth, c["tgt"], c["tsdf"], F, W, b, g2)
    torch.cuda.synchronize()
    ref, bd = tsdf_ref(c, g.ravel())
    assert np.abs(ref).max() > 0
    grad_close(gd.cpu().numpy(), ref, bd, f"tsdf depth gradient, window {window}")


def test_library_maxima():
    """The declared limits: 16 views per call, 4096 bins, and a row of 16384
    pixels (the widest image the host accepts)."""
    c = scenes.small_ring(seed=4, width=9, height=7, k=16, n_ring=17, bins=32, noise=0.01,
                          holes=0.05)
    assert c["depth"].shape[0] == 16
    depth, rgb = to_dev(c)
    check_splat(c, depth, rgb)
    check_tsdf(c, depth)
    c = small(w=6, h=5, k=2, bins=4096)
    depth, _ = to_dev(c)
    check_tsdf(c, depth)
    c = small(w=16384, h=2, k=2, bins=8)
    depth, rgb = to_dev(c)
    check_splat(c, depth, rgb)
    check_tsdf(c, depth)


def test_carried_fusion_both_table_forms():
    """The carried fusion with up to four views reads the view tables with structured loads
    where a table row (the image width plus its closing record) fits the resource's stride
    field, 2047 records, and with range-checked raw loads beyond; widths straddle the limit,
    a carried second frame included, and both forms give the oracle's volume bitwise."""
    for w in (2046, 2047, 4100):
        c = small(w=w, h=3, k=2, bins=32)
        depth, _ = to_dev(c)
        (F, W, _, _), ref = check_tsdf(c, depth)
        check_tsdf(c, depth, F_prev=F, W_prev=W, ref_prev=ref)


def test_single_view_and_many_views():
    for k in (1, 8):
        c = small(k=k)
        depth, rgb = to_dev(c)
        check_splat(c, depth, rgb)
        check_tsdf(c, depth)


def test_invalid_depths_are_holes():
    c = small(holes=0.0)
    d = c["depth"].copy()
    d[0, 3, 4] = np.nan
    d[0, 5, 6] = np.inf
    d[1, 7, 8] = -1.0
    d[2, :, 10:14] = 0.0
    c["depth"] = d
    depth, rgb = to_dev(c)
    check_splat(c, depth, rgb)
    check_tsdf(c, depth)


def test_all_holes():
    c = small()
    c["depth"] = np.zeros_like(c["depth"])
    depth, rgb = to_dev(c)
    out, _ = check_splat(c, depth, rgb)
    assert (out["win_idx"] == -1).all()
    (F, W, dep, b), _ = check_tsdf(c, depth)
    assert (W == 0).all() and (b == -1).all()


def test_mask_carry_and_in_place():
    c = small()
    depth, rgb = to_dev(c)
    (F, W, _, _), ref = check_tsdf(c, depth)
    rng = np.random.default_rng(3)
    mask = rng.uniform(0, 1.2, (c["tgt"].height, c["tgt"].width)).astype(np.float32)
    c2 = dict(c, depth=(c["depth"] * np.float32(1.01)).astype(np.float32))
    d2 = torch.from_numpy(c2["depth"]).to(DEV)
    # in place: F, W are both previous and output
    Fg, Wg, dep, b = gg.tsdf_integrate(c2["src"], d2, c2["tgt"], c2["tsdf"], F_prev=F, W_prev=W,
                                       F=F, W=W, mask=torch.from_numpy(mask).to(DEV))
    torch.cuda.synchronize()
    Fr, Wr = oracle.integrate(c2["src"], c2["depth"], c2["tgt"], c2["tsdf"], mask=mask,
                              F_prev=ref[0], W_prev=ref[1])
    D = c["tsdf"]["num_bins"]
    assert np.array_equal(bits(Fg.reshape(-1, D).cpu().numpy()), bits(Fr))
    assert np.array_equal(bits(Wg.reshape(-1, D).cpu().numpy()), bits(Wr))


def test_standalone_extract_equals_fused():
    c = scenes.config3()
    depth, _ = to_dev(c)
    F, W, dep, b = gg.tsdf_integrate(c["src"], depth, c["tgt"], c["tsdf"])
    d2, b2 = gg.tsdf_extract_depth(c["tgt"], c["tsdf"], F, W)
    torch.cuda.synchronize()
    assert torch.equal(b, b2)
    assert torch.equal(dep.view(torch.int32), d2.view(torch.int32))


def test_repeat_runs_bitwise():
    c = scenes.config1()
    depth, rgb = to_dev(c)
    outs = [gg.splat_views(c["src"], depth, rgb, c["tgt"], c["splat"]) for _ in range(10)]
    vols = [gg.tsdf_integrate(c["src"], depth, c["tgt"], c["tsdf"]) for _ in range(10)]
    torch.cuda.synchronize()
    for o in outs[1:]:
        for key in ("win_idx", "depth", "rgb", "alpha", "tape"):
            assert torch.equal(o[key].view(torch.int32), outs[0][key].view(torch.int32)), key
    for v in vols[1:]:
        for a, b in zip(v, vols[0]):
            assert torch.equal(a.view(torch.int32), b.view(torch.int32))


def test_volume_tile_shape_does_not_change_results():
    """Launch shape and tile order (bands of 1 .. 5 tiles across a row of 6,
    a narrower last band, several bands per row of 12, or row-major) leave
    every output bitwise unchanged."""
    c = small(w=96, h=29, bins=96)
    depth, _ = to_dev(c)
    base = gg.tsdf_integrate(c["src"], depth, c["tgt"], c["tsdf"])
    F, W = base[0], base[1]
    shapes = [(0, 0, 0), (1, 1, 0), (3, 1, 0), (8, 1, 0), (8, 8, 0), (16, 16, 0), (40, 8, 0),
              (32, 32, 0), (16, 16, 16), (16, 16, 48), (16, 16, 80), (8, 8, 24), (32, 16, 32),
              (16, 16, 65536), (40, 8, 80)]
    for vec in (1, 2, 4, 8):
        for ppb in shapes:
            tun = (ppb[0], ppb[1], vec, ppb[2])
            v = gg.tsdf_integrate(c["src"], depth, c["tgt"], c["tsdf"], tuning=tun)
            e = gg.tsdf_extract_depth(c["tgt"], c["tsdf"], F, W, tuning=tun)
            torch.cuda.synchronize()
            for a, b in zip(v, base):
                assert torch.equal(a.view(torch.int32), b.view(torch.int32)), tun
            for a, b in zip(e, base[2:]):
                assert torch.equal(a.view(torch.int32), b.view(torch.int32)), tun


# ---------------------------------------------------------------------------
# adjoints against the oracle's


U32 = 2.0 ** -24
# Roundings along one term beyond the count of summed terms: the term's own
# products and quotients (about a dozen), the extraction factor upstream, the
# 49-term window statistic of a fusion-weight term, and a band's colour sum
# inside the splat's colour difference.
CHAIN = 96


def grad_close(got, ref, bound, what):
    """Gradients against the FP32 oracle: norm-wise within 1e-5, and per
    entry within 1e-5 of the entry or within the running error bound
    (terms + CHAIN) 2^-24 M (+ Q, see below), whichever is larger.  M is the
    oracle's sum of the entry's terms over magnitudes (differences of computed
    values as sums of magnitudes) and terms its number of summed terms: the
    GPU sums the same FP32 terms, the oracle in FP32 one by one, so both lie
    within that bound of the exact sum of the terms.  ``bound`` is (M, terms)
    or (M, terms, Q): Q an absolute allowance per entry, the fixed-point
    quantisation of the fusion adjoint's sums (fusion_quantum)."""
    mag, terms = bound[0], bound[1]
    quant = bound[2] if len(bound) > 2 else 0.0
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    mag = np.asarray(mag, np.float64)
    assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref), what
    allowed = np.maximum(1e-5 * np.abs(ref),
                         (np.asarray(terms, np.float64) + CHAIN) * U32 * mag + quant)
    bad = np.abs(got - ref) > allowed
    assert not bad.any(), f"{what}: {bad.sum()} of {bad.size} beyond the bound; worst " \
                          f"{(np.abs(got - ref)[bad] / np.maximum(allowed[bad], 1e-300)).max():.3g}x"


def fusion_quantum(term_bound, npix):
    """The fusion adjoint accumulates in 64-bit fixed point with the scale
    include/ggeom.h states: the quantum is 2^-E, E = 61 - e, 2^(e-1) <=
    2 npix m < 2^e, m the largest |term| bound (here the oracle's, which the
    library's FP32 evaluation matches to rounding: one power of two of slack)."""
    if term_bound <= 0:
        return 0.0
    e = np.frexp(2.0 * npix * term_bound)[1]
    return 2.0 ** -(61 - e - 1)


def tsdf_ref(c, g, **kw):
    """Oracle fusion adjoint and its bound (terms: the entry's own plus the
    most terms of any fusion-weight adjoint feeding its window terms; Q: the
    entry's error in fixed-point quanta times the quantum)."""
    r, (m, n, ncm, qs, tb) = oracle.tsdf_backward(c["src"], c["depth"], c["tgt"], c["tsdf"], g,
                                                  bound=True, **kw)
    q = fusion_quantum(tb, c["tgt"].width * c["tgt"].height)
    return r, (m, n + ncm, np.asarray(qs, np.float64) * q)


def splat_ref(c, g_rgb, g_z, g_a):
    """Oracle splat adjoints (depth, colour) with their bounds."""
    rd, rc, (md, mc, nd) = oracle.splat_backward(c["src"], c["depth"], c["rgb"], c["tgt"],
                                                 c["splat"], g_rgb, g_z, g_a, bound=True)
    return (rd, (md, nd)), (rc, (mc, nd[..., None]))


def test_tsdf_backward_parity():
    c = scenes.config1()
    depth, _ = to_dev(c)
    F, W, dep, b = gg.tsdf_integrate(c["src"], depth, c["tgt"], c["tsdf"])
    rng = np.random.default_rng(2)
    g = rng.standard_normal(dep.shape).astype(np.float32)
    g2 = gg.tsdf_extract_depth_backward(c["tgt"], c["tsdf"], F, W, b, torch.from_numpy(g).to(DEV))
    gd = gg.tsdf_integrate_backward(c["src"], depth, c["tgt"], c["tsdf"], F, W, b, g2)
    torch.cuda.synchronize()
    ref, bd = tsdf_ref(c, g.ravel())
    grad_close(gd.cpu().numpy(), ref, bd, "tsdf depth gradient")


def test_splat_backward_parity():
    c = scenes.config1()
    depth, rgb = to_dev(c)
    out = gg.splat_views(c["src"], depth, rgb, c["tgt"], c["splat"])
    rng = np.random.default_rng(3)
    g_rgb = rng.standard_normal(out["rgb"].shape).astype(np.float32)
    g_z = rng.standard_normal(out["depth"].shape).astype(np.float32)
    g_a = rng.standard_normal(out["alpha"].shape).astype(np.float32)
    gd, gc = gg.splat_views_backward(c["src"], depth, rgb, c["tgt"], c["splat"], out,
                                     torch.from_numpy(g_rgb).to(DEV), torch.from_numpy(g_z).to(DEV),
                                     torch.from_numpy(g_a).to(DEV))
    torch.cuda.synchronize()
    (rd, bd), (rc, bc) = splat_ref(c, g_rgb, g_z, g_a)
    grad_close(gc.cpu().numpy(), rc, bc, "splat colour gradient")
    grad_close(gd.cpu().numpy(), rd, bd, "splat depth gradient")


def test_two_call_fusion_on_two_streams():
    """tsdf_view_table on a second stream, an event, then tsdf_integrate_tabled
    on the main stream, pipelined over a small video with two workspaces as
    the benchmark does: bitwise the volume and depths of tsdf_integrate."""
    c = scenes.small_video(seed=2, width=96, height=64, k=3, bins=32)
    frames = [c["seq"].frame(t)[0] for t in range(5)]
    K, H, W = frames[0].shape
    tp = c["tsdf"]
    ref = []
    F = Wv = None
    for d in frames:
        F, Wv, dep, b = gg.tsdf_integrate(c["src"], torch.from_numpy(d).to(DEV), c["tgt"], tp,
                                          F_prev=F, W_prev=Wv)
        ref.append((F.clone(), Wv.clone(), dep.clone(), b.clone()))
    need = gg.workspace_size(3, K, W, H, c["tgt"].width, c["tgt"].height, tp["num_bins"])
    wss = [torch.empty(need, dtype=torch.uint8, device=DEV) for _ in range(2)]
    side = torch.cuda.Stream(device=DEV)
    ev_t = [torch.cuda.Event(), torch.cuda.Event()]
    ev_f = [torch.cuda.Event(), torch.cuda.Event()]
    main = torch.cuda.current_stream(DEV)
    dd = [torch.from_numpy(d).to(DEV) for d in frames]
    torch.cuda.synchronize()
    F = Wv = None
    outs = []
    for i, d in enumerate(dd):
        b = i % 2
        side.wait_event(ev_f[b])
        gg.tsdf_view_table(c["src"], d, tp, ws=wss[b], stream=side)
        ev_t[b].record(side)
        main.wait_event(ev_t[b])
        if F is None:
            F, Wv, dep, bb = gg.tsdf_integrate(c["src"], d, c["tgt"], tp, ws=wss[b],
                                               table_ready=True)
        else:
            F, Wv, dep, bb = gg.tsdf_integrate(c["src"], d, c["tgt"], tp, F_prev=F, W_prev=Wv,
                                               F=F, W=Wv, ws=wss[b], table_ready=True)
        ev_f[b].record(main)
        outs.append((dep.clone(), bb.clone()))
    torch.cuda.synchronize()
    Fr, Wr, _, _ = ref[-1]
    assert torch.equal(F.view(torch.int32), Fr.view(torch.int32))
    assert torch.equal(Wv.view(torch.int32), Wr.view(torch.int32))
    for (dep, bb), r in zip(outs, ref):
        assert torch.equal(dep.view(torch.int32), r[2].view(torch.int32))
        assert torch.equal(bb, r[3])


def test_full_video_in_the_benchmark_launch(video_frames):
    """The metric's workload (1280x720, K=4, D=128) in the benchmark's own
    launch configuration: fusion tile (16, 16, 8), the view table and the
    splat on a second stream, the fusion from that table on the main stream,
    two workspaces, two frames with the volume carried in place.  The oracle
    follows 2000 sampled pixel columns through both frames; the second
    frame's splat is compared in full."""
    c, frames = video_frames
    tp, sp = c["tsdf"], c["splat"]
    K, H, W = frames[0][0].shape
    Ht, Wt = c["tgt"].height, c["tgt"].width
    rng = np.random.default_rng(5)
    pix = np.sort(rng.choice(Ht * Wt, 2000, replace=False)).astype(np.int32)
    need = gg.workspace_size(3, K, W, H, Wt, Ht, tp["num_bins"])
    wss = [torch.empty(need, dtype=torch.uint8, device=DEV) for _ in range(2)]
    ws_s = torch.empty(gg.workspace_size(1, K, W, H, Wt, Ht, 2, sp), dtype=torch.uint8,
                       device=DEV)
    side = torch.cuda.Stream(device=DEV)
    main = torch.cuda.current_stream(DEV)
    ev_t = [torch.cuda.Event(), torch.cuda.Event()]
    ev_f = [torch.cuda.Event(), torch.cuda.Event()]
    dev_frames = [(torch.from_numpy(d).to(DEV), torch.from_numpy(r).to(DEV)) for d, r in frames]
    tun = (16, 16, 8)
    F = Wv = None
    outs = []
    torch.cuda.synchronize()
    for i, (d, r) in enumerate(dev_frames):
        b = i % 2
        side.wait_event(ev_f[b])
        gg.tsdf_view_table(c["src"], d, tp, ws=wss[b], stream=side)
        ev_t[b].record(side)
        so = gg.splat_views(c["src"], d, r, c["tgt"], sp, ws=ws_s, stream=side)
        main.wait_event(ev_t[b])
        if F is None:
            F, Wv, dep, bb = gg.tsdf_integrate(c["src"], d, c["tgt"], tp, ws=wss[b],
                                               table_ready=True, tuning=tun)
        else:
            F, Wv, dep, bb = gg.tsdf_integrate(c["src"], d, c["tgt"], tp, F_prev=F,
                                               W_prev=Wv, F=F, W=Wv, ws=wss[b],
                                               table_ready=True, tuning=tun)
        ev_f[b].record(main)
        torch.cuda.synchronize()
        outs.append((F.reshape(-1, tp["num_bins"])[pix].cpu().numpy(),
                     Wv.reshape(-1, tp["num_bins"])[pix].cpu().numpy(),
                     dep.reshape(-1)[pix].cpu().numpy(), bb.reshape(-1)[pix].cpu().numpy()))
    ref = None
    for (d, r), (Fg, Wg, dg, bg) in zip(frames, outs):
        Fr_prev, Wr_prev = ref if ref is not None else (None, None)
        Fr, Wr = oracle.integrate(c["src"], d, c["tgt"], tp, F_prev=Fr_prev, W_prev=Wr_prev,
                                  pixels=pix)
        dr, br = oracle.extract(Fr, Wr, tp)
        assert np.array_equal(bits(Fg), bits(Fr)) and np.array_equal(bits(Wg), bits(Wr))
        assert np.array_equal(bg, br)
        close(dg, dr, what="extracted depth")
        ref = (Fr, Wr)
    d, r = frames[-1]
    sref = oracle.splat(c["src"], d, r, c["tgt"], sp)
    assert np.array_equal(so["win_idx"].cpu().numpy(), sref["win_idx"])
    assert np.array_equal(bits(so["depth"].cpu().numpy()), bits(sref["depth"]))
    close(so["rgb"].cpu().numpy(), sref["rgb"], what="rgb")
    close(so["alpha"].cpu().numpy(), sref["alpha"], what="alpha")


def test_backward_at_the_streaming_size(streaming_frame):
    """The adjoints at 1920x1080, K=8, D=256 (the backward the benchmark
    times there), through properties that hold at any size: a second call
    agrees bitwise, and doubling every upstream gradient doubles every input
    gradient exactly (the fusion's fixed-point scale moves by one power of
    two; every other step is a product with, or a sum of, doubled terms)."""
    c, (d, r) = streaming_frame
    depth, rgb = torch.from_numpy(d).to(DEV), torch.from_numpy(r).to(DEV)
    tp, sp = c["tsdf"], c["splat"]
    F, W, dep, b = gg.tsdf_integrate(c["src"], depth, c["tgt"], tp)
    so = gg.splat_views(c["src"], depth, rgb, c["tgt"], sp)
    rng = np.random.default_rng(6)
    g = torch.from_numpy(rng.standard_normal(dep.shape).astype(np.float32)).to(DEV)
    gs = [torch.from_numpy(rng.standard_normal(so[k].shape).astype(np.float32)).to(DEV)
          for k in ("rgb", "depth", "alpha")]

    def fusion_grad(scale):
        g2 = gg.tsdf_extract_depth_backward(c["tgt"], tp, F, W, b, g * scale)
        return gg.tsdf_integrate_backward(c["src"], depth, c["tgt"], tp, F, W, b, g2)

    def splat_grad(scale):
        return gg.splat_views_backward(c["src"], depth, rgb, c["tgt"], sp, so,
                                       *(x * scale for x in gs))

    a1, a2, a3 = fusion_grad(1.0), fusion_grad(1.0), fusion_grad(2.0)
    s1, s2, s3 = splat_grad(1.0), splat_grad(1.0), splat_grad(2.0)
    torch.cuda.synchronize()
    assert torch.isfinite(a1).all() and (a1 != 0).sum() > 0.05 * a1.numel()
    assert torch.equal(a1.view(torch.int32), a2.view(torch.int32)), "fusion gradient repeat"
    assert torch.equal((2 * a1).view(torch.int32), a3.view(torch.int32)), "fusion gradient x2"
    for x, y, z, what in zip(s1, s2, s3, ("depth", "colour")):
        assert torch.isfinite(x).all() and (x != 0).any(), what
        assert torch.equal(x.view(torch.int32), y.view(torch.int32)), f"splat {what} repeat"
        assert torch.equal((2 * x).view(torch.int32), z.view(torch.int32)), f"splat {what} x2"


def test_backward_at_the_differentiation_size():
    """The three adjoints the benchmark times at 640x360, K=4, D=96 (random
    upstream gradients on every output) against the oracle's adjoints, to the
    gradient tolerance."""
    c = scenes.config3()
    depth, rgb = to_dev(c)
    F, W, dep, b = gg.tsdf_integrate(c["src"], depth, c["tgt"], c["tsdf"])
    so = gg.splat_views(c["src"], depth, rgb, c["tgt"], c["splat"])
    rng = np.random.default_rng(7)
    g_t = rng.standard_normal(dep.shape).astype(np.float32)
    g_rgb, g_z, g_a = (rng.standard_normal(so[k].shape).astype(np.float32)
                       for k in ("rgb", "depth", "alpha"))
    gd, gc = gg.splat_views_backward(c["src"], depth, rgb, c["tgt"], c["splat"], so,
                                     *(torch.from_numpy(x).to(DEV) for x in (g_rgb, g_z, g_a)))
    g2 = gg.tsdf_extract_depth_backward(c["tgt"], c["tsdf"], F, W, b,
                                        torch.from_numpy(g_t).to(DEV))
    gt = gg.tsdf_integrate_backward(c["src"], depth, c["tgt"], c["tsdf"], F, W, b, g2)
    torch.cuda.synchronize()
    (rd, bd), (rc, bc) = splat_ref(c, g_rgb, g_z, g_a)
    rt, bt = tsdf_ref(c, g_t.ravel())
    grad_close(gc.cpu().numpy(), rc, bc, "splat colour gradient")
    grad_close(gd.cpu().numpy(), rd, bd, "splat depth gradient")
    grad_close(gt.cpu().numpy(), rt, bt, "fusion depth gradient")


def test_backward_at_the_streaming_size_against_the_oracle(streaming_frame):
    """Both adjoints at 1920x1080, K=8, D=256 (the streaming workload) against
    the oracle's, with the upstream gradients nonzero on 2000 sampled target
    pixels only: every other pixel contributes nothing, so the oracle forms
    only those pixels' voxels, while the GPU runs its full launch (every
    pixel, zero gradients elsewhere).  Tolerance: the gradient bound."""
    c, (d, r) = streaming_frame
    ct = dict(c, depth=d, rgb=r)
    depth, rgb = torch.from_numpy(d).to(DEV), torch.from_numpy(r).to(DEV)
    tp, sp = c["tsdf"], c["splat"]
    Ht, Wt = c["tgt"].height, c["tgt"].width
    rng = np.random.default_rng(8)
    pix = np.sort(rng.choice(Ht * Wt, 2000, replace=False)).astype(np.int32)
    sel = np.zeros(Ht * Wt, bool)
    sel[pix] = True
    sel = sel.reshape(Ht, Wt)
    g = np.zeros((Ht, Wt), np.float32)
    g[sel] = rng.standard_normal(sel.sum()).astype(np.float32)
    F, W, dep, b = gg.tsdf_integrate(c["src"], depth, c["tgt"], tp)
    so = gg.splat_views(c["src"], depth, rgb, c["tgt"], sp)
    K = d.shape[0]
    g_rgb = np.zeros((K, 3, Ht, Wt), np.float32)
    g_z = np.zeros((K, Ht, Wt), np.float32)
    g_a = np.zeros((K, Ht, Wt), np.float32)
    g_rgb[:, :, sel] = rng.standard_normal((K, 3, sel.sum())).astype(np.float32)
    g_z[:, sel] = rng.standard_normal((K, sel.sum())).astype(np.float32)
    g_a[:, sel] = rng.standard_normal((K, sel.sum())).astype(np.float32)
    g2 = gg.tsdf_extract_depth_backward(c["tgt"], tp, F, W, b, torch.from_numpy(g).to(DEV))
    gt = gg.tsdf_integrate_backward(c["src"], depth, c["tgt"], tp, F, W, b, g2)
    gd, gc = gg.splat_views_backward(c["src"], depth, rgb, c["tgt"], sp, so,
                                     *(torch.from_numpy(x).to(DEV) for x in (g_rgb, g_z, g_a)))
    torch.cuda.synchronize()
    rt, bt = tsdf_ref(ct, g.ravel()[pix], pixels=pix)
    assert (rt != 0).sum() > 10000
    grad_close(gt.cpu().numpy(), rt, bt, "fusion depth gradient (streaming size)")
    (rd, bd), (rc, bc) = splat_ref(ct, g_rgb, g_z, g_a)
    assert (rd != 0).sum() > 1000
    grad_close(gd.cpu().numpy(), rd, bd, "splat depth gradient (streaming size)")
    grad_close(gc.cpu().numpy(), rc, bc, "splat colour gradient (streaming size)")


@pytest.mark.parametrize("vec", [8, 4, 2])
def test_fusion_stream_probe(vec):
    """The fusion kernel launched with no views (the benchmark's ceiling
    probe of the volume stream) only decays the carried weight, in place:
    W = min(decay W_prev, cap), F = (W F_prev) / W (0 where W is 0), in that
    FP32 order; its fused extraction equals tsdf_extract_depth on the
    result."""
    c = small(w=61, h=35, k=3, bins=32)
    depth, _ = to_dev(c)
    tp = c["tsdf"]
    F, W, _, _ = gg.tsdf_integrate(c["src"], depth, c["tgt"], tp)
    Fp, Wp = F.cpu().numpy(), W.cpu().numpy()
    od = torch.empty(F.shape[:2], device=DEV)
    ob = torch.empty(F.shape[:2], dtype=torch.int32, device=DEV)
    gg.ops.fusion_stream_probe(c["tgt"], tp, F, W, F, W, od, ob, tuning=(16, 16, vec))
    torch.cuda.synchronize()
    wn = np.minimum(np.float32(tp["decay"]) * Wp, np.float32(tp["weight_cap"]))
    with np.errstate(invalid="ignore", divide="ignore"):
        fn = np.where(wn > 0, (wn * Fp) / wn, np.float32(0)).astype(np.float32)
    assert np.array_equal(bits(W.cpu().numpy()), bits(wn))
    assert np.array_equal(bits(F.cpu().numpy()), bits(fn))
    d2, b2 = gg.tsdf_extract_depth(c["tgt"], tp, F, W)
    torch.cuda.synchronize()
    assert torch.equal(od.view(torch.int32), d2.view(torch.int32))
    assert torch.equal(ob, b2)
