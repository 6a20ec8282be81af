"""The batched path (persistent kernels in one hipGraph launch) against the
plain calls, item by item, bitwise, for several launch tunings, item orders
and graph replays; and against the oracle directly, in full at half size and
on sampled pixel columns at full size."""
import os

import numpy as np
import pytest
import torch

import paper_2505_18932_amd as gg
import scenes

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _items(scale=4, n=24):
    out = []
    for desc in scenes.config4_items()[:n]:
        c = scenes.config4_item(desc, scale=scale)
        out.append(dict(src=c["src"], tgt=c["tgt"], depth=torch.from_numpy(c["depth"]).to(DEV),
                        rgb=torch.from_numpy(c["rgb"]).to(DEV), splat=c["splat"], tsdf=c["tsdf"]))
    return out


def _plain(it, F_prev=None, W_prev=None):
    s = None
    if it.get("rgb") is not None:
        s = gg.splat_views(it["src"], it["depth"], it["rgb"], it["tgt"], it["splat"])
    mask = it.get("mask")
    F, W, d, b = gg.tsdf_integrate(it["src"], it["depth"], it["tgt"], it["tsdf"], F_prev=F_prev,
                                   W_prev=W_prev, mask=mask)
    return s, F, W, d, b


def _same(a, b, what):
    assert torch.equal(a.view(torch.int32), b.view(torch.int32)), what


def _check(plan_items, refs):
    for i, (it, (s, F, W, d, b)) in enumerate(zip(plan_items, refs)):
        _same(it["F"], F, f"item {i} F")
        _same(it["W"], W, f"item {i} W")
        _same(it["depth_out"], d, f"item {i} depth")
        _same(it["bin_out"], b, f"item {i} bin")
        if s is not None:
            for key in ("win_idx", "depth", "rgb", "alpha", "tape"):
                _same(it["splat_out"][key], s[key], f"item {i} splat {key}")


# (pixels per fusion workgroup, light-phase workgroups per CU, bins per thread, branches)
@pytest.mark.parametrize("tuning", [(0, 0, 0, 0), (64, 1, 0, 0), (512, 2, 8, 2), (1024, 8, 4, 1),
                                    (16, 0, 8, 1), (3, 0, 8, 0)])
def test_batch_equals_plain(tuning):
    items = _items()
    refs = [_plain(it) for it in items]
    plan = gg.BatchPlan(items, *tuning)
    plan.launch()
    torch.cuda.synchronize()
    _check(items, refs)
    plan.close()


# each item's own fusion launch shape (gg_batch_item.volume): pixels per workgroup, per
# wavefront row, bins per thread and band width, cycled over the items
ITEM_SHAPES = [(16, 16, 8, 0), (32, 16, 8, 128), (64, 16, 8, 0), (16, 16, 8, 192),
               (0, 0, 4, 0), (32, 8, 4, 0), (8, 8, 2, 0), (16, 16, 8, 65536), None]


@pytest.mark.parametrize("plan_tuning", [(0, 0, 0, 0), (32, 1, 4, 1)])
def test_batch_items_with_their_own_launch_shapes(plan_tuning):
    """Items that bring their own fusion launch shape (several items sharing one, some none)
    give the plain calls' results bitwise, whatever the plan's own tuning."""
    items = _items(n=18)
    refs = [_plain(it) for it in items]
    for i, it in enumerate(items):
        shape = ITEM_SHAPES[i % len(ITEM_SHAPES)]
        if shape is not None:
            it["volume"] = shape
    plan = gg.BatchPlan(items, *plan_tuning)
    plan.launch()
    torch.cuda.synchronize()
    _check(items, refs)
    plan.close()


def test_batch_shuffled_order_and_replays():
    items = _items(n=10)
    refs = [_plain(it) for it in items]
    order = np.random.default_rng(0).permutation(len(items))
    shuffled = [items[i] for i in order]
    plan = gg.BatchPlan(shuffled)
    for rep in range(3):
        # eager work between replays (the graph must not depend on it)
        junk = torch.randn(1 << 20, device=DEV).sum()
        plan.launch()
        torch.cuda.synchronize()
        _check(shuffled, [refs[i] for i in order])
        del junk
    plan.close()


def test_batch_mixed_items_carry_and_mask():
    """Items without splat, odd and tiny bin counts, a single view, a mask,
    an in-place carried volume and confidence windows other than 7."""
    base = _items(n=4)
    small = scenes.small_ring(seed=3, width=41, height=23, k=1, bins=7)
    base.append(dict(src=small["src"], tgt=small["tgt"], depth=torch.from_numpy(small["depth"]).to(DEV),
                     tsdf=small["tsdf"]))  # no rgb, K=1, D=7 (one bin per thread)
    base[1]["tsdf"] = dict(base[1]["tsdf"], num_bins=66, conf_window=11)  # two bins per thread
    base[0]["tsdf"] = dict(base[0]["tsdf"], conf_window=15)
    base[4]["tsdf"] = dict(base[4]["tsdf"], conf_window=1)
    rng = np.random.default_rng(1)
    it = base[2]
    it["mask"] = torch.from_numpy(rng.uniform(0, 1, (it["tgt"].height, it["tgt"].width))
                                  .astype(np.float32)).to(DEV)
    # carried state for item 3: previous frame from the plain path, updated in place
    _, F0, W0, _, _ = _plain(base[3])
    refs = []
    for i, x in enumerate(base):
        if i == 3:
            refs.append(_plain(x, F_prev=F0.clone(), W_prev=W0.clone()))
        else:
            refs.append(_plain(x))
    base[3]["F"] = F0.clone()
    base[3]["W"] = W0.clone()
    base[3]["F_prev"] = base[3]["F"]
    base[3]["W_prev"] = base[3]["W"]
    plan = gg.BatchPlan(base)
    plan.launch()
    torch.cuda.synchronize()
    _check(base, refs)
    plan.close()


@pytest.mark.parametrize("vec", [8, 2])
def test_batch_bins_per_thread(vec):
    """Other fusion specialisations (bins per thread) in the batch: still the
    plain results, which do not depend on that choice either."""
    items = _items(n=8)
    refs = [_plain(it) for it in items]
    plan = gg.BatchPlan(items, bins_per_thread=vec)
    plan.launch()
    torch.cuda.synchronize()
    _check(items, refs)
    plan.close()


# GG_BATCH_CASES widens the random mixes (the default keeps the suite quick)
BATCH_CASES = int(os.environ.get("GG_BATCH_CASES", "4"))


@pytest.mark.parametrize("seed", range(BATCH_CASES))
def test_batch_random_mix(seed):
    """Seeded random mixes of 3 to 12 small ring items: view counts 1 to 8,
    ragged sizes, 2 to 199 bins, any confidence window, some items without
    colour (no splat) or with a temporal mask, some with their own fusion
    launch shape; the one graph launch equals the plain calls bitwise, on two
    replays."""
    rng = np.random.default_rng(2000 + seed)
    shapes = np.random.default_rng(3000 + seed)
    items = []
    for n in range(int(rng.integers(3, 13))):
        k = int(rng.integers(1, 9))
        c = scenes.small_ring(seed=100 * seed + n, width=int(rng.integers(1, 120)),
                              height=int(rng.integers(1, 80)), k=k, n_ring=max(8, k + 2),
                              bins=int(rng.integers(2, 200)), noise=0.01,
                              holes=float(rng.uniform(0.0, 0.2)))
        it = dict(src=c["src"], tgt=c["tgt"], depth=torch.from_numpy(c["depth"]).to(DEV),
                  splat=c["splat"],
                  tsdf=dict(c["tsdf"], conf_window=int(rng.choice([1, 3, 5, 7, 9, 11, 13, 15]))))
        if rng.uniform() < 0.8:
            it["rgb"] = torch.from_numpy(c["rgb"]).to(DEV)
        if rng.uniform() < 0.3:
            it["mask"] = torch.from_numpy(
                rng.uniform(0, 1.2, (c["tgt"].height, c["tgt"].width)).astype(np.float32)).to(DEV)
        if shapes.uniform() < 0.4:
            it["volume"] = (int(shapes.choice([0, 1, 3, 8, 16, 32, 64])),
                            int(shapes.choice([0, 4, 8, 16])), int(shapes.choice([0, 1, 2, 4, 8])),
                            int(shapes.choice([0, 64, 128, 65536])))
        items.append(it)
    refs = [_plain(it) for it in items]
    plan = gg.BatchPlan(items)
    for rep in range(2):
        plan.launch()
        torch.cuda.synchronize()
        _check(items, refs)
    plan.close()


def _full_size_items():
    """The 24 batching items at their full resolutions.  Each item's views
    are rendered at 1/8 scale (rendering all of them at full size takes
    minutes on the host) and upsampled by repetition: full-size depth and
    colour maps with the scene's structure, for the full-size cameras."""
    out = []
    for desc in scenes.config4_items():
        w, h = desc["width"], desc["height"]
        lo = scenes.config4_item(desc, scale=8)
        seq = scenes.RingSequence(4, desc["seed"], 16, 1.0, w, h, desc["k"],
                                  scenes.MovingSpheres(desc["seed"], 4),
                                  target_angle=desc["angle"])
        ys = np.minimum(np.arange(h) // 8, lo["depth"].shape[1] - 1)
        xs = np.minimum(np.arange(w) // 8, lo["depth"].shape[2] - 1)
        depth = np.ascontiguousarray(lo["depth"][:, ys][:, :, xs])
        rgb = np.ascontiguousarray(lo["rgb"][:, ys][:, :, xs])
        out.append(dict(src=seq.src, tgt=seq.tgt, depth=torch.from_numpy(depth).to(DEV),
                        rgb=torch.from_numpy(rgb).to(DEV), splat=lo["splat"], tsdf=lo["tsdf"]))
    return out


def test_batch_full_size_benchmark_tuning():
    """All 24 items at full size (2.6 G voxels) with the launch tuning the
    benchmark measures (512 threads per fusion workgroup, 4 persistent
    workgroups per CU): one graph launch equals the 24 plain call pairs."""
    import oracle
    from tests.test_parity_gpu import bits

    items = _full_size_items()
    refs = [_plain(it) for it in items]
    plan = gg.BatchPlan(items, 512, 4)
    plan.launch()
    torch.cuda.synchronize()
    _check(items, refs)
    # and the batched volume against the oracle on 1500 sampled pixel columns
    # of three items: 1280x720 K=8 D=128, 1920x1080 K=6 D=128, 1920x1080 K=8 D=64
    rng = np.random.default_rng(9)
    for i in (0, 3, 14):
        it = items[i]
        D = it["tsdf"]["num_bins"]
        npix = it["tgt"].width * it["tgt"].height
        pix = np.sort(rng.choice(npix, 1500, replace=False)).astype(np.int32)
        Fr, Wr = oracle.integrate(it["src"], it["depth"].cpu().numpy(), it["tgt"], it["tsdf"],
                                  pixels=pix)
        _, br = oracle.extract(Fr, Wr, it["tsdf"])
        assert np.array_equal(bits(it["F"].reshape(-1, D)[pix].cpu().numpy()), bits(Fr)), i
        assert np.array_equal(bits(it["W"].reshape(-1, D)[pix].cpu().numpy()), bits(Wr)), i
        assert np.array_equal(it["bin_out"].reshape(-1)[pix].cpu().numpy(), br), i
    plan.close()


def test_batch_against_the_oracle():
    """Four batching items rendered at half their resolution -- 640x360 K=8
    D=128, 960x540 K=6 D=128, 320x180 K=4 D=128 and 960x540 K=8 D=64 -- in
    one graph launch, compared with the oracle directly: the volume and the
    bins bitwise, the extracted depth within 1e-5, splat winners and winner
    depth bitwise, colour and opacity within 1e-5."""
    import oracle
    from tests.test_parity_gpu import bits, close

    descs = scenes.config4_items()
    cs = [scenes.config4_item(descs[i], scale=2) for i in (0, 3, 12, 14)]
    items = [dict(src=c["src"], tgt=c["tgt"], depth=torch.from_numpy(c["depth"]).to(DEV),
                  rgb=torch.from_numpy(c["rgb"]).to(DEV), splat=c["splat"], tsdf=c["tsdf"])
             for c in cs]
    assert (len(cs[0]["src"]), cs[0]["tsdf"]["num_bins"]) == (8, 128)
    plan = gg.BatchPlan(items)
    plan.launch()
    torch.cuda.synchronize()
    for n, (c, it) in enumerate(zip(cs, items)):
        D = c["tsdf"]["num_bins"]
        Fr, Wr = oracle.integrate(c["src"], c["depth"], c["tgt"], c["tsdf"])
        dr, br = oracle.extract(Fr, Wr, c["tsdf"])
        Fg = it["F"].reshape(-1, D).cpu().numpy()
        Wg = it["W"].reshape(-1, D).cpu().numpy()
        assert np.array_equal(bits(Fg), bits(Fr)), f"item {n}: F"
        assert np.array_equal(bits(Wg), bits(Wr)), f"item {n}: W"
        assert np.array_equal(it["bin_out"].reshape(-1).cpu().numpy(), br), f"item {n}: bins"
        close(it["depth_out"].reshape(-1).cpu().numpy(), dr, what=f"item {n}: depth")
        sr = oracle.splat(c["src"], c["depth"], c["rgb"], c["tgt"], c["splat"])
        so = it["splat_out"]
        assert np.array_equal(so["win_idx"].cpu().numpy(), sr["win_idx"]), f"item {n}: winners"
        assert np.array_equal(bits(so["depth"].cpu().numpy()), bits(sr["depth"])), \
            f"item {n}: winner depth"
        close(so["rgb"].cpu().numpy(), sr["rgb"], what=f"item {n}: rgb")
        close(so["alpha"].cpu().numpy(), sr["alpha"], what=f"item {n}: alpha")
    plan.close()
