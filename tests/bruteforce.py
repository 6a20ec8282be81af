"""Direct FP64 brute force of the per-ray TSDF and of the z-buffered splat.

Used only to pin the oracle.  It is written independently of ``oracle.c``: it
back-projects and projects through world space literally
(``x_c = R p + t``, ``(x, y) = K x_c / z``), never forms the relative
projection, computes the window statistic with array shifts, and runs in FP64
without the FP32 operation order.  Where its FP64 decisions sit within a small
margin of a boundary (a pixel edge, the occlusion cut, the coverage radius,
equal depths) it reports the sample as ambiguous so that the comparison skips
it instead of depending on rounding.
"""
import numpy as np


def kmat(cam):
    return np.array([[cam.fx, 0, cam.cx], [0, cam.fy, cam.cy], [0, 0, 1.0]])


def backproject(cam, i, j, z):
    """World point of pixel centre (i, j) at camera depth z."""
    xc = np.stack([(i + 0.5 - cam.cx) / cam.fx * z, (j + 0.5 - cam.cy) / cam.fy * z,
                   np.broadcast_to(z, np.broadcast(i, j, z).shape)], -1)
    return (xc - cam.t) @ cam.R  # R^T (xc - t)


def project(cam, P):
    Xc = P @ cam.R.T + cam.t
    return Xc @ kmat(cam).T  # (x_k, y_k, z_k) = K (R p + t)


def valid(d):
    return np.isfinite(d) & (d > 0)


def confidence(depth, tau, scale, w):
    """omega = min(scale (nu / w^2)^(-1/2), 1), nu over the w x w window of
    min(dD^2, tau^2); out-of-image neighbours skipped, holes count tau^2."""
    depth = np.asarray(depth, np.float64)
    H, W = depth.shape
    r = (w - 1) // 2
    ok = valid(depth)
    pad = np.full((H + 2 * r, W + 2 * r), np.nan)
    pad[r:r + H, r:r + W] = np.where(ok, depth, -1.0)
    nu = np.zeros((H, W))
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            nb = pad[r + dy:r + dy + H, r + dx:r + dx + W]
            inside = ~np.isnan(nb)
            term = np.where(nb > 0, np.minimum((depth - np.where(nb > 0, nb, 0)) ** 2, tau * tau),
                            tau * tau)
            nu += np.where(inside, term, 0.0)
    with np.errstate(divide="ignore"):
        om = np.where(nu == 0, 1.0, np.minimum(scale / np.sqrt(nu / (w * w)), 1.0))
    return np.where(ok, om, 0.0)


def bins(prm):
    D = prm["num_bins"]
    un, uf = 1.0 / prm["z_near"], 1.0 / prm["z_far"]
    u = un - np.arange(D) * (un - uf) / (D - 1)
    z = 1.0 / u
    tau = prm["trunc"] * (un - uf) / (D - 1) * z * z if prm["trunc_in_bins"] else \
        np.full(D, float(prm["trunc"]))
    return z, tau


def tsdf(src, depth, tgt, prm, margin=1e-4):
    """Per-ray brute force.  Returns F, W (Ht*Wt, D) and a boolean mask of
    voxels whose decisions are within ``margin`` of a boundary."""
    K = len(src)
    z, tau = bins(prm)
    D = len(z)
    Ht, Wt = tgt.height, tgt.width
    jj, ii = np.meshgrid(np.arange(Ht, dtype=np.float64), np.arange(Wt, dtype=np.float64),
                         indexing="ij")
    conf = [confidence(depth[k], prm["conf_tau"], prm["conf_scale"], prm["conf_window"])
            for k in range(K)]
    F = np.zeros((Ht * Wt, D))
    Wv = np.zeros((Ht * Wt, D))
    amb = np.zeros((Ht * Wt, D), bool)
    for d in range(D):
        P = backproject(tgt, ii, jj, np.full_like(ii, z[d])).reshape(-1, 3)
        S = np.zeros(len(P))
        Wo = np.zeros(len(P))
        for k in range(K):
            X = project(src[k], P)
            zk = X[:, 2]
            front = zk > 0
            with np.errstate(divide="ignore", invalid="ignore"):
                u = X[:, 0] / zk
                v = X[:, 1] / zk
            Hs, Ws = depth[k].shape
            near_edge = front & ((np.abs(u - np.round(u)) < margin) | (np.abs(v - np.round(v)) < margin))
            inb = front & (u >= 0) & (u < Ws) & (v >= 0) & (v < Hs)
            ui = np.where(inb, np.floor(u), 0).astype(int)
            vi = np.where(inb, np.floor(v), 0).astype(int)
            Dk = np.asarray(depth[k], np.float64)[vi, ui]
            ok = inb & valid(Dk)
            s = Dk - zk
            near_cut = ok & (np.abs(s + tau[d]) < margin * 1e-2 * (1 + np.abs(s)))
            use = ok & (s >= -tau[d])
            c = np.minimum(s, tau[d])
            w = conf[k][vi, ui]
            S += np.where(use, w * c, 0.0)
            Wo += np.where(use, w, 0.0)
            amb[:, d] |= near_edge | near_cut
        F[:, d] = np.where(Wo > 0, S / np.where(Wo > 0, Wo, 1), 0.0)
        Wv[:, d] = Wo
    return F, Wv, amb


def extract(F, W, prm):
    z, _ = bins(prm)
    n, D = F.shape
    depth = np.zeros(n)
    b = np.full(n, -1)
    for p in range(n):
        for d in range(D - 1):
            if W[p, d] > 0 and W[p, d + 1] > 0 and F[p, d] > 0 and F[p, d + 1] <= 0:
                depth[p] = z[d] + (z[d + 1] - z[d]) * F[p, d] / (F[p, d] - F[p, d + 1])
                b[p] = d
                break
    return depth, b


def zbuffer(src, depth, rgb, tgt, sp, margin=1e-6, mask=None):
    """O(N^2) splat: every source pixel against every target pixel.
    Returns win (K, Ht, Wt), depth, rgb (K,3,Ht,Wt), alpha, ambiguous mask;
    with ``mask`` (K, Hs, Ws) also the band blend of the mask (K, Ht, Wt)."""
    K = len(src)
    Ht, Wt = tgt.height, tgt.width
    bj, bi = np.meshgrid(np.arange(Ht), np.arange(Wt), indexing="ij")
    cent = np.stack([bi.ravel() + 0.5, bj.ravel() + 0.5], -1)  # (Nt, 2)
    win = np.full((K, Ht * Wt), -1)
    zw = np.zeros((K, Ht * Wt))
    col = np.zeros((K, 3, Ht * Wt))
    alpha = np.zeros((K, Ht * Wt))
    msk = np.zeros((K, Ht * Wt))
    amb = np.zeros((K, Ht * Wt), bool)
    for k in range(K):
        Hs, Ws = depth[k].shape
        sj, si = np.meshgrid(np.arange(Hs), np.arange(Ws), indexing="ij")
        Dq = np.asarray(depth[k], np.float64).ravel()
        q = np.arange(Hs * Ws)
        ok = valid(Dq)
        P = backproject(src[k], si.ravel().astype(float), sj.ravel().astype(float),
                        np.where(ok, Dq, 1.0))
        X = project(tgt, P)
        zt = X[:, 2]
        ok &= zt > sp["z_min"]
        x = X[:, 0] / np.where(ok, zt, 1)
        y = X[:, 1] / np.where(ok, zt, 1)
        sig = sp["sigma_px"] * tgt.fx / src[k].fx * Dq / np.where(ok, zt, 1)
        R2 = np.minimum(2 * sig * sig, sp["r_max_px"] ** 2)
        d2 = (cent[:, None, 0] - x[None]) ** 2 + (cent[:, None, 1] - y[None]) ** 2  # (Nt, Ns)
        cov = ok[None] & (d2 <= R2[None])
        amb[k] |= (ok[None] & (np.abs(d2 - R2[None]) < margin * 1e2 * R2[None])).any(1)
        big = np.where(cov, zt[None], np.inf)
        best = np.argmin(np.where(cov, zt[None] * (1 + 0 * q[None]), np.inf), axis=1)
        has = cov.any(1)
        zmin = big.min(1)
        # ties within margin are ambiguous in FP64 vs FP32
        close = cov & (np.abs(big - zmin[:, None]) <= margin * np.abs(zmin[:, None])) & \
            (big != zmin[:, None])
        amb[k] |= close.any(1)
        # exact ties pick the smaller source index
        tie = cov & (big == zmin[:, None])
        first = np.argmax(tie, axis=1)
        win[k] = np.where(has, first, -1)
        zw[k] = np.where(has, zmin, 0)
        thr = zmin * (1 + sp["band_rel"])
        band = cov & (zt[None] <= thr[:, None])
        amb[k] |= (cov & (np.abs(zt[None] - thr[:, None]) < margin * 10 * thr[:, None])).any(1)
        G = np.where(band, np.exp(-0.5 * d2 / (sig * sig)[None]), 0.0)
        n = G.sum(1)
        c = np.asarray(rgb[k], np.float64).reshape(-1, 3) / 255.0
        for ch in range(3):
            col[k, ch] = np.where(has, (G * c[None, :, ch]).sum(1) / np.where(has, n, 1), 0)
        alpha[k] = np.where(has, 1 - np.prod(np.where(band, 1 - G, 1.0), axis=1), 0)
        if mask is not None:
            m = np.asarray(mask[k], np.float64).ravel()
            msk[k] = np.where(has, (G * m[None]).sum(1) / np.where(has, n, 1), 0)
        del best
    sh = (K, Ht, Wt)
    out = (win.reshape(sh), zw.reshape(sh), col.reshape(K, 3, Ht, Wt), alpha.reshape(sh),
           amb.reshape(sh))
    return out if mask is None else out + (msk.reshape(sh),)


def difference_mask(rgb, rgb_prev, factor, beta, lam):
    """Eq. 1 mask of one (H, W, 3) frame pair in FP64 with array operations:
    box means by reduceat, the 3x3 max-pool as a maximum of nine shifted
    copies (-inf padding), bilinear upsampling by index arrays."""
    a = np.asarray(rgb, np.float64) / 255.0
    b = np.asarray(rgb_prev, np.float64) / 255.0
    H, W = a.shape[:2]
    rs, cs = np.arange(0, H, factor), np.arange(0, W, factor)
    cnt = np.add.reduceat(np.add.reduceat(np.ones((H, W)), rs, 0), cs, 1)
    ma = np.add.reduceat(np.add.reduceat(a, rs, 0), cs, 1) / cnt[..., None]
    mb = np.add.reduceat(np.add.reduceat(b, rs, 0), cs, 1) / cnt[..., None]
    low = np.minimum(np.abs(ma - mb).mean(-1) / lam + beta, 1.0)
    Hq, Wq = low.shape
    pad = np.pad(low, 1, constant_values=-np.inf)
    pool = np.max([pad[1 + dy:1 + dy + Hq, 1 + dx:1 + dx + Wq]
                   for dy in (-1, 0, 1) for dx in (-1, 0, 1)], axis=0)
    x = np.clip((np.arange(W) + 0.5) / factor - 0.5, 0, Wq - 1)
    y = np.clip((np.arange(H) + 0.5) / factor - 0.5, 0, Hq - 1)
    x0, y0 = np.floor(x).astype(int), np.floor(y).astype(int)
    x1, y1 = np.minimum(x0 + 1, Wq - 1), np.minimum(y0 + 1, Hq - 1)
    fx, fy = (x - x0)[None, :], (y - y0)[:, None]
    top = pool[y0][:, x0] * (1 - fx) + pool[y0][:, x1] * fx
    bot = pool[y1][:, x0] * (1 - fx) + pool[y1][:, x1] * fx
    return top * (1 - fy) + bot * fy
