"""Seeded synthetic multi-view RGB-D inputs for the geometry stage.

This module only *generates inputs*: camera rigs, analytic scenes ray-cast in
FP64, depth noise, holes and procedural textures.  It holds none of the
arithmetic of the method itself (no splatting, no TSDF, no relative
projection), so both the CPU oracle and the HIP path can consume what it makes
without sharing any of their computation.

Conventions (the camera model of the paper's Suppl. A.1 projection
``(x_k, y_k, z_k) = K_k (R_k p + t_k)``):

* world -> camera is ``x_c = R x_w + t`` with R row-major, camera axes
  x right, y down, z forward; world is right-handed with +y up;
* pixel (i, j) = (column, row) has its centre at (i + 0.5, j + 0.5);
* depth maps hold camera-frame z in metres; a hole is depth 0.

Configurations follow the five workload descriptions of the build contract
(tiny plain forward, video ring, differentiation, batching, large streaming).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence

import numpy as np

# ----------------------------------------------------------------------------
# cameras


@dataclasses.dataclass
class Camera:
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray  # (3, 3) float64, world -> camera rotation
    t: np.ndarray  # (3,) float64
    width: int
    height: int

    def center(self) -> np.ndarray:
        return -self.R.T @ self.t

    def packed(self) -> np.ndarray:
        """fx, fy, cx, cy, R(9, row-major), t(3) as float32 (the ABI layout)."""
        return np.concatenate([[self.fx, self.fy, self.cx, self.cy],
                               self.R.reshape(-1), self.t]).astype(np.float32)

    def quantized(self) -> "Camera":
        """The same camera with every parameter rounded to FP32 (what the
        kernels and the oracle actually see)."""
        p = self.packed().astype(np.float64)
        return Camera(p[0], p[1], p[2], p[3], p[4:13].reshape(3, 3).copy(),
                      p[13:16].copy(), self.width, self.height)


def look_at(eye, target, down=(0.0, -1.0, 0.0)):
    """World->camera (R, t) of a camera at ``eye`` looking at ``target``."""
    eye = np.asarray(eye, np.float64)
    z = np.asarray(target, np.float64) - eye
    z /= np.linalg.norm(z)
    x = np.cross(np.asarray(down, np.float64), z)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z])
    return R, -R @ eye


def make_camera(width, height, f, eye, target, cx=None, cy=None) -> Camera:
    R, t = look_at(eye, target)
    return Camera(float(f), float(f),
                  float(width) / 2 if cx is None else float(cx),
                  float(height) / 2 if cy is None else float(cy),
                  R, t, int(width), int(height))


def ring_rig(n, radius, width, height, f=None, height_m=0.2, look_y=-0.1):
    """``n`` cameras on a horizontal circle, each aimed at the circle's axis."""
    f = 0.9375 * width if f is None else f
    cams = []
    for i in range(n):
        th = 2.0 * math.pi * i / n
        eye = (radius * math.cos(th), height_m, radius * math.sin(th))
        cams.append(make_camera(width, height, f, eye, (0.0, look_y, 0.0)))
    return cams


def ring_target(angle, radius, width, height, f=None, height_m=0.2, look_y=-0.1):
    f = 0.9375 * width if f is None else f
    eye = (radius * math.cos(angle), height_m, radius * math.sin(angle))
    return make_camera(width, height, f, eye, (0.0, look_y, 0.0))


def closest_views(cams: Sequence[Camera], target: Camera, k: int) -> List[int]:
    """Indices of the ``k`` cameras whose centres are closest to the target's
    (the input-view selection of the paper's evaluation procedure); a camera
    that coincides with the target is excluded."""
    c = target.center()
    d = [float(np.linalg.norm(cam.center() - c)) for cam in cams]
    order = [i for i in np.argsort(d, kind="stable") if d[i] > 1e-9]
    return sorted(int(i) for i in order[:k])


def rays(cam: Camera):
    """Per-pixel world ray origin (the centre) and direction with unit
    camera-z, so that the hit parameter equals camera-frame depth."""
    j, i = np.meshgrid(np.arange(cam.height, dtype=np.float64),
                       np.arange(cam.width, dtype=np.float64), indexing="ij")
    dc = np.stack([(i + 0.5 - cam.cx) / cam.fx, (j + 0.5 - cam.cy) / cam.fy,
                   np.ones_like(i)], axis=-1)
    dw = dc @ cam.R  # == (R^T dc^T)^T
    return cam.center(), dw


# ----------------------------------------------------------------------------
# procedural texture (seeded value noise)

_M1 = np.uint64(0x9E3779B97F4A7C15)
_M2 = np.uint64(0xBF58476D1CE4E5B9)
_M3 = np.uint64(0x94D049BB133111EB)


def _hash2(ix, iy, seed):
    with np.errstate(over="ignore"):
        h = (ix.astype(np.int64).astype(np.uint64) * _M1) ^ \
            (iy.astype(np.int64).astype(np.uint64) * _M2) ^ (np.uint64(seed) * _M3)
        h ^= h >> np.uint64(31)
        h *= _M2
        h ^= h >> np.uint64(29)
        h *= _M3
        h ^= h >> np.uint64(32)
    return (h >> np.uint64(40)).astype(np.float64) / float(1 << 24)


def value_noise(s, t, seed, cells=12.0):
    s = s * cells
    t = t * cells
    i0 = np.floor(s)
    j0 = np.floor(t)
    fs = s - i0
    ft = t - j0
    fs = fs * fs * (3 - 2 * fs)
    ft = ft * ft * (3 - 2 * ft)
    v00 = _hash2(i0, j0, seed)
    v10 = _hash2(i0 + 1, j0, seed)
    v01 = _hash2(i0, j0 + 1, seed)
    v11 = _hash2(i0 + 1, j0 + 1, seed)
    return (v00 * (1 - fs) + v10 * fs) * (1 - ft) + (v01 * (1 - fs) + v11 * fs) * ft


def texture_rgb(s, t, seed, base):
    n1 = value_noise(s, t, seed * 7)
    n2 = value_noise(s, t, seed * 7 + 3, 40.0)
    n3 = value_noise(s, t, seed * 7 + 5, 5.0)
    out = np.empty(s.shape + (3,), np.float64)
    mix = (0.5 * n1 + 0.3 * n2, 0.5 * n1 + 0.3 * n3, 0.3 * n2 + 0.5 * n3)
    for c in range(3):
        out[..., c] = base[c] * (0.25 + 0.75 * (mix[c] + 0.2))
    return np.clip(out, 0.0, 1.0)


# ----------------------------------------------------------------------------
# analytic primitives: each returns (hit parameter, s, t) with inf on a miss


class Primitive:
    seed = 0
    base = (0.8, 0.8, 0.8)

    def hit(self, o, d):  # pragma: no cover - interface
        raise NotImplementedError


class Sphere(Primitive):
    def __init__(self, center, radius, seed, base):
        self.c = np.asarray(center, np.float64)
        self.r = float(radius)
        self.seed, self.base = seed, base

    def window(self, cam):
        """Conservative pixel window (y0, y1, x0, x1) of the sphere's image,
        or None for the whole image."""
        corners = np.array([[sx, sy, sz] for sx in (-1, 1) for sy in (-1, 1)
                            for sz in (-1, 1)], np.float64) * self.r + self.c
        pc = corners @ cam.R.T + cam.t
        if (pc[:, 2] <= 1e-3).any():
            return None
        u = cam.fx * pc[:, 0] / pc[:, 2] + cam.cx
        v = cam.fy * pc[:, 1] / pc[:, 2] + cam.cy
        x0 = max(int(np.floor(u.min())) - 2, 0)
        x1 = min(int(np.ceil(u.max())) + 2, cam.width)
        y0 = max(int(np.floor(v.min())) - 2, 0)
        y1 = min(int(np.ceil(v.max())) + 2, cam.height)
        return (y0, max(y0, y1), x0, max(x0, x1))

    def hit(self, o, d):
        oc = o - self.c
        a = np.einsum("...i,...i->...", d, d)
        b = 2.0 * np.einsum("...i,...i->...", d, oc)
        cc = float(oc @ oc) - self.r * self.r
        disc = b * b - 4 * a * cc
        lam = np.full(a.shape, np.inf)
        ok = disc >= 0
        sq = np.sqrt(np.where(ok, disc, 0.0))
        l0 = (-b - sq) / (2 * a)
        l1 = (-b + sq) / (2 * a)
        l = np.where(l0 > 1e-6, l0, l1)
        ok &= l > 1e-6
        lam[ok] = l[ok]
        p = o + lam[..., None] * d - self.c
        with np.errstate(invalid="ignore"):
            s = np.arctan2(p[..., 2], p[..., 0]) / (2 * math.pi) * 3.0
            t = np.arccos(np.clip(p[..., 1] / self.r, -1, 1)) / math.pi * 1.5
        return lam, s, t


class Quad(Primitive):
    """A textured rectangle: centre, two half-extent edge vectors."""

    def __init__(self, center, u, v, seed, base):
        self.c = np.asarray(center, np.float64)
        self.u = np.asarray(u, np.float64)
        self.v = np.asarray(v, np.float64)
        self.n = np.cross(self.u, self.v)
        self.n /= np.linalg.norm(self.n)
        self.seed, self.base = seed, base

    def hit(self, o, d):
        den = d @ self.n
        with np.errstate(divide="ignore", invalid="ignore"):
            lam = ((self.c - o) @ self.n) / den
        p = o + lam[..., None] * d - self.c
        s = (p @ self.u) / (self.u @ self.u)
        t = (p @ self.v) / (self.v @ self.v)
        ok = (np.abs(den) > 1e-12) & (lam > 1e-6) & (np.abs(s) <= 1) & (np.abs(t) <= 1)
        lam = np.where(ok, lam, np.inf)
        return lam, s * np.linalg.norm(self.u), t * np.linalg.norm(self.v)


class Floor(Primitive):
    def __init__(self, y, seed, base):
        self.y = float(y)
        self.seed, self.base = seed, base

    def hit(self, o, d):
        with np.errstate(divide="ignore", invalid="ignore"):
            lam = (self.y - o[1]) / d[..., 1]
        ok = np.isfinite(lam) & (lam > 1e-6)
        lam = np.where(ok, lam, np.inf)
        p = o + np.where(ok, lam, 0.0)[..., None] * d
        return lam, p[..., 0], p[..., 2]


class Backdrop(Primitive):
    """Inside of a vertical cylinder around the origin."""

    def __init__(self, radius, seed, base):
        self.r = float(radius)
        self.seed, self.base = seed, base

    def hit(self, o, d):
        a = d[..., 0] ** 2 + d[..., 2] ** 2
        b = 2 * (d[..., 0] * o[0] + d[..., 2] * o[2])
        cc = o[0] ** 2 + o[2] ** 2 - self.r ** 2
        with np.errstate(invalid="ignore", divide="ignore"):
            lam = (-b + np.sqrt(b * b - 4 * a * cc)) / (2 * a)
        ok = np.isfinite(lam) & (lam > 1e-6)
        lam = np.where(ok, lam, np.inf)
        p = o + np.where(ok, lam, 0.0)[..., None] * d
        s = np.arctan2(p[..., 2], p[..., 0]) * self.r
        return lam, s, p[..., 1]


class Box(Primitive):
    """Oriented box: centre, rotation (box->world columns), half extents."""

    def __init__(self, center, rot, half, seed, base):
        self.c = np.asarray(center, np.float64)
        self.Rb = np.asarray(rot, np.float64)
        self.h = np.asarray(half, np.float64)
        self.seed, self.base = seed, base

    def hit(self, o, d):
        ol = (o - self.c) @ self.Rb
        dl = d @ self.Rb
        with np.errstate(divide="ignore", invalid="ignore"):
            t1 = (-self.h - ol) / dl
            t2 = (self.h - ol) / dl
        tmin = np.nanmax(np.minimum(t1, t2), axis=-1)
        tmax = np.nanmin(np.maximum(t1, t2), axis=-1)
        ok = (tmax >= tmin) & (tmin > 1e-6)
        lam = np.where(ok, tmin, np.inf)
        p = ol + np.where(ok, lam, 0.0)[..., None] * dl
        ax = np.argmax(np.abs(p) / self.h, axis=-1)
        s = np.where(ax == 0, p[..., 1], p[..., 0])
        t = np.where(ax == 2, p[..., 1], p[..., 2])
        return lam, s, t


def rot_y(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])


def render(cam: Camera, prims: Sequence[Primitive], static_cache=None):
    """FP64 ray cast: z-depth (inf on a miss) and linear RGB in [0, 1].

    ``static_cache`` (a dict) memoises the hit parameters of primitives
    flagged ``static`` for this camera, so a sequence re-renders only what
    moves."""
    o, d = rays(cam) if static_cache is None or "rays" not in static_cache \
        else static_cache["rays"]
    if static_cache is not None:
        static_cache["rays"] = (o, d)
    shape = d.shape[:-1]
    depth = np.full(shape, np.inf)
    owner = np.full(shape, -1, np.int32)
    st = []
    for n, p in enumerate(prims):
        key = getattr(p, "static_key", None)
        win = p.window(cam) if hasattr(p, "window") else None
        if static_cache is not None and key is not None and key in static_cache:
            lam, s, t = static_cache[key]
        elif win is not None:
            y0, y1, x0, x1 = win
            lam = np.full(shape, np.inf)
            s = np.zeros(shape)
            t = np.zeros(shape)
            if y1 > y0 and x1 > x0:
                lw, sw, tw = p.hit(o, d[y0:y1, x0:x1])
                lam[y0:y1, x0:x1] = lw
                s[y0:y1, x0:x1] = sw
                t[y0:y1, x0:x1] = tw
        else:
            lam, s, t = p.hit(o, d)
            if static_cache is not None and key is not None:
                static_cache[key] = (lam, s, t)
        st.append((s, t))
        closer = lam < depth
        depth = np.where(closer, lam, depth)
        owner = np.where(closer, n, owner)
    rgb = np.zeros(shape + (3,))
    for n, p in enumerate(prims):
        m = owner == n
        if m.any():
            key = getattr(p, "static_key", None)
            if static_cache is not None and key is not None:
                if key + ":rgb" not in static_cache:
                    s, t = st[n]
                    fin = np.isfinite(static_cache[key][0])
                    full = np.zeros(shape + (3,))
                    full[fin] = texture_rgb(s[fin], t[fin], p.seed, p.base)
                    static_cache[key + ":rgb"] = full
                rgb[m] = static_cache[key + ":rgb"][m]
            else:
                s, t = st[n]
                rgb[m] = texture_rgb(s[m], t[m], p.seed, p.base)
    return depth, rgb


def to_inputs(depth, rgb, rng, noise=0.0, holes=0.0):
    """Round a rendered view to the stage's input format: FP32 depth with
    multiplicative Gaussian noise and random holes (depth 0), uint8 RGB."""
    dep = depth.copy()
    if noise > 0:
        dep = dep * (1.0 + noise * rng.standard_normal(dep.shape))
    dep = np.where(np.isfinite(dep), dep, 0.0)
    if holes > 0:
        dep[rng.random(dep.shape) < holes] = 0.0
    col = np.clip(np.round(rgb * 255.0), 0, 255).astype(np.uint8)
    return dep.astype(np.float32), col


# ----------------------------------------------------------------------------
# parameter sets


def splat_params(**kw):
    p = dict(sigma_px=0.5, band_rel=0.01, z_min=0.05, r_max_px=8.0)
    p.update(kw)
    return p


def tsdf_params(**kw):
    p = dict(z_near=0.5, z_far=5.0, num_bins=64, trunc=3.0, trunc_in_bins=1,
             conf_tau=0.02, conf_scale=0.001, conf_window=7, decay=0.9, weight_cap=32.0)
    p.update(kw)
    return p


# ----------------------------------------------------------------------------
# the workloads


def _cfg1_scene(seed):
    return [
        Quad((0.0, 0.0, 4.0), (2.5, 0, 0), (0, 1.8, 0), seed + 1, (0.9, 0.8, 0.6)),        # back wall
        Quad((-0.75, 0.05, 2.6), 0.7 * np.array([math.cos(0.6), 0, -math.sin(0.6)]),
             (0, 0.65, 0), seed + 2, (0.5, 0.8, 0.9)),                                    # slanted
        Floor(-0.8, seed + 3, (0.7, 0.7, 0.5)),                                           # floor
        Sphere((0.35, 0.0, 2.0), 0.5, seed + 4, (0.9, 0.4, 0.3)),
    ]


def parallel_rig(xs, width, height, f):
    return [make_camera(width, height, f, (x, 0.0, 0.0), (x, 0.0, 1.0)) for x in xs]


def _quantize_all(cams):
    return [c.quantized() for c in cams]


def make_frame(src, tgt, prims, rng, noise, holes, caches=None):
    depth, rgb = [], []
    for v, cam in enumerate(src):
        d, c = render(cam, prims, None if caches is None else caches[v])
        d, c = to_inputs(d, c, rng, noise, holes)
        depth.append(d)
        rgb.append(c)
    return np.stack(depth), np.stack(rgb)


def config1(seed=0):
    """K=2 parallel 320x240 views (f=300, principal point at the centre),
    baseline 0.1 m, target midway; 3 planes + sphere; 1% noise; D=64
    inverse-depth bins over 0.5-5 m, truncation 3 bins."""
    src = _quantize_all(parallel_rig([-0.05, 0.05], 320, 240, 300.0))
    tgt = parallel_rig([0.0], 320, 240, 300.0)[0].quantized()
    rng = np.random.default_rng([1, seed])
    depth, rgb = make_frame(src, tgt, _cfg1_scene(seed), rng, 0.01, 0.0)
    return dict(name="plain-tiny", src=src, tgt=tgt, depth=depth, rgb=rgb,
                splat=splat_params(), tsdf=tsdf_params(num_bins=64, trunc=3.0))


def config3(seed=0):
    """The tiny scene at 640x360, f=600, K=4 parallel views at x=+-0.05,
    +-0.15 m, target at x=0, D=96."""
    src = _quantize_all(parallel_rig([-0.15, -0.05, 0.05, 0.15], 640, 360, 600.0))
    tgt = parallel_rig([0.0], 640, 360, 600.0)[0].quantized()
    rng = np.random.default_rng([3, seed])
    depth, rgb = make_frame(src, tgt, _cfg1_scene(seed), rng, 0.01, 0.0)
    return dict(name="differentiation", src=src, tgt=tgt, depth=depth, rgb=rgb,
                splat=splat_params(), tsdf=tsdf_params(num_bins=96, trunc=3.0))


class MovingSpheres:
    """Spheres moving at a fixed speed inside a disc of radius ``r_max``,
    reflecting at its edge, over a textured floor and a cylinder backdrop."""

    def __init__(self, seed, n, speed=0.02, r_disc=0.6, floor_y=-0.5, backdrop=3.0,
                 boxes=0):
        rng = np.random.default_rng([99, seed])
        self.floor_y = floor_y
        self.backdrop = backdrop
        self.speed = speed
        self.r_disc = r_disc
        self.radii = rng.uniform(0.1, 0.25, n)
        ang = rng.uniform(0, 2 * math.pi, n)
        rad = rng.uniform(0, r_disc * 0.8, n)
        self.pos0 = np.stack([rad * np.cos(ang), rad * np.sin(ang)], -1)
        dang = rng.uniform(0, 2 * math.pi, n)
        self.vel = speed * np.stack([np.cos(dang), np.sin(dang)], -1)
        self.height = floor_y + self.radii + rng.uniform(0, 0.3, n)
        self.cols = rng.uniform(0.3, 1.0, (n, 3))
        self.seed = seed
        self.nbox = boxes
        self.box_pos = rng.uniform(-0.4, 0.4, (boxes, 2))
        self.box_half = rng.uniform(0.08, 0.18, (boxes, 3))

    def positions(self, frame):
        p = self.pos0.copy()
        v = self.vel.copy()
        for _ in range(frame):  # reflecting walk, exact and seeded
            p = p + v
            r = np.linalg.norm(p, axis=-1)
            out = r > self.r_disc
            if out.any():
                nrm = p[out] / r[out, None]
                v[out] = v[out] - 2 * (v[out] * nrm).sum(-1, keepdims=True) * nrm
                p[out] = nrm * self.r_disc
        return p

    def prims(self, frame):
        pr = [Floor(self.floor_y, self.seed * 31 + 1, (0.75, 0.7, 0.55)),
              Backdrop(self.backdrop, self.seed * 31 + 2, (0.6, 0.7, 0.85))]
        pr[0].static_key = "floor"
        pr[1].static_key = "backdrop"
        for b in range(self.nbox):
            half = self.box_half[b]
            c = (self.box_pos[b, 0], self.floor_y + half[1], self.box_pos[b, 1])
            pr.append(Box(c, rot_y(0.05 * frame + b), half, self.seed * 31 + 10 + b,
                          (0.9, 0.6, 0.4)))
        p = self.positions(frame)
        for s in range(len(self.radii)):
            pr.append(Sphere((p[s, 0], self.height[s], p[s, 1]), self.radii[s],
                             self.seed * 31 + 100 + s, tuple(self.cols[s])))
        return pr


def _render_job(args):
    cam, prims = args
    return render(cam, prims, None)


class RingSequence:
    """A K-of-N ring rig looking at a dynamic scene; frames generated on
    demand and seeded by (config, seed, frame)."""

    def __init__(self, cfg_id, seed, n_ring, radius, width, height, k, scene,
                 noise=0.01, holes=0.02, target_angle=None):
        self.ring = ring_rig(n_ring, radius, width, height)
        ang = (2 * math.pi * 0.5 / n_ring) if target_angle is None else target_angle
        self.tgt = ring_target(ang, radius, width, height).quantized()
        self.views = closest_views(self.ring, self.tgt, k)
        self.src = _quantize_all([self.ring[i] for i in self.views])
        self.scene = scene
        self.cfg_id, self.seed, self.noise, self.holes = cfg_id, seed, noise, holes
        self.caches = [dict() for _ in self.src]

    def frame(self, t, procs=1):
        """Depth and colour of every view at frame t.  With procs > 1 the
        views are ray-cast in a process pool and the seeded noise and holes
        are then applied in view order: the same frame as procs = 1."""
        rng = np.random.default_rng([self.cfg_id, self.seed, t])
        if procs <= 1:
            return make_frame(self.src, self.tgt, self.scene.prims(t), rng, self.noise,
                              self.holes, self.caches)
        import multiprocessing as mp
        prims = self.scene.prims(t)
        with mp.get_context("fork").Pool(min(procs, len(self.src))) as pool:
            views = pool.map(_render_job, [(cam, prims) for cam in self.src])
        depth, rgb = [], []
        for d, c in views:
            d, c = to_inputs(d, c, rng, self.noise, self.holes)
            depth.append(d)
            rgb.append(c)
        return np.stack(depth), np.stack(rgb)


def _coarse_job(args):
    cam, prims, f, seeds, noise, holes = args
    lo = Camera(cam.fx / f, cam.fy / f, cam.cx / f, cam.cy / f, cam.R, cam.t,
                -(-cam.width // f), -(-cam.height // f))
    d, c = render(lo, prims, None)
    ys = np.arange(cam.height) // f
    xs = np.arange(cam.width) // f
    return to_inputs(d[ys][:, xs], c[ys][:, xs], np.random.default_rng(seeds), noise, holes)


def coarse_frame(seq, t, factor=2, procs=1):
    """Frame t of ``seq`` ray-cast at 1/factor resolution (the same cameras
    with scaled intrinsics) and repeated to the full maps, then rounded to
    inputs with the sequence's noise and holes per full-resolution pixel
    (seeded per view): full-size depth and colour with the scene's structure
    and motion, cheaper to generate on the host (for long sequences at large
    sizes)."""
    prims = seq.scene.prims(t)
    jobs = [(cam, prims, factor, [seq.cfg_id, seq.seed, t, factor, v], seq.noise, seq.holes)
            for v, cam in enumerate(seq.src)]
    if procs <= 1:
        views = [_coarse_job(j) for j in jobs]
    else:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(min(procs, len(jobs))) as pool:
            views = pool.map(_coarse_job, jobs)
    # C order whatever the rendering's strides (one process returns views of them)
    return (np.ascontiguousarray(np.stack([d for d, _ in views])),
            np.ascontiguousarray(np.stack([c for _, c in views])))


def config2(seed=0):
    """Video: K=4 of a 16-camera ring (radius 1 m, aimed inward) at
    1280x720, target between two ring cameras; 5 spheres moving
    0.02 m/frame over a textured floor; 1% noise, 2% holes; D=128,
    truncation 4 bins, decay 0.9, weight cap 32; 30 frames."""
    seq = RingSequence(2, seed, 16, 1.0, 1280, 720, 4, MovingSpheres(seed, 5))
    return dict(name="video", seq=seq, src=seq.src, tgt=seq.tgt, frames=30,
                splat=splat_params(), tsdf=tsdf_params(num_bins=128, trunc=4.0))


def paper_shape(seed=0):
    """The video workload's scene and rig at the paper's DyNeRF test shape,
    1352x1014, K=4 of the 16-camera ring, D=128 (a context run beside the
    metric's 1280x720)."""
    seq = RingSequence(6, seed, 16, 1.0, 1352, 1014, 4, MovingSpheres(seed, 5))
    return dict(name="paper shape", seq=seq, src=seq.src, tgt=seq.tgt,
                splat=splat_params(), tsdf=tsdf_params(num_bins=128, trunc=4.0))


def small_video(seed=0, width=96, height=64, k=3, bins=32):
    """A small version of the video workload (ring rig, moving spheres) for
    tests of the temporal path."""
    seq = RingSequence(7, seed, 16, 1.0, width, height, k, MovingSpheres(seed, 5))
    return dict(name="small video", seq=seq, src=seq.src, tgt=seq.tgt,
                splat=splat_params(), tsdf=tsdf_params(num_bins=bins, trunc=4.0))


def config5(seed=0):
    """Large streaming: K=8 of a 16-camera ring (radius 1.5 m), 1920x1080,
    D=256, truncation 4 bins, 20 moving spheres + 2 rotating boxes."""
    seq = RingSequence(5, seed, 16, 1.5, 1920, 1080, 8,
                       MovingSpheres(seed, 20, r_disc=0.9, boxes=2))
    return dict(name="streaming", seq=seq, src=seq.src, tgt=seq.tgt, frames=300,
                splat=splat_params(), tsdf=tsdf_params(num_bins=256, trunc=4.0))


BATCH_RES = [(640, 360), (960, 540), (1280, 720), (1920, 1080)]
BATCH_K = [2, 3, 4, 6, 8]
BATCH_D = [64, 128]


def config4_items(seed=0, n_items=24):
    """Batching: descriptors of ``n_items`` target views of uneven
    resolution, view count and bin count (no pixels rendered yet)."""
    rng = np.random.default_rng([4, seed])
    items = []
    for it in range(n_items):
        w, h = BATCH_RES[rng.integers(len(BATCH_RES))]
        items.append(dict(width=w, height=h, k=int(BATCH_K[rng.integers(len(BATCH_K))]),
                          d=int(BATCH_D[rng.integers(len(BATCH_D))]),
                          angle=float(rng.uniform(0, 2 * math.pi)), seed=int(seed * 1000 + it)))
    return items


def config4_item(desc, scale=1):
    """Render one batching item (optionally downscaled by ``scale``)."""
    w, h = desc["width"] // scale, desc["height"] // scale
    scene = MovingSpheres(desc["seed"], 4)
    seq = RingSequence(4, desc["seed"], 16, 1.0, w, h, desc["k"], scene,
                       target_angle=desc["angle"])
    depth, rgb = seq.frame(0)
    return dict(name="batch-item", src=seq.src, tgt=seq.tgt, depth=depth, rgb=rgb,
                splat=splat_params(), tsdf=tsdf_params(num_bins=desc["d"], trunc=4.0))


def small_ring(seed=0, width=8, height=8, k=2, n_ring=8, radius=1.0, bins=24,
               f=None, noise=0.0, holes=0.0, frame=0):
    """A tiny rotated-camera case (default 8x8) for brute-force checks."""
    seq = RingSequence(7, seed, n_ring, radius, width, height, k, MovingSpheres(seed, 3),
                       noise=noise, holes=holes, target_angle=2 * math.pi * 0.37 / n_ring)
    if f is not None:
        for c in seq.src + [seq.tgt]:
            c.fx = c.fy = float(np.float32(f))
    depth, rgb = seq.frame(frame)
    return dict(name="small-ring", src=seq.src, tgt=seq.tgt, depth=depth, rgb=rgb,
                splat=splat_params(), tsdf=tsdf_params(num_bins=bins, trunc=3.0))
