"""The relative projection (H, c) of camera pairs, from the oracle and from the
library, against its exact value: H = K_b R_b R_a^T K_a^-1 and
c = K_b (t_b - R_b R_a^T t_a), in rational arithmetic from the FP32 camera
parameters, rounded to the nearest FP32 with ties to even.  An entry below
2^-50 of its monomials' summed magnitudes is 0 on both sides (exactly zero
here).  Rigs aligned with the axes make exact ties: the first view of the
random sweep's seed 1348 has one in H[1][0], which binary128 rounding alone
had sent different ways on the two sides."""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
import scenes
from tests.test_unorm8_cpu import rn32


def _params(cam):
    g = oracle.cam(cam)
    F = lambda v: Fr(float(np.float32(v)))  # noqa: E731
    return (F(g.fx), F(g.fy), F(g.cx), F(g.cy), [F(v) for v in g.R], [F(v) for v in g.t])


def _mul(A, B):
    return [[sum(A[r][m] * B[m][k] for m in range(3)) for k in range(3)] for r in range(3)]


def _vec(A, x):
    return [sum(A[r][m] * x[m] for m in range(3)) for r in range(3)]


def exact_relproj(a, b):
    """(H, c) as exact rationals, and the same products over magnitudes."""
    fxa, fya, cxa, cya, Ra, ta = _params(a)
    fxb, fyb, cxb, cyb, Rb, tb = _params(b)
    out = []
    for mag in (False, True):
        f = abs if mag else (lambda v: v)
        Kb = [[f(fxb), 0, f(cxb)], [0, f(fyb), f(cyb)], [0, 0, 1]]
        Kai = [[f(1 / fxa), 0, f(-cxa / fxa)], [0, f(1 / fya), f(-cya / fya)], [0, 0, 1]]
        Rbm = [[f(Rb[3 * r + k]) for k in range(3)] for r in range(3)]
        RaT = [[f(Ra[3 * k + r]) for k in range(3)] for r in range(3)]
        H = _mul(Kb, _mul(Rbm, _mul(RaT, Kai)))
        v = _vec(Rbm, _vec(RaT, [f(x) for x in ta]))
        e = [f(tb[r]) + v[r] if mag else tb[r] - v[r] for r in range(3)]
        out.append(([H[r][k] for r in range(3) for k in range(3)], _vec(Kb, e)))
    return out[0], out[1]


def expected_f32(val, mag):
    if abs(val) < Fr(1, 2 ** 50) * mag:
        return np.float32(0.0)
    return np.float32(float(rn32(val)))


def sweep_rig(seed):
    """The cameras of the GPU random sweep's case ``seed`` (its rig draws, without rendering)."""
    rng = np.random.default_rng(1000 + seed)
    k = int(rng.integers(1, 9))
    w, h = int(rng.integers(1, 90)), int(rng.integers(1, 60))
    n_ring = max(8, k + 2)
    seq = scenes.RingSequence(7, seed, n_ring, 1.0, w, h, k, scenes.MovingSpheres(seed, 3),
                              target_angle=2 * math.pi * 0.37 / n_ring)
    return seq.src, seq.tgt


def _pairs():
    for seed in list(range(300)) + [1348]:
        src, tgt = sweep_rig(seed)
        for s in src:
            yield f"sweep seed {seed}", s, tgt
    ring = scenes.ring_rig(16, 1.0, 1280, 720)
    tgt = scenes.ring_target(0.5, 1.0, 1280, 720)
    for k in range(0, 16, 3):
        yield f"ring view {k}", ring[k], tgt
        yield f"ring view {k} from the target", tgt, ring[k]


def _expected(a, b):
    (H, c), (Hm, cm) = exact_relproj(a, b)
    return np.array([expected_f32(v, m) for v, m in zip(H + c, Hm + cm)], np.float32)


def test_oracle_rounds_the_exact_projection():
    for what, a, b in _pairs():
        Ho, co = oracle.relproj(a, b)
        got = np.concatenate([Ho.astype(np.float32).ravel(), co.astype(np.float32)])
        want = _expected(a, b)
        assert got.tobytes() == want.tobytes(), (what, got, want)


def test_library_rounds_the_exact_projection():
    ops = pytest.importorskip("paper_2505_18932_amd.ops")
    for what, a, b in _pairs():
        H, c = ops.relative_projection(a, b)
        got = np.concatenate([np.array(H, np.float32).ravel(), np.array(c, np.float32)])
        want = _expected(a, b)
        assert got.tobytes() == want.tobytes(), (what, got, want)


def test_the_tie_of_seed_1348():
    src, tgt = sweep_rig(1348)
    (H, _), _ = exact_relproj(src[0], tgt)
    lo = np.float32(0.17127085)
    hi = np.nextafter(lo, np.float32(1))
    assert H[3] == (Fr(float(lo)) + Fr(float(hi))) / 2  # exactly halfway
    even = lo if (lo.view(np.uint32) & 1) == 0 else hi
    Ho, _ = oracle.relproj(src[0], tgt)
    assert Ho.astype(np.float32).ravel()[3] == even
