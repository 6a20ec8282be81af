"""The splat's fixed-point terms: the FP32 route that the raster kernel takes
(floor, the exact fraction, one round-half-to-even of the fraction times 2^32;
negative terms through their magnitude, negated back) gives exactly
round(t 2^32) as the FP64 product and a 64-bit rint would, for every FP32 t
the kernel feeds it (G and G c in [0, 1] times 2^8, the mask term of either
sign, log(1 - G) in [-17, 0]).  IEEE FP32 arithmetic in numpy follows the same
rules as the device's, so this checks the exactness argument itself -- and
shows why negative terms need the detour: the fraction 1 - |t| of a small
negative t is not exact."""
import numpy as np


def nonneg_fp32(t):
    """round(t 2^32) for t >= 0 the kernel's way."""
    t = np.asarray(t, dtype=np.float32)
    assert np.all(np.signbit(t) == False) or np.all(t[np.signbit(t)] == 0)  # noqa: E712
    hi = np.floor(t).astype(np.float32)
    f = (t - hi).astype(np.float32)
    lo = np.rint((f * np.float32(4294967296.0)).astype(np.float32)).astype(np.float32)
    assert np.all(lo < 2.0 ** 32)
    return hi.astype(np.int64) * (1 << 32) + lo.astype(np.int64)


def signed_fp32(t):
    """Either sign: through |t|, negated back (round half to even is symmetric)."""
    t = np.asarray(t, dtype=np.float32)
    m = nonneg_fp32(np.abs(t))
    return np.where(t < 0, -m, m)


def reference(t):
    # t 2^32 is exact in FP64 (24 significant bits); rint rounds half to even
    return np.rint(np.asarray(t, dtype=np.float32).astype(np.float64) * 2.0 ** 32).astype(np.int64)


def test_unit_interval_terms_times_256():
    rng = np.random.default_rng(11)
    x = np.concatenate([rng.random(400000, dtype=np.float32),
                        np.float32(2.0) ** -rng.integers(0, 60, 50000).astype(np.float32)
                        * rng.random(50000, dtype=np.float32),
                        np.array([0.0, 1.0, np.nextafter(np.float32(1), np.float32(0)),
                                  np.float32(2.0 ** -40), np.float32(2.0 ** -41),
                                  np.float32(3 * 2.0 ** -42), np.float32(1.5 * 2.0 ** -40)],
                                 dtype=np.float32)])
    t = (x * np.float32(256.0)).astype(np.float32)
    assert np.array_equal(nonneg_fp32(t), reference(t))
    assert np.array_equal(signed_fp32(-t), reference(-t))


def test_log_terms():
    rng = np.random.default_rng(12)
    G = rng.random(400000, dtype=np.float32)
    L = np.log((np.float32(1) - G).astype(np.float32)).astype(np.float32)
    L = np.concatenate([L, np.array([0.0, -0.0, -16.635532, -1.0, -2.0 ** -30, -17.0],
                                    dtype=np.float32)])
    # the kernel's log term: 0 - round(-L 2^32)
    assert np.array_equal(-nonneg_fp32(-L), reference(L))


def test_halfway_cases_round_to_even():
    # fractions whose 2^32 multiple ends in exactly one half
    t = np.array([2.0 ** -33, 3 * 2.0 ** -33, 5 * 2.0 ** -33, 1 + 2.0 ** -23, 255.5,
                  -(2.0 ** -33), -(3 * 2.0 ** -33), -(2.0 ** -30), -0.75], dtype=np.float32)
    assert np.array_equal(signed_fp32(t), reference(t))
