"""The fusion kernels take 1/z from the hardware reciprocal refined by one
fused Newton step; they are bitwise equal to the oracle only if that is the
correctly rounded reciprocal.  Checked exhaustively on the device against
IEEE division, and on a random sample against the host's division."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2505_18932_amd import _lib as L

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def test_reciprocal_exhaustive_fast_range():
    # biased exponents 27 .. 226: every FP32 in [2^-100, 2^100) (2e9 values)
    cnt = torch.zeros(1, dtype=torch.int64, device=DEV)
    s = C.c_void_p(torch.cuda.current_stream(DEV).cuda_stream)
    L.check(L.lib().gg_selftest_reciprocal(27, 226, C.c_void_p(cnt.data_ptr()), s))
    torch.cuda.synchronize()
    assert int(cnt.item()) == 0


def test_reciprocal_matches_host_division():
    rng = np.random.default_rng(0)
    e = rng.uniform(-140, 127, 2_000_000)
    z = np.float32(2.0) ** e.astype(np.float32) * rng.uniform(1, 2, e.size).astype(np.float32)
    z = z[np.isfinite(z) & (z > 0)].astype(np.float32)
    zt = torch.from_numpy(z).to(DEV)
    out = torch.empty_like(zt)
    s = C.c_void_p(torch.cuda.current_stream(DEV).cuda_stream)
    L.check(L.lib().gg_fast_reciprocal(C.c_void_p(zt.data_ptr()), C.c_void_p(out.data_ptr()),
                                       z.size, s))
    torch.cuda.synchronize()
    ref = np.float32(1.0) / z
    got = out.cpu().numpy()
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
