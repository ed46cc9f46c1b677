"""The allocation-free encode (dino_encode_noalloc) against dino_encode, through the C ABI.

Both run the same transform kernels on the same inputs, so their outputs must be
identical; they are also checked against the oracle's encoder (the bar of the encode
parity test, 1e-12). Two calls in a row, the second with fewer fields, share the
library's static scratch; sizes beyond the scratch are refused.
"""
import ctypes as ct

import numpy as np
import pytest

from oracle import prior

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _encode(ctx, fn, fields):
    n, d_m = fields.shape
    x = torch.full((n, ctx.r), np.nan, dtype=torch.float64, device="cuda:0")
    zp = torch.full((n, d_m - ctx.r), np.nan, dtype=torch.float64, device="cuda:0")
    st = ct.c_void_p(torch.cuda.current_stream().cuda_stream)
    status = fn(ctx.h, n, ct.c_void_p(fields.data_ptr()), ct.c_void_p(x.data_ptr()), ct.c_void_p(zp.data_ptr()), st)
    torch.cuda.synchronize()
    return status, x.cpu().numpy(), zp.cpu().numpy()


def test_encode_noalloc_matches_encode_twice():
    from paper_2403_08220_amd import Context
    from paper_2403_08220_amd._lib import check

    n, r = 65, 50
    ctx = Context(0)
    try:
        ctx.load_prior(n, 0.1, 1.0, r)
        basis = prior.KLEBasis(n, 0.1, 1.0, r)
        rng = np.random.default_rng(21)
        for nf in (9, 4):  # the second call is smaller: stale scratch from the first must not matter
            print(f"encode_noalloc: {nf} fields on {n}x{n}", flush=True)
            m = rng.standard_normal((nf, n * n))
            fields = torch.tensor(m, dtype=torch.float64, device="cuda:0")
            s1, x1, z1 = _encode(ctx, ctx.lib.dino_encode, fields)
            s2, x2, z2 = _encode(ctx, ctx.lib.dino_encode_noalloc, fields)
            check(s1)
            check(s2)
            np.testing.assert_array_equal(x2, x1)
            np.testing.assert_array_equal(z2, z1)
            zref = basis.whiten_full(m)
            scale = np.max(np.abs(zref))
            assert np.max(np.abs(x2 - zref[:, :r])) / scale < 1e-12
            assert np.max(np.abs(z2 - zref[:, r:])) / scale < 1e-12
    finally:
        ctx.close()


def test_encode_noalloc_refuses_sizes_beyond_its_scratch():
    from paper_2403_08220_amd import Context, DinoError
    from paper_2403_08220_amd._lib import check

    n, r = 129, 200
    ctx = Context(0)
    try:
        ctx.load_prior(n, 0.1, 1.0, r)
        cap = (16 << 20) // (2 * 8 * n * n)          # 63 fields fit
        fields = torch.zeros((cap + 1, n * n), dtype=torch.float64, device="cuda:0")
        status, _, _ = _encode(ctx, ctx.lib.dino_encode_noalloc, fields)
        with pytest.raises(DinoError, match="too large for the encode scratch"):
            check(status)
        status, _, _ = _encode(ctx, ctx.lib.dino_encode_noalloc, fields[:cap])
        check(status)
    finally:
        ctx.close()
