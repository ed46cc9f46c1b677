"""Encode / decode of nodal fields in whitened KLE coordinates (all d_m modes) against
the oracle's closed-form basis (dense DCT-II products in KLE order).

Tolerance: the device transform is two passes of n-term FP64 dot products with DCT
entries of size sqrt(2/n); 1e-12 relative covers the rounding at n = 129.
"""
import numpy as np
import pytest

from oracle import prior

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("n,r,nf", [(33, 32, 5), (129, 200, 3), (10, 7, 2)])
def test_encode_decode_against_oracle(n, r, nf):
    from paper_2403_08220_amd import Context
    print(f"encode n={n} r={r}", flush=True)
    ctx = Context(0)
    ctx.load_prior(n, 0.1, 1.0, r)
    B = prior.KLEBasis(n, 0.1, 1.0, r)
    rng = np.random.default_rng(n)
    m = rng.standard_normal((nf, n * n))
    x, zp = ctx.encode(torch.tensor(m, device="cuda:0"))
    ref = B.whiten_full(m)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(x.cpu().numpy() - ref[:, :r])) < 1e-12 * scale
    assert np.max(np.abs(zp.cpu().numpy() - ref[:, r:])) < 1e-12 * scale
    back = ctx.decode(x, zp).cpu().numpy()
    assert np.max(np.abs(back - m)) < 1e-12 * np.max(np.abs(m))
    xr = rng.standard_normal((nf, r))
    dec = ctx.decode(torch.tensor(xr, device="cuda:0")).cpu().numpy()
    ref_dec = xr @ B.dec.T
    assert np.max(np.abs(dec - ref_dec)) < 1e-12 * np.max(np.abs(ref_dec))
    ctx.close()
