"""The allocation-free surrogate forward (sl_mlp_forward_noalloc) against sl_mlp_forward.

Two calls in a row through the C ABI, the second with a smaller batch (the
static scratch keeps the first call's contents, which the second must fully
overwrite): each must equal sl_mlp_forward on the same inputs bit for bit,
since both run the same kernels.  Also checks the host-side rejection of a
batch beyond the maximum.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _params(sl, seed):
    rng = np.random.default_rng(seed)
    w = []
    for a, b in ((7, 256), (256, 256), (256, 1)):
        lim = np.sqrt(6.0 / a)
        w.append((rng.uniform(-lim, lim, size=(a, b)), 0.1 * rng.standard_normal(b)))
    return sl.mlp_pack(w, DEV)


def test_noalloc_forward_matches_workspace_forward():
    import paper_1101_5803_amd as sl
    assert torch.cuda.is_available()
    rng = np.random.default_rng(5)
    for call, (batch, seed) in enumerate(((8192, 1), (1000, 2))):
        params = _params(sl, seed)
        x = torch.tensor(rng.uniform(-1, 1, (batch, 7)), dtype=torch.float32, device=DEV)
        y_ref = sl.mlp_forward(params, x)
        y = torch.full((batch,), float("nan"), dtype=torch.float32, device=DEV)
        sl.mlp_forward_noalloc(params, x, y)
        torch.cuda.synchronize()
        assert torch.isfinite(y).all(), call
        assert torch.equal(y, y_ref), (call, float((y - y_ref).abs().max()))
    # a batch beyond the maximum is refused on the host, before any launch
    L = sl._lib
    x1 = torch.zeros((1, 7), dtype=torch.float32, device=DEV)
    rc = L.lib().sl_mlp_forward_noalloc(L.ptr(params), L.ptr(x1), L.MLP_MAX_BATCH + 1, L.ptr(y), None)
    assert rc == L.SL_EINVAL
    assert b"batch" in L.lib().sl_last_error()
