"""The allocation-free network forward (lagot_mlp_forward_noalloc, for callers that cannot
allocate device memory) against lagot_mlp_forward, through the C-ABI.

Both run the same kernels on the same parameters and inputs; only the hidden-activation
buffers differ (the library's static device array against the context's workspace), so the
outputs must agree bit for bit. Two calls in a row, the second with fewer rows (the array
keeps the first call's contents), and the row limit of the static array."""
import sys

import numpy as np
import pytest

from oracle import mlp

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _bf16_bits(a):
    a = np.asarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16).view(np.int16)


def test_forward_noalloc_matches_forward():
    import torch
    import paper_2601_05765_amd as L
    assert torch.cuda.is_available()
    ctx = L.Context()
    params = np.concatenate([p.ravel() for p in mlp.init_params(21)]).astype(np.float32)
    ctx.mlp_set_params(torch.tensor(params, device="cuda"))
    rng = np.random.default_rng(22)
    for m in (20_000, 3_001):  # the second call is smaller: rows past m hold the first call's values
        _say(f"case: noalloc forward, m = {m}")
        X = rng.normal(size=(m, 64))
        X[:, 50:] = 0
        feats = torch.tensor(_bf16_bits(X), device="cuda")
        ref = ctx.mlp_forward(feats)
        out = torch.full((m,), float("nan"), dtype=torch.float32, device="cuda")
        ctx.mlp_forward_noalloc(feats, out)
        torch.cuda.synchronize()
        a, b = ref.cpu().numpy(), out.cpu().numpy()
        assert np.all(np.isfinite(b))
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), float(np.max(np.abs(a - b)))


def test_forward_noalloc_row_limit():
    import torch
    import paper_2601_05765_amd as L
    ctx = L.Context()
    params = np.concatenate([p.ravel() for p in mlp.init_params(23)]).astype(np.float32)
    ctx.mlp_set_params(torch.tensor(params, device="cuda"))
    m = L.NOALLOC_MAX_ROWS + 1
    _say(f"case: noalloc forward beyond its row limit, m = {m}")
    feats = torch.zeros((m, 64), dtype=torch.int16, device="cuda")
    out = torch.zeros(m, dtype=torch.float32, device="cuda")
    with pytest.raises(L.LagotError) as e:
        ctx.mlp_forward_noalloc(feats, out)
    assert e.value.code == L.ECAPACITY
