"""lambda_predict_noalloc, the variant of lambda_predict for callers that
cannot allocate: the network's activations live in the library's static
device array instead of the model's workspace.  It runs the same kernels
with the same grid on the same inputs, so its outputs must equal
lambda_predict's bit for bit, on two calls in a row (the second smaller, so
that stale rows of the first call sit in the array), without any change in
the device's free memory; too many rows are refused."""
import numpy as np
import pytest

from tests.gpu_util import require_gpu, say

pytestmark = pytest.mark.gpu


def test_predict_noalloc_matches_predict():
    require_gpu()
    import torch
    from paper_2311_15393_amd import (KP_ERR_WORKSPACE, KP_PREDICT_NOALLOC_MAX_ROWS, KPError,
                                      Mlp)
    from paper_2311_15393_amd.lambda_net import init_params
    dev = torch.device("cuda:0")
    cap = KP_PREDICT_NOALLOC_MAX_ROWS
    mlp = Mlp(max_batch=cap)
    mlp.set_params(init_params(3))
    g = torch.Generator(device=dev)
    g.manual_seed(7)
    for call, nb in enumerate((cap, 300)):
        say(f"noalloc predict call {call}: {nb} rows")
        feats = torch.randn((nb, 128), device=dev, generator=g) * 3.0 + 0.5
        if call == 0:
            mlp.fit_normalizer(feats)
        ref = mlp.predict(feats)
        out = torch.full((nb,), float("nan"), device=dev, dtype=torch.float64)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        mlp.predict_noalloc(feats, out)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        assert free1 == free0, (free0, free1)
        assert bool(torch.isfinite(out).all())
        assert torch.equal(out, ref), float((out - ref).abs().max())
    big = torch.zeros((cap + 1, 128), device=dev)
    out = torch.empty(cap + 1, device=dev, dtype=torch.float64)
    with pytest.raises(KPError) as ei:
        mlp.predict_noalloc(big, out)
    assert ei.value.status == KP_ERR_WORKSPACE
    mlp.close()
