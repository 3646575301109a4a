"""The backward entry point that allocates nothing (bx_mlp_backward_noalloc)
against bx_mlp_backward with a caller work buffer: the same kernels, so the
gradients agree bit for bit, on two calls in a row (the second with fewer
samples, over the scratch the first one left), and a batch beyond the static
scratch is refused before any device work."""
import ctypes

import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

import paper_1608_05288_amd as bx

F, H = 32, 128


def _inputs(m, B, seed):
    import torch
    rng = np.random.default_rng(seed)
    x = torch.from_numpy(rng.uniform(-0.5, 1.5, (B, F)).astype(np.float32)).cuda()
    dy = torch.from_numpy(rng.normal(0, 1, B).astype(np.float32)).cuda()
    _, act = m.forward(x)
    return x, act, dy


def test_noalloc_backward_matches_buffered_backward():
    import torch
    p = bx.PartitionMLP.init_params(F, H, 7) + np.random.default_rng(7).normal(0, 0.05, bx.lib().bx_mlp_num_params(F, H)).astype(np.float32)
    m = bx.PartitionMLP(F, H, params=p.astype(np.float32))
    for B, seed in ((bx.MLP_NOALLOC_MAX_BATCH, 1), (1000, 2), (37, 3)):
        x, act, dy = _inputs(m, B, seed)
        ref = m.backward(x, act, dy).clone()
        torch.cuda.synchronize()
        m.grads.fill_(float("nan"))
        got = m.backward_noalloc(x, act, dy).clone()
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (B, int((got != ref).sum()))
    with pytest.raises(bx.BxError) as e:
        x, act, dy = _inputs(m, bx.MLP_NOALLOC_MAX_BATCH + 1, 4)
        m.backward_noalloc(x, act, dy)
    assert e.value.status == -3
