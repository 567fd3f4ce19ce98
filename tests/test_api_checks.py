"""Argument checks of the Python binding: every device buffer the kernels read
or write is validated (device, type, contiguity, size) before any launch, so
a wrong argument raises instead of reaching the GPU.

The CPU tests need no GPU (host tensors are rejected first); the GPU tests
build valid device tensors of the wrong shape and check that nothing runs.
"""
import numpy as np
import pytest
import torch

import paper_2502_20392_amd as sk

OFFSETS = np.array([0, 40, 100, 130], dtype=np.int64)
PAIRS = np.array([[0, 1], [1, 2], [2, 2]], dtype=np.int32)


def test_host_tensors_are_rejected():
    x = torch.zeros(10, 3, dtype=torch.float64)
    with pytest.raises(TypeError):
        sk.pair(x, x)
    with pytest.raises(TypeError):
        sk.gram(x[None])
    plan = sk.RaggedPlan(OFFSETS, PAIRS, 3, order=8)
    pool = torch.zeros(130, 3, dtype=torch.float64)
    with pytest.raises(TypeError):
        plan.run(pool)
    with pytest.raises(TypeError):
        plan.backward(pool, torch.ones(3, dtype=torch.float64))
    with pytest.raises(TypeError):
        sk.gram_ragged(pool, OFFSETS, PAIRS)
    with pytest.raises(TypeError):
        sk.backward(pool, OFFSETS, PAIRS, torch.ones(3, dtype=torch.float64))


@pytest.mark.gpu
def test_device_buffers_are_validated(dev):
    pool = torch.randn(130, 3, dtype=torch.float64, device=dev).cumsum(0) * 0.1
    plan = sk.RaggedPlan(OFFSETS, PAIRS, 3, order=8)
    with pytest.raises(ValueError):  # fewer points than the offsets address
        plan.run(pool[:129])
    with pytest.raises(ValueError):  # channel count differs from the plan's
        plan.run(torch.zeros(130, 4, dtype=torch.float64, device=dev))
    with pytest.raises(ValueError):  # output too small
        plan.run(pool, torch.empty(2, dtype=torch.float64, device=dev))
    with pytest.raises(TypeError):  # output of the wrong type
        plan.run(pool, torch.empty(3, dtype=torch.float32, device=dev))
    with pytest.raises(ValueError):  # non-contiguous output
        plan.run(pool, torch.empty(3, 2, dtype=torch.float64, device=dev)[:, 0])
    with pytest.raises(TypeError):  # weights on the host
        plan.backward(pool, torch.ones(3, dtype=torch.float64))
    with pytest.raises(ValueError):  # wrong number of weights
        plan.backward(pool, torch.ones(4, dtype=torch.float64, device=dev))
    with pytest.raises(ValueError):  # gradient buffer not the pool's shape
        plan.backward(pool, torch.ones(3, dtype=torch.float64, device=dev),
                      torch.zeros(129, 3, dtype=torch.float64, device=dev))
    with pytest.raises(ValueError):  # non-contiguous gradient buffer
        plan.backward(pool, torch.ones(3, dtype=torch.float64, device=dev),
                      torch.zeros(3, 130, dtype=torch.float64, device=dev).t())
    with pytest.raises(ValueError):
        sk.gram_ragged(pool[:100], OFFSETS, PAIRS)
    with pytest.raises(ValueError):
        sk.backward(pool[:100], OFFSETS, PAIRS, torch.ones(3, dtype=torch.float64, device=dev))
    x = pool[:40].contiguous()
    with pytest.raises(TypeError):  # workspace on the host
        sk.pair(x, x, order=8, ws=torch.empty(1 << 20, dtype=torch.uint8))
    # the plan still works after the rejected calls
    out = plan.run(pool)
    torch.cuda.synchronize()
    assert torch.isfinite(out).all()
