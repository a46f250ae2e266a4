"""The streaming kernel of include/yoro_measure.h computes what it says
(c = a ^ b), including a ragged tail of fewer than four elements."""
from __future__ import annotations

import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [1, 3, 4, 4099, 1 << 20])
def test_stream_kernel_is_exact(cuda, n):
    import torch

    from paper_2506_15183_amd import yoro

    g = torch.Generator().manual_seed(n)
    a = torch.randint(-2**31, 2**31 - 1, (n,), dtype=torch.int32, generator=g).cuda()
    b = torch.randint(-2**31, 2**31 - 1, (n,), dtype=torch.int32, generator=g).cuda()
    c = torch.full_like(a, 7)
    yoro.measure_stream(a, b, c)
    torch.cuda.synchronize()
    assert torch.equal(c.cpu(), a.cpu() ^ b.cpu())
