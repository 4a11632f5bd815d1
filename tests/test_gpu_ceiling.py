"""The library's reference streams (gpop_stream_ceiling): the copy and the
widening copy write exactly what they read, over sizes that end inside a
workgroup's span and span several workgroups; the reads (whole array, and
scattered 512-byte segments) write nothing."""
import pytest
import torch

import paper_1806_08092_amd as gp

pytestmark = pytest.mark.gpu

# bytes of source: one vector, a partial workgroup span (16 KiB per
# workgroup), several spans with a ragged tail
SIZES = [16, 4096 + 48, 3 * 16384 + 1040, 1 << 22]


@pytest.mark.parametrize("nbytes", SIZES)
def test_copy_is_exact(nbytes):
    g = torch.Generator().manual_seed(nbytes)
    src = torch.randint(-2**31, 2**31 - 1, (nbytes // 4,), generator=g, dtype=torch.int32).cuda()
    dst = torch.full((nbytes // 4 + 64,), 7, dtype=torch.int32, device="cuda")
    gp.stream_ceiling(gp.STREAM_COPY, src, dst, nbytes)
    torch.cuda.synchronize()
    assert torch.equal(dst[: nbytes // 4], src)
    assert bool((dst[nbytes // 4:] == 7).all())  # nothing past the end


@pytest.mark.parametrize("nbytes", [8, 4096 + 24, 3 * 8192 + 520, 1 << 21])
def test_widen_is_exact(nbytes):
    n = nbytes // 2
    g = torch.Generator().manual_seed(n)
    src = torch.randint(0, 1 << 16, (n,), generator=g, dtype=torch.int32)
    src16 = src.to(torch.int16).cuda()  # wraps to the same 16 bits
    dst = torch.full((n + 64,), 7, dtype=torch.int32, device="cuda")
    gp.stream_ceiling(gp.STREAM_WIDEN, src16, dst, nbytes)
    torch.cuda.synchronize()
    assert torch.equal(dst[:n].cpu(), src)
    assert bool((dst[n:] == 7).all())


def test_read_writes_nothing():
    src = torch.ones((1 << 20) // 4, dtype=torch.int32, device="cuda")  # XOR of ones: 0
    sink = torch.full((16,), 5, dtype=torch.int32, device="cuda")
    gp.stream_ceiling(gp.STREAM_READ, src, sink, 1 << 20)
    torch.cuda.synchronize()
    assert bool((sink == 5).all())


@pytest.mark.parametrize("nbytes", [512, 1 << 20])
def test_scattered_segments_write_nothing(nbytes):
    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")  # XOR of ones: 0
    sink = torch.full((16,), 5, dtype=torch.int32, device="cuda")
    gp.stream_ceiling(gp.STREAM_SEGMENTS, src, sink, nbytes)
    torch.cuda.synchronize()
    assert bool((sink == 5).all())
