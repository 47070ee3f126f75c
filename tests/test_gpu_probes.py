"""The streaming probes (the read/write-mix ceilings the fused kernels are
compared with) move the bytes they claim, in every launch shape: the copy
reproduces its source, the 2:1 mix writes a XOR b, the write-only probe writes
its index pattern, the read-only probe leaves its output alone on random data;
the tiled probes (16384-row column-major streams moved tile by tile) copy and
XOR every element of every column in each tile shape."""
import numpy as np
import pytest

from gpu_util import need_gpu, torch

pytestmark = pytest.mark.gpu

from paper_2308_03120_amd import coot  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    coot.init(0)


@pytest.mark.parametrize("shape", [0, 1, 2, 3])
@pytest.mark.parametrize("nbytes", [16, 16 * 1000 + 16 * 37, 16 * (1 << 20) + 48])
def test_probes_move_their_bytes(shape, nbytes):
    g = torch.Generator(device="cuda")
    g.manual_seed(nbytes + shape)
    n32 = nbytes // 4
    src = torch.randint(-2 ** 31, 2 ** 31 - 1, (2 * n32,), generator=g, device="cuda", dtype=torch.int32)
    dst = torch.zeros(n32, device="cuda", dtype=torch.int32)
    coot.bandwidth_probe(coot.PROBE_COPY | (shape << 8), dst, src, nbytes)
    torch.cuda.synchronize()
    assert torch.equal(dst, src[:n32])
    coot.bandwidth_probe(coot.PROBE_READ2_WRITE1 | (shape << 8), dst, src, nbytes)
    torch.cuda.synchronize()
    assert torch.equal(dst, src[:n32] ^ src[n32:])
    coot.bandwidth_probe(coot.PROBE_WRITE | (shape << 8), dst, src, nbytes)
    torch.cuda.synchronize()
    want = np.zeros((n32 // 4, 4), np.int32)
    want[:, 0] = np.arange(n32 // 4)
    assert np.array_equal(dst.cpu().numpy().reshape(-1, 4), want)
    dst.fill_(7)
    coot.bandwidth_probe(coot.PROBE_READ | (shape << 8), dst, src, nbytes)
    torch.cuda.synchronize()
    assert bool((dst == 7).all())


@pytest.mark.parametrize("shape", [0, 1, 2, 3])
def test_tiled_probes_move_every_element(shape):
    cols = 128
    n = 16384 * cols
    g = torch.Generator(device="cuda")
    g.manual_seed(100 + shape)
    src = torch.randint(-2 ** 31, 2 ** 31 - 1, (2 * n,), generator=g, device="cuda", dtype=torch.int32)
    dst = torch.zeros(n, device="cuda", dtype=torch.int32)
    coot.bandwidth_probe(coot.PROBE_TILED_COPY | (shape << 8), dst, src, 4 * n)
    torch.cuda.synchronize()
    assert torch.equal(dst, src[:n])
    dst.zero_()
    coot.bandwidth_probe(coot.PROBE_TILED_READ2_WRITE1 | (shape << 8), dst, src, 4 * n)
    torch.cuda.synchronize()
    assert torch.equal(dst, src[:n] ^ src[n:])
