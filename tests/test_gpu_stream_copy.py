"""The library's plain streaming copy (the bandwidth reference of the bench):
every byte copied, nothing written outside the destination range."""
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1309_3452_amd as P
    assert torch.cuda.is_available(), "needs a GPU"
    P.lib()
    return P


@pytest.mark.parametrize("n8", [1, 7, 255, 256, 257, 65536 * 256 + 3, 40_000_123])
def test_stream_copy_exact(P, n8):
    print("stream_copy %d x 8 B" % n8, flush=True)
    g = torch.Generator(device="cuda").manual_seed(n8)
    src = torch.randint(-2 ** 31, 2 ** 31 - 1, (2 * n8,), dtype=torch.int32, device="cuda", generator=g)
    # a guard element on each side of the destination stays untouched
    buf = torch.full((2 * n8 + 4,), 12345, dtype=torch.int32, device="cuda")
    dst = buf[2:2 + 2 * n8]
    P.stream_copy(dst, src)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    assert torch.equal(buf[:2], torch.full((2,), 12345, dtype=torch.int32, device="cuda"))
    assert torch.equal(buf[-2:], torch.full((2,), 12345, dtype=torch.int32, device="cuda"))
