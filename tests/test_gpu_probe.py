"""The streaming-ceiling probe of the measurement section: its copies move
the bytes exactly, its read sweep touches every word, and it rejects
misaligned or empty buffers."""
import pytest

from paper_2609_36267_amd import binding as ww

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    ww.load()
    return torch


@pytest.mark.parametrize("mode", [0, 2])
@pytest.mark.parametrize("nbytes", [16, 4096 + 48, (3 << 20) + 16 * 7])
def test_copy_modes_copy_exactly(torch_cuda, mode, nbytes):
    torch = torch_cuda
    g = torch.Generator(device="cuda").manual_seed(nbytes + mode)
    src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device="cuda", generator=g)
    dst = torch.zeros_like(src)
    ms = ww.stream_probe(src, dst, mode=mode, reps=2)
    torch.cuda.synchronize()
    assert ms > 0
    assert torch.equal(src, dst)


def test_read_mode_folds_every_word(torch_cuda):
    """One non-zero word among zeros: the XOR of the workgroups' results is
    that word, wherever it sits."""
    torch = torch_cuda
    n = 1 << 22
    for pos in (0, 12345, n // 16 - 1):
        src = torch.zeros(n, dtype=torch.uint8, device="cuda")
        src.view(torch.int32)[pos * 4:pos * 4 + 4] = torch.tensor([1, 2, 3, 4], dtype=torch.int32,
                                                                     device="cuda")
        out = torch.zeros(32 << 10, dtype=torch.uint8, device="cuda")
        ww.stream_probe(src, out, mode=1, reps=1)
        torch.cuda.synchronize()
        words = out.view(torch.int32).view(-1, 4)
        acc = words[0].clone()
        for k in range(1, words.shape[0]):
            acc ^= words[k]
        assert acc.tolist() == [1, 2, 3, 4]


def test_bad_arguments_rejected(torch_cuda):
    torch = torch_cuda
    a = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    b = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    with pytest.raises(ww.WWError):
        ww.stream_probe(a[:4008], b, mode=0)       # not a multiple of 16
    with pytest.raises(ww.WWError):
        ww.stream_probe(a[1:17], b, mode=0)        # misaligned source
    with pytest.raises(ww.WWError):
        ww.stream_probe(a, b, mode=3)
