"""The library's plain streaming copy and write (the attainable-bandwidth
references of the benchmark) copy and write exactly, at sizes around their
unrolled block and with a ragged tail (needs an MI355X)."""
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("words", [1, 255, 1024, 4096 * 3 + 7, (1 << 20) + 13])
def test_stream_copy_is_exact(words):
    from paper_1410_1937_amd import nfa
    g = torch.Generator(device="cuda").manual_seed(words)
    src = torch.randint(-2 ** 31, 2 ** 31 - 1, (4 * words,), dtype=torch.int32, device="cuda", generator=g)
    buf = torch.full((4 * words + 64,), 7, dtype=torch.int32, device="cuda")
    nfa.stream_copy(buf[:4 * words], src)
    torch.cuda.synchronize()
    assert torch.equal(buf[:4 * words], src)
    assert bool((buf[4 * words:] == 7).all())     # nothing written past the end


@pytest.mark.parametrize("words", [1, 255, 1024, 4096 * 3 + 7, (1 << 20) + 13])
def test_stream_fill_is_exact(words):
    from paper_1410_1937_amd import nfa
    buf = torch.full((4 * words + 64,), 7, dtype=torch.int32, device="cuda")
    nfa.stream_fill(buf[:4 * words], 0xDEADBEEF)
    torch.cuda.synchronize()
    assert bool((buf[:4 * words] == 0xDEADBEEF - (1 << 32)).all())     # the word as a signed int32
    assert bool((buf[4 * words:] == 7).all())     # nothing written past the end
