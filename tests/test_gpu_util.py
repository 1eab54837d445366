"""GPU test of the library's streaming copy (the measurement reference)."""
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def chx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2101_06550_amd import chx as m
    m.load()
    return m


@pytest.mark.parametrize("n", [1, 2047, 2048, 2049, 1 << 20, (1 << 20) + 333])
def test_stream_copy_exact(chx, n):
    print(f"[case] stream copy n={n}", flush=True)
    src = torch.rand(n, dtype=torch.float64, device="cuda")
    dst = torch.full_like(src, -1.0)
    guard = torch.full((4096,), 5.0, dtype=torch.float64, device="cuda")
    chx.chx_stream_copy(src, dst)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    assert torch.all(guard == 5.0)


def test_stream_copy_rejects_overlap_and_misalignment(chx):
    buf = torch.zeros(4096, dtype=torch.float64, device="cuda")
    with pytest.raises(chx.ChxError):
        chx.chx_stream_copy(buf[:2048], buf[1024:3072])
    with pytest.raises(chx.ChxError):
        chx.chx_stream_copy(buf[1:1001], buf[2048:3048])
