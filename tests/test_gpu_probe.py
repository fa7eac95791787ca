"""GPU: the streaming-read reference of the rooflines (amg_stream_read): every
16-byte element read exactly once, and argument errors."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_stream_read_sums_every_element_once():
    print("case stream read", flush=True)
    from paper_2511_21268_amd import amg
    assert torch.cuda.is_available()
    for n, threads in ((1 << 20, 2048 * 256), (3 * 1000 + 2, 256), (2, 512)):
        buf = torch.arange(n, dtype=torch.float64, device="cuda")
        sink = torch.full((threads,), float("nan"), dtype=torch.float64, device="cuda")
        amg.stream_read(buf, sink)
        torch.cuda.synchronize()
        assert float(sink.sum()) == n * (n - 1) / 2, n     # integers below 2^53: exact
    with pytest.raises(amg.AmgError):
        amg.stream_read(torch.zeros(3, dtype=torch.float64, device="cuda"), sink)   # 24 bytes
    with pytest.raises(amg.AmgError):
        amg.stream_read(buf, torch.zeros(100, dtype=torch.float64, device="cuda"))  # sink below 256
