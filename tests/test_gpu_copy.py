"""The library's streaming copy (HBM ceiling and counter calibration):
bitwise copy for sizes below, at and above one block's chunk (64 KiB, more
above 512 MiB), with ragged tails, and nothing written past the end."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes", [16, 4096, 65536, 65536 + 48, 3 * 65536 + 16 * 7, (64 << 20) + 16 * 1001, (600 << 20) + 48])
def test_stream_copy_bitwise(nbytes):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_05264_amd import lbmflow as L

    print(f"case: stream_copy {nbytes} bytes", flush=True)
    # distinct words, so a misplaced element shows
    src = torch.arange(nbytes // 4, dtype=torch.int32, device="cuda") ^ 0x5A5A5A5
    dst = torch.full_like(src, -1)
    guard = torch.full((64,), -7, dtype=torch.int32, device="cuda")
    pad = torch.cat([dst, guard])  # bytes past the copy stay untouched
    L.stream_copy(pad.data_ptr(), src.data_ptr(), nbytes)
    torch.cuda.synchronize()
    assert torch.equal(pad[: nbytes // 4], src)
    assert torch.equal(pad[nbytes // 4:], guard)
