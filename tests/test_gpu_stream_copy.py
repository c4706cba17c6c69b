"""dd_stream_copy, the bandwidth reference of the benchmark: an exact copy for
whole tiles, a partial last tile and a single vector, nothing written past
the end, and its argument checks."""
import numpy as np
import pytest

from paper_1710_07041_amd import ddsap

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nvec", [1, 3, 1024, 1025, 4096 + 17, 3 * 1024 * 1024 + 511])
def test_copy_is_exact(nvec):
    import torch
    gen = torch.Generator(device="cuda")
    gen.manual_seed(nvec)
    src = torch.randint(-2 ** 31, 2 ** 31 - 1, (nvec * 4,), dtype=torch.int32, device="cuda", generator=gen)
    dst = torch.full((nvec * 4 + 64,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
    ddsap.stream_copy(src, dst, nvec * 16)
    torch.cuda.synchronize()
    assert torch.equal(dst[: nvec * 4], src)
    assert bool((dst[nvec * 4:] == 0x5A5A5A5A).all())


def test_argument_checks():
    import torch
    a = torch.zeros(64, dtype=torch.int32, device="cuda")
    b = torch.zeros(64, dtype=torch.int32, device="cuda")
    for nbytes in (0, 8, 100):
        with pytest.raises(ddsap.DDError):
            ddsap.stream_copy(a, b, nbytes)
    torch.cuda.synchronize()
    assert np.all(b.cpu().numpy() == 0)
