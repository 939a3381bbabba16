"""The streaming copy and read kernels (the achievable-bandwidth references of the benchmark):
the copy moves every byte (ragged sizes, nothing written past the end); the read leaves its
input untouched; both refuse misaligned arguments."""
import numpy as np
import pytest

from gpu_util import announce

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("units", [1, 3, 4, 255, 1024, 4097, 1 << 20, (1 << 23) + 5])
def test_stream_copy_exact(units):
    import torch
    import paper_1611_00728_amd as ks
    announce("stream copy", units)
    rng = np.random.default_rng(units)
    src = torch.from_numpy(rng.integers(0, 2 ** 31, size=4 * units, dtype=np.int32)).cuda()
    big = torch.full((4 * units + 64,), -1, dtype=torch.int32, device="cuda")
    dst = big[:4 * units]
    ks.stream_copy(dst, src)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    assert torch.all(big[4 * units:] == -1)    # nothing written past the end


def test_stream_copy_errors():
    import torch
    import paper_1611_00728_amd as ks
    announce("stream copy errors")
    a = torch.zeros(64, dtype=torch.int32, device="cuda")
    with pytest.raises(ValueError):
        ks.stream_copy(a[:8], a[8:24])
    with pytest.raises(ks.KSError):
        ks.stream_copy(a[1:5], a[8:12])     # 4-byte offset: not 16-byte aligned


@pytest.mark.parametrize("units", [1, 255, 4097, (1 << 23) + 5])
def test_stream_read_leaves_input(units):
    import torch
    import paper_1611_00728_amd as ks
    announce("stream read", units)
    rng = np.random.default_rng(units)
    src = torch.from_numpy(rng.integers(0, 2 ** 31, size=4 * units, dtype=np.int32)).cuda()
    keep = src.clone()
    ks.stream_read(src)
    torch.cuda.synchronize()
    assert torch.equal(src, keep)


def test_stream_read_errors():
    import torch
    import paper_1611_00728_amd as ks
    announce("stream read errors")
    a = torch.zeros(64, dtype=torch.int32, device="cuda")
    with pytest.raises(ks.KSError):
        ks.stream_read(a[1:5])              # 4-byte offset
    with pytest.raises(ks.KSError):
        ks.stream_read(a[:3])               # 12 bytes
