"""Reference streaming kernels (ldpm_stream_probe), which the benchmark uses
for the practical HBM ceiling: each moves exactly the bytes it is asked to
and computes what its description says (checked element by element, with a
ragged tail), and bad arguments are refused before any launch."""
import ctypes as C

import pytest

pytestmark = pytest.mark.gpu


def _t():
    import torch
    return torch


def test_copy_fill_mix_and_read_results():
    torch = _t()
    from paper_2603_13190_amd.ldpm import stream_probe
    n2 = 1000 * 256 + 17                     # 16-byte elements: several blocks and a ragged tail
    g = torch.Generator().manual_seed(7)
    a = torch.rand(3 * 2 * n2, generator=g, dtype=torch.float64).cuda()
    b = torch.full((2 * 2 * n2 + 8,), -7.0, dtype=torch.float64, device="cuda")

    stream_probe("copy", a, b, 32 * n2)
    torch.cuda.synchronize()
    assert torch.equal(b[:2 * n2], a[:2 * n2])
    assert bool((b[2 * n2:] == -7.0).all())  # nothing past the end

    b.fill_(-7.0)
    stream_probe("fill", None, b, 16 * n2)
    torch.cuda.synchronize()
    assert bool((b[0:2 * n2:2] == 1.0).all()) and bool((b[1:2 * n2:2] == -1.0).all())
    assert bool((b[2 * n2:] == -7.0).all())

    b.fill_(-7.0)
    stream_probe("mix", a, b, 80 * n2)
    torch.cuda.synchronize()
    x, y, z = a[:2 * n2], a[2 * n2:4 * n2], a[4 * n2:6 * n2]
    assert torch.equal(b[:2 * n2], x + y)
    assert torch.equal(b[2 * n2:4 * n2], y + z)
    assert bool((b[4 * n2:] == -7.0).all())

    blocks = (n2 + 255) // 256
    b.fill_(-7.0)
    stream_probe("read", a, b, 16 * n2)
    torch.cuda.synchronize()
    ref = torch.nn.functional.pad(a[:2 * n2].cpu(), (0, 2 * 256 * blocks - 2 * n2)).view(blocks, 512).sum(1)
    assert torch.allclose(b[:blocks].cpu(), ref, rtol=1e-13, atol=0)
    assert bool((b[blocks:] == -7.0).all())


def test_probe_errors():
    torch = _t()
    from paper_2603_13190_amd.ldpm import lib, LdpmError, stream_probe
    a = torch.zeros(1024, dtype=torch.float64, device="cuda")
    b = torch.zeros(1024, dtype=torch.float64, device="cuda")
    with pytest.raises(LdpmError):
        stream_probe("copy", a, b, 48)          # not a multiple of 32
    with pytest.raises(LdpmError):
        stream_probe("mix", a, b, 160 + 16)     # not a multiple of 80
    with pytest.raises(LdpmError):
        stream_probe("copy", a, b, 0)
    with pytest.raises(LdpmError):
        stream_probe("read", None, b, 64)       # null source
    assert lib().ldpm_stream_probe(9, C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), 64, None) != 0
    assert lib().ldpm_stream_probe(0, C.c_void_p(a.data_ptr() + 8), C.c_void_p(b.data_ptr()), 64, None) != 0
