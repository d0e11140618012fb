"""The library's streaming copy (``gft_stream_copy``), the HBM reference the bench quotes
beside the transform kernels: byte-exact copies at sizes across the grid-stride step and its
ragged tail, and its argument checks (which launch nothing)."""
import ctypes

import pytest

import paper_1907_07875_amd as G
from tests.gpu_helpers import device, torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes", [16, 4096, 16 * 1023, 16 * (256 * 4 * 64 * 256 + 37), 64 << 20])
def test_stream_copy_is_byte_exact(nbytes):
    dev = device()
    g = torch.Generator(device=dev).manual_seed(nbytes % 1000)
    src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device=dev, generator=g)
    dst = torch.zeros_like(src)
    G.gft_stream_copy(src, dst)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)


def test_stream_copy_leaves_bytes_past_the_end_alone():
    dev = device()
    src = torch.full((4096 + 64,), 7, dtype=torch.uint8, device=dev)
    dst = torch.zeros_like(src)
    lib = G.load_library()
    st = lib.gft_stream_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), 4096,
                             G._stream_ptr(None))
    assert st == 0
    torch.cuda.synchronize()
    assert int(dst[:4096].sum()) == 7 * 4096 and int(dst[4096:].sum()) == 0


def test_stream_copy_rejects_bad_arguments():
    dev = device()
    buf = torch.zeros(1 << 16, dtype=torch.uint8, device=dev)
    lib = G.load_library()
    s = G._stream_ptr(None)
    p = buf.data_ptr()
    cases = [
        ((p, p + 8192, 100), "GFT_ERR_INVALID_ARG"),      # not a multiple of 16
        ((p, p + 8192, -16), "GFT_ERR_INVALID_ARG"),
        ((0, p + 8192, 4096), "GFT_ERR_INVALID_ARG"),     # NULL
        ((p + 4, p + 8192, 4096), "GFT_ERR_ALIGNMENT"),
        ((p, p + 4096, 8192), "GFT_ERR_ALIGNMENT"),       # overlap
    ]
    for (a, b, nb), want in cases:
        st = lib.gft_stream_copy(ctypes.c_void_p(a), ctypes.c_void_p(b), nb, s)
        assert G.STATUS[st] == want, (a - p, b - p, nb, G.STATUS[st])
    assert lib.gft_stream_copy(ctypes.c_void_p(p), ctypes.c_void_p(p + 8192), 0, s) == 0
    torch.cuda.synchronize()
    assert int(buf.sum()) == 0
