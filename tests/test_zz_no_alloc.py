"""The entry point that allocates nothing (rsg_gauss_filter_noalloc) against
rsg_gauss_filter, through the C ABI: the same image filtered by both must
agree bit for bit for uint8 and within 1e-5 of max|result| for FP32, on two
calls in a row with the second smaller, on the two-pass path (which uses the
scratch array) and on the fused path (which needs none); an intermediate
larger than the scratch array is refused before any launch."""
import ctypes

import numpy as np
import pytest

import synthimg
from gpu_util import from_device, rel_max_err, to_device

pytestmark = pytest.mark.gpu


def _both(img, dt, sigma, K, boundary=0):
    import torch
    import paper_1107_4958_amd as rsg
    src = to_device(img, dt)
    H, W = img.shape[:2]
    C = img.shape[2] if img.ndim == 3 else 1
    ref = torch.empty_like(src)
    out = torch.full_like(src, 7)
    st = torch.cuda.current_stream().cuda_stream
    code = rsg.DTYPE_NAMES[dt]
    rsg.rsg_gauss_filter(src.data_ptr(), ref.data_ptr(), H, W, C, code, sigma, K, boundary, st)
    rsg.rsg_gauss_filter_noalloc(src.data_ptr(), out.data_ptr(), H, W, C, code, sigma, K, boundary, st)
    torch.cuda.synchronize()
    return from_device(out, dt), from_device(ref, dt)


def _agree(a, b, dt):
    if dt == "f32":
        assert rel_max_err(a, b.astype(np.float64)) <= 1e-5
    else:
        assert np.array_equal(a, b)


@pytest.mark.parametrize("dt", ["u8", "f32", "f16"])
def test_two_calls_two_pass_then_smaller(dt):
    """The two-pass path (forced for both entry points): the intermediate is
    the scratch array; the second, smaller call reuses it with the first
    call's values still beyond its own size."""
    import paper_1107_4958_amd as rsg
    rsg.rsg_tune_path(rsg.RSG_PATH_TWO_PASS)         # both entry points plan the two-pass path
    try:
        for (H, W, C, seed) in ((1000, 1900, 2, 5), (300, 517, 1, 6)):
            img = synthimg.image(H, W, C, dt, seed)
            out, ref = _both(img, dt, 32.0, 4)
            _agree(out, ref, dt)
    finally:
        rsg.rsg_tune_path(rsg.RSG_PATH_AUTO)


@pytest.mark.parametrize("dt", ["u8", "f32"])
def test_two_calls_fused(dt):
    for (H, W, C, seed) in ((700, 640, 1, 7), (65, 129, 3, 8)):
        img = synthimg.image(H, W, C, dt, seed)
        out, ref = _both(img, dt, 5.0, 3, boundary=2)
        _agree(out, ref, dt)


def test_too_large_intermediate_is_refused():
    """A 4096 x 4096 x 3 FP32 image at sigma = 32 would need a 192 MiB
    intermediate: RSG_ENOMEM, nothing launched, the destination untouched."""
    import torch
    import paper_1107_4958_amd as rsg
    src = torch.zeros((4096, 4096, 3), dtype=torch.float32, device="cuda")
    dst = torch.full_like(src, 3.0)
    with pytest.raises(rsg.RsgError) as e:
        rsg.rsg_gauss_filter_noalloc(src.data_ptr(), dst.data_ptr(), 4096, 4096, 3, rsg.RSG_F32, 32.0, 4, 0,
                                     torch.cuda.current_stream().cuda_stream)
    assert e.value.code == rsg.RSG_ENOMEM and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool(torch.all(dst == 3.0))
