"""Pitched rows and unaligned window bases, through the batch entry point
(the one that takes row strides).  Each image is a window cut out of a wider
device buffer and is written into a window of another wider buffer.  A
window base that is not 16-byte aligned turns every chunk load into element
loads; an aligned base with a pitch keeps the vector loads.  The samples
around the source window hold a sentinel that would show in the result if
read, and the samples around the destination window must stay untouched.
Bars as in the other parity tests: uint8 bit-exact, FP32 1e-5 of max|ref|,
FP16 one ulp."""
import numpy as np
import pytest

import oracle
import synthimg
from gpu_util import decode, from_device, half_ulp_diff, rel_max_err, to_device

pytestmark = pytest.mark.gpu

ES = {"u8": 1, "f32": 4, "f16": 2}
NP = {"u8": np.uint8, "f32": np.float32, "f16": np.float16}
SRC_FILL = {"u8": 77, "f32": 1.0e4, "f16": 2000.0}
DST_FILL = {"u8": 171, "f32": -7.5, "f16": -3.0}

# dtype, H, W, C, source window column x0 and extra pixels, destination x1 and extra, sigma, K, boundary
CASES = [
    ("f32", 300, 257, 1, 1, 11, 3, 5, 5.0, 3, oracle.REPLICATE),      # unaligned: element loads only
    ("f32", 150, 640, 1, 4, 12, 0, 9, 8.0, 3, oracle.REFLECT),        # aligned base, pitched rows
    ("f32", 97, 130, 3, 2, 5, 1, 4, 3.0, 4, oracle.ZERO),
    ("f32", 2000, 200, 1, 1, 3, 2, 2, 2.0, 3, oracle.REPLICATE),      # tall and narrow: mostly border strips
    ("u8", 200, 333, 1, 3, 9, 5, 7, 6.0, 4, oracle.REPLICATE),
    ("u8", 129, 500, 3, 16, 20, 1, 3, 20.0, 5, oracle.REFLECT),       # wide boxes: the two-pass path
    ("u8", 64, 64, 4, 1, 1, 0, 1, 1.5, 3, oracle.ZERO),
    ("f16", 120, 300, 2, 1, 7, 3, 1, 4.0, 3, oracle.REPLICATE),
]


@pytest.mark.parametrize("dt,H,W,C,x0,pad0,x1,pad1,sigma,K,boundary", CASES)
def test_pitched_window(dt, H, W, C, x0, pad0, x1, pad1, sigma, K, boundary):
    import torch
    import paper_1107_4958_amd as rsg
    img = synthimg.image(H, W, C, dt, seed=H * 13 + W + C)
    img3 = img.reshape(H, W, C)
    Ws, Wd = W + x0 + pad0, W + x1 + pad1
    big_src = np.full((H, Ws, C), SRC_FILL[dt], dtype=NP[dt])
    big_src[:, x0:x0 + W, :] = img3
    big_dst = np.full((H, Wd, C), DST_FILL[dt], dtype=NP[dt])
    ts, td = to_device(big_src, dt), to_device(big_dst, dt)
    es = ES[dt]

    d = rsg.rsg_image_desc()
    d.src = ts.data_ptr() + x0 * C * es
    d.dst = td.data_ptr() + x1 * C * es
    d.H, d.W, d.C = H, W, C
    d.src_stride, d.dst_stride = Ws * C, Wd * C
    d.dt = rsg.tensor_dtype_code(ts)
    d.sigma, d.K, d.b = sigma, K, boundary
    d.boxes = None
    nbytes = rsg.rsg_filter_batch_workspace([d])
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device="cuda")
    rsg.rsg_filter_batch([d], ws.data_ptr(), ws.numel(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    out_big = from_device(td, dt)

    outside = np.ones((H, Wd), dtype=bool)
    outside[:, x1:x1 + W] = False
    assert np.all(out_big[outside] == NP[dt](DST_FILL[dt])), "a sample outside the destination window changed"
    out = out_big[:, x1:x1 + W, :].reshape(img.shape)

    b = oracle.boxes(sigma, K)
    if dt == "u8":
        ref = oracle.box_filter_u8(img, b["r"], b["m"], b["G"], boundary)
        assert np.array_equal(out, ref), "uint8 mismatch in %d samples" % int(np.sum(out != ref))
    elif dt == "f32":
        ref = oracle.box_filter(decode(img, dt), b["r"], b["w32"].astype(np.float64), boundary)
        e = rel_max_err(out, ref)
        assert e <= 1e-5, "FP32 rel err %.3g" % e
    else:
        ref = oracle.box_filter(decode(img, dt), b["r"], b["w32"].astype(np.float64), boundary)
        assert half_ulp_diff(out, ref, dt) <= 1


@pytest.mark.parametrize("nbytes", [16, 4096 + 7, (1 << 20) + 5, 33 << 20])
def test_stream_copy(nbytes):
    """The bandwidth reference of the benchmark copies exactly, tail bytes
    included, and leaves the bytes after the range alone."""
    import torch
    import paper_1107_4958_amd as rsg
    src = torch.randint(0, 256, (nbytes + 64,), dtype=torch.uint8, device="cuda")
    dst = torch.zeros(nbytes + 64, dtype=torch.uint8, device="cuda")
    rsg.rsg_stream_copy(src.data_ptr(), dst.data_ptr(), nbytes, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes], src[:nbytes])
    assert int(dst[nbytes:].sum()) == 0
