"""Staged stores of the cooperative fused kernel: FP32 images planned with
them (the tuning table's store form, rsg_tune_stores, else four or five
taps), whose interior tasks write 16-byte-aligned output rows, stage each
wave's 8 x 64 results in LDS and store them as 16-byte row pieces.  Checked
against the oracle (FP32 max|err| / max|oracle| <= 1e-5) on ragged heights
(tasks that end inside a wave's block), single rows, several channels and a
large image element by element; bit-identical to the per-lane stores that a
destination without 16-byte alignment takes; and, through pitched windows,
no sample outside the destination window written."""
import numpy as np
import pytest

import oracle
import synthimg
import test_gpu_parity as par
import test_gpu_pitch as pitch
from gpu_util import from_device, to_device

pytestmark = pytest.mark.gpu

# (H, W, C, sigma, K): many interior strips; heights that are not multiples
# of the 32-row step
STAGED_SHAPES = [
    (1, 700, 1, 2.0, 4), (9, 513, 1, 3.0, 5), (203, 1000, 1, 5.0, 4), (77, 640, 3, 2.0, 5),
    (130, 900, 2, 4.0, 4), (300, 2048, 1, 8.0, 5), (65, 300, 4, 1.0, 4),
]


@pytest.mark.parametrize("boundary", [oracle.REPLICATE, oracle.REFLECT])
@pytest.mark.parametrize("H,W,C,sigma,K", STAGED_SHAPES)
def test_staged_parity(boundary, H, W, C, sigma, K):
    img = synthimg.image(H, W, C, "f32", seed=H * 31 + W + K)
    par._check(img, "f32", sigma, K, boundary)


@pytest.mark.parametrize("K", [4, 5])
def test_staged_full_image(K):
    """1024 x 4096, sigma 8, every sample against the oracle."""
    img = synthimg.image(1024, 4096, 1, "f32", seed=40 + K)
    par._check(img, "f32", 8.0, K, oracle.REPLICATE)


@pytest.mark.parametrize("H,W,C,sigma,K", [(203, 1000, 1, 5.0, 4), (77, 640, 3, 2.0, 5), (300, 2048, 1, 8.0, 5)])
def test_staged_identical_to_lane_stores(H, W, C, sigma, K):
    """The same image into an aligned destination (staged stores) and into
    one 4 bytes past alignment (per-lane stores): bit-identical."""
    import torch
    import paper_1107_4958_amd as rsg
    img = synthimg.image(H, W, C, "f32", seed=H + W)
    src = to_device(img, "f32")
    outs = []
    for shift in (0, 1):
        big = torch.zeros(H * W * C + 4, dtype=torch.float32, device="cuda")
        d = rsg.rsg_image_desc()
        d.src = src.data_ptr()
        d.dst = big.data_ptr() + 4 * shift
        d.H, d.W, d.C = H, W, C
        d.src_stride, d.dst_stride = W * C, W * C
        d.dt = rsg.RSG_F32
        d.sigma, d.K, d.b = sigma, K, oracle.REPLICATE
        d.boxes = None
        nbytes = rsg.rsg_filter_batch_workspace([d])
        ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device="cuda")
        rsg.rsg_filter_batch([d], ws.data_ptr(), ws.numel(), torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        outs.append(from_device(big, "f32")[shift:shift + H * W * C])
    assert np.array_equal(outs[0].view(np.uint32), outs[1].view(np.uint32))


@pytest.mark.parametrize("case", [
    ("f32", 150, 640, 1, 4, 12, 0, 12, 4.0, 4, oracle.REPLICATE),    # pitched, aligned: staged
    ("f32", 90, 520, 1, 0, 8, 4, 4, 3.0, 5, oracle.REFLECT),         # base 16 bytes in: staged
    ("f32", 90, 520, 1, 0, 8, 2, 6, 3.0, 5, oracle.REPLICATE),       # base 8 bytes in: lane stores
    ("f32", 60, 400, 3, 4, 4, 0, 4, 2.0, 4, oracle.REPLICATE),       # 3 channels, pitched: staged
])
def test_staged_pitched_window(case):
    pitch.test_pitched_window(*case)


def test_staged_batch_identical_to_alone():
    """FP32 images with three, four and five taps in one batch, each
    bit-identical to filtering it alone."""
    import torch
    import paper_1107_4958_amd as rsg
    specs = [(203, 1000, 1, 5.0, 4), (77, 640, 3, 2.0, 5), (300, 517, 1, 8.0, 3), (64, 4096, 1, 1.5, 5),
             (500, 300, 2, 3.0, 4)]
    imgs = [synthimg.image(H, W, C, "f32", 90 + i) for i, (H, W, C, _, _) in enumerate(specs)]
    srcs = [to_device(im, "f32") for im in imgs]
    dsts = [torch.empty_like(s) for s in srcs]
    rsg.filter_batch_tensors(srcs, dsts, [s[3] for s in specs], [s[4] for s in specs])
    torch.cuda.synchronize()
    for i, s in enumerate(specs):
        alone = rsg.filter_tensor(srcs[i], s[3], s[4])
        torch.cuda.synchronize()
        assert np.array_equal(from_device(dsts[i], "f32").view(np.uint32), from_device(alone, "f32").view(np.uint32)), i


@pytest.mark.parametrize("H,W,C,sigma,K", [(203, 1000, 1, 5.0, 3), (77, 640, 3, 2.0, 3), (300, 2048, 1, 8.0, 5),
                                           (100, 777, 2, 3.0, 4)])
def test_forced_store_forms(H, W, C, sigma, K):
    """rsg_tune_stores(2) (staged, three taps included) against the oracle,
    and bit-identical to rsg_tune_stores(1) (one store per lane and row)."""
    import paper_1107_4958_amd as rsg
    from gpu_util import gpu_filter
    img = synthimg.image(H, W, C, "f32", seed=H * 3 + K)
    outs = []
    try:
        for form in (2, 1):
            rsg.rsg_tune_stores(form)
            if form == 2:
                par._check(img, "f32", sigma, K, oracle.REPLICATE)
            outs.append(gpu_filter(img, "f32", sigma, K))
    finally:
        rsg.rsg_tune_stores(0)
    assert np.array_equal(outs[0].view(np.uint32), outs[1].view(np.uint32))
