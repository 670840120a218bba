"""The fused kernel's wide column form (rsg_tune_columns > 1): each lane owns
two adjacent columns at C = 1 (strips of 128 samples) and one pixel's three
channels at C = 3 (strips of 64 pixels).  Same bars as the other parity
tests (uint8 bit-exact against the exact-integer oracle; FP32 max|err| /
max|oracle| <= 1e-5; FP16 / BF16 one ulp), on ragged shapes whose last lane
holds only part of its columns, on pitched and unaligned destinations (which
turn the lanes' vector stores into element stores), through the batch, the
stacked-slice volume launch, and on the full 4096 x 4096 image."""
import numpy as np
import pytest

import oracle
import synthimg
import test_gpu_parity as par
import test_gpu_pitch as pitch
from gpu_util import from_device, gpu_filter, rel_max_err, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def wide_columns():
    import paper_1107_4958_amd as rsg
    rsg.rsg_tune_columns(2)
    yield
    rsg.rsg_tune_columns(0)


# (H, W, C, sigma, K): odd widths leave the last lane of a C = 1 row with one
# live column; 3-channel rows of every residue; boxes wider than the image
WIDE_SHAPES = [
    (1, 1, 1, 2.0, 3), (1, 129, 1, 1.0, 3), (5, 3, 1, 8.0, 5), (17, 301, 1, 5.0, 3),
    (65, 127, 1, 3.0, 2), (200, 333, 1, 8.0, 3), (33, 521, 1, 0.5, 5), (129, 1001, 1, 12.0, 4),
    (61, 211, 3, 6.0, 5), (130, 77, 3, 20.0, 4), (40, 64, 3, 2.0, 3), (7, 65, 3, 4.0, 3),
]


@pytest.mark.parametrize("dtype", ["f32", "u8"])
@pytest.mark.parametrize("boundary", [oracle.REPLICATE, oracle.ZERO, oracle.REFLECT])
@pytest.mark.parametrize("H,W,C,sigma,K", WIDE_SHAPES)
def test_wide_parity(dtype, boundary, H, W, C, sigma, K):
    img = synthimg.image(H, W, C, dtype, seed=H * 29 + W)
    par._check(img, dtype, sigma, K, boundary)


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
@pytest.mark.parametrize("H,W,C,sigma,K", WIDE_SHAPES[1::2])
def test_wide_half_formats(dtype, H, W, C, sigma, K):
    img = synthimg.image(H, W, C, dtype, seed=H * 5 + W)
    par._check(img, dtype, sigma, K, oracle.ZERO if W % 2 else oracle.REPLICATE)


@pytest.mark.parametrize("dtype", ["u8", "f32"])
@pytest.mark.parametrize("H,W,C,sigma,K", [(300, 1001, 1, 6.0, 4), (257, 300, 3, 9.0, 3)])
def test_wide_agrees_with_one_column(dtype, H, W, C, sigma, K):
    """uint8 results are bit-identical to the one-column form's; FP32 ones
    agree to rounding."""
    import paper_1107_4958_amd as rsg
    img = synthimg.image(H, W, C, dtype, seed=3)
    a = gpu_filter(img, dtype, sigma, K)
    rsg.rsg_tune_columns(1)
    b = gpu_filter(img, dtype, sigma, K)
    if dtype == "u8":
        assert np.array_equal(a, b)
    else:
        assert rel_max_err(a, b.astype(np.float64)) <= 2e-6


@pytest.mark.parametrize("case", [c for c in pitch.CASES if c[3] in (1, 3)] + [
    ("u8", 90, 301, 1, 0, 3, 1, 2, 4.0, 3, oracle.REPLICATE),       # odd destination base: byte stores
    ("u8", 90, 300, 1, 0, 4, 2, 6, 4.0, 3, oracle.ZERO),            # even base and pitch: 2-byte stores
    ("f16", 60, 257, 1, 3, 1, 1, 4, 2.0, 4, oracle.REFLECT),        # 2-byte aligned base: element stores
    ("f16", 60, 256, 1, 0, 0, 2, 2, 2.0, 4, oracle.REPLICATE),      # 4-byte aligned: 4-byte stores
])
def test_wide_pitched_window(case):
    pitch.test_pitched_window(*case)


def test_wide_batch_identical_to_alone():
    """A batch of C = 1 and C = 3 images (uint8 and FP32) under the wide form:
    every image bit-identical to filtering it alone."""
    import torch
    import paper_1107_4958_amd as rsg
    specs = [(37, 523, 3, "u8", 7.5, 4), (300, 17, 1, "f32", 5.0, 3), (129, 1001, 1, "f32", 12.0, 5),
             (513, 127, 1, "u8", 0.7, 2), (1024, 768, 3, "u8", 3.0, 4), (5, 3000, 1, "f32", 1.0, 1),
             (200, 199, 1, "u8", 9.0, 3)]
    imgs = [synthimg.crop_pool(H, W, C, dt, 80 + i) for i, (H, W, C, dt, _, _) in enumerate(specs)]
    srcs = [to_device(im, s[3]) for im, s in zip(imgs, specs)]
    dsts = [torch.empty_like(s) for s in srcs]
    rsg.filter_batch_tensors(srcs, dsts, [s[4] for s in specs], [s[5] for s in specs])
    torch.cuda.synchronize()
    for i, s in enumerate(specs):
        alone = rsg.filter_tensor(srcs[i], s[4], s[5])
        torch.cuda.synchronize()
        assert np.array_equal(from_device(dsts[i], s[3]), from_device(alone, s[3])), i


@pytest.mark.parametrize("D,H,W,C", [(5, 7, 9, 1), (17, 33, 201, 1), (9, 30, 65, 3)])
@pytest.mark.parametrize("boundary", [oracle.REPLICATE, oracle.ZERO])
def test_wide_volume(D, H, W, C, boundary):
    rng = np.random.default_rng(D * 11 + W)
    vol = rng.uniform(0, 255, size=(D, H, W, C) if C > 1 else (D, H, W)).astype(np.float32)
    b = oracle.boxes(4.0, 4)
    out = par._volume_gpu(vol, 4.0, 4, boundary)
    ref = oracle.box_filter_3d(vol.astype(np.float64), b["r"], b["w32"].astype(np.float64), boundary)
    assert rel_max_err(out, ref) <= par.FP32_TOL


@pytest.mark.parametrize("dtype", ["f32", "u8"])
def test_wide_full_image_4096(dtype):
    """4096 x 4096, sigma 8, K 3, replicate: the whole image."""
    img = synthimg.image(4096, 4096, 1, dtype, seed=2)
    par._check(img, dtype, 8.0, 3, oracle.REPLICATE)
