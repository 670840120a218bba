"""Channel-planar tasks (rsg_tune_columns(3)): each task filters 64 pixels of
one channel of a multi-channel image with the one-channel kernel, reading
and writing its samples C apart.  Same bars as the other parity tests
(uint8 bit-exact against the exact-integer oracle; FP32 max|err| /
max|oracle| <= 1e-5; FP16 / BF16 one ulp), on ragged shapes of every
channel count, every boundary, pitched and unaligned windows, through the
batch and the server's batched launch, against the interleaved form, and on
a full 2048 x 2048 three-channel image."""
import numpy as np
import pytest

import oracle
import synthimg
import test_gpu_parity as par
import test_gpu_pitch as pitch
from gpu_util import from_device, gpu_filter, rel_max_err, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def planar_tasks():
    import paper_1107_4958_amd as rsg
    rsg.rsg_tune_columns(3)
    yield
    rsg.rsg_tune_columns(0)


PLANAR_SHAPES = [
    (1, 1, 2, 2.0, 3), (3, 5, 3, 8.0, 5), (17, 65, 3, 5.0, 3), (97, 250, 2, 4.0, 4),
    (61, 211, 3, 6.0, 5), (70, 90, 4, 2.5, 3), (130, 77, 3, 20.0, 4), (40, 130, 4, 9.0, 3),
    (33, 129, 3, 0.5, 5), (200, 333, 2, 12.0, 3),
]


@pytest.mark.parametrize("dtype", ["f32", "u8"])
@pytest.mark.parametrize("boundary", [oracle.REPLICATE, oracle.ZERO, oracle.REFLECT])
@pytest.mark.parametrize("H,W,C,sigma,K", PLANAR_SHAPES)
def test_planar_parity(dtype, boundary, H, W, C, sigma, K):
    img = synthimg.image(H, W, C, dtype, seed=H * 17 + W + C)
    par._check(img, dtype, sigma, K, boundary)


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
@pytest.mark.parametrize("H,W,C,sigma,K", PLANAR_SHAPES[1::2])
def test_planar_half_formats(dtype, H, W, C, sigma, K):
    img = synthimg.image(H, W, C, dtype, seed=H * 3 + W)
    par._check(img, dtype, sigma, K, oracle.ZERO if W % 2 else oracle.REPLICATE)


@pytest.mark.parametrize("dtype", ["u8", "f32"])
@pytest.mark.parametrize("H,W,C,sigma,K", [(300, 301, 3, 6.0, 4), (257, 300, 2, 9.0, 3), (129, 200, 4, 3.0, 5)])
def test_planar_agrees_with_interleaved(dtype, H, W, C, sigma, K):
    """uint8 results are bit-identical to the interleaved tasks'; FP32 ones
    agree to rounding."""
    import paper_1107_4958_amd as rsg
    img = synthimg.image(H, W, C, dtype, seed=5)
    a = gpu_filter(img, dtype, sigma, K)
    rsg.rsg_tune_columns(1)
    b = gpu_filter(img, dtype, sigma, K)
    if dtype == "u8":
        assert np.array_equal(a, b)
    else:
        assert rel_max_err(a, b.astype(np.float64)) <= 2e-6


@pytest.mark.parametrize("case", [c for c in pitch.CASES if c[3] >= 2])
def test_planar_pitched_window(case):
    pitch.test_pitched_window(*case)


def test_planar_batch_identical_to_alone():
    """A batch mixing one- and multi-channel images of every dtype: every
    image bit-identical to filtering it alone under the same plan."""
    import torch
    import paper_1107_4958_amd as rsg
    specs = [(37, 523, 3, "u8", 7.5, 4), (300, 17, 1, "f32", 5.0, 3), (129, 1001, 4, "f32", 12.0, 5),
             (513, 127, 2, "u8", 0.7, 2), (1024, 768, 3, "u8", 3.0, 4), (61, 211, 3, "f16", 6.0, 5),
             (70, 90, 4, "bf16", 2.5, 3), (200, 199, 3, "f32", 9.0, 3)]
    imgs = [synthimg.crop_pool(H, W, C, dt, 90 + i) for i, (H, W, C, dt, _, _) in enumerate(specs)]
    srcs = [to_device(im, s[3]) for im, s in zip(imgs, specs)]
    dsts = [torch.empty_like(s) for s in srcs]
    rsg.filter_batch_tensors(srcs, dsts, [s[4] for s in specs], [s[5] for s in specs])
    torch.cuda.synchronize()
    for i, s in enumerate(specs):
        alone = rsg.filter_tensor(srcs[i], s[4], s[5])
        torch.cuda.synchronize()
        assert np.array_equal(from_device(dsts[i], s[3]), from_device(alone, s[3])), i


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_planar_full_image_2048_c3(dtype):
    """2048 x 2048 x 3, sigma 8, K 4, replicate: the whole image."""
    img = synthimg.image(2048, 2048, 3, dtype, seed=4)
    par._check(img, dtype, 8.0, 4, oracle.REPLICATE)


def test_planar_volume_keeps_interleaved_tasks():
    """Volumes take the slice index for the stack, so they keep interleaved
    tasks under the planar setting (results as the oracle's)."""
    D, H, W, C = 9, 30, 65, 3
    rng = np.random.default_rng(3)
    vol = rng.uniform(0, 255, size=(D, H, W, C)).astype(np.float32)
    b = oracle.boxes(4.0, 4)
    out = par._volume_gpu(vol, 4.0, 4, oracle.REPLICATE)
    ref = oracle.box_filter_3d(vol.astype(np.float64), b["r"], b["w32"].astype(np.float64), oracle.REPLICATE)
    assert rel_max_err(out, ref) <= par.FP32_TOL


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_planar_fallback_for_boxes_too_wide_otherwise(dtype):
    """C = 4, sigma 64: neither the interleaved span nor the two-pass window
    holds the boxes; channel-planar tasks do (sampled against the oracle)."""
    import paper_1107_4958_amd as rsg
    rsg.rsg_tune_columns(0)
    H, W, C = 300, 420, 4
    img = synthimg.image(H, W, C, dtype, seed=11)
    par._check(img, dtype, 64.0, 5, oracle.REPLICATE)
