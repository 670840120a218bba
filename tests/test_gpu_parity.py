"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bars: uint8 bit-exact against the exact-integer oracle; FP32 max|err| /
max|ref| <= 1e-5 against the FP64 oracle run with the same FP32 weights;
FP16 / BF16 within one unit in the last place of the oracle's FP64 result
rounded to the storage format (FP32 accumulation error is far below half an
ulp of the output, so only ties decided by it can differ)."""
import numpy as np
import pytest

import oracle
import synthimg
from gpu_util import decode, from_device, gpu_filter, half_ulp_diff, rel_max_err, to_device

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5


def _check(img, dtype, sigma, K, boundary):
    b = oracle.boxes(sigma, K)
    out = gpu_filter(img, dtype, sigma, K, boundary)
    if dtype == "u8":
        ref = oracle.box_filter_u8(img, b["r"], b["m"], b["G"], boundary)
        bad = np.argwhere(out != ref)
        assert bad.size == 0, "uint8 mismatch at %s: gpu %s oracle %s" % (
            bad[:3].tolist(), out[tuple(bad[0])], ref[tuple(bad[0])])
        return 0.0
    ref = oracle.box_filter(decode(img, dtype), b["r"], b["w32"].astype(np.float64), boundary)
    if dtype == "f32":
        e = rel_max_err(out, ref)
        assert e <= FP32_TOL, "FP32 rel err %.3g" % e
        return e
    d = half_ulp_diff(out, ref, dtype)
    assert d <= 1, "%s differs by %d ulp" % (dtype, d)
    return d


# (H, W, C, sigma, K): ragged sizes, boxes wider than the image, every C and K
SHAPES = [
    (1, 1, 1, 2.0, 3), (1, 37, 1, 1.0, 3), (41, 1, 1, 1.5, 4), (3, 5, 1, 8.0, 5),
    (17, 300, 1, 5.0, 3), (300, 17, 1, 5.0, 3), (64, 64, 1, 2.0, 1), (65, 129, 1, 3.0, 2),
    (200, 333, 1, 8.0, 3), (97, 250, 2, 4.0, 4), (61, 211, 3, 6.0, 5), (70, 90, 4, 2.5, 3),
    (130, 77, 3, 20.0, 4), (257, 259, 1, 32.0, 5), (33, 520, 1, 0.5, 5), (129, 1000, 1, 12.0, 3),
]


@pytest.mark.parametrize("dtype", ["f32", "u8"])
@pytest.mark.parametrize("boundary", [oracle.REPLICATE, oracle.ZERO, oracle.REFLECT])
@pytest.mark.parametrize("H,W,C,sigma,K", SHAPES)
def test_parity_shapes(dtype, boundary, H, W, C, sigma, K):
    img = synthimg.image(H, W, C, dtype, seed=H * 31 + W)
    _check(img, dtype, sigma, K, boundary)


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
@pytest.mark.parametrize("H,W,C,sigma,K", SHAPES[::2])
def test_parity_half_formats(dtype, H, W, C, sigma, K):
    img = synthimg.image(H, W, C, dtype, seed=H * 7 + W)
    _check(img, dtype, sigma, K, oracle.REPLICATE)


@pytest.mark.parametrize("dtype", ["f32", "u8", "f16", "bf16"])
def test_plain_method_512(dtype):
    """512 x 512 single channel, sigma 5, K 3, replicate: the whole image."""
    img = synthimg.image(512, 512, 1, dtype, seed=1)
    _check(img, dtype, 5.0, 3, oracle.REPLICATE)


@pytest.mark.parametrize("sigma,K", [(2.0, 3), (8.0, 4), (32.0, 5), (64.0, 5)])
def test_u8_constant_and_impulse(sigma, K):
    b = oracle.boxes(sigma, K)
    for v in (0, 1, 128, 255):
        img = np.full((150, 190), v, dtype=np.uint8)
        assert np.all(gpu_filter(img, "u8", sigma, K) == v)
    n = 2 * int(b["r"].max()) + 9
    img = np.zeros((n, n + 3), dtype=np.uint8)
    img[n // 2, n // 2] = 255
    out = gpu_filter(img, "u8", sigma, K, oracle.ZERO)
    ref = oracle.box_filter_u8(img, b["r"], b["m"], b["G"], oracle.ZERO)
    assert np.array_equal(out, ref)


def test_row_then_column_equals_transposed_u8():
    img = synthimg.image(300, 211, 1, "u8", seed=5)
    a = gpu_filter(img, "u8", 6.0, 4)
    t = gpu_filter(np.ascontiguousarray(img.T), "u8", 6.0, 4).T
    assert np.array_equal(a, t)


def test_deterministic_repeat():
    img = synthimg.image(700, 900, 1, "f32", seed=8)
    a = gpu_filter(img, "f32", 8.0, 3)
    b = gpu_filter(img, "f32", 8.0, 3)
    assert np.array_equal(a, b)


# --------------------------------------------------------------------------
# Full-size configurations: sampled outputs computed one by one by the oracle
# --------------------------------------------------------------------------
def _sample_points(H, W, C, n, seed):
    rng = np.random.default_rng(seed)
    ys = list(rng.integers(0, H, n))
    xs = list(rng.integers(0, W, n))
    # corners and edges
    for y in (0, 1, 7, 23, H // 2, H - 24, H - 8, H - 2, H - 1):
        for x in (0, 1, 7, 23, W // 2, W - 24, W - 8, W - 2, W - 1):
            ys.append(max(0, y))
            xs.append(max(0, x))
    ys = np.array(ys) % H
    xs = np.array(xs) % W
    cs = rng.integers(0, C, len(ys))
    return ys, xs, cs


def _sampled_check(H, W, C, dtype, sigma, K, npts=1500, seed=0, boundary=oracle.REPLICATE):
    b = oracle.boxes(sigma, K)
    img = synthimg.image(H, W, C, dtype, seed=seed)
    out = gpu_filter(img, dtype, sigma, K, boundary)
    if out.ndim == 2:
        out = out[..., None]
    img3 = img if img.ndim == 3 else img[..., None]
    ys, xs, cs = _sample_points(H, W, C, npts, seed + 1)
    if dtype == "u8":
        ref = oracle.box_filter_u8_points(img3, b["r"], b["m"], b["G"], ys, xs, cs, boundary=boundary)
        got = out[ys, xs, cs]
        assert np.array_equal(got, ref), "uint8 sampled mismatch"
        return
    ref = oracle.box_filter_points(decode(img3, dtype), b["r"], b["w32"].astype(np.float64), ys, xs, cs,
                                   boundary=boundary)
    got = out[ys, xs, cs]
    if dtype == "f32":
        assert rel_max_err(got, ref) <= FP32_TOL
    else:
        assert half_ulp_diff(got, ref, dtype) <= 1


@pytest.mark.parametrize("dtype", ["f32", "u8"])
@pytest.mark.parametrize("sigma", [2.0, 8.0, 32.0])
@pytest.mark.parametrize("K", [3, 4, 5])
def test_at_scale_4096(dtype, sigma, K):
    _sampled_check(4096, 4096, 1, dtype, sigma, K, npts=800, seed=2)


@pytest.mark.parametrize("dtype", ["f32", "u8"])
@pytest.mark.parametrize("sigma", [8.0, 32.0])
def test_at_scale_4096_reflect(dtype, sigma):
    _sampled_check(4096, 4096, 1, dtype, sigma, 3, npts=800, seed=3, boundary=oracle.REFLECT)


@pytest.mark.parametrize("dtype", ["f32", "u8", "f16", "bf16"])
@pytest.mark.parametrize("sigma", [4.0, 64.0])
def test_precision_8192(dtype, sigma):
    _sampled_check(8192, 8192, 1, dtype, sigma, 5, npts=500, seed=4)


@pytest.mark.parametrize("dtype,H,W,C,sigma,K", [("u8", 300, 517, 3, 5.0, 4), ("f32", 700, 300, 1, 12.0, 5),
                                                 ("u8", 90, 1100, 1, 30.0, 3)])
def test_any_segment_height_gives_the_oracle(dtype, H, W, C, sigma, K):
    """The segment height only changes how rows are split into tasks: every
    height (1, ragged, one task per strip) must match the oracle."""
    import paper_1107_4958_amd as rsg
    img = synthimg.image(H, W, C, dtype, 31)
    try:
        for hs in (1, 7, 64, 333, 100000):
            rsg.rsg_tune_override(hs)
            _check(img, dtype, sigma, K, oracle.REPLICATE)
    finally:
        rsg.rsg_tune_override(0)


TWO_PASS_SHAPES = [
    (1, 1, 1, 2.0, 3, 0), (5, 3, 1, 8.0, 5, 1), (1, 300, 1, 3.0, 3, 0), (300, 1, 1, 3.0, 4, 1),
    (97, 250, 2, 4.0, 4, 0), (61, 211, 3, 6.0, 5, 1), (200, 333, 1, 8.0, 3, 0), (130, 77, 3, 20.0, 4, 0),
    (257, 259, 1, 32.0, 5, 1), (700, 300, 1, 12.0, 5, 0), (1000, 129, 1, 40.0, 3, 0), (33, 2000, 4, 5.0, 3, 1),
    (520, 1030, 1, 64.0, 5, 0), (64, 64, 1, 1.0, 1, 0),
    # reflect: boxes many times wider than the axis, and every channel count
    (5, 3, 1, 8.0, 5, 2), (300, 1, 1, 3.0, 4, 2), (61, 211, 3, 6.0, 5, 2), (257, 259, 1, 32.0, 5, 2),
    (33, 2000, 4, 5.0, 3, 2), (97, 250, 2, 4.0, 4, 2),
    # windows too wide for 16-row workgroups: pass A runs 8 rows per workgroup
    (130, 300, 3, 64.0, 5, 0), (97, 520, 4, 40.0, 4, 2), (400, 90, 2, 64.0, 5, 1),
]


@pytest.mark.parametrize("dtype", ["u8", "f32", "f16", "bf16"])
@pytest.mark.parametrize("H,W,C,sigma,K,boundary", TWO_PASS_SHAPES)
def test_two_pass_path(dtype, H, W, C, sigma, K, boundary):
    """The two-pass path (row filter into a transposed intermediate, twice)
    forced on every shape: uint8 bit-exact, floats within the same bars."""
    import paper_1107_4958_amd as rsg
    img = synthimg.image(H, W, C, dtype, 41)
    rsg.rsg_tune_path(rsg.RSG_PATH_TWO_PASS)
    try:
        _check(img, dtype, sigma, K, boundary)
    finally:
        rsg.rsg_tune_path(rsg.RSG_PATH_AUTO)


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_paths_agree(dtype):
    """Fused and two-pass results of one image: identical for uint8, within
    the FP32 bar for floats."""
    import paper_1107_4958_amd as rsg
    img = synthimg.image(384, 700, 3, dtype, 43)
    outs = []
    for path in (rsg.RSG_PATH_FUSED, rsg.RSG_PATH_TWO_PASS):
        rsg.rsg_tune_path(path)
        try:
            outs.append(gpu_filter(img, dtype, 16.0, 4, 0))
        finally:
            rsg.rsg_tune_path(rsg.RSG_PATH_AUTO)
    if dtype == "u8":
        assert np.array_equal(outs[0], outs[1])
    else:
        assert rel_max_err(outs[1], outs[0].astype(np.float64)) <= FP32_TOL


@pytest.mark.parametrize("dtype", ["u8", "f32"])
@pytest.mark.parametrize("H,W,C,sigma,K,boundary", [(200, 333, 1, 8.0, 3, 0), (97, 250, 2, 4.0, 4, 1),
                                                    (61, 211, 3, 6.0, 5, 0), (33, 520, 1, 0.5, 5, 1),
                                                    (70, 90, 4, 2.5, 3, 2), (130, 77, 3, 20.0, 4, 2)])
def test_one_wave_fused_form(dtype, H, W, C, sigma, K, boundary):
    """The fused kernel with one wave per task (the form batched launches
    run) forced for single images."""
    import paper_1107_4958_amd as rsg
    img = synthimg.image(H, W, C, dtype, 47)
    rsg.rsg_tune_path(rsg.RSG_PATH_FUSED_ONE_WAVE)
    try:
        _check(img, dtype, sigma, K, boundary)
    finally:
        rsg.rsg_tune_path(rsg.RSG_PATH_AUTO)


# --------------------------------------------------------------------------
# Other fit methods: the direct fit at sigma and the l2 fit, through
# rsg_box_filter, against the oracle's own fit of the same method
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["u8", "f32"])
@pytest.mark.parametrize("method,sigma,K", [("direct", 0.5, 5), ("direct", 1.0, 3), ("direct", 2.5, 4),
                                            ("direct", 6.0, 5), ("l2", 2.0, 3), ("l2", 9.0, 5)])
@pytest.mark.parametrize("H,W,C,boundary", [(130, 77, 3, 0), (257, 259, 1, 2), (33, 520, 2, 1)])
def test_fit_methods_filter(dtype, method, sigma, K, H, W, C, boundary):
    import paper_1107_4958_amd as rsg
    img = synthimg.image(H, W, C, dtype, 53)
    if method == "direct":
        b = rsg.rsg_fit_boxes_ex(sigma, K, rsg.RSG_FIT_DIRECT)
        o = oracle.boxes_direct(sigma, K)
    else:
        b = rsg.rsg_fit_boxes_ex(sigma, K, rsg.RSG_FIT_SCALED_L2)
        o = oracle.boxes(sigma, K, use_qf=False)
    out = gpu_filter(img, dtype, sigma, K, boundary, boxes=b)
    if dtype == "u8":
        if o["m"] is None:
            pytest.skip("no integer weights for these boxes")
        ref = oracle.box_filter_u8(img, o["r"], o["m"], o["G"], boundary)
        assert np.array_equal(out, ref)
    else:
        ref = oracle.box_filter(decode(img, dtype), o["r"], o["w32"].astype(np.float64), boundary)
        assert rel_max_err(out, ref) <= FP32_TOL


# --------------------------------------------------------------------------
# Strided (downsampling) evaluation: every step-th row and pixel
# --------------------------------------------------------------------------
STRIDED = [
    (1, 1, 1, 2.0, 3, 0, 2), (7, 5, 1, 1.5, 3, 0, 3), (257, 259, 1, 8.0, 5, 1, 2), (130, 77, 3, 6.0, 4, 2, 3),
    (97, 250, 2, 4.0, 4, 0, 4), (33, 2000, 4, 5.0, 3, 0, 7), (300, 17, 1, 20.0, 5, 0, 16), (64, 64, 1, 3.0, 3, 0, 100),
    (200, 333, 1, 8.0, 3, 2, 1),
]


def _strided_gpu(img, dtype, sigma, K, boundary, step, boxes=None):
    import torch
    import paper_1107_4958_amd as rsg
    src = to_device(img, dtype)
    out = rsg.filter_strided_tensor(src, sigma, K, step, boundary, boxes=boxes)
    torch.cuda.synchronize()
    return from_device(out, dtype)


@pytest.mark.parametrize("dtype", ["u8", "f32", "f16"])
@pytest.mark.parametrize("H,W,C,sigma,K,boundary,step", STRIDED)
def test_strided_output(dtype, H, W, C, sigma, K, boundary, step):
    img = synthimg.image(H, W, C, dtype, 59)
    out = _strided_gpu(img, dtype, sigma, K, boundary, step)
    b = oracle.boxes(sigma, K)
    if dtype == "u8":
        ref = oracle.box_filter_u8(img, b["r"], b["m"], b["G"], boundary)[::step, ::step]
        assert out.shape == ref.shape and np.array_equal(out, ref)
        return
    ref = oracle.box_filter(decode(img, dtype), b["r"], b["w32"].astype(np.float64), boundary)[::step, ::step]
    assert out.shape == ref.shape
    if dtype == "f32":
        assert rel_max_err(out, ref) <= FP32_TOL
    else:
        assert half_ulp_diff(out, ref, dtype) <= 1


def test_strided_step1_and_direct_boxes():
    """step = 1 reproduces the single-image result (uint8: bit for bit), and
    caller boxes pass through."""
    import paper_1107_4958_amd as rsg
    img = synthimg.image(211, 190, 3, "u8", 61)
    assert np.array_equal(_strided_gpu(img, "u8", 7.0, 4, 0, 1), gpu_filter(img, "u8", 7.0, 4, 0))
    b = rsg.rsg_fit_boxes_ex(1.2, 4, rsg.RSG_FIT_DIRECT)
    o = oracle.boxes_direct(1.2, 4)
    out = _strided_gpu(img, "u8", 0.0, 0, 2, 3, boxes=b)
    assert np.array_equal(out, oracle.box_filter_u8(img, o["r"], o["m"], o["G"], 2)[::3, ::3])


@pytest.mark.parametrize("dtype,step", [("f32", 2), ("u8", 4)])
def test_strided_at_scale_4096(dtype, step):
    b = oracle.boxes(8.0, 3)
    img = synthimg.image(4096, 4096, 1, dtype, seed=2)
    out = _strided_gpu(img, dtype, 8.0, 3, 0, step)
    Ho, Wo = out.shape
    ys, xs, _ = _sample_points(Ho, Wo, 1, 800, 5)
    img3 = img[..., None]
    cs = np.zeros_like(ys)
    if dtype == "u8":
        ref = oracle.box_filter_u8_points(img3, b["r"], b["m"], b["G"], ys * step, xs * step, cs)
        assert np.array_equal(out[ys, xs], ref)
    else:
        ref = oracle.box_filter_points(img3.astype(np.float64), b["r"], b["w32"].astype(np.float64),
                                       ys * step, xs * step, cs)
        assert rel_max_err(out[ys, xs], ref) <= FP32_TOL


# --------------------------------------------------------------------------
# Volumes: x, y per slice, then z
# --------------------------------------------------------------------------
VOLUMES = [(1, 1, 1, 1), (5, 7, 9, 1), (17, 33, 20, 2), (40, 64, 65, 3), (9, 3, 300, 4), (130, 17, 19, 1)]


def _volume_gpu(vol, sigma, K, boundary, boxes=None):
    import torch
    import paper_1107_4958_amd as rsg
    src = torch.from_numpy(np.ascontiguousarray(vol, dtype=np.float32)).cuda()
    out = rsg.filter_volume_tensor(src, sigma, K, boundary, boxes=boxes)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("D,H,W,C", VOLUMES)
@pytest.mark.parametrize("boundary", [oracle.REPLICATE, oracle.ZERO, oracle.REFLECT])
@pytest.mark.parametrize("sigma,K", [(1.5, 3), (4.0, 5), (12.0, 4)])
def test_volume_parity(D, H, W, C, boundary, sigma, K):
    rng = np.random.default_rng(D * 7 + H * 3 + W + C)
    vol = rng.uniform(0, 255, size=(D, H, W, C) if C > 1 else (D, H, W)).astype(np.float32)
    b = oracle.boxes(sigma, K)
    out = _volume_gpu(vol, sigma, K, boundary)
    ref = oracle.box_filter_3d(vol.astype(np.float64), b["r"], b["w32"].astype(np.float64), boundary)
    assert rel_max_err(out, ref) <= FP32_TOL


def test_volume_at_size_and_direct_boxes():
    """A 96 x 160 x 200 one-over-f stack, every voxel; and the direct fit at
    small sigma passed as boxes."""
    import paper_1107_4958_amd as rsg
    vol = np.stack([synthimg.image(160, 200, 1, "f32", 70 + z) for z in range(96)])
    b = oracle.boxes(3.0, 3)
    out = _volume_gpu(vol, 3.0, 3, oracle.REPLICATE)
    ref = oracle.box_filter_3d(vol.astype(np.float64), b["r"], b["w32"].astype(np.float64))
    assert rel_max_err(out, ref) <= FP32_TOL
    bd = rsg.rsg_fit_boxes_ex(0.9, 3, rsg.RSG_FIT_DIRECT)
    o = oracle.boxes_direct(0.9, 3)
    out = _volume_gpu(vol[:20], 0.0, 0, oracle.REFLECT, boxes=bd)
    ref = oracle.box_filter_3d(vol[:20].astype(np.float64), o["r"], o["w32"].astype(np.float64), oracle.REFLECT)
    assert rel_max_err(out, ref) <= FP32_TOL


# --------------------------------------------------------------------------
# Zero extension with boxes much wider than the image: the outputs are a small
# fraction of the inputs (most of each box lies outside), so any rounding that
# scales with the inputs rather than the outputs shows against max|oracle|.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("path", ["auto", "two_pass", "fused"])
@pytest.mark.parametrize("H,W,C,sigma,K", [(2, 91, 1, 32.012, 2), (91, 2, 1, 32.012, 2), (3, 40, 3, 30.0, 5),
                                           (5, 200, 1, 64.0, 3), (1, 1, 1, 64.0, 5)])
def test_zero_extension_wide_boxes(path, H, W, C, sigma, K):
    """A 2 x 91 FP32 image with half-widths (31, 66) under zero extension (and
    its transpose, and similar shapes): outputs of about 2 from inputs up to
    255.  FP32 within 1e-5 of max|oracle| on every path."""
    import paper_1107_4958_amd as rsg
    forced = {"auto": rsg.RSG_PATH_AUTO, "two_pass": rsg.RSG_PATH_TWO_PASS, "fused": rsg.RSG_PATH_FUSED}[path]
    img = synthimg.image(H, W, C, "f32", 38)
    rsg.rsg_tune_path(forced)
    try:
        try:
            e = _check(img, "f32", sigma, K, oracle.ZERO)
        except rsg.RsgError as err:
            assert err.code == rsg.RSG_EUNSUPPORTED and path != "auto"
            pytest.skip("path infeasible for this shape: %s" % err)
    finally:
        rsg.rsg_tune_path(rsg.RSG_PATH_AUTO)
    assert e <= FP32_TOL


@pytest.mark.parametrize("dtype", ["f32", "u8"])
@pytest.mark.parametrize("sigma", [2.0, 8.0])
def test_full_image_4096(dtype, sigma):
    """The 4096 x 4096 headline shape (K = 3, replicate) compared element by
    element over the whole image, in the launch configuration the benchmark
    times (Section 3.4 composes the passes over every pixel)."""
    img = synthimg.image(4096, 4096, 1, dtype, seed=2)
    _check(img, dtype, sigma, 3, oracle.REPLICATE)


@pytest.mark.parametrize("layout", [1, 2, 3])
@pytest.mark.parametrize("dtype", ["f32", "u8"])
@pytest.mark.parametrize("H,W,C,sigma,K,boundary", [(97, 250, 1, 2.0, 3, oracle.REPLICATE),
                                                     (61, 211, 3, 1.0, 4, oracle.ZERO),
                                                     (130, 300, 2, 3.0, 5, oracle.REFLECT)])
def test_forced_row_layouts(layout, dtype, H, W, C, sigma, K, boundary):
    """Narrow boxes on the wider row-scan layouts the tuner may choose
    (rsg_tune_layout): tiles much wider than the span a task needs."""
    import paper_1107_4958_amd as rsg
    img = synthimg.image(H, W, C, dtype, seed=H + 3 * layout)
    rsg.rsg_tune_layout(layout)
    try:
        _check(img, dtype, sigma, K, boundary)
    finally:
        rsg.rsg_tune_layout(0)
