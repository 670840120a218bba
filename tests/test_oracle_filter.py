"""Pins of the oracle's filters (Section 3, Section 3.4) against brute force,
invariants, a library Gaussian and Young's inequality."""
import math

import numpy as np
import pytest
from scipy import ndimage

import oracle
import synthimg


def _pad(img, R, mode):
    if img.ndim == 2:
        return np.pad(img, R, mode=mode)
    return np.pad(img, ((R, R), (R, R), (0, 0)), mode=mode)


# numpy's padding modes for the oracle's boundaries; "symmetric" is the
# half-sample reflection (d c b a | a b c d | d c b a), repeated for pads
# wider than the axis
PAD_MODE = {oracle.REPLICATE: "edge", oracle.ZERO: "constant", oracle.REFLECT: "symmetric"}
BOUNDARIES = [oracle.REPLICATE, oracle.ZERO, oracle.REFLECT]


def _brute_2d(img, h, boundary):
    """Direct 2D convolution with the outer product h x h (never separable)."""
    R = (len(h) - 1) // 2
    mode = PAD_MODE[boundary]
    x = _pad(img.astype(np.float64), R, mode)
    H, W = img.shape[:2]
    K2 = np.outer(h, h)
    out = np.zeros(img.shape, dtype=np.float64)
    for dy in range(-R, R + 1):
        for dx in range(-R, R + 1):
            out += K2[dy + R, dx + R] * x[R + dy:R + dy + H, R + dx:R + dx + W]
    return out


def _brute_2d_int(img, hm, boundary):
    R = (len(hm) - 1) // 2
    mode = PAD_MODE[boundary]
    x = _pad(img.astype(np.int64), R, mode)
    H, W = img.shape[:2]
    K2 = np.outer(hm, hm).astype(np.int64)
    out = np.zeros(img.shape, dtype=np.int64)
    for dy in range(-R, R + 1):
        for dx in range(-R, R + 1):
            out += K2[dy + R, dx + R] * x[R + dy:R + dy + H, R + dx:R + dx + W]
    return out


SHAPES = [(1, 1, 1), (1, 9, 1), (9, 1, 1), (7, 5, 1), (13, 11, 3), (2, 31, 2), (17, 4, 4), (23, 29, 1)]


@pytest.mark.parametrize("H,W,C", SHAPES)
@pytest.mark.parametrize("boundary", BOUNDARIES)
@pytest.mark.parametrize("sigma,k", [(1.0, 3), (2.0, 4), (5.0, 3), (3.3, 5)])
def test_box_f64_equals_2d_brute_force(H, W, C, boundary, sigma, k):
    b = oracle.boxes(sigma, k)
    rng = np.random.default_rng(H * 1000 + W * 10 + C)
    img = rng.uniform(0, 255, size=(H, W, C) if C > 1 else (H, W))
    out = oracle.box_filter(img, b["r"], b["w"], boundary)
    ref = _brute_2d(img, oracle.kernel_1d(b["r"], b["w"]), boundary)
    assert np.max(np.abs(out - ref)) <= 1e-12 * 255


@pytest.mark.parametrize("H,W,C", SHAPES)
@pytest.mark.parametrize("boundary", BOUNDARIES)
@pytest.mark.parametrize("sigma,k", [(1.0, 3), (5.0, 3), (3.3, 5)])
def test_box_u8_equals_exact_2d_brute_force(H, W, C, boundary, sigma, k):
    b = oracle.boxes(sigma, k)
    rng = np.random.default_rng(H * 7 + W * 3 + C)
    img = rng.integers(0, 256, size=(H, W, C) if C > 1 else (H, W), dtype=np.uint8)
    out = oracle.box_filter_u8(img, b["r"], b["m"], b["G"], boundary)
    hm = oracle.kernel_1d(b["r"], b["m"].astype(np.float64)).astype(np.int64)
    U = _brute_2d_int(img, hm, boundary)
    G2 = b["G"] ** 2
    ref = (U + G2 // 2) // G2
    assert np.array_equal(out.astype(np.int64), ref)


@pytest.mark.parametrize("sigma,k", [(0.5, 3), (2.0, 3), (8.0, 3), (8.0, 5), (30.0, 4), (64.0, 5)])
def test_constant_image_maps_to_itself(sigma, k):
    b = oracle.boxes(sigma, k)
    for v in (0, 1, 37, 128, 254, 255):
        img = np.full((9, 40), v, dtype=np.uint8)
        assert np.all(oracle.box_filter_u8(img, b["r"], b["m"], b["G"]) == v)
        out = oracle.box_filter(img.astype(np.float64), b["r"], b["w"])
        assert np.max(np.abs(out - v)) <= 1e-12 * max(v, 1)


@pytest.mark.parametrize("sigma,k", [(2.0, 3), (5.0, 4), (8.0, 5)])
def test_impulse_response_is_outer_product(sigma, k):
    b = oracle.boxes(sigma, k)
    R = int(b["r"].max())
    n = 2 * R + 5
    img = np.zeros((n, n))
    img[n // 2, n // 2] = 1.0
    out = oracle.box_filter(img, b["r"], b["w"], oracle.ZERO)
    h = oracle.kernel_1d(b["r"], b["w"])
    expect = np.zeros((n, n))
    expect[n // 2 - R:n // 2 + R + 1, n // 2 - R:n // 2 + R + 1] = np.outer(h, h)
    assert np.max(np.abs(out - expect)) <= 1e-15
    # uint8 impulse of 255
    img8 = np.zeros((n, n), dtype=np.uint8)
    img8[n // 2, n // 2] = 255
    out8 = oracle.box_filter_u8(img8, b["r"], b["m"], b["G"], oracle.ZERO)
    hm = oracle.kernel_1d(b["r"], b["m"].astype(np.float64)).astype(np.int64)
    G2 = b["G"] ** 2
    exp8 = np.zeros((n, n), dtype=np.int64)
    exp8[n // 2 - R:n // 2 + R + 1, n // 2 - R:n // 2 + R + 1] = (255 * np.outer(hm, hm) + G2 // 2) // G2
    assert np.array_equal(out8.astype(np.int64), exp8)


@pytest.mark.parametrize("sigma,k", [(3.0, 3), (8.0, 4)])
def test_row_then_column_equals_column_then_row(sigma, k):
    b = oracle.boxes(sigma, k)
    img = synthimg.image(61, 47, 1, "f32", seed=9).astype(np.float64)
    a = oracle.box_filter(img, b["r"], b["w"])
    t = oracle.box_filter(np.ascontiguousarray(img.T), b["r"], b["w"]).T
    assert np.max(np.abs(a - t)) <= 1e-11
    img8 = synthimg.image(61, 47, 1, "u8", seed=9)
    a8 = oracle.box_filter_u8(img8, b["r"], b["m"], b["G"])
    t8 = oracle.box_filter_u8(np.ascontiguousarray(img8.T), b["r"], b["m"], b["G"]).T
    assert np.array_equal(a8, t8)


def test_linearity():
    b = oracle.boxes(4.0, 4)
    rng = np.random.default_rng(3)
    f = rng.uniform(0, 255, (20, 33))
    g = rng.uniform(0, 255, (20, 33))
    lhs = oracle.box_filter(2.5 * f - 0.75 * g, b["r"], b["w"])
    rhs = 2.5 * oracle.box_filter(f, b["r"], b["w"]) - 0.75 * oracle.box_filter(g, b["r"], b["w"])
    assert np.max(np.abs(lhs - rhs)) <= 1e-10


def test_channels_are_independent():
    b = oracle.boxes(2.5, 3)
    img = synthimg.image(19, 23, 3, "f32", seed=4).astype(np.float64)
    out = oracle.box_filter(img, b["r"], b["w"])
    for c in range(3):
        one = oracle.box_filter(np.ascontiguousarray(img[..., c]), b["r"], b["w"])
        assert np.array_equal(out[..., c], one)


def test_u8_is_within_half_a_level_of_the_rational_result():
    b = oracle.boxes(6.0, 5)
    img8 = synthimg.image(40, 50, 1, "u8", seed=2)
    out8 = oracle.box_filter_u8(img8, b["r"], b["m"], b["G"])
    outf = oracle.box_filter(img8.astype(np.float64), b["r"], b["m"].astype(np.float64) / b["G"])
    assert np.max(np.abs(out8 - outf)) <= 0.5 + 1e-9


@pytest.mark.parametrize("sigma,k", [(1.0, 3), (5.0, 3), (9.0, 5)])
def test_reflect_matches_scipy_correlate1d(sigma, k):
    """Reflect boundary against scipy's separable correlation in its
    half-sample 'reflect' mode, with the fitted 1D step kernel along each
    axis; the smallest shapes put boxes many times wider than the image."""
    b = oracle.boxes(sigma, k)
    h = oracle.kernel_1d(b["r"], b["w"])
    for H, W in ((40, 33), (3, 50), (1, 2)):
        img = synthimg.image(H, W, 1, "f32", seed=H + W).astype(np.float64)
        ref = ndimage.correlate1d(ndimage.correlate1d(img, h, axis=1, mode="reflect"), h, axis=0, mode="reflect")
        out = oracle.box_filter(img, b["r"], b["w"], oracle.REFLECT)
        assert np.max(np.abs(out - ref)) <= 1e-11 * 255


@pytest.mark.parametrize("boundary", BOUNDARIES)
def test_points_match_full_filter(boundary):
    b = oracle.boxes(7.0, 4)
    img = synthimg.image(50, 70, 3, "f32", seed=6).astype(np.float64)
    img8 = synthimg.image(50, 70, 3, "u8", seed=6)
    full = oracle.box_filter(img, b["r"], b["w"], boundary)
    full8 = oracle.box_filter_u8(img8, b["r"], b["m"], b["G"], boundary)
    rng = np.random.default_rng(0)
    ys, xs, cs = rng.integers(0, 50, 200), rng.integers(0, 70, 200), rng.integers(0, 3, 200)
    pts = oracle.box_filter_points(img, b["r"], b["w"], ys, xs, cs, boundary=boundary)
    pts8 = oracle.box_filter_u8_points(img8, b["r"], b["m"], b["G"], ys, xs, cs, boundary=boundary)
    assert np.max(np.abs(pts - full[ys, xs, cs])) <= 1e-11
    assert np.array_equal(pts8, full8[ys, xs, cs])


# --------------------------------------------------------------------------
# Gaussian reference
# --------------------------------------------------------------------------
@pytest.mark.parametrize("sigma", [0.7, 2.0, 5.0, 8.0])
def test_gauss_matches_scipy(sigma):
    img = synthimg.image(64, 48, 1, "f32", seed=1).astype(np.float64)
    R = int(math.ceil(6 * sigma))
    ref = ndimage.gaussian_filter(img, sigma, mode="nearest", radius=R)
    out = oracle.gauss_filter(img, sigma)
    assert np.max(np.abs(out - ref)) <= 1e-10
    ref = ndimage.gaussian_filter(img, sigma, mode="reflect", radius=R)
    out = oracle.gauss_filter(img, sigma, oracle.REFLECT)
    assert np.max(np.abs(out - ref)) <= 1e-10


@pytest.mark.parametrize("sigma,k", [(2.0, 3), (5.0, 3), (8.0, 4), (8.0, 5)])
def test_young_bound_between_box_and_gauss(sigma, k):
    """max |box - gauss| <= max|f| * || h x h - g x g ||_1 (Young's inequality)."""
    b = oracle.boxes(sigma, k)
    img = synthimg.image(80, 80, 1, "f32", seed=3).astype(np.float64)
    box = oracle.box_filter(img, b["r"], b["w"])
    gau = oracle.gauss_filter(img, sigma)
    R = max(int(math.ceil(6 * sigma)), int(b["r"].max()))
    h = np.zeros(2 * R + 1)
    hr = oracle.kernel_1d(b["r"], b["w"])
    rb = (len(hr) - 1) // 2
    h[R - rb:R + rb + 1] = hr
    t = np.arange(-R, R + 1)
    Rg = int(math.ceil(6 * sigma))
    g = np.where(np.abs(t) <= Rg, np.exp(-t ** 2 / (2 * sigma ** 2)), 0.0)
    g /= g.sum()
    bound = np.abs(np.outer(h, h) - np.outer(g, g)).sum() * np.abs(img).max()
    assert np.max(np.abs(box - gau)) <= bound + 1e-9


def test_method_accuracy_on_one_over_f_image():
    """The box approximation is close to the Gaussian on a 1/f image, and more
    boxes help (Section 5's qualitative finding)."""
    img = synthimg.image(256, 256, 1, "f32", seed=1).astype(np.float64)
    g = oracle.gauss_filter(img, 8.0)
    errs = []
    for k in (3, 4, 5):
        b = oracle.boxes(8.0, k)
        errs.append(oracle.nrms(oracle.box_filter(img, b["r"], b["w"]), g))
    assert errs[0] < 1e-2 and errs[2] < errs[0]


def test_metrics():
    ref = np.full((4, 4), 100.0)
    y = ref + 1.0
    assert abs(oracle.nrms(y, ref) - 0.01) < 1e-15
    assert abs(oracle.psnr(y, ref) - (-10 * math.log10((1 / 255) ** 2))) < 1e-12


def test_gauss_points_match_full_filter():
    img = synthimg.image(70, 90, 3, "f32", seed=5).astype(np.float64)
    rng = np.random.default_rng(2)
    ys, xs, cs = rng.integers(0, 70, 200), rng.integers(0, 90, 200), rng.integers(0, 3, 200)
    for boundary in BOUNDARIES:
        full = oracle.gauss_filter(img, 3.5, boundary)
        pts = oracle.gauss_filter_points(img, 3.5, ys, xs, cs, boundary=boundary)
        assert np.max(np.abs(pts - full[ys, xs, cs])) <= 1e-9


# --------------------------------------------------------------------------
# Volumes: one more separable pass along z
# --------------------------------------------------------------------------
def _brute_3d(vol, h, boundary):
    """Direct 3D correlation with the outer product h x h x h."""
    R = (len(h) - 1) // 2
    mode = PAD_MODE[boundary]
    v = vol.astype(np.float64)
    if v.ndim == 3:
        v = v[..., None]
    x = np.pad(v, ((R, R), (R, R), (R, R), (0, 0)), mode=mode)
    D, H, W = v.shape[:3]
    out = np.zeros(v.shape, dtype=np.float64)
    for dz in range(-R, R + 1):
        for dy in range(-R, R + 1):
            for dx in range(-R, R + 1):
                out += h[dz + R] * h[dy + R] * h[dx + R] * x[R + dz:R + dz + D, R + dy:R + dy + H, R + dx:R + dx + W]
    return out.reshape(vol.shape)


@pytest.mark.parametrize("D,H,W,C", [(1, 1, 1, 1), (5, 3, 4, 1), (7, 6, 5, 2), (9, 4, 11, 3), (2, 13, 1, 1)])
@pytest.mark.parametrize("boundary", BOUNDARIES)
@pytest.mark.parametrize("sigma,k", [(1.0, 3), (2.5, 4)])
def test_box3_equals_3d_brute_force(D, H, W, C, boundary, sigma, k):
    b = oracle.boxes(sigma, k)
    rng = np.random.default_rng(D * 100 + H * 10 + W + C)
    vol = rng.uniform(0, 255, size=(D, H, W, C) if C > 1 else (D, H, W))
    out = oracle.box_filter_3d(vol, b["r"], b["w"], boundary)
    ref = _brute_3d(vol, oracle.kernel_1d(b["r"], b["w"]), boundary)
    assert np.max(np.abs(out - ref)) <= 1e-11 * 255


def test_box3_matches_scipy_and_constant():
    """Three scipy 1D correlations (reflect mode) on a larger volume; a
    constant volume maps to itself."""
    b = oracle.boxes(3.0, 3)
    h = oracle.kernel_1d(b["r"], b["w"])
    rng = np.random.default_rng(5)
    vol = rng.uniform(0, 255, size=(12, 20, 17))
    ref = vol.copy()
    for ax in range(3):
        ref = ndimage.correlate1d(ref, h, axis=ax, mode="reflect")
    out = oracle.box_filter_3d(vol, b["r"], b["w"], oracle.REFLECT)
    assert np.max(np.abs(out - ref)) <= 1e-11 * 255
    const = np.full((6, 7, 8), 77.25)
    assert np.max(np.abs(oracle.box_filter_3d(const, b["r"], b["w"]) - 77.25)) <= 1e-12
