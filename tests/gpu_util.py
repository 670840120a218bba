"""Helpers for the GPU tests: move seeded numpy inputs to the device, run the
HIP path through the C ABI, and read results back."""
import numpy as np

import synthimg


def to_device(img: np.ndarray, dtype: str):
    import torch
    if dtype == "bf16":
        t = torch.from_numpy(np.ascontiguousarray(img).view(np.int16)).view(torch.bfloat16)
    else:
        t = torch.from_numpy(np.ascontiguousarray(img))
    return t.to("cuda")


def from_device(t, dtype: str) -> np.ndarray:
    import torch
    if dtype == "bf16":
        return t.view(torch.int16).cpu().numpy().view(np.uint16)
    return t.cpu().numpy()


def decode(img: np.ndarray, dtype: str) -> np.ndarray:
    """Exact FP64 value of each stored sample."""
    if dtype == "bf16":
        return synthimg.bf16_bits_to_f32(img).astype(np.float64)
    return img.astype(np.float64)


def gpu_filter(img: np.ndarray, dtype: str, sigma: float, K: int, boundary: int = 0, boxes=None) -> np.ndarray:
    import torch
    import paper_1107_4958_amd as rsg
    src = to_device(img, dtype)
    out = rsg.filter_tensor(src, sigma, K, boundary, boxes=boxes)
    torch.cuda.synchronize()
    return from_device(out, dtype)


def rel_max_err(y: np.ndarray, ref: np.ndarray) -> float:
    den = float(np.max(np.abs(ref)))
    return float(np.max(np.abs(y.astype(np.float64) - ref))) / (den if den > 0 else 1.0)


def half_ulp_diff(y_bits: np.ndarray, ref: np.ndarray, dtype: str) -> int:
    """Largest difference in units in the last place between the device's
    16-bit result and the FP64 reference rounded to the same format."""
    if dtype == "f16":
        a = y_bits.astype(np.float16).view(np.int16).astype(np.int64)
        b = ref.astype(np.float32).astype(np.float16).view(np.int16).astype(np.int64)
    else:
        a = y_bits.view(np.int16).astype(np.int64)
        b = synthimg.f32_to_bf16_bits(ref.astype(np.float32)).view(np.int16).astype(np.int64)
    return int(np.max(np.abs(a - b))) if a.size else 0
