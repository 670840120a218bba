"""Running-sum Gaussian filtering on AMD Instinct MI355X (gfx950).

Python binding of ``librsg.so`` (C ABI in ``include/rsg.h``): ctypes
marshalling only.  Every step of the filter runs in the library's HIP kernels;
PyTorch tensors are used only as device memory and their streams.  If the
library has not been built this module raises ImportError: there is no
fallback path.

Entry points carry the C names (``rsg_fit_boxes``, ``rsg_fit_boxes_ex``,
``rsg_gauss_filter``, ``rsg_gauss_filter_noalloc``, ``rsg_box_filter``, ``rsg_gauss_filter_strided``,
``rsg_gauss_filter_3d``, ``rsg_filter_batch_workspace``, ``rsg_filter_batch``,
``rsg_server_create``, ``rsg_submit``, ``rsg_poll``, ``rsg_server_destroy``,
``rsg_plan_shape``, ``rsg_tune_override``, ``rsg_tune_path``, ``rsg_tune_columns``, ``rsg_tune_layout``, ``rsg_tune_stores``,
``rsg_stream_copy``, ``rsg_last_error``); ``filter_tensor``, ``filter_strided_tensor``,
``filter_volume_tensor`` and ``filter_batch_tensors`` wrap them for torch
tensors.

Unless ``RSG_TUNE_TABLE`` is already set, the library reads the segment
heights measured by ``autotune.py`` from ``tune_gfx950.txt`` beside it.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librsg.so")
TUNE_TABLE = os.path.join(_HERE, "tune_gfx950.txt")
if os.path.exists(TUNE_TABLE):
    os.environ.setdefault("RSG_TUNE_TABLE", TUNE_TABLE)

RSG_OK = 0
RSG_EINVAL = -1
RSG_ENOMEM = -2
RSG_EBUSY = -3
RSG_ENOTFOUND = -4
RSG_EDEVICE = -5
RSG_EUNSUPPORTED = -6

RSG_U8, RSG_F32, RSG_F16, RSG_BF16 = 0, 1, 2, 3
RSG_REPLICATE, RSG_ZERO, RSG_REFLECT = 0, 1, 2
RSG_FIT_SCALED, RSG_FIT_SCALED_L2, RSG_FIT_DIRECT = 0, 1, 2
RSG_MAX_K = 5

DTYPE_NAMES = {"u8": RSG_U8, "f32": RSG_F32, "f16": RSG_F16, "bf16": RSG_BF16}


class RsgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("rsg error %d: %s" % (code, msg))
        self.code = code


class rsg_boxes(ctypes.Structure):
    _fields_ = [
        ("K", ctypes.c_int32),
        ("p", ctypes.c_int32 * RSG_MAX_K),
        ("c", ctypes.c_double * RSG_MAX_K),
        ("fit_err", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("r", ctypes.c_int32 * RSG_MAX_K),
        ("w", ctypes.c_double * RSG_MAX_K),
        ("w32", ctypes.c_float * RSG_MAX_K),
        ("m", ctypes.c_uint32 * RSG_MAX_K),
        ("G", ctypes.c_uint64),
        ("s", ctypes.c_int32),
        ("u8_ok", ctypes.c_int32),
    ]


class rsg_image_desc(ctypes.Structure):
    _fields_ = [
        ("src", ctypes.c_void_p),
        ("dst", ctypes.c_void_p),
        ("H", ctypes.c_int32),
        ("W", ctypes.c_int32),
        ("C", ctypes.c_int32),
        ("src_stride", ctypes.c_int64),
        ("dst_stride", ctypes.c_int64),
        ("dt", ctypes.c_int),
        ("sigma", ctypes.c_double),
        ("K", ctypes.c_int32),
        ("b", ctypes.c_int),
        ("boxes", ctypes.c_void_p),          # const rsg_boxes* or NULL
    ]


class rsg_server_config(ctypes.Structure):
    _fields_ = [
        ("d_arena", ctypes.c_void_p),
        ("arena_bytes", ctypes.c_size_t),
        ("hbm_budget", ctypes.c_size_t),
        ("max_inflight", ctypes.c_int32),
        ("n_streams", ctypes.c_int32),
        ("queue_depth", ctypes.c_int32),
        ("max_batch", ctypes.c_int32),
    ]


class rsg_req_stats(ctypes.Structure):
    _fields_ = [
        ("done", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("t_submit_ns", ctypes.c_uint64),
        ("t_admit_ns", ctypes.c_uint64),
        ("t_start_ns", ctypes.c_uint64),
        ("t_done_ns", ctypes.c_uint64),
    ]


SYMBOLS = ("rsg_fit_boxes", "rsg_gauss_filter", "rsg_filter_batch_workspace", "rsg_filter_batch",
           "rsg_server_create", "rsg_submit", "rsg_poll", "rsg_server_destroy", "rsg_plan_shape",
           "rsg_tune_override", "rsg_tune_path", "rsg_tune_columns", "rsg_tune_layout", "rsg_tune_stores", "rsg_fit_boxes_ex", "rsg_box_filter", "rsg_gauss_filter_strided",
           "rsg_gauss_filter_3d", "rsg_gauss_filter_noalloc", "rsg_stream_copy", "rsg_last_error")


def _load():
    # One HIP runtime per process: torch ships its own copy of the HIP and HSA
    # runtimes (same sonames as /opt/rocm's).  Loading torch first makes
    # librsg.so bind to that copy, so the device pointers and stream handles
    # torch hands over belong to the runtime the library launches on; loaded
    # the other way round, a process holds two runtimes and the second may see
    # no device at all.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError("librsg.so is not built (run paper_1107_4958_amd.build.build()); "
                          "there is no non-HIP fallback")
    lib = ctypes.CDLL(LIB_PATH)
    V, I, D, S = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    lib.rsg_fit_boxes.argtypes = [D, I, ctypes.POINTER(rsg_boxes)]
    lib.rsg_gauss_filter.argtypes = [V, V, I, I, I, I, D, I, I, V]
    lib.rsg_gauss_filter_noalloc.argtypes = [V, V, I, I, I, I, D, I, I, V]
    lib.rsg_stream_copy.argtypes = [V, V, S, V]
    lib.rsg_fit_boxes_ex.argtypes = [D, I, I, ctypes.POINTER(rsg_boxes)]
    lib.rsg_box_filter.argtypes = [V, V, I, I, I, I, ctypes.POINTER(rsg_boxes), I, V]
    lib.rsg_gauss_filter_strided.argtypes = [V, V, I, I, I, I, D, I, ctypes.POINTER(rsg_boxes), I, I, V]
    lib.rsg_gauss_filter_3d.argtypes = [V, V, I, I, I, I, I, D, I, ctypes.POINTER(rsg_boxes), I, V]
    lib.rsg_filter_batch_workspace.argtypes = [ctypes.POINTER(rsg_image_desc), I, ctypes.POINTER(S)]
    lib.rsg_filter_batch.argtypes = [ctypes.POINTER(rsg_image_desc), I, V, S, V]
    lib.rsg_server_create.argtypes = [ctypes.POINTER(rsg_server_config), ctypes.POINTER(V)]
    lib.rsg_submit.argtypes = [V, ctypes.POINTER(rsg_image_desc), ctypes.POINTER(ctypes.c_uint64)]
    lib.rsg_poll.argtypes = [V, ctypes.c_uint64, ctypes.POINTER(rsg_req_stats)]
    lib.rsg_server_destroy.argtypes = [V]
    lib.rsg_plan_shape.argtypes = [ctypes.POINTER(rsg_image_desc), ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_uint32)]
    lib.rsg_tune_override.argtypes = [ctypes.c_int32]
    lib.rsg_tune_path.argtypes = [ctypes.c_int32]
    lib.rsg_tune_columns.argtypes = [ctypes.c_int32]
    lib.rsg_tune_layout.argtypes = [ctypes.c_int32]
    lib.rsg_tune_stores.argtypes = [ctypes.c_int32]
    lib.rsg_last_error.argtypes = []
    lib.rsg_last_error.restype = ctypes.c_char_p
    for name in SYMBOLS[:-1]:
        getattr(lib, name).restype = ctypes.c_int
    return lib


_lib = _load()


def lib():
    return _lib


def rsg_last_error() -> str:
    return _lib.rsg_last_error().decode()


def _check(rc: int) -> int:
    if rc != RSG_OK:
        raise RsgError(rc, rsg_last_error())
    return rc


# ---------------------------------------------------------------------------
# C entry points (same names, plain values and device pointers)
# ---------------------------------------------------------------------------
def rsg_fit_boxes(sigma: float, K: int) -> rsg_boxes:
    out = rsg_boxes()
    _check(_lib.rsg_fit_boxes(float(sigma), int(K), ctypes.byref(out)))
    return out


def rsg_fit_boxes_ex(sigma: float, K: int, method: int) -> rsg_boxes:
    out = rsg_boxes()
    _check(_lib.rsg_fit_boxes_ex(float(sigma), int(K), int(method), ctypes.byref(out)))
    return out


def rsg_gauss_filter(d_src: int, d_dst: int, H: int, W: int, C: int, dt: int, sigma: float, K: int,
                     boundary: int = RSG_REPLICATE, stream: int = 0) -> None:
    _check(_lib.rsg_gauss_filter(ctypes.c_void_p(d_src), ctypes.c_void_p(d_dst), H, W, C, dt,
                                 float(sigma), K, boundary, ctypes.c_void_p(stream)))


def rsg_gauss_filter_noalloc(d_src: int, d_dst: int, H: int, W: int, C: int, dt: int, sigma: float, K: int,
                             boundary: int = RSG_REPLICATE, stream: int = 0) -> None:
    _check(_lib.rsg_gauss_filter_noalloc(ctypes.c_void_p(d_src), ctypes.c_void_p(d_dst), H, W, C, dt,
                                         float(sigma), K, boundary, ctypes.c_void_p(stream)))


def rsg_stream_copy(d_src: int, d_dst: int, nbytes: int, stream: int = 0) -> None:
    _check(_lib.rsg_stream_copy(ctypes.c_void_p(d_src), ctypes.c_void_p(d_dst), int(nbytes), ctypes.c_void_p(stream)))


def rsg_box_filter(d_src: int, d_dst: int, H: int, W: int, C: int, dt: int, boxes: rsg_boxes,
                   boundary: int = RSG_REPLICATE, stream: int = 0) -> None:
    _check(_lib.rsg_box_filter(ctypes.c_void_p(d_src), ctypes.c_void_p(d_dst), H, W, C, dt, ctypes.byref(boxes),
                               boundary, ctypes.c_void_p(stream)))


def _desc_array(descs):
    arr = (rsg_image_desc * len(descs))()
    for i, d in enumerate(descs):
        arr[i] = d
    return arr


def rsg_filter_batch_workspace(descs) -> int:
    arr = _desc_array(descs)
    nbytes = ctypes.c_size_t(0)
    _check(_lib.rsg_filter_batch_workspace(arr, len(descs), ctypes.byref(nbytes)))
    return nbytes.value


def rsg_filter_batch(descs, d_workspace: int, ws_bytes: int, stream: int = 0) -> None:
    arr = _desc_array(descs)
    _check(_lib.rsg_filter_batch(arr, len(descs), ctypes.c_void_p(d_workspace), ws_bytes,
                                 ctypes.c_void_p(stream)))


def rsg_server_create(cfg: rsg_server_config) -> int:
    h = ctypes.c_void_p(0)
    _check(_lib.rsg_server_create(ctypes.byref(cfg), ctypes.byref(h)))
    return h.value


def rsg_submit(server: int, desc: rsg_image_desc) -> int:
    t = ctypes.c_uint64(0)
    _check(_lib.rsg_submit(ctypes.c_void_p(server), ctypes.byref(desc), ctypes.byref(t)))
    return t.value


def rsg_poll(server: int, ticket: int) -> rsg_req_stats:
    st = rsg_req_stats()
    _check(_lib.rsg_poll(ctypes.c_void_p(server), ctypes.c_uint64(ticket), ctypes.byref(st)))
    return st


def rsg_server_destroy(server: int) -> None:
    _check(_lib.rsg_server_destroy(ctypes.c_void_p(server)))


def rsg_plan_shape(desc: rsg_image_desc):
    """(segment height, tasks, LDS bytes per task) of the plan for `desc`."""
    hs, nt, lds = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_uint32(0)
    _check(_lib.rsg_plan_shape(ctypes.byref(desc), ctypes.byref(hs), ctypes.byref(nt), ctypes.byref(lds)))
    return hs.value, nt.value, lds.value


def rsg_tune_override(seg_height: int) -> None:
    _check(_lib.rsg_tune_override(int(seg_height)))


RSG_PATH_AUTO, RSG_PATH_FUSED, RSG_PATH_TWO_PASS, RSG_PATH_FUSED_ONE_WAVE = 0, 1, 2, 3


def rsg_tune_path(path: int) -> None:
    _check(_lib.rsg_tune_path(int(path)))


def rsg_tune_columns(columns: int) -> None:
    _check(_lib.rsg_tune_columns(int(columns)))


def rsg_tune_layout(first: int) -> None:
    _check(_lib.rsg_tune_layout(int(first)))


def rsg_tune_stores(form: int) -> None:
    _check(_lib.rsg_tune_stores(int(form)))


# ---------------------------------------------------------------------------
# torch-tensor helpers (device memory and streams only)
# ---------------------------------------------------------------------------
def tensor_dtype_code(t) -> int:
    import torch
    m = {torch.uint8: RSG_U8, torch.float32: RSG_F32, torch.float16: RSG_F16, torch.bfloat16: RSG_BF16}
    if t.dtype not in m:
        raise TypeError("unsupported dtype %s" % t.dtype)
    return m[t.dtype]


def _hwc(t):
    if t.dim() == 2:
        return t.shape[0], t.shape[1], 1
    if t.dim() == 3:
        return t.shape[0], t.shape[1], t.shape[2]
    raise ValueError("expected H x W or H x W x C tensor")


def _stream_handle(t, stream):
    import torch
    if stream is None:
        return torch.cuda.current_stream(t.device).cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def rsg_gauss_filter_strided(d_src: int, d_dst: int, H: int, W: int, C: int, dt: int, sigma: float, K: int,
                             boxes=None, boundary: int = RSG_REPLICATE, step: int = 1, stream: int = 0) -> None:
    _check(_lib.rsg_gauss_filter_strided(ctypes.c_void_p(d_src), ctypes.c_void_p(d_dst), H, W, C, dt, float(sigma),
                                         int(K), ctypes.byref(boxes) if boxes is not None else None, boundary,
                                         int(step), ctypes.c_void_p(stream)))


def filter_strided_tensor(src, sigma: float, K: int, step: int, boundary: int = RSG_REPLICATE, out=None,
                          stream=None, boxes=None):
    """Every step-th row and pixel of the filtered image, as a new
    ceil(H/step) x ceil(W/step) (x C) tensor (or into `out`)."""
    import torch
    if not src.is_cuda or not src.is_contiguous():
        raise ValueError("src must be a contiguous device tensor")
    H, W, C = _hwc(src)
    shape = ((H + step - 1) // step, (W + step - 1) // step) + ((C,) if src.dim() == 3 else ())
    if out is None:
        out = torch.empty(shape, dtype=src.dtype, device=src.device)
    elif tuple(out.shape) != shape or not out.is_contiguous():
        raise ValueError("out must be a contiguous tensor of shape %r" % (shape,))
    rsg_gauss_filter_strided(src.data_ptr(), out.data_ptr(), H, W, C, tensor_dtype_code(src), sigma, K, boxes,
                             boundary, step, _stream_handle(src, stream))
    return out


def rsg_gauss_filter_3d(d_src: int, d_dst: int, D: int, H: int, W: int, C: int, dt: int, sigma: float, K: int,
                        boxes=None, boundary: int = RSG_REPLICATE, stream: int = 0) -> None:
    _check(_lib.rsg_gauss_filter_3d(ctypes.c_void_p(d_src), ctypes.c_void_p(d_dst), D, H, W, C, dt, float(sigma),
                                    int(K), ctypes.byref(boxes) if boxes is not None else None, boundary,
                                    ctypes.c_void_p(stream)))


def filter_volume_tensor(vol, sigma: float, K: int, boundary: int = RSG_REPLICATE, out=None, stream=None,
                         boxes=None):
    """Filter a contiguous D x H x W (x C) FP32 device tensor along all three axes."""
    import torch
    if not vol.is_cuda or not vol.is_contiguous() or vol.dim() not in (3, 4):
        raise ValueError("vol must be a contiguous D x H x W (x C) device tensor")
    D, H, W = vol.shape[:3]
    C = vol.shape[3] if vol.dim() == 4 else 1
    if out is None:
        out = torch.empty_like(vol)
    rsg_gauss_filter_3d(vol.data_ptr(), out.data_ptr(), D, H, W, C, tensor_dtype_code(vol), sigma, K, boxes,
                        boundary, _stream_handle(vol, stream))
    return out


def filter_tensor(src, sigma: float, K: int, boundary: int = RSG_REPLICATE, out=None, stream=None, boxes=None):
    """Filter a contiguous H x W (x C) device tensor; returns `out`.  With
    `boxes` (an rsg_boxes, e.g. from rsg_fit_boxes_ex) those boxes are used
    and sigma, K are ignored."""
    import torch
    if not src.is_cuda or not src.is_contiguous():
        raise ValueError("src must be a contiguous device tensor")
    if out is None:
        out = torch.empty_like(src)
    H, W, C = _hwc(src)
    if boxes is not None:
        rsg_box_filter(src.data_ptr(), out.data_ptr(), H, W, C, tensor_dtype_code(src), boxes, boundary,
                       _stream_handle(src, stream))
    else:
        rsg_gauss_filter(src.data_ptr(), out.data_ptr(), H, W, C, tensor_dtype_code(src), sigma, K, boundary,
                         _stream_handle(src, stream))
    return out


def make_desc(src, dst, sigma: float, K: int, boundary: int = RSG_REPLICATE, boxes=None) -> rsg_image_desc:
    H, W, C = _hwc(src)
    d = rsg_image_desc()
    d.src = src.data_ptr()
    d.dst = dst.data_ptr()
    d.H, d.W, d.C = H, W, C
    d.src_stride = 0
    d.dst_stride = 0
    d.dt = tensor_dtype_code(src)
    d.sigma = float(sigma)
    d.K = int(K)
    d.b = boundary
    if boxes is not None:
        d.boxes = ctypes.addressof(boxes)
        d._boxes_ref = boxes                 # keeps the struct alive with the descriptor
    return d


def filter_batch_tensors(srcs, dsts, sigmas, Ks, boundary: int = RSG_REPLICATE, workspace=None, stream=None):
    """One persistent launch over a list of device tensors; returns the workspace."""
    import torch
    descs = [make_desc(s, d, sg, k, boundary) for s, d, sg, k in zip(srcs, dsts, sigmas, Ks)]
    need = rsg_filter_batch_workspace(descs)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=srcs[0].device)
    rsg_filter_batch(descs, workspace.data_ptr(), workspace.numel(), _stream_handle(srcs[0], stream))
    return workspace
