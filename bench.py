"""Benchmark of the running-sum Gaussian filter on one MI355X.

A step is one filter of one image through the C ABI (rsg_gauss_filter: the
host fit is cached, the fused row + column kernel runs on the device).  The
headline workload is one 4096 x 4096 single-channel FP32 synthetic 1/f image,
sigma = 8, K = 3 boxes, replicate boundary.  Inputs rotate over enough buffer
pairs (> 512 MB) that no step finds its image in the 256 MB last-level cache,
and are resident in HBM before the timed region starts.

Prints ONE JSON line: metric/value/unit of the headline, the roofline of the
fused kernel (algorithmic bytes per launch / launch time, against 8 TB/s
HBM3E; the --steps timed launches run as 5 repetitions bracketed by HIP
events on the launch stream and the median repetition is reported; beside it
the bandwidth of the library's streaming copy kernel on the same buffer
rotation, replayed from a captured HIP graph; HBM traffic, and for uint8 the VALU work, from the committed
rocprofv3 counter summary when it was taken on the current kernel sources),
the CPU oracle baseline, the uint8 form of the headline and, unless
--quick: the sigma x K grid at 4096^2 (uint8 and FP32), the plain method at
512^2 with its accuracy against the sampled Gaussian, the mixed batch (256
three-channel uint8 images in one launch per kernel class against the same
images filtered one launch each), the 8192^2 precision forms with their
normalised RMS error against the FP64 box oracle and the sampled Gaussian,
and the served request streams (p50/p99 latency and throughput at fractions
of the measured saturation rate).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gpixel/s + %HBM roofline (4096², σ=8, K=3); served p50/p99 latency"
HBM_PEAK_GBS = 8000.0
ES = {"u8": 1, "f32": 4, "f16": 2, "bf16": 2}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("rsg_device.h", "rsg_dispatch.h", "rsg_plan.cpp", "rsg_internal.h", "rsg_launch.cpp"):
        with open(os.path.join(ROOT, "paper_1107_4958_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    tune = os.path.join(ROOT, "paper_1107_4958_amd", "tune_gfx950.txt")
    if os.path.exists(tune):
        with open(tune, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_record(workload_key: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel sources and tuning table; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            rec = json.load(f).get(workload_key)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("kernel_sha") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def to_dev(img, dtype):
    import torch
    if dtype == "bf16":
        return torch.from_numpy(np.ascontiguousarray(img).view(np.int16)).view(torch.bfloat16).cuda()
    return torch.from_numpy(np.ascontiguousarray(img)).cuda()


def from_dev(t, dtype):
    import torch
    if dtype == "bf16":
        return t.view(torch.int16).cpu().numpy().view(np.uint16)
    return t.cpu().numpy()


def decode(a, dtype):
    import synthimg
    if dtype == "bf16":
        return synthimg.bf16_bits_to_f32(a).astype(np.float64)
    return a.astype(np.float64)


def _pool(base, min_pool_bytes):
    import torch
    pair = 2 * base.numel() * base.element_size()
    npairs = max(2, int(math.ceil(min_pool_bytes / pair)))
    srcs = [base] + [base.clone() for _ in range(npairs - 1)]
    dsts = [torch.empty_like(base) for _ in range(npairs)]
    return srcs, dsts


def _timed_reps(launch, steps, reps):
    """Time `steps` launches as `reps` consecutive repetitions (HIP events on
    the launch stream between them, synchronised before and after); returns
    the median per-launch time of the repetitions (ms) and every repetition's."""
    import torch
    stream = torch.cuda.current_stream()
    reps = max(1, min(reps, steps))
    sizes = [steps // reps + (1 if r < steps % reps else 0) for r in range(reps)]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    i = 0
    for r in range(reps):
        for _ in range(sizes[r]):
            launch(i)
            i += 1
        ev[r + 1].record(stream)
    torch.cuda.synchronize()
    per = [ev[r].elapsed_time(ev[r + 1]) / sizes[r] for r in range(reps)]
    return float(np.median(per)), per


def time_image(img, dtype, sigma, K, steps, warmup, min_pool_bytes=640 << 20, reps=5, with_reps=False):
    """Launch time (ms) of rsg_gauss_filter on `img`: `steps` launches on
    rotating buffers in `reps` repetitions timed with HIP events on the launch
    stream, the median repetition's per-launch time.  Returns (ms, last output
    tensor) or, with_reps, (ms, output, per-repetition ms)."""
    import torch
    import paper_1107_4958_amd as rsg
    base = to_dev(img, dtype)
    H, W = img.shape[:2]
    C = img.shape[2] if img.ndim == 3 else 1
    srcs, dsts = _pool(base, min_pool_bytes)
    npairs = len(srcs)
    stream = torch.cuda.current_stream()
    code = rsg.tensor_dtype_code(base)

    def launch(i):
        rsg.rsg_gauss_filter(srcs[i % npairs].data_ptr(), dsts[i % npairs].data_ptr(), H, W, C, code, sigma, K,
                             rsg.RSG_REPLICATE, stream.cuda_stream)

    for i in range(warmup):
        launch(i)
    ms, per = _timed_reps(launch, steps, reps)
    out = dsts[(steps - 1) % npairs]
    return (ms, out, per) if with_reps else (ms, out)


def copy_ceiling(nbytes, steps, min_pool_bytes=640 << 20, reps=5):
    """GB/s (read + write) of the library's streaming copy kernel over
    buffers of the workload's size, on the same rotation as the filter.  A
    copy of one image is shorter than a Python-side launch, so the launches
    are captured once in a HIP graph and replayed back to back: the device
    never idles between copies.  Median of `reps` replays of `steps` copies."""
    import torch
    import paper_1107_4958_amd as rsg
    base = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    srcs, dsts = _pool(base, min_pool_bytes)
    npairs = len(srcs)
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        for i in range(3):
            rsg.rsg_stream_copy(srcs[i % npairs].data_ptr(), dsts[i % npairs].data_ptr(), nbytes, side.cuda_stream)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        st = torch.cuda.current_stream().cuda_stream
        for i in range(steps):
            rsg.rsg_stream_copy(srcs[i % npairs].data_ptr(), dsts[i % npairs].data_ptr(), nbytes, st)
    graph.replay()
    torch.cuda.synchronize()
    per = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        graph.replay()
        e1.record()
        torch.cuda.synchronize()
        per.append(e0.elapsed_time(e1) / steps)
    del graph
    return 2.0 * nbytes / (float(np.median(per)) * 1e-3) / 1e9


def valu_record(workload_key: str, ms: float, pixels: int):
    """VALU work of the fused kernel from the committed rocprofv3 counter
    summary (SQ_INSTS_VALU per launch, taken on the current kernel sources):
    lane-operations per pixel, and the busy fraction at this run's launch
    time (wave64 instructions take 4 cycles on a 16-lane SIMD; 1024 SIMDs at
    2.4 GHz); None without a current record."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f).get(workload_key)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("kernel_sha") != kernel_source_hash() or not rec.get("valu_insts_per_launch"):
        return None
    insts = float(rec["valu_insts_per_launch"])
    return {"insts_per_launch": insts, "lane_ops_per_px": round(insts * 64 / pixels, 2),
            "busy_frac": round(insts * 4 / (1024 * ms * 1e-3 * 2.4e9), 3),
            "source": "profiles/traffic.json (rocprofv3 --pmc SQ_INSTS_VALU)"}


def roofline(dtype, H, W, C, ms, traffic=None, copy_gbs=None):
    alg = 2.0 * H * W * C * ES[dtype]              # read once + write once
    achieved = alg / (ms * 1e-3) / 1e9
    r = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
         "algorithmic_bytes_per_launch": int(alg)}
    if copy_gbs:
        r["copy_ceiling"] = round(copy_gbs, 1)
        r["frac_of_copy"] = round(achieved / copy_gbs, 4)
    return r


def cpu_baseline(img, dtype, sigma, K, min_seconds=10.0, max_passes=200):
    """The oracle (FP64 direct box sums, OpenMP) timed on the host cores: whole
    passes over the workload image, repeated until at least `min_seconds` of
    CPU work (a bounded sample), scaled to Gpixel/s."""
    import oracle
    b = oracle.boxes(sigma, K)
    src = np.ascontiguousarray(img)
    src64 = None if dtype == "u8" else src.astype(np.float64)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    passes = 0
    t0 = time.perf_counter()
    while True:
        if dtype == "u8":
            oracle.box_filter_u8(src, b["r"], b["m"], b["G"])
        else:
            oracle.box_filter(src64, b["r"], b["w32"].astype(np.float64))
        passes += 1
        dt = time.perf_counter() - t0
        if dt >= min_seconds or passes >= max_passes:
            break
    H, W = src.shape[:2]
    return {"value": round(passes * H * W / dt / 1e9, 5), "unit": "Gpixel/s", "cores": cores, "kind": "oracle",
            "sample": "%d whole passes over the %s workload image (%dx%d), sigma=%g K=%d, FP64 direct box sums, "
                      "%.1f s" % (passes, dtype, H, W, sigma, K, dt)}


def sampled_parity(img, out, dtype, sigma, K, n=300):
    """Spot-check a timed output against the oracle (a few hundred points)."""
    import oracle
    b = oracle.boxes(sigma, K)
    H, W = img.shape[:2]
    rng = np.random.default_rng(7)
    ys, xs = rng.integers(0, H, n), rng.integers(0, W, n)
    o = from_dev(out, dtype)
    im3 = img[..., None] if img.ndim == 2 else img
    o3 = o[..., None] if o.ndim == 2 else o
    if dtype == "u8":
        ref = oracle.box_filter_u8_points(im3, b["r"], b["m"], b["G"], ys, xs)
        return bool(np.array_equal(o3[ys, xs, 0], ref))
    ref = oracle.box_filter_points(decode(im3, dtype), b["r"], b["w32"].astype(np.float64), ys, xs)
    return float(np.max(np.abs(o3[ys, xs, 0].astype(np.float64) - ref)) / max(np.max(np.abs(ref)), 1e-30)) <= 1e-5


# ---------------------------------------------------------------------------
# further workloads
# ---------------------------------------------------------------------------
def plain_workload(steps):
    """The plain method on one 512 x 512 single-channel FP32 1/f image,
    sigma = 5, K = 3: parity with the box oracle over the whole image, and
    the method's accuracy against the sampled Gaussian (NRMS, PSNR)."""
    import oracle
    import synthimg
    img = synthimg.image(512, 512, 1, "f32", 1)
    ms, out = time_image(img, "f32", 5.0, 3, steps, 10, min_pool_bytes=64 << 20)
    o = from_dev(out, "f32").astype(np.float64)
    b = oracle.boxes(5.0, 3)
    x = img.astype(np.float64)
    ref = oracle.box_filter(x, b["r"], b["w32"].astype(np.float64)).reshape(o.shape)
    g = oracle.gauss_filter(x, 5.0).reshape(o.shape)
    return {"H": 512, "W": 512, "sigma": 5.0, "K": 3, "r": [int(v) for v in b["r"]], "us": round(ms * 1000, 2),
            "gpix_s": round(512 * 512 / (ms * 1e-3) / 1e9, 2),
            "parity_max_rel_err": float("%.3g" % (np.max(np.abs(o - ref)) / np.max(np.abs(ref)))),
            "nrms_vs_gauss": float("%.4g" % oracle.nrms(o, g)), "psnr_vs_gauss_db": round(oracle.psnr(o, g), 2),
            "note": "2 MiB: resident in the last-level cache, no roofline"}


def fit_study():
    """The fit methods compared on the method's own accuracy (the analogue of
    the paper's parameter comparison): a 1024 x 1024 FP32 1/f image filtered
    on the device with the boxes of each method, PSNR and NRMS against the
    sampled Gaussian (FP64 oracle), for sigma in {1, 2, 4, 8, 16} and K in
    {3, 4, 5}.  Methods: the paper's rescaled quadratic-form fit, the
    rescaled l2 fit, and the direct quadratic-form fit at sigma."""
    import oracle
    import paper_1107_4958_amd as rsg
    import synthimg
    img = synthimg.image(1024, 1024, 1, "f32", 21)
    x = img.astype(np.float64)
    src = to_dev(img, "f32")
    methods = (("scaled_qf", rsg.RSG_FIT_SCALED), ("scaled_l2", rsg.RSG_FIT_SCALED_L2), ("direct_qf", rsg.RSG_FIT_DIRECT))
    out = []
    for sigma in (1.0, 2.0, 4.0, 8.0, 16.0):
        g = oracle.gauss_filter(x, sigma).reshape(img.shape)
        for K in (3, 4, 5):
            row = {"sigma": sigma, "K": K}
            for name, m in methods:
                b = rsg.rsg_fit_boxes_ex(sigma, K, m)
                o = from_dev(rsg.filter_tensor(src, sigma, K, boxes=b), "f32").astype(np.float64)
                row[name] = {"r": [int(v) for v in b.r[:K]], "psnr_db": round(oracle.psnr(o, g), 2),
                             "nrms": float("%.4g" % oracle.nrms(o, g))}
            out.append(row)
    return out


def strided_workload(steps):
    """Strided (downsampling) evaluation at 8192 x 8192 FP32, sigma = 8,
    K = 3: every step-th row and pixel for step in {1, 2, 4} (step 1 through
    the strided entry point too), against the full single-image filter.
    Algorithmic bytes: the input read once plus the strided output written
    once; sampled parity against the oracle."""
    import torch
    import oracle
    import paper_1107_4958_amd as rsg
    import synthimg
    H = W = 8192
    img = synthimg.to_dtype(synthimg.one_over_f(H, W, 13), "f32")
    base = to_dev(img, "f32")
    srcs = [base, base.clone(), base.clone()]
    stream = torch.cuda.current_stream()
    b = oracle.boxes(8.0, 3)
    rng = np.random.default_rng(9)
    out = []
    ms_full, _ = time_image(img, "f32", 8.0, 3, steps, 3, min_pool_bytes=1 << 30)
    for step in (1, 2, 4):
        Ho, Wo = (H + step - 1) // step, (W + step - 1) // step
        dsts = [torch.empty((Ho, Wo), dtype=torch.float32, device="cuda") for _ in srcs]

        def launch(i):
            rsg.rsg_gauss_filter_strided(srcs[i % 3].data_ptr(), dsts[i % 3].data_ptr(), H, W, 1, rsg.RSG_F32, 8.0,
                                         3, None, rsg.RSG_REPLICATE, step, stream.cuda_stream)

        for i in range(3):
            launch(i)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(steps):
            launch(i)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        o = dsts[(steps - 1) % 3].cpu().numpy()
        ys, xs = rng.integers(0, Ho, 400), rng.integers(0, Wo, 400)
        ref = oracle.box_filter_points(img[..., None].astype(np.float64), b["r"], b["w32"].astype(np.float64),
                                       ys * step, xs * step)
        err = float(np.max(np.abs(o[ys, xs] - ref)) / np.max(np.abs(img)))
        alg = 4.0 * (H * W + Ho * Wo)
        out.append({"step": step, "ms": round(ms, 5), "input_gpix_s": round(H * W / (ms * 1e-3) / 1e9, 2),
                    "hbm_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                    "vs_full_filter": round(ms_full / ms, 3), "parity_max_rel_err": float("%.3g" % err)})
        del dsts
    return {"H": H, "W": W, "sigma": 8.0, "K": 3, "ms_full_filter": round(ms_full, 5), "steps": out}


def volume_workload(steps):
    """A 256 x 256 x 256 FP32 volume (a stack of seeded 1/f slices), sigma
    in {2, 4}, K = 3, filtered along x, y (slices, one batched launch) and z:
    time per volume, its HBM fraction on the algorithmic bytes (read once +
    write once), and the largest error against the FP64 volume oracle."""
    import torch
    import oracle
    import paper_1107_4958_amd as rsg
    import synthimg
    D = H = W = 256
    vol = np.stack([synthimg.image(H, W, 1, "f32", 300 + z) for z in range(D)])
    srcs = [to_dev(vol, "f32"), None]
    srcs[1] = srcs[0].clone()
    dsts = [torch.empty_like(srcs[0]) for _ in srcs]
    stream = torch.cuda.current_stream()
    out = []
    for sigma in (2.0, 4.0):
        def launch(i):
            rsg.rsg_gauss_filter_3d(srcs[i % 2].data_ptr(), dsts[i % 2].data_ptr(), D, H, W, 1, rsg.RSG_F32, sigma, 3,
                                    None, rsg.RSG_REPLICATE, stream.cuda_stream)

        for i in range(3):
            launch(i)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(steps):
            launch(i)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        got = dsts[(steps - 1) % 2].cpu().numpy().astype(np.float64)
        b = oracle.boxes(sigma, 3)
        ref = oracle.box_filter_3d(vol.astype(np.float64), b["r"], b["w32"].astype(np.float64))
        err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
        alg = 2.0 * D * H * W * 4
        out.append({"sigma": sigma, "K": 3, "ms": round(ms, 4), "gvox_s": round(D * H * W / (ms * 1e-3) / 1e9, 2),
                    "hbm_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "parity_max_rel_err": float("%.3g" % err)})
    return {"D": D, "H": H, "W": W, "runs": out}


def sigma_k_grid(imgs, steps):
    """Gpixel/s and HBM fraction at 4096^2 for sigma in {2, 8, 32}, K in {3, 4, 5}."""
    out = []
    for dtype, img in imgs.items():
        H, W = img.shape[:2]
        for sigma in (2.0, 8.0, 32.0):
            for K in (3, 4, 5):
                ms, _ = time_image(img, dtype, sigma, K, steps, 5)
                out.append({"dtype": dtype, "sigma": sigma, "K": K, "ms": round(ms, 5),
                            "gpix_s": round(H * W / (ms * 1e-3) / 1e9, 2),
                            "hbm_frac": roofline(dtype, H, W, 1, ms)["frac"]})
    return out


def batch_workload(steps, headline_gsamples=None):
    """256 three-channel uint8 images (sides 64..2048, sigma log-uniform in
    [1, 30], K = 4) in one persistent launch, against the same images
    filtered with one launch each."""
    import torch
    import paper_1107_4958_amd as rsg
    import synthimg
    specs = synthimg.batch_specs(256)
    srcs = [to_dev(synthimg.crop_pool(s["H"], s["W"], s["C"], "u8", s["seed"]), "u8") for s in specs]
    dsts = [torch.empty_like(s) for s in srcs]
    sig = [s["sigma"] for s in specs]
    Ks = [s["K"] for s in specs]
    ws = rsg.filter_batch_tensors(srcs, dsts, sig, Ks)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        rsg.filter_batch_tensors(srcs, dsts, sig, Ks, workspace=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_batch = e0.elapsed_time(e1) / steps
    e0.record(stream)
    for _ in range(steps):
        for s, d, sg, k in zip(srcs, dsts, sig, Ks):
            rsg.filter_tensor(s, sg, k, out=d)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_single = e0.elapsed_time(e1) / steps
    px = sum(s["H"] * s["W"] for s in specs)
    byt = 2 * sum(s["H"] * s["W"] * s["C"] for s in specs)
    gs = byt / 2 / (ms_batch * 1e-3) / 1e9
    return {"images": len(specs), "pixels": px, "ms_per_batch": round(ms_batch, 4),
            "gpix_s": round(px / (ms_batch * 1e-3) / 1e9, 2),
            "channel_gsamples_s": round(gs, 2),
            "vs_single_image_fp32_gsamples": round(gs / headline_gsamples, 3) if headline_gsamples else None,
            "hbm_frac": round(byt / (ms_batch * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "ms_one_launch_per_image": round(ms_single, 4),
            "speedup_vs_one_launch_per_image": round(ms_single / ms_batch, 2)}


def precision_workload(steps, npts=8000, ngauss=2000):
    """8192^2 single-channel image in uint8 (exact integer sums), FP16 and
    BF16 storage (FP32 accumulation) and FP32; sigma in {4, 64}, K = 5.
    NRMS error on sampled points against the FP64 oracle of the same boxes
    (the arithmetic's error) and against the sampled Gaussian (the method's
    error), both on each form's own input."""
    import oracle
    import synthimg
    H = W = 8192
    x = synthimg.one_over_f(H, W, 11)
    forms = {dt: synthimg.to_dtype(x, dt) for dt in ("u8", "f16", "bf16", "f32")}
    del x
    rng = np.random.default_rng(5)
    ys, xs = rng.integers(0, H, npts), rng.integers(0, W, npts)
    out = []
    for sigma in (4.0, 64.0):
        b = oracle.boxes(sigma, 5)
        for dtype, img in forms.items():
            ms, res = time_image(img, dtype, sigma, 5, steps, 3, min_pool_bytes=1 << 30)
            o = from_dev(res, dtype)[ys, xs]
            im3 = decode(img, dtype)[..., None]
            ref = oracle.box_filter_points(im3, b["r"], b["w"], ys, xs)     # FP64 weights
            gref = oracle.gauss_filter_points(im3, sigma, ys[:ngauss], xs[:ngauss])
            rec = {"dtype": dtype, "sigma": sigma, "K": 5, "ms": round(ms, 4),
                   "gpix_s": round(H * W / (ms * 1e-3) / 1e9, 2),
                   "hbm_frac": roofline(dtype, H, W, 1, ms)["frac"],
                   "nrms_vs_fp64_boxes": float("%.3g" % oracle.nrms(decode(o, dtype), ref)),
                   "nrms_vs_gauss": float("%.3g" % oracle.nrms(decode(o, dtype)[:ngauss], gref))}
            if dtype == "u8":
                exact = oracle.box_filter_u8_points(img[..., None], b["r"], b["m"], b["G"], ys, xs)
                rec["bit_exact_vs_integer_oracle"] = bool(np.array_equal(o, exact))
            out.append(rec)
    return out


class _ServingRig:
    """Device-resident 4096^2 source images (one per dtype and channel
    count; a request is a window of one, row stride = the resident image's),
    and a ring of output slots of the largest request's size."""

    def __init__(self, nslots=128):
        import torch
        import synthimg
        fields = [synthimg.one_over_f(4096, 4096, 48 + c) for c in range(3)]
        self.resident = {}
        for dt in ("u8", "f32"):
            for C in (1, 3):
                self.resident[(dt, C)] = to_dev(np.stack([synthimg.to_dtype(f, dt) for f in fields[:C]], axis=-1), dt)
        self.slot_bytes = 4096 * 4096 * 3 * 4
        self.nslots = nslots
        self.out = torch.empty(self.slot_bytes * nslots, dtype=torch.uint8, device="cuda")
        # the server's arena: 8 slots of 1 GiB, each holding a launch's work
        # list and the intermediates of its two-pass requests (up to 4 H W C
        # bytes each: 192 MiB for the largest request)
        self.arena = torch.empty(8 << 30, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()

    def desc(self, r, i):
        import paper_1107_4958_amd as rsg
        src = self.resident[(r["dtype"], r["C"])]
        d = rsg.rsg_image_desc()
        d.src = src.data_ptr()
        d.dst = self.out.data_ptr() + (i % self.nslots) * self.slot_bytes
        d.H, d.W, d.C = r["H"], r["W"], r["C"]
        d.src_stride, d.dst_stride = 4096 * r["C"], 0
        d.dt = rsg.tensor_dtype_code(src)
        d.sigma, d.K, d.b = r["sigma"], r["K"], rsg.RSG_REPLICATE
        return d

    def run(self, reqs, open_loop=True, timeout_s=120.0):
        """Submit reqs at their arrival times (or all at once), poll to
        completion; per-request (submit, done) ns.  A request reuses an
        output slot only after the request that held it has completed."""
        import paper_1107_4958_amd as rsg
        cfg = rsg.rsg_server_config()
        cfg.d_arena, cfg.arena_bytes = self.arena.data_ptr(), self.arena.numel()
        cfg.hbm_budget = 16 << 30
        cfg.max_inflight, cfg.n_streams, cfg.queue_depth, cfg.max_batch = 8, 4, 1024, 16
        srv = rsg.rsg_server_create(cfg)
        n = len(reqs)
        ticket = [None] * n
        stats = [None] * n
        busy = 0
        try:
            t0 = time.perf_counter()
            i = 0
            done = 0
            pending = []
            while done < n:
                now = time.perf_counter() - t0
                while i < n and (not open_loop or reqs[i]["t_arrive"] <= now):
                    if i >= self.nslots and stats[i - self.nslots] is None:
                        break                                      # its output slot is still in use
                    try:
                        ticket[i] = rsg.rsg_submit(srv, self.desc(reqs[i], i))
                    except rsg.RsgError as e:
                        if e.code != rsg.RSG_EBUSY:
                            raise
                        busy += 1
                        break
                    pending.append(i)
                    i += 1
                still = []
                for j in pending:
                    st = rsg.rsg_poll(srv, ticket[j])
                    if st.done:
                        if st.status != rsg.RSG_OK:
                            raise RuntimeError("request %d failed with %d" % (j, st.status))
                        stats[j] = (st.t_submit_ns, st.t_done_ns)
                        done += 1
                    else:
                        still.append(j)
                pending = still
                if now > timeout_s:
                    raise RuntimeError("serving run did not finish in %.0f s" % timeout_s)
        finally:
            rsg.rsg_server_destroy(srv)
        lat = np.array([(d - s_) * 1e-6 for s_, d in stats])
        span = (max(d for _, d in stats) - min(s_ for s_, _ in stats)) * 1e-9
        px = sum(r["H"] * r["W"] for r in reqs)
        return lat, span, px, busy


def serving_workload(n=10000, fractions=(0.25, 0.5, 0.8, 0.95)):
    """Poisson request streams (sides uniform in [128, 4096], C in {1, 3},
    uint8 or FP32, sigma log-uniform in [0.5, 50], K in {3, 5}) served with
    continuous batching under an HBM budget.  Saturation is the completion
    rate of a closed burst; then open-loop streams at fractions of it.
    Latency = done - submit per request (images device-resident)."""
    import synthimg
    rig = _ServingRig()
    burst = synthimg.request_stream(min(n, 2000), 1e9, seed=6)
    _, span, _, _ = rig.run(burst, open_loop=False)
    sat = len(burst) / span
    out = {"saturation_qps": round(sat, 1), "requests_per_rate": n, "rates": []}
    for f in fractions:
        reqs = synthimg.request_stream(n, f * sat, seed=5)
        lat, span, px, busy = rig.run(reqs)
        out["rates"].append({"fraction_of_saturation": f, "qps": round(f * sat, 1),
                             "p50_ms": round(float(np.percentile(lat, 50)), 3),
                             "p99_ms": round(float(np.percentile(lat, 99)), 3),
                             "gpix_s": round(px / span / 1e9, 2), "ebusy_retries": busy})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500, help="timed launches, split into 5 repetitions")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--sigma", type=float, default=8.0)
    ap.add_argument("--K", type=int, default=3)
    ap.add_argument("--dtype", default="f32", choices=["f32", "u8", "f16", "bf16"])
    ap.add_argument("--quick", action="store_true", help="headline and its uint8 form only")
    ap.add_argument("--grid-only", action="store_true",
                    help="only the sigma x K grid at 4096^2 (FP32 and uint8), for profiling its kernels")
    ap.add_argument("--only", choices=["strided", "volume", "batch", "precision"],
                    help="only one of the other workloads (--steps timed repetitions), for profiling its kernels")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--copy-ref", type=int, default=0, metavar="MIB",
                    help="first run 3 copies of MIB MiB with the library's streaming copy kernel "
                         "(a known-size reference for the HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    import paper_1107_4958_amd  # noqa: F401  (fails loudly if the HIP library is missing)
    import synthimg

    if args.copy_ref:           # the library's streaming copy kernel over MIB MiB, three times
        import paper_1107_4958_amd as rsg
        a = torch.empty(args.copy_ref << 20, dtype=torch.uint8, device="cuda").fill_(1)
        b = torch.empty_like(a)
        for _ in range(3):
            rsg.rsg_stream_copy(a.data_ptr(), b.data_ptr(), a.numel(), torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        del a, b

    if args.grid_only:
        imgs = {"f32": synthimg.image(4096, 4096, 1, "f32", 2), "u8": synthimg.image(4096, 4096, 1, "u8", 2)}
        print(json.dumps({"sigma_K_grid_4096": sigma_k_grid(imgs, args.steps)}), flush=True)
        return

    if args.only:
        run = {"strided": ("strided_8192", strided_workload), "volume": ("volume_256", volume_workload),
               "batch": ("batch", batch_workload), "precision": ("precision_8192", precision_workload)}
        name, fn = run[args.only]
        print(json.dumps({name: fn(args.steps)}), flush=True)
        return

    H = W = args.size
    img = synthimg.image(H, W, 1, args.dtype, 2)
    ms, out, ms_reps = time_image(img, args.dtype, args.sigma, args.K, args.steps, args.warmup, with_reps=True)
    copy_gbs = copy_ceiling(H * W * ES[args.dtype], 100)
    gpx = H * W / (ms * 1e-3) / 1e9
    key = "%s_%dx%d_s%g_K%d" % (args.dtype, H, W, args.sigma, args.K)
    result = {
        "metric": METRIC,
        "value": round(gpx, 2),
        "unit": "Gpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic (seeded 1/f-spectrum image scaled to [0, 255])",
        "config": {"workload": "%dx%d single-channel %s 1/f image, sigma=%g, K=%d constant boxes, replicate "
                               "boundary, one fused kernel launch per step" % (H, W, args.dtype, args.sigma, args.K),
                   "H": H, "W": W, "C": 1, "sigma": args.sigma, "K": args.K},
        "roofline": roofline(args.dtype, H, W, 1, ms, traffic_record(key), copy_gbs),
        "timing": {"reps": len(ms_reps), "launches_per_rep": args.steps // max(1, len(ms_reps)),
                   "ms_per_launch_reps": [round(x, 5) for x in ms_reps], "statistic": "median of repetitions"},
        "parity_spot_check": sampled_parity(img, out, args.dtype, args.sigma, args.K),
        # the paper states no run times, throughputs or hardware: only the
        # per-pixel operation count (Table 1) and a speed ranking whose figure
        # carries no data in its source
        "paper_context": {"published_timings": None,
                          "ops_per_pixel": 6 * args.K, "ops_note": "4K additions + 2K multiplications per pixel (Table 1)",
                          "achieved_gops": round(6 * args.K * gpx, 1)},
    }
    imgs = {args.dtype: img}
    if args.dtype != "u8":          # the uint8 form of the same configuration (exact integer path)
        img8 = synthimg.image(H, W, 1, "u8", 2)
        imgs["u8"] = img8
        ms8, out8 = time_image(img8, "u8", args.sigma, args.K, args.steps, args.warmup)
        key8 = "u8_%dx%d_s%g_K%d" % (H, W, args.sigma, args.K)
        result["u8_variant"] = {"value": round(H * W / (ms8 * 1e-3) / 1e9, 2), "unit": "Gpixel/s",
                                "ms_per_step": round(ms8, 5),
                                "roofline": roofline("u8", H, W, 1, ms8, traffic_record(key8),
                                                     copy_ceiling(H * W, 100)),
                                "valu": valu_record(key8, ms8, H * W),
                                "parity_spot_check": sampled_parity(img8, out8, "u8", args.sigma, args.K)}
    if not args.quick:
        print("bench: sigma x K grid", file=sys.stderr, flush=True)
        result["sigma_K_grid_4096"] = sigma_k_grid(imgs, max(20, args.steps // 4))
        print("bench: plain 512^2", file=sys.stderr, flush=True)
        result["plain_512"] = plain_workload(200)
        print("bench: fit methods", file=sys.stderr, flush=True)
        result["fit_study_1024"] = fit_study()
        print("bench: strided", file=sys.stderr, flush=True)
        result["strided_8192"] = strided_workload(20)
        print("bench: volume", file=sys.stderr, flush=True)
        result["volume_256"] = volume_workload(20)
        print("bench: batch", file=sys.stderr, flush=True)
        result["batch"] = batch_workload(5, gpx if args.dtype == "f32" else None)
        print("bench: precision", file=sys.stderr, flush=True)
        result["precision_8192"] = precision_workload(10)
        print("bench: serving", file=sys.stderr, flush=True)
        result["serving"] = serving_workload()
    if not args.no_cpu:
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(img, args.dtype, args.sigma, args.K)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
