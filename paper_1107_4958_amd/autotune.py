"""Measure the fastest tile shape (segment height, strip width, first
row-scan layout and, for FP32, the output store form) per tuning bucket on
the device and write the table the planner reads.

    python -m paper_1107_4958_amd.autotune [--out PATH] [--quick]

A task of the fused kernel covers 64 consecutive samples of a row and a
segment of hs output rows, streaming 2R + 1 extra rows above the segment
(R: largest box half-width).  Short segments give many tasks but re-read
the halo often; long ones give few tasks.  The best hs depends on the
element type, the channel count, R and the amount of work (strips x rows),
so the table is keyed on exactly those: lines "dtype C rlo rhi nlo nhi hs
nc lo st", with hs = -1 selecting the two-pass path (row filter into a
transposed intermediate, twice), which wins for wide boxes.  nc is the strip
form (rsg_tune_columns): 1 for strips of 64 interleaved samples, 2 for the
wide form that C = 1 and C = 3 images have (lanes owning two columns or one
pixel), which shortens the row span per output but needs a larger LDS ring,
3 for channel-planar tasks of multi-channel images (one channel of 64
pixels per task).  lo is the first row-scan layout the planner tries
(rsg_tune_layout): 0 the narrowest whose rows cover the span, higher ones
scan fewer, wider rows per group.  st is the output store form of FP32
one-column tasks (rsg_tune_stores): 1 one 4-byte store per lane and row,
2 staged 16-byte stores through the wave's LDS row tile, 0 the planner's
rule (staged at four or five taps).  Each point is measured at one tap
count while its bucket also serves the others, so the table records a
measured form only where it departs from the rule at that tap count (see
store_field).

For every (dtype, C, image side, sigma, K) point the script times each
candidate (height, width, layout, store form) through rsg_tune_override,
rsg_tune_columns, rsg_tune_layout and rsg_tune_stores,
and the two-pass path through rsg_tune_path, on rotating synthetic images
resident in HBM (timed with HIP events on the launch stream) and keeps the
fastest.  Points are then turned into buckets: R ranges split halfway
between measured R values, work ranges split at the geometric middle
between measured sizes.  BF16 shares the FP16 lines (same element size and
kernel structure).
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "tune_gfx950.txt")

CANDIDATES = (16, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 2048)
TWO_PASS = -1                      # table value for the two-pass path
DEFAULT = -2                       # key of the built-in rule's timing
POINTS = ((1.0, 3), (2.0, 3), (4.0, 5), (8.0, 3), (16.0, 4), (32.0, 5), (64.0, 5))
SIDES = (512, 1024, 2048, 4096, 8192)
MAX_SAMPLES = 8192 * 8192          # per image (side^2 * C)
POOL_BYTES = 640 << 20             # rotate through more than the last-level cache


def _torch_dtype(torch, dt):
    return {"u8": torch.uint8, "f32": torch.float32, "f16": torch.float16}[dt]


WIDE_C = (1, 3)                    # channel counts with a wide column form
WIDE_MARGIN = 0.05                 # the wide form must beat the best other shape by this fraction
LAYOUTS = 4                        # row-scan layouts (rsg_tune_layout)


def _time_config(rsg, torch, dt, side, C, sigma, K, reps):
    """{(hs, nc, lo, st): microseconds} for every candidate height, strip
    width, first layout and store form the planner accepts (layouts that
    plan the same tile as a lower one are skipped)."""
    shape = (side, side, C) if C > 1 else (side, side)
    tdt = _torch_dtype(torch, dt)
    if dt == "u8":
        base = torch.randint(0, 256, shape, dtype=torch.uint8, device="cuda")
    else:
        base = (torch.rand(shape, device="cuda") * 255).to(tdt)
    nbytes = 2 * base.numel() * base.element_size()
    npairs = max(2, min(8, math.ceil(POOL_BYTES / nbytes)))
    srcs = [base] + [base.clone() for _ in range(npairs - 1)]
    dsts = [torch.empty_like(base) for _ in range(npairs)]
    stream = torch.cuda.current_stream()
    code = rsg.tensor_dtype_code(base)
    out = {}
    # (0, 0, 0, 0): the built-in rule; (h, nc, lo, st), h > 0: the fused
    # kernel with segment height h, strip width nc, first layout lo and
    # store form st; (TWO_PASS, 0, 0, 0): the two-pass path
    shapes = [(0, 0, 0, 0)]
    for nc in (1,) + ((2,) if C in WIDE_C else ()) + ((3,) if C >= 2 else ()):
        for st in ((1, 2) if dt == "f32" and nc == 1 else (0,)):
            for lo in range(LAYOUTS):
                shapes += [(h, nc, lo, st) for h in CANDIDATES if h <= side]
    shapes.append((TWO_PASS, 0, 0, 0))
    seen_lds = {}
    for hs, nc, lo, st in shapes:
        rsg.rsg_tune_path(rsg.RSG_PATH_TWO_PASS if hs == TWO_PASS else
                          (rsg.RSG_PATH_FUSED if hs > 0 else rsg.RSG_PATH_AUTO))
        rsg.rsg_tune_override(max(hs, 0))
        rsg.rsg_tune_columns(nc)
        rsg.rsg_tune_layout(lo)
        rsg.rsg_tune_stores(st)
        try:
            d = rsg.make_desc(srcs[0], dsts[0], sigma, K)
            plan_hs, plan_tasks, plan_lds = rsg.rsg_plan_shape(d)
        except rsg.RsgError:
            continue
        if hs > 0 and plan_hs != hs:
            continue                                  # clamped to another candidate
        if nc == 2 and plan_tasks > -(-side * C // (64 * (2 if C == 1 else 3))) * -(-side // hs):
            continue                                  # the wide form did not fit: same as nc = 1
        if hs > 0:
            key = (hs, nc, plan_lds, st)
            if key in seen_lds:
                continue                              # the same tile as a lower first layout
            seen_lds[key] = lo

        def launch(i):
            rsg.rsg_gauss_filter(srcs[i % npairs].data_ptr(), dsts[i % npairs].data_ptr(), side, side, C, code,
                                 sigma, K, rsg.RSG_REPLICATE, stream.cuda_stream)

        for i in range(3):
            launch(i)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(reps):
            launch(i)
        e1.record(stream)
        torch.cuda.synchronize()
        out[(hs, nc, lo, st) if hs else DEFAULT] = e0.elapsed_time(e1) / reps * 1000.0
    rsg.rsg_tune_override(0)
    rsg.rsg_tune_path(rsg.RSG_PATH_AUTO)
    rsg.rsg_tune_columns(0)
    rsg.rsg_tune_layout(0)
    rsg.rsg_tune_stores(0)
    del srcs, dsts, base
    return out


def store_field(st: int, K: int) -> int:
    """Table value for a measured store form st (1 per lane, 2 staged; 0
    where no form was measured) at a point with K taps: a staged win at
    three taps and a per-lane win at four or five are recorded, anything
    else leaves the rule."""
    if st == 2 and K <= 3:
        return 2
    if st == 1 and K >= 4:
        return 1
    return 0


def _buckets(values, log=False):
    """Ranges [lo, hi] covering all integers, split between sorted values."""
    v = sorted(set(values))
    cuts = []
    for a, b in zip(v, v[1:]):
        cuts.append(int(math.sqrt(a * b)) if log else (a + b) // 2)
    los = [0] + [c + 1 for c in cuts]
    his = cuts + [2 ** 62 if log else 1 << 30]
    return dict(zip(v, zip(los, his)))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--quick", action="store_true", help="fewer sides and points (a smoke run)")
    ap.add_argument("--dtypes", default="u8,f32,f16")
    ap.add_argument("--channels", default="1,2,3,4")
    args = ap.parse_args(argv)

    os.environ["RSG_TUNE_TABLE"] = ""                 # measure against the built-in rule, not an old table
    import torch
    if not torch.cuda.is_available():
        print("autotune needs a GPU", file=sys.stderr)
        return 1
    sys.path.insert(0, os.path.dirname(HERE))
    import paper_1107_4958_amd as rsg

    sides = SIDES[1::2] if args.quick else SIDES
    points = POINTS[::3] if args.quick else POINTS
    rows = []
    t_start = time.time()
    for dt in args.dtypes.split(","):
        for C in (int(c) for c in args.channels.split(",")):
            for side in sides:
                if side * side * C > MAX_SAMPLES:
                    continue
                for sigma, K in points:
                    R = int(max(rsg.rsg_fit_boxes(sigma, K).r[:K]))
                    reps = 10 if side * side * C >= 4096 * 4096 else 30
                    res = _time_config(rsg, torch, dt, side, C, sigma, K, reps)
                    if not res:
                        continue
                    default = [v for k, v in res.items() if k == DEFAULT]
                    tuned = {k: v for k, v in res.items() if k != DEFAULT}
                    best = min(tuned, key=tuned.get)
                    narrow = {k: v for k, v in tuned.items() if k[1] not in (2, 3)}
                    if best[1] in (2, 3) and narrow:
                        # the wide and channel-planar forms only where they
                        # clearly win: a batch whose images mix forms runs one
                        # launch per form
                        alt = min(narrow, key=narrow.get)
                        if narrow[alt] <= tuned[best] * (1.0 + WIDE_MARGIN):
                            best = alt
                    n = -(-side * C // 64) * side
                    rows.append(dict(dt=dt, C=C, R=R, n=n, hs=best[0], nc=best[1], lo=best[2], st=best[3], us=tuned[best],
                                     default_us=default[0] if default else float("nan"),
                                     side=side, sigma=sigma, K=K))
                    tp = (TWO_PASS, 0, 0, 0)
                    print("%-4s C=%d side=%5d sigma=%5.1f K=%d R=%3d: best %s %8.1f us (built-in rule %8.1f us%s)"
                          % (dt, C, side, sigma, K, R,
                             "two-pass" if best == tp else "hs=%4d nc=%d lo=%d st=%d" % best,
                             tuned[best], rows[-1]["default_us"],
                             ", two-pass %.1f us" % tuned[tp] if tp in tuned else ""), flush=True)

    code = {"u8": 0, "f32": 1, "f16": 2, "bf16": 3}
    lines = ["# tile shapes measured by paper_1107_4958_amd/autotune.py on %s (%.0f s)"
             % (torch.cuda.get_device_name(0), time.time() - t_start),
             "# dtype C rlo rhi nlo nhi hs nc lo st   # measured point: side sigma K, best / built-in-rule microseconds"]
    for dt in sorted({r["dt"] for r in rows}, key=code.get):
        for C in sorted({r["C"] for r in rows if r["dt"] == dt}):
            pts = [r for r in rows if r["dt"] == dt and r["C"] == C]
            nb = _buckets([r["n"] for r in pts], log=True)
            for n in sorted(nb):
                at_n = [r for r in pts if r["n"] == n]
                rb = _buckets([r["R"] for r in at_n])
                for R in sorted(rb):
                    r = min((x for x in at_n if x["R"] == R), key=lambda x: x["us"])
                    for dcode in ((code["f16"], code["bf16"]) if dt == "f16" else (code[dt],)):
                        lines.append("%d %d %d %d %d %d %d %d %d %d   # %d %g %d: %.1f / %.1f" % (
                            dcode, C, rb[R][0], rb[R][1], nb[n][0], nb[n][1], r["hs"], r["nc"], r["lo"], store_field(r["st"], r["K"]),
                            r["side"], r["sigma"], r["K"], r["us"], r["default_us"]))
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote %d lines to %s" % (len(lines) - 2, args.out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
