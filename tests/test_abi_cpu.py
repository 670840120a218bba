"""Host-side checks of the C ABI library (no device work): exports, the
library's own FP64 fit against the oracle's, and argument validation."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _rsg():
    import paper_1107_4958_amd as rsg
    return rsg


def test_library_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "rsg.h")).read()
    declared = set(re.findall(r"^\s*(?:int|const char\*)\s+(rsg_\w+)\s*\(", header, re.M))
    assert len(declared) >= 16
    rsg = _rsg()
    lib = ctypes.CDLL(rsg.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(rsg.SYMBOLS)


@pytest.mark.parametrize("K", [1, 2, 3, 4, 5])
def test_library_fit_matches_oracle_fit(K):
    """Two independent searches (incremental Cholesky vs summed-area table)
    land on the same partition and constants."""
    rsg = _rsg()
    b = rsg.rsg_fit_boxes(8.0, K)
    p, c, e = oracle.fit(K)
    assert list(b.p[:K]) == list(p)
    assert np.allclose(list(b.c[:K]), c, rtol=0, atol=1e-12)
    # E2 = gAg - v.c cancels ~1e3-sized terms: compare at 1e-9 absolute
    assert abs(b.fit_err - e) <= 1e-9


SIGMAS = [0.5, 0.8, 1.0, 1.7, 2.0, 3.3, 5.0, 8.0, 12.5, 100.0 / math.pi, 32.0, 47.3, 64.0]


@pytest.mark.parametrize("K", [1, 2, 3, 4, 5])
def test_library_boxes_bit_identical_to_oracle(K):
    rsg = _rsg()
    for sigma in SIGMAS:
        b = rsg.rsg_fit_boxes(sigma, K)
        o = oracle.boxes(sigma, K)
        assert list(b.r[:K]) == o["r"].tolist(), sigma
        # the two least-squares solves agree to ~1e-12; the roundings below must not see it
        assert np.allclose(list(b.w[:K]), o["w"], rtol=1e-10, atol=0), sigma
        assert np.array_equal(np.array(b.w32[:K], dtype=np.float32), o["w32"]), sigma
        if o["m"] is not None:
            assert b.u8_ok == 1
            assert list(b.m[:K]) == o["m"].tolist() and b.G == o["G"] and b.s == o["s"], sigma
        else:
            assert b.u8_ok == 0


def test_fit_boxes_errors():
    rsg = _rsg()
    lib = rsg.lib()
    out = rsg.rsg_boxes()
    assert lib.rsg_fit_boxes(1.0, 0, ctypes.byref(out)) == rsg.RSG_EINVAL
    assert lib.rsg_fit_boxes(1.0, 6, ctypes.byref(out)) == rsg.RSG_EUNSUPPORTED
    assert lib.rsg_fit_boxes(0.0, 3, ctypes.byref(out)) == rsg.RSG_EINVAL
    assert lib.rsg_fit_boxes(float("nan"), 3, ctypes.byref(out)) == rsg.RSG_EINVAL
    assert lib.rsg_fit_boxes(-2.0, 3, ctypes.byref(out)) == rsg.RSG_EINVAL
    assert lib.rsg_fit_boxes(float("inf"), 3, ctypes.byref(out)) == rsg.RSG_EINVAL
    assert lib.rsg_fit_boxes(1.0, 3, None) == rsg.RSG_EINVAL
    assert "sigma" in rsg.rsg_last_error() or "NULL" in rsg.rsg_last_error()


def test_gauss_filter_rejects_bad_arguments_before_any_device_call():
    rsg = _rsg()
    lib = rsg.lib()
    A, B = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x900000)
    cases = [
        ((None, B, 8, 8, 1, rsg.RSG_F32, 2.0, 3, rsg.RSG_REPLICATE), rsg.RSG_EINVAL),
        ((A, None, 8, 8, 1, rsg.RSG_F32, 2.0, 3, rsg.RSG_REPLICATE), rsg.RSG_EINVAL),
        ((A, B, 0, 8, 1, rsg.RSG_F32, 2.0, 3, rsg.RSG_REPLICATE), rsg.RSG_EINVAL),
        ((A, B, 8, -1, 1, rsg.RSG_F32, 2.0, 3, rsg.RSG_REPLICATE), rsg.RSG_EINVAL),
        ((A, B, 8, 8, 5, rsg.RSG_F32, 2.0, 3, rsg.RSG_REPLICATE), rsg.RSG_EINVAL),
        ((A, B, 8, 8, 0, rsg.RSG_F32, 2.0, 3, rsg.RSG_REPLICATE), rsg.RSG_EINVAL),
        ((A, B, 8, 8, 1, 7, 2.0, 3, rsg.RSG_REPLICATE), rsg.RSG_EINVAL),
        ((A, B, 8, 8, 1, rsg.RSG_F32, 0.0, 3, rsg.RSG_REPLICATE), rsg.RSG_EINVAL),
        ((A, B, 8, 8, 1, rsg.RSG_F32, 2.0, 0, rsg.RSG_REPLICATE), rsg.RSG_EINVAL),
        ((A, B, 8, 8, 1, rsg.RSG_F32, 2.0, 6, rsg.RSG_REPLICATE), rsg.RSG_EUNSUPPORTED),
        ((A, B, 8, 8, 1, rsg.RSG_F32, 2.0, 3, 3), rsg.RSG_EINVAL),
        ((A, B, 8, 8, 1, rsg.RSG_F32, 2.0, 3, 9), rsg.RSG_EINVAL),
        ((A, ctypes.c_void_p(0x100000 + 64), 8, 8, 1, rsg.RSG_F32, 2.0, 3, rsg.RSG_REPLICATE), rsg.RSG_EINVAL),
    ]
    for args, want in cases:
        assert lib.rsg_gauss_filter(*args, None) == want, args
        assert rsg.rsg_last_error() != ""


def test_batch_workspace_is_host_only_and_validates():
    rsg = _rsg()
    d = rsg.rsg_image_desc()
    d.src, d.dst = 0x100000, 0x90000000
    d.H, d.W, d.C = 1000, 700, 3
    d.src_stride = d.dst_stride = 0
    d.dt, d.sigma, d.K, d.b = rsg.RSG_U8, 6.0, 4, rsg.RSG_REPLICATE
    n = rsg.rsg_filter_batch_workspace([d, d])
    assert n > 0
    bad = rsg.rsg_image_desc.from_buffer_copy(d)
    bad.C = 9
    with pytest.raises(rsg.RsgError) as ei:
        rsg.rsg_filter_batch_workspace([d, bad])
    assert ei.value.code == rsg.RSG_EINVAL and "image 1" in str(ei.value)
    with pytest.raises(rsg.RsgError):
        rsg.rsg_filter_batch_workspace([])


def test_uint8_unsupported_where_no_integer_scale_exists():
    rsg = _rsg()
    b = rsg.rsg_fit_boxes(2000.0, 5)         # r_K = 5340: no s >= 1 keeps 255 G (2 r + 1) below 2^32
    assert b.u8_ok == 0
    lib = rsg.lib()
    rc = lib.rsg_gauss_filter(ctypes.c_void_p(0x100000), ctypes.c_void_p(0x90000000), 8, 8, 1, rsg.RSG_U8,
                              2000.0, 5, rsg.RSG_REPLICATE, None)
    assert rc == rsg.RSG_EUNSUPPORTED


def test_one_hip_runtime_per_process():
    """The library must bind to the HIP runtime torch already uses (the
    pointers and streams it receives come from torch), whatever the import
    order: a fresh process that imports the package first maps exactly one
    libamdhip64."""
    import subprocess
    import sys
    code = ("import paper_1107_4958_amd, torch\n"
            "m = {l.split()[-1] for l in open('/proc/self/maps').read().splitlines() if 'libamdhip64' in l}\n"
            "print(len(m))\n")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300,
                         env=dict(os.environ, PYTHONPATH=ROOT))
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "1"


# --------------------------------------------------------------------------
# Fit methods and caller-supplied boxes (host only)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("sigma,K", [(0.5, 5), (0.8, 3), (1.0, 4), (2.0, 3), (3.7, 5), (8.0, 4), (12.0, 5),
                                     (100.0 / math.pi, 3)])
def test_direct_fit_matches_oracle(sigma, K):
    """The product's direct fit at sigma against the oracle's (independent
    code): partition, half-widths and uint8 form exact, weights to rounding."""
    import oracle
    rsg = _rsg()
    b = rsg.rsg_fit_boxes_ex(sigma, K, rsg.RSG_FIT_DIRECT)
    o = oracle.boxes_direct(sigma, K)
    assert list(b.p[:K]) == list(o["p"]) and list(b.r[:K]) == list(o["r"])
    # two independent Cholesky solves: agreement to rounding, absolutely for
    # the vanishing weights of an exact fit at small sigma (c_k = g(k))
    assert np.allclose(np.array(b.w[:K]), o["w"], rtol=1e-11, atol=1e-13)
    assert np.allclose(np.array(b.w32[:K], dtype=np.float32), o["w32"], rtol=2 ** -23, atol=1e-13)
    assert bool(b.u8_ok) == (o["m"] is not None)
    if b.u8_ok:
        assert list(b.m[:K]) == list(o["m"]) and b.G == o["G"] and b.s == o["s"]


@pytest.mark.parametrize("sigma,K", [(2.0, 3), (8.0, 4), (30.0, 5)])
def test_scaled_l2_fit_matches_oracle(sigma, K):
    import oracle
    rsg = _rsg()
    b = rsg.rsg_fit_boxes_ex(sigma, K, rsg.RSG_FIT_SCALED_L2)
    o = oracle.boxes(sigma, K, use_qf=False)
    assert list(b.p[:K]) == list(o["p"]) and list(b.r[:K]) == list(o["r"])
    assert np.allclose(np.array(b.w[:K]), o["w"], rtol=1e-11, atol=0)
    s = rsg.rsg_fit_boxes_ex(sigma, K, rsg.RSG_FIT_SCALED)
    r = rsg.rsg_fit_boxes(sigma, K)
    assert list(s.r[:K]) == list(r.r[:K]) and list(s.w[:K]) == list(r.w[:K])


def test_fit_method_errors():
    rsg = _rsg()
    with pytest.raises(rsg.RsgError) as e:
        rsg.rsg_fit_boxes_ex(2.0, 3, 7)
    assert e.value.code == rsg.RSG_EINVAL
    with pytest.raises(rsg.RsgError) as e:
        rsg.rsg_fit_boxes_ex(40.0, 3, rsg.RSG_FIT_DIRECT)
    assert e.value.code == rsg.RSG_EUNSUPPORTED


def test_caller_boxes_are_validated():
    """Descriptors carrying boxes: planned like the fitted ones when valid,
    refused when inconsistent (checked on the host, nothing launched)."""
    rsg = _rsg()
    d = rsg.rsg_image_desc()
    d.src, d.dst = 0x10000, 0x100000000000
    d.H, d.W, d.C = 300, 200, 1
    d.dt, d.sigma, d.K, d.b = rsg.RSG_U8, 2.0, 3, rsg.RSG_REPLICATE
    base = rsg.rsg_plan_shape(d)
    b = rsg.rsg_fit_boxes(2.0, 3)
    d.boxes = ctypes.addressof(b)
    assert rsg.rsg_plan_shape(d) == base
    bad = rsg.rsg_boxes.from_buffer_copy(b)
    bad.G = bad.G + 1                                  # G no longer sum m_k (2 r_k + 1)
    d.boxes = ctypes.addressof(bad)
    with pytest.raises(rsg.RsgError) as e:
        rsg.rsg_plan_shape(d)
    assert e.value.code == rsg.RSG_EINVAL
    bad = rsg.rsg_boxes.from_buffer_copy(b)
    bad.r[1] = -1
    d.boxes = ctypes.addressof(bad)
    with pytest.raises(rsg.RsgError):
        rsg.rsg_plan_shape(d)
    bad = rsg.rsg_boxes.from_buffer_copy(b)
    bad.K = 0
    d.boxes = ctypes.addressof(bad)
    with pytest.raises(rsg.RsgError):
        rsg.rsg_plan_shape(d)


def test_strided_validation():
    """Refusals of the strided entry point happen on the host, before any launch."""
    rsg = _rsg()
    lib = rsg.lib()
    A, B = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x9000000)
    assert lib.rsg_gauss_filter_strided(A, B, 64, 64, 1, rsg.RSG_F32, 2.0, 3, None, 0, 0, None) == rsg.RSG_EINVAL
    assert lib.rsg_gauss_filter_strided(A, B, 64, 64, 4, rsg.RSG_F32, 60.0, 5, None, 0, 2, None) == rsg.RSG_EUNSUPPORTED
    assert lib.rsg_gauss_filter_strided(None, B, 64, 64, 1, rsg.RSG_F32, 2.0, 3, None, 0, 2, None) == rsg.RSG_EINVAL


def test_volume_validation():
    """Refusals of the volume entry point happen on the host, before any allocation or launch."""
    rsg = _rsg()
    lib = rsg.lib()
    A, B = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x90000000)
    assert lib.rsg_gauss_filter_3d(A, B, 4, 8, 8, 1, rsg.RSG_U8, 2.0, 3, None, 0, None) == rsg.RSG_EUNSUPPORTED
    assert lib.rsg_gauss_filter_3d(A, B, 0, 8, 8, 1, rsg.RSG_F32, 2.0, 3, None, 0, None) == rsg.RSG_EINVAL
    assert lib.rsg_gauss_filter_3d(A, B, 4, 8, 8, 5, rsg.RSG_F32, 2.0, 3, None, 0, None) == rsg.RSG_EINVAL
    assert lib.rsg_gauss_filter_3d(A, ctypes.c_void_p(0x100000 + 64), 4, 8, 8, 1, rsg.RSG_F32, 2.0, 3, None, 0,
                                   None) == rsg.RSG_EINVAL


def test_fits_and_plans_from_many_threads():
    """Host entry points called from 8 threads at once (ctypes releases the
    GIL): the fit caches and the tuning-table load give every thread the
    sequential results."""
    import threading
    rsg = _rsg()
    jobs = [(s, K, m) for s in (0.6, 1.3, 2.7, 5.5, 9.0) for K in (3, 4, 5) for m in (0, 1, 2)]

    def key(b):
        return (b.K, tuple(b.r[:b.K]), tuple(b.w[:b.K]), tuple(b.m[:b.K]), b.G)

    seq = {j: key(rsg.rsg_fit_boxes_ex(*j)) for j in jobs}
    out, errors = {}, []

    def worker(t):
        try:
            for j in jobs[t::8] + jobs[::-1][t::8]:
                got = key(rsg.rsg_fit_boxes_ex(*j))
                out.setdefault(j, set()).add(got)
                d = rsg.rsg_image_desc()
                d.src, d.dst = 0x10000, 0x100000000000
                d.H, d.W, d.C, d.dt, d.sigma, d.K, d.b = 300 + t, 200, 1 + t % 4, t % 4, j[0], j[1], t % 3
                rsg.rsg_plan_shape(d)
        except Exception as e:          # noqa: BLE001  (reported below)
            errors.append(e)

    threads = [threading.Thread(target=worker, args=(t,)) for t in range(8)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    assert not errors, errors
    for j, got in out.items():
        assert got == {seq[j]}, j
