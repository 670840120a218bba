"""Host-side tile planning through the C ABI (no device needed): the plan
query, the tuning-table lookup and the process-wide override."""
import os
import subprocess
import sys

import pytest

import paper_1107_4958_amd as rsg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _desc(H, W, C=1, dt=rsg.RSG_F32, sigma=8.0, K=3, stride=0):
    d = rsg.rsg_image_desc()
    d.src, d.dst = 0x10000, 0x100000000000       # distinct ranges; never dereferenced
    d.H, d.W, d.C = H, W, C
    d.src_stride = d.dst_stride = stride
    d.dt, d.sigma, d.K, d.b = dt, sigma, K, rsg.RSG_REPLICATE
    return d


def test_plan_shape_basics():
    hs, tasks, lds = rsg.rsg_plan_shape(_desc(4096, 4096))
    assert 1 <= hs <= 4096 and lds > 0
    try:
        rsg.rsg_tune_columns(1)
        hs, tasks, lds = rsg.rsg_plan_shape(_desc(4096, 4096))
        assert tasks == 64 * -(-4096 // hs)         # 64-sample strips x segments
        # the wide form: lanes own two columns at C = 1 and one pixel (three
        # samples) at C = 3, strips of 128 and 192 samples
        rsg.rsg_tune_columns(2)
        hs2, tasks2, lds2 = rsg.rsg_plan_shape(_desc(4096, 4096))
        assert tasks2 == 32 * -(-4096 // hs2) and lds2 > lds
        rsg.rsg_tune_path(rsg.RSG_PATH_FUSED)
        hs3, tasks3, _ = rsg.rsg_plan_shape(_desc(100, 70, C=3, dt=rsg.RSG_U8))
        assert tasks3 == -(-210 // 192) * -(-100 // hs3)
        rsg.rsg_tune_columns(1)
        hs3, tasks3, _ = rsg.rsg_plan_shape(_desc(100, 70, C=3, dt=rsg.RSG_U8))
        assert tasks3 == -(-210 // 64) * -(-100 // hs3)
        with pytest.raises(rsg.RsgError):
            rsg.rsg_tune_columns(-1)
    finally:
        rsg.rsg_tune_path(rsg.RSG_PATH_AUTO)
        rsg.rsg_tune_columns(0)
    hs3, tasks3, _ = rsg.rsg_plan_shape(_desc(100, 70, C=3, dt=rsg.RSG_U8))
    if hs3 == 100:                                  # two passes: workgroups of 16 rows in each
        assert tasks3 == -(-100 // 16) + -(-210 // 16)


def test_override_and_clamp():
    try:
        rsg.rsg_tune_override(200)
        assert rsg.rsg_plan_shape(_desc(4096, 4096))[0] == 200
        assert rsg.rsg_plan_shape(_desc(150, 4096))[0] == 150      # clamped to H
        with pytest.raises(rsg.RsgError):
            rsg.rsg_tune_override(-1)
    finally:
        rsg.rsg_tune_override(0)


def test_huge_stride_shrinks_segments_or_is_refused():
    """Every offset a task touches must stay below 2^30 bytes: a wide stride
    makes the planner shorten segments, an absurd one is refused."""
    hs, _, _ = rsg.rsg_plan_shape(_desc(4096, 64, stride=1 << 20))
    assert hs * (1 << 22) < (1 << 30)
    try:
        rsg.rsg_tune_path(rsg.RSG_PATH_FUSED)
        with pytest.raises(rsg.RsgError) as e:
            rsg.rsg_plan_shape(_desc(64, 64, sigma=30.0, stride=1 << 26))
        assert e.value.code == rsg.RSG_EUNSUPPORTED
    finally:
        rsg.rsg_tune_path(rsg.RSG_PATH_AUTO)
    # the two-pass path addresses each row on its own: any stride is fine
    assert rsg.rsg_plan_shape(_desc(64, 64, sigma=30.0, stride=1 << 26))[0] == 64


def _plans_with_table(path):
    code = ("import paper_1107_4958_amd as r, sys; sys.path.insert(0, %r)\n"
            "from test_plan_cpu import _desc\n"
            "print(r.rsg_plan_shape(_desc(4096, 4096))[0], r.rsg_plan_shape(_desc(4096, 2048))[0],"
            " r.rsg_plan_shape(_desc(4096, 4096, dt=r.RSG_U8))[0], r.rsg_plan_shape(_desc(4096, 4096, sigma=2.0))[0])"
            % os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, RSG_TUNE_TABLE=str(path), PYTHONPATH=ROOT)
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    return list(map(int, out.stdout.split()))


def test_tuning_table_lookup(tmp_path):
    """A table line applies only inside its (dtype, C, R, work) bucket;
    outside every line the built-in rule decides."""
    R = int(max(rsg.rsg_fit_boxes(8.0, 3).r[:3]))
    n = 64 * 4096
    table = tmp_path / "t.txt"
    table.write_text("# comment\n1 1 %d %d %d %d 96\n0 1 0 1000 0 %d 40  # other dtype\n" % (R, R, n, n, 1 << 40))
    empty = tmp_path / "empty.txt"
    empty.write_text("")
    a, b, c, d = _plans_with_table(table)
    _, b0, _, d0 = _plans_with_table(empty)
    assert a == 96                 # inside the bucket
    assert b == b0                 # work size outside the line: built-in rule
    assert c == 40                 # uint8 line
    assert d == d0                 # R outside the line's range: built-in rule


def _run_planner_code(code, table_text=""):
    """Run planner checks in a fresh process whose tuning table holds
    `table_text` (empty: the built-in rule decides)."""
    import tempfile
    with tempfile.NamedTemporaryFile("w", suffix=".txt", delete=False) as f:
        f.write(table_text)
    env = dict(os.environ, RSG_TUNE_TABLE=f.name, PYTHONPATH=ROOT)
    pre = ("import sys; sys.path.insert(0, %r)\nimport paper_1107_4958_amd as rsg, pytest\n"
           "from test_plan_cpu import _desc\n" % os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", pre + code], env=env, capture_output=True, text=True, timeout=300)
    os.unlink(f.name)
    assert out.returncode == 0, out.stderr
    return out.stdout


def test_wide_boxes_take_the_two_pass_path():
    """Built-in rule: wide boxes (R * C >= 40) take the two passes, narrow
    ones the fused kernel; a table line with hs = -1 selects two passes;
    the path override wins over both."""
    _run_planner_code(
        "hs, tasks, lds = rsg.rsg_plan_shape(_desc(8192, 8192, sigma=64.0, K=5))\n"
        "assert hs == 8192 and tasks == 8192 // 16 + 8192 // 16\n"
        "assert rsg.rsg_plan_shape(_desc(4096, 4096, sigma=8.0, K=3))[0] < 4096\n"
        "rsg.rsg_tune_path(rsg.RSG_PATH_FUSED)\n"
        "assert rsg.rsg_plan_shape(_desc(8192, 8192, sigma=64.0, K=5))[0] < 8192\n"
        "rsg.rsg_tune_path(rsg.RSG_PATH_TWO_PASS)\n"
        "assert rsg.rsg_plan_shape(_desc(64, 64, sigma=1.0, K=3))[0] == 64\n"
        "with pytest.raises(rsg.RsgError):\n    rsg.rsg_tune_path(4)\n")
    R = int(max(rsg.rsg_fit_boxes(8.0, 3).r[:3]))
    _run_planner_code("assert rsg.rsg_plan_shape(_desc(4096, 4096, sigma=8.0, K=3))[0] == 4096\n",
                      "1 1 %d %d 0 %d -1\n" % (R, R, 1 << 40))


def test_plan_does_not_depend_on_the_boundary():
    """Every boundary mode plans the same tile (the extension only changes
    which samples the border loads read)."""
    for H, W, C, sigma in ((4096, 4096, 1, 8.0), (37, 523, 3, 7.5), (1, 1, 1, 2.0), (96, 96, 4, 40.0)):
        shapes = []
        for b in (rsg.RSG_REPLICATE, rsg.RSG_ZERO, rsg.RSG_REFLECT):
            d = _desc(H, W, C, sigma=sigma)
            d.b = b
            shapes.append(rsg.rsg_plan_shape(d))
        assert shapes[0] == shapes[1] == shapes[2], (H, W, C, shapes)


def test_table_strip_width_field():
    """A table line's optional last field selects the strip width: 2 the wide
    form (128-sample strips at C = 1, 64-pixel strips at C = 3), 1 or no
    field one column per lane; the override wins over the table."""
    R = int(max(rsg.rsg_fit_boxes(8.0, 3).r[:3]))
    _run_planner_code(
        "hs, tasks, _ = rsg.rsg_plan_shape(_desc(4096, 4096, sigma=8.0, K=3))\n"
        "assert hs == 256 and tasks == 32 * 16, (hs, tasks)\n"
        "rsg.rsg_tune_columns(1)\n"
        "hs, tasks, _ = rsg.rsg_plan_shape(_desc(4096, 4096, sigma=8.0, K=3))\n"
        "assert tasks == 64 * 16, tasks\n",
        "1 1 %d %d 0 %d 256 2\n" % (R, R, 1 << 40))
    _run_planner_code(
        "hs, tasks, _ = rsg.rsg_plan_shape(_desc(4096, 4096, sigma=8.0, K=3))\n"
        "assert hs == 256 and tasks == 64 * 16, (hs, tasks)\n",
        "1 1 %d %d 0 %d 256\n1 1 0 1000 0 %d 128 1\n" % (R, R, 1 << 40, 1 << 40))


def test_table_first_layout_field():
    """The table's layout field (and rsg_tune_layout) starts the planner's
    search at a wider row-scan layout: same strips and segments, another
    row tile (fewer, wider rows per group); out-of-range values are refused."""
    R = int(max(rsg.rsg_fit_boxes(8.0, 3).r[:3]))
    _run_planner_code(
        "hs, tasks, lds = rsg.rsg_plan_shape(_desc(4096, 4096, sigma=8.0, K=3))\n"
        "rsg.rsg_tune_layout(0)\n"
        "hs0, tasks0, lds0 = rsg.rsg_plan_shape(_desc(4096, 4096, sigma=8.0, K=3))\n"
        "assert (hs, tasks) == (hs0, tasks0) == (256, 64 * 16) and lds == lds0, (hs, tasks, lds)\n"
        "rsg.rsg_tune_layout(2)\n"
        "hs2, tasks2, lds2 = rsg.rsg_plan_shape(_desc(4096, 4096, sigma=8.0, K=3))\n"
        "assert (hs2, tasks2) == (256, 64 * 16) and lds2 != lds, (lds2, lds)\n"
        "with pytest.raises(rsg.RsgError):\n    rsg.rsg_tune_layout(4)\n",
        "1 1 %d %d 0 %d 256 1 0\n" % (R, R, 1 << 40))
    a = _run_planner_code("print(rsg.rsg_plan_shape(_desc(4096, 4096, sigma=8.0, K=3))[2])\n",
                          "1 1 %d %d 0 %d 256 1 1\n" % (R, R, 1 << 40))
    b = _run_planner_code("print(rsg.rsg_plan_shape(_desc(4096, 4096, sigma=8.0, K=3))[2])\n",
                          "1 1 %d %d 0 %d 256 1\n" % (R, R, 1 << 40))
    assert int(a) != int(b)


def test_table_store_form_field():
    """The table's store-form field (and rsg_tune_stores) is read with the
    plan: staged stores use the wave's existing row tile, so the segments,
    tasks and LDS are those of the per-lane stores; out-of-range values are
    refused."""
    R = int(max(rsg.rsg_fit_boxes(8.0, 3).r[:3]))
    shapes = [_run_planner_code("print(*rsg.rsg_plan_shape(_desc(4096, 4096, sigma=8.0, K=3)))\n",
                                "1 1 %d %d 0 %d 256 1 0 %d\n" % (R, R, 1 << 40, st)) for st in (1, 2)]
    assert shapes[0] == shapes[1] and shapes[0].split()[:2] == ["256", str(64 * 16)], shapes
    _run_planner_code(
        "for form in (0, 1, 2, 0):\n    rsg.rsg_tune_stores(form)\n"
        "for bad in (-1, 3):\n    with pytest.raises(rsg.RsgError):\n        rsg.rsg_tune_stores(bad)\n",
        "1 1 %d %d 0 %d 256 1 0 2\n" % (R, R, 1 << 40))


def test_channel_planar_plan():
    """Channel-planar tasks: one task per 64 pixels of one channel; the row
    span (and so the tile) is that of a one-channel image."""
    try:
        rsg.rsg_tune_columns(1)
        hs1, t1, lds1 = rsg.rsg_plan_shape(_desc(2048, 2048, C=3, dt=rsg.RSG_U8, sigma=8.0, K=4))
        rsg.rsg_tune_columns(3)
        hs3, t3, lds3 = rsg.rsg_plan_shape(_desc(2048, 2048, C=3, dt=rsg.RSG_U8, sigma=8.0, K=4))
        assert t1 == -(-2048 * 3 // 64) * -(-2048 // hs1)
        assert t3 == 3 * (2048 // 64) * -(-2048 // hs3)
        h, t, _ = rsg.rsg_plan_shape(_desc(100, 70, C=1, dt=rsg.RSG_U8))   # one channel: unchanged
        assert t == 2 * -(-100 // h)
        with pytest.raises(rsg.RsgError):
            rsg.rsg_tune_columns(4)
    finally:
        rsg.rsg_tune_columns(0)


def test_too_wide_for_interleaved_and_two_pass_takes_planar_tasks():
    """Four channels with boxes too wide for both the interleaved span and
    the two-pass window: the planner falls back to channel-planar tasks
    (was RSG_EUNSUPPORTED)."""
    _run_planner_code(
        "hs, tasks, lds = rsg.rsg_plan_shape(_desc(1024, 1024, C=4, dt=rsg.RSG_U8, sigma=64.0, K=5))\n"
        "assert tasks == 4 * (1024 // 64) * -(-1024 // hs), (hs, tasks)\n"
        "rsg.rsg_tune_path(rsg.RSG_PATH_FUSED_ONE_WAVE)\n"
        "with pytest.raises(rsg.RsgError):\n"
        "    rsg.rsg_plan_shape(_desc(1024, 1024, C=4, dt=rsg.RSG_U8, sigma=64.0, K=5))\n")


def test_autotune_store_field():
    """The tuner records a measured store form only where it departs from
    the planner's rule at the measured tap count (staged at four and five
    taps): a staged win at three taps, a per-lane win at four or five."""
    from paper_1107_4958_amd.autotune import store_field
    assert [store_field(st, 3) for st in (0, 1, 2)] == [0, 0, 2]
    for K in (4, 5):
        assert [store_field(st, K) for st in (0, 1, 2)] == [0, 1, 0]
