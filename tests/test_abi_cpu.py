"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/hbt.h, and rejects bad arguments on the host before
anything is enqueued (no compute call is made here)."""
import ctypes as C
import os
import re
from pathlib import Path

import pytest

from paper_2605_08048_amd import hbt

ROOT = Path(__file__).resolve().parents[1]
HEADER = ROOT / "include" / "hbt.h"

pytestmark = pytest.mark.skipif(not hbt.LIB_PATH.exists(), reason="libhbt.so not built")


def declared_functions():
    text = re.sub(r"/\*.*?\*/", "", HEADER.read_text(), flags=re.S)
    return sorted(set(re.findall(r"\b(hbt_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_three_calls():
    names = declared_functions()
    for f in ["hbt_align", "hbt_perm_test", "hbt_perm_test_batched"]:
        assert f in names


def test_library_exports_every_declared_symbol():
    L = hbt.lib()
    missing = [f for f in declared_functions() if not hasattr(L, f)]
    assert not missing, missing
    assert L.hbt_abi_version() == 2


def test_struct_sizes_match_header():
    assert C.sizeof(hbt.HbtResult) == 112
    assert C.sizeof(hbt.HbtPermParams) == 96
    assert hbt.HbtPermParams.masks.offset == 88 and hbt.HbtPermParams.block_perms.offset == 80


def test_status_strings():
    L = hbt.lib()
    for s in range(11):
        assert L.hbt_status_string(s)
    assert L.hbt_status_string(99) == b"unknown status"


FAKE = C.c_void_p(0x1000)  # never dereferenced: every case below fails validation first


def _call(prm, X=FAKE, Y=FAKE, res=FAKE, ws=FAKE, ws_bytes=1 << 40):
    return hbt.lib().hbt_perm_test(X, Y, C.byref(prm), res, None, None, ws, ws_bytes, None)


@pytest.mark.parametrize("n,m,d,B,status", [
    (1, 10, 8, 10, hbt.ERR_SIZE), (10, 1, 8, 10, hbt.ERR_SIZE), (10, 10, 0, 10, hbt.ERR_SIZE),
    (10, 10, 8, 0, hbt.ERR_SIZE), (40000, 30000, 8, 10, hbt.ERR_SIZE), (10, 10, 9000, 10, hbt.ERR_SIZE),
])
def test_perm_test_rejects_bad_sizes(n, m, d, B, status):
    assert _call(hbt.make_params(n, m, d, B)) == status
    assert hbt.lib().hbt_last_error()


def test_perm_test_rejects_null_pointers_and_enums():
    prm = hbt.make_params(10, 12, 8, 10)
    assert _call(prm, X=None) == hbt.ERR_ARG
    assert _call(prm, res=None) == hbt.ERR_ARG
    assert hbt.lib().hbt_perm_test(FAKE, FAKE, None, FAKE, None, None, FAKE, 1 << 40, None) == hbt.ERR_ARG
    for field, bad, st in [("precision", 7, hbt.ERR_ARG), ("input_dtype", 5, hbt.ERR_DTYPE),
                           ("gd", 3, hbt.ERR_ARG), ("alternative", 2, hbt.ERR_ARG),
                           ("align", 2, hbt.ERR_ARG), ("flags", 8, hbt.ERR_ARG),
                           ("stat_route", 5, hbt.ERR_ARG), ("block_perms", -1, hbt.ERR_ARG)]:
        p = hbt.make_params(10, 12, 8, 10)
        setattr(p, field, bad)
        assert _call(p) == st, field


def test_perm_offset_overflow():
    prm = hbt.make_params(10, 12, 8, 100, perm_offset=2**32 - 50)
    assert _call(prm) == hbt.ERR_ARG
    # offsets whose sum with B wraps around 2^64 are rejected too
    for off in (2**64 - 1, 2**64 - 50, 2**33):
        assert _call(hbt.make_params(10, 12, 8, 100, perm_offset=off)) == hbt.ERR_ARG, off
    # the last valid window ends exactly at 2^32 (it fails later, on the fake workspace pointer's size)
    assert _call(hbt.make_params(10, 12, 8, 100, perm_offset=2**32 - 100), ws_bytes=0) == hbt.ERR_WORKSPACE


def test_bindings_check_operands_before_any_device_call():
    """Shapes, lengths and row ranges the library cannot see are checked in the
    binding, and host tensors are refused before a pointer reaches the library."""
    torch = pytest.importorskip("torch")
    Z = torch.zeros(10, 8)
    with pytest.raises(hbt.HbtError, match="outside Z_all's 10 rows"):
        hbt.perm_test_batched(Z, [0, 4], [2, 3], [2, 4], 10)
    with pytest.raises(hbt.HbtError, match="outside Z_all's 10 rows"):
        hbt.perm_test_batched(Z, [-1], [2], [2], 10)
    with pytest.raises(hbt.HbtError, match="one entry per pair"):
        hbt.perm_test_batched(Z, [0], [2, 2], [2, 2], 10)
    with pytest.raises(hbt.HbtError, match="must be \\(rows, d\\)"):
        hbt.perm_test_batched(torch.zeros(10), [0], [2], [2], 10)
    with pytest.raises(hbt.HbtError, match="Z_all must be a GPU tensor"):
        hbt.perm_test_batched(Z, [0, 4], [2, 3], [2, 3], 10)
    # a cumulative offset table (P + 1 entries) is accepted; too few entries are not
    with pytest.raises(hbt.HbtError, match="Z_all must be a GPU tensor"):
        hbt.perm_test_batched(Z, [0, 4, 10], [2, 3], [2, 3], 10)
    with pytest.raises(hbt.HbtError, match="one entry per pair"):
        hbt.perm_test_batched(Z, [0], [2, 3], [2, 3], 10)
    X, Y = torch.zeros(5, 8), torch.zeros(6, 8)
    with pytest.raises(hbt.HbtError, match="must be \\(n, d\\) and \\(m, d\\)"):
        hbt.perm_test(X, torch.zeros(6, 7), 10)
    with pytest.raises(hbt.HbtError, match="X must be a GPU tensor"):
        hbt.perm_test(X, Y, 10)
    with pytest.raises(hbt.HbtError, match="X must be a GPU tensor"):
        hbt.align(X, Y)


def test_allocator_bindings_refuse_host_tensors():
    torch = pytest.importorskip("torch")
    F, T = torch.zeros(4, hbt.MLP_FEATURES), torch.zeros(4, 2)
    th = torch.zeros(hbt.MLP_PARAMS)
    res = torch.zeros(4 * hbt.RESULT_BYTES, dtype=torch.uint8)
    for call in (lambda: hbt.budget_features(res, 8), lambda: hbt.null_targets(res),
                 lambda: hbt.feature_norm(F, th), lambda: hbt.target_norm(T, th),
                 lambda: hbt.mlp_forward(F, th), lambda: hbt.mlp_grad(F, T, th),
                 lambda: hbt.mlp_adam(th, th, th, th, 1), lambda: hbt.budgets(T, res, 0.01, 0.1, 10, 100)):
        with pytest.raises(hbt.HbtError, match="must be a GPU tensor"):
            call()


def test_workspace_size_and_too_small_workspace():
    L = hbt.lib()
    prm = hbt.make_params(2000, 1500, 768, 10000, precision="bf16x2")
    need = L.hbt_perm_test_workspace_size(C.byref(prm))
    # Z planes alone: 3520 rows x 768 x 4 bytes
    assert need > 3520 * 768 * 4
    assert _call(prm, ws_bytes=need - 1) == hbt.ERR_WORKSPACE
    assert _call(prm, ws=None) == hbt.ERR_WORKSPACE
    bad = hbt.make_params(1, 1500, 768, 10)
    assert L.hbt_perm_test_workspace_size(C.byref(bad)) == 0
    # more splits per block need more workspace; B0 = 1 needs the least
    small = hbt.make_params(2000, 1500, 768, 10000, precision="bf16x2", block_perms=1)
    assert L.hbt_perm_test_workspace_size(C.byref(small)) < need


def test_align_validation():
    L = hbt.lib()
    assert L.hbt_align(0, None, 10, FAKE, 10, 8, 1, 0, FAKE, None, FAKE, FAKE, 1 << 30, None) == hbt.ERR_ARG
    assert L.hbt_align(0, FAKE, 1, FAKE, 10, 8, 1, 0, FAKE, None, FAKE, FAKE, 1 << 30, None) == hbt.ERR_SIZE
    assert L.hbt_align(3, FAKE, 10, FAKE, 10, 8, 1, 0, FAKE, None, FAKE, FAKE, 1 << 30, None) == hbt.ERR_DTYPE
    need = L.hbt_align_workspace_size(10, 10, 8)
    assert need > 0
    assert L.hbt_align(0, FAKE, 10, FAKE, 10, 8, 1, 0, FAKE, None, FAKE, FAKE, need - 1, None) == hbt.ERR_WORKSPACE


def test_batched_validation():
    import numpy as np
    L = hbt.lib()
    P = 3
    n = np.array([10, 20, 1], dtype=np.int64)
    m = np.array([10, 20, 30], dtype=np.int64)
    B = np.array([5, 5, 5], dtype=np.int64)
    off = np.array([0, 20, 60, 91], dtype=np.int64)
    ptr = lambda a: a.ctypes.data_as(C.c_void_p)
    prm = hbt.make_params(0, 0, 8, 0, precision="bf16x2")
    assert L.hbt_perm_test_batched_workspace_size(P, ptr(n), ptr(m), ptr(B), 8, C.byref(prm)) == 0
    st = L.hbt_perm_test_batched(P, FAKE, ptr(off), ptr(n), ptr(m), ptr(B), None, 8, C.byref(prm), FAKE,
                                 FAKE, 1 << 40, None)
    assert st == hbt.ERR_SIZE and b"pair 2" in L.hbt_last_error()
    n[2] = 3
    need = L.hbt_perm_test_batched_workspace_size(P, ptr(n), ptr(m), ptr(B), 8, C.byref(prm))
    assert need > 0
    st = L.hbt_perm_test_batched(P, FAKE, ptr(off), ptr(n), ptr(m), ptr(B), None, 8, C.byref(prm), FAKE,
                                 FAKE, need - 1, None)
    assert st == hbt.ERR_WORKSPACE
    st = L.hbt_perm_test_batched(0, FAKE, ptr(off), ptr(n), ptr(m), ptr(B), None, 8, C.byref(prm), FAKE,
                                 FAKE, need, None)
    assert st == hbt.ERR_SIZE
    # the point-to-centroid route needs more workspace (centroids, an FP32
    # copy of the rows, its partial sums), and the int8 planes do not have it
    prm.stat_route = 1
    need2 = L.hbt_perm_test_batched_workspace_size(P, ptr(n), ptr(m), ptr(B), 8, C.byref(prm))
    assert need2 > need
    st = L.hbt_perm_test_batched(P, FAKE, ptr(off), ptr(n), ptr(m), ptr(B), None, 8, C.byref(prm), FAKE,
                                 FAKE, need, None)
    assert st == hbt.ERR_WORKSPACE
    for prec in ("i8x3", "bf16e4m3", "bf16lazy"):  # route 0 only
        prm.precision = hbt.PRECISION[prec]
        st = L.hbt_perm_test_batched(P, FAKE, ptr(off), ptr(n), ptr(m), ptr(B), None, 8, C.byref(prm), FAKE,
                                     FAKE, need2, None)
        assert st == hbt.ERR_UNSUPPORTED, prec
    # the lazy precision stores as split BF16 and adds its refinement lists
    prm.stat_route = 0
    prm.precision = hbt.PRECISION["bf16lazy"]
    need_lazy = L.hbt_perm_test_batched_workspace_size(P, ptr(n), ptr(m), ptr(B), 8, C.byref(prm))
    assert need_lazy > need
    st = L.hbt_perm_test_batched(P, FAKE, ptr(off), ptr(n), ptr(m), ptr(B), None, 8, C.byref(prm), FAKE,
                                 FAKE, need, None)
    assert st == hbt.ERR_WORKSPACE


def test_lazy_precision_workspace_and_route():
    """The lazy split-BF16 precision stores as split BF16 and adds its
    refinement list, so the single-pair call needs a little more workspace;
    the point-to-centroid route refuses it before anything is enqueued."""
    L = hbt.lib()
    lazy = hbt.make_params(300, 400, 64, 5000, precision="bf16lazy")
    split = hbt.make_params(300, 400, 64, 5000, precision="bf16x2")
    assert L.hbt_perm_test_workspace_size(C.byref(lazy)) > L.hbt_perm_test_workspace_size(C.byref(split)) > 0
    assert _call(hbt.make_params(10, 12, 8, 10, precision="bf16lazy", stat_route=1)) == hbt.ERR_UNSUPPORTED
    # its tuning entry is the split-BF16 one
    e = hbt.HbtTuneEntry()
    for f in (L.hbt_tune_entry_get, L.hbt_tune_entry_set):
        assert f(hbt.PRECISION["bf16lazy"], 768, C.byref(e)) == hbt.ERR_ARG
        assert b"split-BF16 entry" in L.hbt_last_error()


def test_clouds_validation():
    """The shared-clouds call refuses what it does not cover before anything
    is enqueued: other precisions, a cloud index out of range, odd d, a cloud
    of fewer than 2 rows, a too-small workspace."""
    L = hbt.lib()
    ptr = lambda a: a.ctypes.data_as(C.c_void_p)
    import numpy as np
    FAKE = C.c_void_p(256)
    rows = np.array([40, 70, 33], dtype=np.int64)
    off = np.array([0, 40, 110], dtype=np.int64)
    px, py = np.array([0, 1], dtype=np.int64), np.array([1, 2], dtype=np.int64)
    B = np.array([100, 200], dtype=np.int64)
    prm = hbt.make_params(0, 0, 64, 0, precision="bf16x2")
    need = L.hbt_perm_test_clouds_workspace_size(3, ptr(rows), 2, ptr(px), ptr(py), ptr(B), 64, C.byref(prm))
    assert need > 0
    call = lambda prm, rows=rows, px=px, d=64, ws=need: L.hbt_perm_test_clouds(
        3, FAKE, ptr(off), ptr(rows), 2, ptr(px), ptr(py), ptr(B), None, d, C.byref(prm), FAKE, FAKE, ws, None)
    assert call(prm, ws=need - 1) == hbt.ERR_WORKSPACE
    assert call(prm, px=np.array([0, 3], dtype=np.int64)) == hbt.ERR_ARG
    assert call(prm, rows=np.array([40, 1, 33], dtype=np.int64)) == hbt.ERR_SIZE
    assert call(prm, d=66) == hbt.ERR_UNSUPPORTED
    for prec in ("f32", "i8x3", "bf16e4m3", "bf16lazy"):
        assert call(hbt.make_params(0, 0, 64, 0, precision=prec)) == hbt.ERR_UNSUPPORTED
    assert call(hbt.make_params(0, 0, 64, 0, precision="bf16x2", stat_route=1)) == hbt.ERR_UNSUPPORTED


def test_tile_width_rule_and_tuning_table(tmp_path):
    """Per pair, the width w in {1024, 256} minimising cost_w * round_up(B, w)."""
    import numpy as np
    d = 4160  # a dimension no other test tunes
    (cw, c256), tuned = hbt.tune_get(d)
    assert (cw, c256) == (1.0, 1.15) and not tuned
    B = np.array([1, 200, 250, 256, 257, 300, 512, 700, 1000, 1025, 2000, 20000])
    want = [256 if c256 * -(-b // 256) * 256 < cw * -(-b // 1024) * 1024 else 1024 for b in B]
    assert list(hbt.tile_widths(B, d)) == want
    assert list(hbt.tile_widths([200, 2000], d)) == [256, 1024]
    hbt.tune_set(d, [1.0, 5.0])
    assert list(hbt.tile_widths(B, d)) == [1024] * len(B)
    assert hbt.tune_get(d) == ((1.0, 5.0), True)
    # whole entries, per precision; the JSON cache round-trips through the
    # library's table
    e = hbt.tune_entry_get("bf16x2", d)
    assert e["cost"] == (1.0, 5.0) and e["tuned"] and (e["grid_wide"], e["grid_narrow"]) == (16, 32)
    assert (e["split_cap"], e["chunks"]) == (6, 1)
    i8 = hbt.tune_entry_get("i8x3", d)
    assert not i8["tuned"] and i8["grid_narrow"] == 16
    hbt.tune_entry_set("i8x3", d, dict(cost=(1.0, 1.0), grid_wide=8, grid_narrow=24, split_cap=5, chunks=2))
    f = tmp_path / "tune.json"
    hbt.save_tuning(f)
    hbt.tune_set(d, [2.0, 1.0])
    hbt.tune_entry_set("i8x3", d, dict(cost=(3.0, 3.0), grid_wide=1, grid_narrow=1, split_cap=1, chunks=1))
    hbt.load_tuning(f)
    assert hbt.tune_get(d) == ((1.0, 5.0), True)
    got = hbt.tune_entry_get("i8x3", d)
    assert (got["grid_wide"], got["grid_narrow"], got["split_cap"], got["chunks"]) == (8, 24, 5, 2)
    # a malformed file changes nothing
    bad = tmp_path / "bad.json"
    bad.write_text(f.read_text().replace('"chunks": 2', '"chunks": 99'))
    with pytest.raises(hbt.HbtError):
        hbt.load_tuning(bad)
    assert hbt.tune_entry_get("i8x3", d)["chunks"] == 2
    with pytest.raises(hbt.HbtError):
        hbt.tune_entry_set("i8x3", d, dict(cost=(1.0, 1.0), grid_wide=0, grid_narrow=24, split_cap=5, chunks=2))
    L = hbt.lib()
    assert L.hbt_tune_set(d, (C.c_double * 2)(1.0, -1.0)) == hbt.ERR_ARG
    assert L.hbt_tile_widths(1, (C.c_int64 * 1)(0), d, (C.c_int32 * 1)()) == hbt.ERR_SIZE


def test_tuning_cache_is_read_on_first_use(tmp_path):
    """HBT_TUNE_CACHE names a JSON file the library reads on first use."""
    import subprocess
    import sys
    import textwrap
    f = tmp_path / "cache.json"
    f.write_text('{"hbt_tune_version": 1, "entries": [\n'
                 ' {"precision": 2, "d_pad": 320, "cost": [2.5, 1.5], "grid_wide": 8, "grid_narrow": 4, '
                 '"split_cap": 5, "chunks": 3}\n]}\n')
    code = textwrap.dedent(f"""
        import sys
        sys.path.insert(0, {str(ROOT)!r})
        from paper_2605_08048_amd import hbt
        e = hbt.tune_entry_get("bf16x2", 300)
        assert e == {{"cost": (2.5, 1.5), "grid_wide": 8, "grid_narrow": 4, "split_cap": 5, "chunks": 3,
                      "tuned": True}}, e
        assert not hbt.tune_entry_get("bf16x2", 1000)["tuned"]
        print("ok")
    """)
    env = dict(os.environ, HBT_TUNE_CACHE=str(f))
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stderr


def test_plans_whose_tile_lists_overflow_are_refused():
    """The product kernels number tiles with 32-bit integers: a plan that
    would need more (4096 pairs of about 2^20 splits at d = 8192 in the lazy
    precision, whose refinement could list every split; one pair in a single
    block of 2^32 - 1 splits at d = 8192) is refused with HBT_ERR_SIZE before
    anything is enqueued, and its workspace size is reported as 0."""
    import numpy as np
    L = hbt.lib()
    P = 4096
    n = np.full(P, 2, dtype=np.int64)
    m = np.full(P, 2, dtype=np.int64)
    B = np.full(P, (1 << 20) - 1, dtype=np.int64)
    off = np.arange(P + 1, dtype=np.int64) * 4
    ptr = lambda a: a.ctypes.data_as(C.c_void_p)
    lazy = hbt.make_params(0, 0, 8192, 0, precision="bf16lazy")
    assert L.hbt_perm_test_batched_workspace_size(P, ptr(n), ptr(m), ptr(B), 8192, C.byref(lazy)) == 0
    st = L.hbt_perm_test_batched(P, FAKE, ptr(off), ptr(n), ptr(m), ptr(B), None, 8192, C.byref(lazy), FAKE,
                                 FAKE, 1 << 60, None)
    assert st == hbt.ERR_SIZE and b"product tiles" in L.hbt_last_error()
    # the same batch in split BF16 takes 1024-split tiles and fits
    split = hbt.make_params(0, 0, 8192, 0, precision="bf16x2")
    assert L.hbt_perm_test_batched_workspace_size(P, ptr(n), ptr(m), ptr(B), 8192, C.byref(split)) > 0
    one = hbt.make_params(300, 200, 8192, (1 << 32) - 1, precision="bf16x2", block_perms=(1 << 32) - 1)
    assert L.hbt_perm_test_workspace_size(C.byref(one)) == 0
    assert _call(one) == hbt.ERR_SIZE and b"product tiles" in L.hbt_last_error()
    one.block_perms = 0  # blocks of 32768 splits
    assert L.hbt_perm_test_workspace_size(C.byref(one)) > 0
