"""C-ABI boundary checks that need no GPU: the library loads, exports every
function include/mpjsvd.h declares, and validates arguments before touching
the device."""
import ctypes
import os
import re

import pytest

import paper_2209_04626_amd as mp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "mpjsvd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_]\w*\s*\**\s*((?:svd|eig)_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_function():
    lib = mp.load()
    declared = header_functions()
    assert len(declared) >= 10
    assert set(declared) == set(mp.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def test_default_options_are_the_papers():
    o = mp.default_opts(mixed=True)
    assert o.tol_alg == 1e-2 and o.tol_orth == 1e-5 and o.tol_cond_coef == 1.5
    assert o.pivot_precision == 32 and o.want_u == 1 and o.want_v == 1
    assert mp.default_opts(mixed=False).pivot_precision == 64
    # right singular vectors: Section 3.4's solve in the mixed path,
    # accumulated rotations in the plain one
    assert o.v_method == 1 and mp.default_opts(mixed=False).v_method == 0
    assert o.tol_vsolve == 0.0 and o.diagnostics == 0 and o.inner_pairs == 0


def test_workspace_size_monotone_and_invalid():
    sizes = [mp.workspace_size(n, n) for n in (1, 16, 64, 65, 200, 1024)]
    assert all(a <= b for a, b in zip(sizes, sizes[1:]))
    assert mp.workspace_size(10, 20) == 0          # m < n
    assert mp.workspace_size(100, 50) > mp.workspace_size(50, 50)


@pytest.mark.parametrize("mode", ["plain", "mixed"])
def test_argument_errors_return_before_device_work(mode):
    # LAPACK convention: -k for invalid argument k; nothing is launched
    assert mp.call_raw(mode, 3, 5, 1, 3, 1, 1, 3, 1, 5, 1, 1 << 30, None, 0)[0] == -2
    assert mp.call_raw(mode, 5, 3, 0, 5, 1, 1, 5, 1, 3, 1, 1 << 30, None, 0)[0] == -3
    assert mp.call_raw(mode, 5, 3, 1, 4, 1, 1, 5, 1, 3, 1, 1 << 30, None, 0)[0] == -4
    assert mp.call_raw(mode, 5, 3, 1, 5, 1, 1, 4, 1, 3, 1, 1 << 30, None, 0)[0] == -7
    assert mp.call_raw(mode, 5, 3, 1, 5, 1, 1, 5, 1, 2, 1, 1 << 30, None, 0)[0] == -9
    assert mp.call_raw(mode, 5, 3, 1, 5, 1, 1, 5, 1, 3, 0, 1 << 30, None, 0)[0] == -10
    assert mp.call_raw(mode, 5, 3, 1, 5, 1, 1, 5, 1, 3, 1, 16, None, 0)[0] == -11
    # n = 0 is a no-op
    assert mp.call_raw(mode, 4, 0, 0, 4, 0, 0, 4, 0, 1, 0, 0, None, 0)[0] == 0


def test_backward_argument_errors():
    lib = mp.load()
    assert lib.svd_backward(1, 3, 5, 1, 15, 1, 5, 1, 25, None, None, None, 1, 15, 0.0, 1, 1 << 20, None) == -2
    assert mp.load().svd_backward_workspace_size(2, 8, 4) > 0


def test_status_strings():
    lib = mp.load()
    assert lib.svd_status_string(0) == b"ok"
    assert b"NaN" in lib.svd_status_string(2)
    assert b"invalid" in lib.svd_status_string(-3)


def test_tuning_table_parse_lookup_and_reject():
    """svd_set_tuning: the smallest nmax >= n applies, unknown members are
    ignored, malformed or invalid tables are rejected and leave the loaded
    table unchanged; the committed table (if any) is restored afterwards."""
    lib = mp.load()
    saved = open(mp.TUNE_PATH).read() if os.path.exists(mp.TUNE_PATH) else None
    try:
        mp.set_tuning('{"arch": "gfx950", "note": [1, {"x": "y"}], "flag": true,'
                      ' "single": [{"nmax": 4096, "b_low": 16, "b_work": 32},'
                      '            {"nmax": 128, "b_low": 32, "b_work": 16, "ms": 1.5}],'
                      ' "batched": [{"nmax": 256, "wg_per_cu": 3}]}')
        assert mp.tuning_lookup(100) == {"b_low": 32, "b_work": 16, "wg_per_cu": 3}
        assert mp.tuning_lookup(128) == {"b_low": 32, "b_work": 16, "wg_per_cu": 3}
        assert mp.tuning_lookup(129) == {"b_low": 16, "b_work": 32, "wg_per_cu": 3}
        assert mp.tuning_lookup(257) == {"b_low": 16, "b_work": 32, "wg_per_cu": 0}
        assert mp.tuning_lookup(5000) == {"b_low": 0, "b_work": 0, "wg_per_cu": 0}
        for bad, code in (('{', -2), ('{"single": [1, 2]}', -2), ('{"a": tru}', -2),
                          ('{"single": [{"nmax": 0, "b_low": 16, "b_work": 16}]}', -3),
                          ('{"single": [{"nmax": 9, "b_low": 8, "b_work": 16}]}', -3),
                          ('{"batched": [{"nmax": 9, "wg_per_cu": 99}]}', -3)):
            assert lib.svd_set_tuning(bad.encode()) == code, bad
        assert mp.tuning_lookup(100)["b_low"] == 32          # unchanged
        mp.set_tuning(None)
        assert lib.svd_tuning_lookup(100, None, None, None) == 0
    finally:
        mp.set_tuning(saved)


def test_committed_tuning_table_is_loaded():
    if not os.path.exists(mp.TUNE_PATH):
        pytest.skip("no tuning table committed")
    import json
    table = json.load(open(mp.TUNE_PATH))
    mp.load()
    for e in table["single"]:
        got = mp.tuning_lookup(e["nmax"])
        assert (got["b_low"], got["b_work"]) == (e["b_low"], e["b_work"])
    o = mp.default_opts(True)
    assert o.block_cols == 0 and o.block_cols_low == 0 and o.block_cols_work == 0
