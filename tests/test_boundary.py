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
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_]\w*\s*\**\s*(svd_\w+)\s*\(", src, flags=re.M)
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
