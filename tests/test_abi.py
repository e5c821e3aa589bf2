"""The C-ABI library loads, exports every entry point of include/hpm.h, and rejects bad
arguments on the host before any device work (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hpm.h")
LIB = os.path.join(ROOT, "paper_1906_10734_amd", "libhpm.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hpm_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1906_10734_amd.build import build
        build(verbose=False)
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert "hpm_plan_create" in names and "hpm_plan_execute" in names and "hpm_solve" in names
    for name in names:
        assert hasattr(lib, name), name


def test_binding_covers_the_header():
    from paper_1906_10734_amd import hpm
    assert set(declared_functions()) == set(hpm.SIGNATURES)


def _problem(**kw):
    from paper_1906_10734_amd import hpm
    raw = ("abi", "kernel_id", "m2l_mode", "extended_id", "reserved")
    p = hpm.Problem(**{k: v for k, v in kw.items() if k not in raw}).c()
    if "abi" in kw:
        p.abi = kw["abi"]
    if "kernel_id" in kw:
        p.kernel = kw["kernel_id"]
    if "m2l_mode" in kw:
        p.m2l_mode = kw["m2l_mode"]
    if "extended_id" in kw:
        p.extended = kw["extended_id"]
    if "reserved" in kw:
        p.reserved = kw["reserved"]
    return p


@pytest.mark.parametrize("kw,status", [
    (dict(ng=5), 6), (dict(ng=0), 1), (dict(ng=7), 6), (dict(ng=8), 6), (dict(box_size=0.0), 1),
    (dict(softening=-1.0), 1), (dict(gconst=0.0), 1), (dict(uniform_depth=11), 1),
    (dict(max_depth=11), 1), (dict(leaf_capacity=0), 1), (dict(abi=1), 1), (dict(abi=99), 1),
    (dict(kernel_id=2), 1), (dict(kernel="yukawa", screening=0.0), 1),
    (dict(kernel="yukawa", screening=float("nan")), 1), (dict(m2l_mode=2), 1), (dict(abi=3), 1),
    (dict(extended=True), 6), (dict(extended_id=2, m2l="cells"), 1), (dict(reserved=1), 1),
])
def test_bad_problem_rejected_on_host(kw, status):
    from paper_1906_10734_amd import hpm
    lib = hpm._lib
    p = _problem(**kw)
    out = ctypes.c_void_p(123)
    dummy = ctypes.c_void_p(1)
    st = lib.hpm_plan_create(ctypes.byref(p), 16, dummy, dummy, dummy, None, ctypes.byref(out))
    assert st == status
    assert out.value is None
    assert len(lib.hpm_last_error()) > 0


def test_null_and_size_checks():
    from paper_1906_10734_amd import hpm
    lib = hpm._lib
    p = _problem()
    out = ctypes.c_void_p()
    dummy = ctypes.c_void_p(1)
    assert lib.hpm_plan_create(ctypes.byref(p), 0, dummy, dummy, dummy, None, ctypes.byref(out)) == 1
    assert lib.hpm_plan_create(ctypes.byref(p), 16, None, dummy, dummy, None, ctypes.byref(out)) == 1
    assert lib.hpm_plan_create(None, 16, dummy, dummy, dummy, None, ctypes.byref(out)) == 1
    assert lib.hpm_plan_execute(None, dummy, dummy, dummy, dummy, dummy, None) == 1
    assert lib.hpm_direct_sum(7, 16, dummy, dummy, dummy, dummy, 1, dummy, 1.0, 0.0, 0, 0.0, dummy,
                              dummy, dummy, dummy, None) == 1
    # unknown kernel, and the screened kernel without a screening length
    assert lib.hpm_direct_sum(0, 16, dummy, dummy, dummy, dummy, 1, dummy, 1.0, 0.0, 5, 0.0, dummy,
                              dummy, dummy, dummy, None) == 1
    assert lib.hpm_direct_sum(0, 16, dummy, dummy, dummy, dummy, 1, dummy, 1.0, 0.0, 1, 0.0, dummy,
                              dummy, dummy, dummy, None) == 1
    assert lib.hpm_status_string(2) == b"HPM_ERR_OUT_OF_BOX"
    lib.hpm_plan_destroy(None)
