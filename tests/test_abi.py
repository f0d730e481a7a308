"""The C-ABI library loads and exports every entry point include/cpd.h declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cpd.h")
LIB = os.path.join(ROOT, "paper_1812_05961_amd", "libcpd.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cpd_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("cpd_csf_build", "cpd_mttkrp", "cpd_als", "cpd_gram", "cpd_solve_normalize",
                 "cpd_fit", "cpd_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "libcpd.so not built"
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (cpd_[a-z0-9_]+)", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing
    L = ctypes.CDLL(LIB)
    for n in declared():
        getattr(L, n)


def test_binding_covers_the_header():
    from paper_1812_05961_amd import cpd
    assert sorted(cpd.exported_symbols()) == declared()


def test_abi_version_and_error_string_without_gpu():
    L = ctypes.CDLL(LIB)
    L.cpd_abi_version.restype = ctypes.c_int32
    assert L.cpd_abi_version() == 2
    L.cpd_last_error.restype = ctypes.c_char_p
    assert L.cpd_last_error() == b""


def test_argument_errors_return_einval_without_touching_the_gpu():
    from paper_1812_05961_amd import cpd
    L = cpd.lib()
    h = ctypes.c_void_p()
    dims = (ctypes.c_int64 * 3)(4, 4, 4)
    # nmodes out of range
    assert L.cpd_csf_build(1, dims, 10, None, None, None, None, ctypes.byref(h)) == cpd.CPD_EINVAL
    assert b"nmodes" in L.cpd_last_error()
    # nnz out of range
    ptrs = (ctypes.c_void_p * 3)(1, 1, 1)
    assert L.cpd_csf_build(3, dims, 0, ptrs, 1, None, None, ctypes.byref(h)) == cpd.CPD_EINVAL
    # order not a permutation
    order = (ctypes.c_int32 * 3)(0, 0, 1)
    assert L.cpd_csf_build(3, dims, 5, ptrs, 1, order, None, ctypes.byref(h)) == cpd.CPD_EINVAL
    # the rooted set checks the same arguments and leaves every output NULL
    hs = (ctypes.c_void_p * 3)(7, 7, 7)
    assert L.cpd_csf_build_rooted(3, dims, 0, ptrs, 1, None, hs) == cpd.CPD_EINVAL
    assert list(hs) == [None, None, None]
    assert L.cpd_csf_build_rooted(1, dims, 10, ptrs, 1, None, hs) == cpd.CPD_EINVAL
    assert L.cpd_csf_build_rooted(3, dims, 5, ptrs, 1, None, None) == cpd.CPD_EINVAL
    # mttkrp on a null handle
    assert L.cpd_mttkrp(None, None, 8, 8, 0, None, 8, None, None) == cpd.CPD_EINVAL
    # als: rank out of range
    f = (ctypes.c_void_p * 3)(1, 1, 1)
    lam = (ctypes.c_double * 8)()
    fit = ctypes.c_double()
    it = ctypes.c_int32()
    assert L.cpd_als(3, dims, 5, ptrs, 1, 0, 5, 0.0, None, f, lam, ctypes.byref(fit),
                     ctypes.byref(it), None) == cpd.CPD_EINVAL
    assert L.cpd_als(3, dims, 5, ptrs, 1, 65, 5, 0.0, None, f, lam, ctypes.byref(fit),
                     ctypes.byref(it), None) == cpd.CPD_EINVAL
