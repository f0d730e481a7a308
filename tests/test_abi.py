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
    assert L.cpd_abi_version() == 4
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


def test_csf_build_rejects_six_to_eight_modes_without_touching_the_gpu():
    """Trees are built for 2..5 modes: 6..8 are refused before any device work
    (the build kernels are instantiated for at most 5 levels)."""
    from paper_1812_05961_amd import cpd
    L = cpd.lib()
    h = ctypes.c_void_p()
    for nm in (6, 7, 8):
        dims = (ctypes.c_int64 * nm)(*([4] * nm))
        ptrs = (ctypes.c_void_p * nm)(*([1] * nm))
        assert L.cpd_csf_build(nm, dims, 10, ptrs, 1, None, None, ctypes.byref(h)) == cpd.CPD_EUNSUPPORTED
        assert b"2..5 modes" in L.cpd_last_error()
        hs = (ctypes.c_void_p * nm)()
        assert L.cpd_csf_build_rooted(nm, dims, 10, ptrs, 1, None, hs) == cpd.CPD_EUNSUPPORTED
    dims = (ctypes.c_int64 * 9)(*([4] * 9))
    ptrs = (ctypes.c_void_p * 9)(*([1] * 9))
    assert L.cpd_csf_build(9, dims, 10, ptrs, 1, None, None, ctypes.byref(h)) == cpd.CPD_EINVAL


def test_mttkrp_plan_rule():
    """The host-side kernel choice: ROW only for 3..5 modes at non-leaf levels,
    with 16-byte rows inside ld and 32-bit row offsets at every gathered level;
    ROUND only at the leaf level, TILED at every level below the root, both
    with ld a multiple of 4 covering the rank; AUTO takes them where eligible,
    LANE otherwise."""
    from paper_1812_05961_amd import cpd
    plan = cpd.mttkrp_plan
    nell = (9000, 12000, 29000)
    assert plan(nell, 0, 35, ld=36) == "row"
    assert plan(nell, 1, 35, ld=36) == "row"       # internal levels too
    assert plan(nell, 1, 35, ld=36, kernel="lane") == "lane"
    assert plan(nell, 1, 35, ld=36, kernel="row") == "row"
    assert plan(nell, 2, 35, ld=36) == "tiled"     # the leaf level
    assert plan(nell, 2, 35, ld=36, kernel="tiled") == "tiled"
    assert plan(nell, 2, 35, ld=36, kernel="round") == "round"
    assert plan(nell, 2, 35, ld=36, kernel="lane") == "lane"
    with pytest.raises(cpd.CpdError) as e:
        plan(nell, 2, 35, ld=36, kernel="row")
    assert e.value.status == cpd.CPD_EUNSUPPORTED
    # ROUND: leaf level, leaf words, ld % 4 == 0 covering the rank rounded up to 4, aligned rows
    assert plan(nell, 2, 35, ld=35) == "lane"
    assert plan(nell, 2, 5, ld=6) == "lane"
    assert plan(nell, 2, 5, ld=8) == "tiled"
    assert plan(nell, 2, 3, ld=4, precision="bf16") == "tiled"
    assert plan(nell, 2, 16, leaf_words=False) == "lane"
    assert plan(nell, 2, 16, rows_aligned=False) == "lane"
    assert plan((300, 500), 1, 16) == "tiled"
    # TILED: every level below the root, on the same row rules
    assert plan(nell, 1, 35, ld=36, kernel="tiled") == "tiled"
    assert plan((30, 40, 50, 60), 2, 16, kernel="tiled") == "tiled"
    for depth, ld, kernel in ((0, 36, "round"), (1, 36, "round"), (2, 35, "round"), (0, 36, "tiled"),
                              (1, 35, "tiled"), (2, 35, "tiled")):
        with pytest.raises(cpd.CpdError) as e:
            plan(nell, depth, 35, ld=ld, kernel=kernel)
        assert e.value.status == cpd.CPD_EUNSUPPORTED
    # two modes: no ROW kernel is built, AUTO takes LANE at the root
    assert plan((300, 500), 0, 16) == "lane"
    with pytest.raises(cpd.CpdError):
        plan((300, 500), 0, 16, kernel="row")
    # padded rank beyond ld, rows not 16-byte multiples, misaligned factors,
    # trees without leaf words
    assert plan(nell, 0, 35, ld=35) == "lane"
    assert plan(nell, 0, 16, ld=18) == "lane"
    assert plan(nell, 0, 16, rows_aligned=False) == "lane"
    assert plan(nell, 0, 16, leaf_words=False) == "lane"
    assert plan(nell, 0, 16, ld=24, precision="bf16") == "row"
    # 32-bit row offsets: rows * ld * 4 <= 2^32 at every gathered level
    big = 2 ** 32 // (128 * 4)                       # 8,388,608 rows of 512 bytes fit exactly
    assert plan((10, big, 100), 0, 32, ld=128) == "row"
    assert plan((10, big + 1, 100), 0, 32, ld=128) == "lane"
    assert plan((10, 100, big + 1), 0, 32, ld=128) == "lane"
    assert plan((big + 1, 100, 100), 0, 32, ld=128) == "row"   # the output level is not gathered
    assert plan((100, big + 1, 100), 1, 32, ld=128, kernel="row") == "row"
    with pytest.raises(cpd.CpdError):
        plan((big + 1, 100, 100), 1, 32, ld=128, kernel="row")  # root rows gathered below the root
    # row ids below 2^24 even when the offsets fit
    assert plan((10, 2 ** 24, 100), 0, 8, ld=8) == "lane"
    assert plan((10, 2 ** 24 - 1, 100), 0, 8, ld=8) == "row"
    # bad requests
    for args in (((4, 4), 2, 8), ((4, 4, 4), 0, 0), ((4, 4, 4), 0, 65)):
        with pytest.raises(cpd.CpdError) as e:
            plan(*args)
        assert e.value.status == cpd.CPD_EINVAL
    with pytest.raises(cpd.CpdError) as e:
        plan((4,) * 6, 0, 8)
    assert e.value.status == cpd.CPD_EUNSUPPORTED


def test_alloc_limit_hook_without_gpu():
    """The allocation-failure test hook sets and clears a process-wide limit
    without touching the GPU."""
    from paper_1812_05961_amd import cpd
    L = cpd.lib()
    assert L.cpd_set_alloc_limit(1 << 20) == cpd.CPD_OK
    assert L.cpd_set_alloc_limit(-1) == cpd.CPD_OK
    cpd.set_alloc_limit(None)
