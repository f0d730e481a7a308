"""Python binding of libcpd (ctypes): argument marshalling only.

Every step runs in the HIP library; this module passes torch tensors' device
pointers, sizes and the current HIP stream through the C ABI of
``include/cpd.h`` under the same names.  It raises if the library is missing:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcpd.so")

CPD_OK, CPD_EINVAL, CPD_ENOMEM, CPD_EHIP, CPD_EUNSUPPORTED = range(5)
FP32, BF16_GATHER = 0, 1
VARIANT = {"auto": 0, "atomic": 1, "private": 2}
KERNEL = {"auto": 0, "row": 1, "lane": 2, "round": 3, "tiled": 4}
PRECISION = {"fp32": FP32, "bf16": BF16_GATHER}
MAX_MODES = 8

_P = ctypes.c_void_p
_I32, _I64, _F64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double


class CpdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("cpd status %d: %s" % (status, msg))
        self.status = status


class MttkrpOpts(ctypes.Structure):
    _fields_ = [("precision", _I32), ("variant", _I32), ("kernel", _I32), ("tile_nnz", _I32)]


class AlsOpts(ctypes.Structure):
    _fields_ = [("precision", _I32), ("variant", _I32), ("kernel", _I32), ("tile_nnz", _I32),
                ("single_csf", _I32), ("fast_fit", _I32), ("order", _P), ("init", _P),
                ("seed", ctypes.c_uint64), ("fit_trace", _P), ("timing_ms", _P),
                ("select", _I32), ("selector_hidden", _I32), ("selector_params", _P)]


class Stats(ctypes.Structure):
    _fields_ = [("nmodes", _I32), ("reserved", _I32), ("nnz", _I64), ("sample", _I64),
                ("dims", _I64 * MAX_MODES), ("top1", _F64 * MAX_MODES),
                ("distinct", _F64 * MAX_MODES), ("alpha", _F64 * MAX_MODES)]

    def as_dict(self):
        n = self.nmodes
        return dict(nmodes=n, nnz=self.nnz, sample=self.sample, dims=list(self.dims[:n]),
                    top1=list(self.top1[:n]), distinct=list(self.distinct[:n]),
                    alpha=list(self.alpha[:n]))


class Choice(ctypes.Structure):
    _fields_ = [("order_kind", _I32), ("depth", _I32), ("order", _I32 * MAX_MODES),
                ("opts", MttkrpOpts)]

    def as_dict(self, nmodes):
        return dict(order_kind=ORDER_KINDS[self.order_kind], depth=self.depth,
                    order=list(self.order[:nmodes]), variant=_VARIANT_NAME[self.opts.variant],
                    kernel=_KERNEL_NAME[self.opts.kernel], tile_nnz=self.opts.tile_nnz)


ORDER_KINDS = ("asc", "first", "last", "desc", "rooted")
_VARIANT_NAME = {v: k for k, v in VARIANT.items()}
_KERNEL_NAME = {v: k for k, v in KERNEL.items()}
SEL_MAX_CAND = 24
SEL_NFEAT = 43
SELECT = {"none": 0, "network": 1, "heuristic": 2}


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "cpd_last_error": (ctypes.c_char_p, []),
    "cpd_set_alloc_limit": (_I32, [_I64]),
    "cpd_abi_version": (_I32, []),
    "cpd_csf_build": (_I32, [_I32, _P, _I64, _P, _P, _P, _P, _P]),
    "cpd_csf_build_rooted": (_I32, [_I32, _P, _I64, _P, _P, _P, _P]),
    "cpd_csf_info": (_I32, [_P, _P, _P, _P]),
    "cpd_csf_export": (_I32, [_P, _I32, _P, _P, _P, _P]),
    "cpd_csf_tiles": (_I32, [_P, _I32, _P, _P, _P]),
    "cpd_csf_free": (None, [_P]),
    "cpd_mttkrp": (_I32, [_P, _P, _I32, _I32, _I32, _P, _I32, _P, _P]),
    "cpd_mttkrp_noalloc": (_I32, [_P, _P, _I32, _I32, _I32, _P, _I32, _P, _P]),
    "cpd_mttkrp_noalloc_workspace_bytes": (ctypes.c_size_t, []),
    "cpd_mttkrp_plan": (_I32, [_I32, _P, _I32, _I32, _I32, _I32, _I32, _I32, _I32, _P]),
    "cpd_gram": (_I32, [_P, _I64, _I32, _I32, _P, _P]),
    "cpd_solve_normalize": (_I32, [_P, _I32, _I32, _P, _I64, _I32, _I32, _P, _I32, _P, _I32, _P,
                                   _P, _P, _P]),
    "cpd_fit": (_I32, [_F64, _P, _P, _I32, _P, _I32, _I64, _I32, _P, _I32, _P, _P]),
    "cpd_sumsq": (_I32, [_P, _I64, _P, _P]),
    "cpd_als": (_I32, [_I32, _P, _I64, _P, _P, _I32, _I32, _F64, _P, _P, _P, _P, _P, _P]),
    "cpd_row_gram": (_I32, [_P, _P, _I64, _I32, _I32, _P, _P]),
    "cpd_row_solve": (_I32, [_P, _P, _I64, _I64, _I32, _F64, _P, _I64, _P, _P]),
    "cpd_complete": (_I32, [_I32, _P, _I64, _P, _P, _I32, _I32, _F64, _F64, _P, _P, _P, _P]),
    "cpd_tensor_stats": (_I32, [_I32, _P, _I64, _P, _P, _P]),
    "cpd_zipf_alpha": (_F64, [_F64, _I64]),
    "cpd_select_candidates": (_I32, [_P, _I32, _I32, _P, _P]),
    "cpd_select_features": (_I32, [_P, _I32, _I32, _P, _I32, _P]),
    "cpd_select_heuristic": (_I32, [_P, _I32, _I32, _P]),
    "cpd_select": (_I32, [_P, _I32, _I32, _P, _I32, _P, _P, _P, _P]),
    "cpd_mlp_param_count": (_I64, [_I32, _I32]),
    "cpd_mlp_init": (_I32, [_P, _I32, _I32, ctypes.c_uint64, _P]),
    "cpd_mlp_forward": (_I32, [_P, _I32, _I32, _P, _I64, _P, _P]),
    "cpd_mlp_loss_grad": (_I32, [_P, _I32, _I32, _P, _P, _I64, _P, _P, _P]),
    "cpd_mlp_adam": (_I32, [_P, _P, _P, _P, _I64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                            ctypes.c_float, _I32, _P]),
    "cpd_mlp_train": (_I32, [_P, _I32, _I32, _P, _P, _I64, _I32, _I32, ctypes.c_float,
                             ctypes.c_uint64, _P, _P]),
}


def lib():
    """The loaded libcpd.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libcpd.so is not built (run python -m paper_1812_05961_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _check(status):
    if status != CPD_OK:
        raise CpdError(status, lib().cpd_last_error().decode())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptrs(ts):
    arr = (ctypes.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = None if t is None else t.data_ptr()
    return arr


def _i64s(xs):
    return (ctypes.c_int64 * len(xs))(*[int(x) for x in xs])


def _need_cuda(t, name, dtype=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a CUDA tensor" % name)
    if dtype is not None and t.dtype != dtype:
        raise ValueError("%s must be %s, not %s" % (name, dtype, t.dtype))
    return t


def _coo_args(inds, vals, dims):
    if isinstance(inds, torch.Tensor):
        inds = [inds[m] for m in range(inds.shape[0])]
    inds = [_need_cuda(i, "inds").to(torch.int32).contiguous() for i in inds]
    vals = _need_cuda(vals, "vals").to(torch.float32).contiguous()
    for i in inds:
        if i.numel() != vals.numel():
            raise ValueError("index and value arrays differ in length")
    return inds, vals, [int(d) for d in dims]


class Csf:
    """A CSF tree held by the library (cpd_csf)."""

    def __init__(self, handle: int):
        self.handle = ctypes.c_void_p(handle)
        nm = _I32()
        order = (_I32 * MAX_MODES)()
        counts = (_I64 * MAX_MODES)()
        _check(lib().cpd_csf_info(self.handle, ctypes.byref(nm), order, counts))
        self.nmodes = nm.value
        self.order = [order[i] for i in range(self.nmodes)]
        self.counts = [counts[i] for i in range(self.nmodes)]

    def free(self):
        if self.handle:
            lib().cpd_csf_free(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def export(self, level: int, stream=None):
        """(fids, fptr or None, vals or None) of one level, as CUDA tensors."""
        dev = torch.device("cuda")
        fids = torch.empty(self.counts[level], dtype=torch.int32, device=dev)
        leaf = level == self.nmodes - 1
        fptr = None if leaf else torch.empty(self.counts[level] + 1, dtype=torch.int32, device=dev)
        vals = torch.empty(self.counts[level], dtype=torch.float32, device=dev) if leaf else None
        _check(lib().cpd_csf_export(self.handle, level, fids.data_ptr(),
                                    None if fptr is None else fptr.data_ptr(),
                                    None if vals is None else vals.data_ptr(), _stream(stream)))
        return fids, fptr, vals

    def tiles(self, tile_nnz: int, stream=None):
        nt = _I64()
        _check(lib().cpd_csf_tiles(self.handle, tile_nnz, None, ctypes.byref(nt), _stream(stream)))
        out = torch.empty((self.nmodes - 1, nt.value), dtype=torch.int32, device="cuda")
        _check(lib().cpd_csf_tiles(self.handle, tile_nnz, out.data_ptr(), ctypes.byref(nt),
                                   _stream(stream)))
        return out


def csf_build(inds, vals, dims, order=None, stream=None) -> Csf:
    """cpd_csf_build from COO on the device (inds: N int tensors or (N, nnz))."""
    inds, vals, dims = _coo_args(inds, vals, dims)
    h = ctypes.c_void_p()
    ordarr = None if order is None else (_I32 * len(dims))(*[int(m) for m in order])
    _check(lib().cpd_csf_build(len(dims), _i64s(dims), vals.numel(), _ptrs(inds), vals.data_ptr(),
                               ordarr, _stream(stream), ctypes.byref(h)))
    c = Csf(h.value)
    c.dims = dims
    return c


def csf_build_rooted(inds, vals, dims, stream=None) -> list:
    """cpd_csf_build_rooted: one tree rooted at each mode (list indexed by
    mode), the other modes by descending length."""
    inds, vals, dims = _coo_args(inds, vals, dims)
    hs = (ctypes.c_void_p * len(dims))()
    _check(lib().cpd_csf_build_rooted(len(dims), _i64s(dims), vals.numel(), _ptrs(inds), vals.data_ptr(),
                                      _stream(stream), hs))
    out = []
    for m in range(len(dims)):
        c = Csf(hs[m])
        c.dims = dims
        out.append(c)
    return out



def mttkrp_plan(dims_by_level, depth, rank, ld=None, precision="fp32", kernel="auto",
                rows_aligned=True, leaf_words=True):
    """Kernel family ("row", "lane", "round" or "tiled") cpd_mttkrp runs for
    this request (host only)."""
    out = _I32()
    nm = len(dims_by_level)
    _check(lib().cpd_mttkrp_plan(nm, _i64s(dims_by_level), int(depth), int(ld or rank), int(rank),
                                 PRECISION[precision], KERNEL[kernel], int(bool(rows_aligned)),
                                 int(bool(leaf_words)), ctypes.byref(out)))
    return _KERNEL_NAME[out.value]


def _mttkrp_call(entry, csf, factors, mode, out, rank, precision, variant, kernel, tile_nnz, stream):
    fdt = torch.float32 if precision == "fp32" else torch.bfloat16
    if out is None and not 0 <= mode < len(csf.dims):
        raise ValueError("mode %d out of range" % mode)
    ref = next(f for m, f in enumerate(factors) if m != mode and f is not None)
    R = int(rank if rank is not None else ref.shape[1])
    ld = int(ref.stride(0))
    for m, f in enumerate(factors):
        if m == mode or f is None:
            continue
        _need_cuda(f, "factor %d" % m, fdt)
        if f.stride(1) != 1 or f.stride(0) != ld:
            raise ValueError("factors need unit column stride and one common row stride")
    if out is None:
        out = torch.empty((csf.dims[mode], R), dtype=torch.float32, device="cuda")
    _need_cuda(out, "out", torch.float32)
    opts = MttkrpOpts(PRECISION[precision], VARIANT[variant], KERNEL[kernel], int(tile_nnz))
    _check(entry(csf.handle, _ptrs([None if m == mode else f for m, f in enumerate(factors)]),
                 ld, R, int(mode), out.data_ptr(), int(out.stride(0)), ctypes.byref(opts), _stream(stream)))
    return out


def mttkrp(csf: Csf, factors, mode: int, out=None, rank=None, precision="fp32", variant="auto",
           kernel="auto", tile_nnz=0, stream=None):
    """cpd_mttkrp: Y (dims[mode] x rank, float32) for the given factors.

    factors: list of N CUDA tensors (row-major, unit column stride; entry
    `mode` may be None): float32 for "fp32", bfloat16 for "bf16"."""
    return _mttkrp_call(lib().cpd_mttkrp, csf, factors, mode, out, rank, precision, variant, kernel,
                        tile_nnz, stream)


def mttkrp_noalloc(csf: Csf, factors, mode: int, out, rank=None, precision="fp32", variant="auto",
                   kernel="auto", tile_nnz=0, stream=None):
    """cpd_mttkrp_noalloc: cpd_mttkrp with every temporary in the library's
    fixed per-device workspace (no device allocation by the library; `out`
    is the caller's).  Calls overlapping on one device race."""
    if out is None:
        raise ValueError("mttkrp_noalloc writes into a caller-allocated out")
    return _mttkrp_call(lib().cpd_mttkrp_noalloc, csf, factors, mode, out, rank, precision, variant, kernel,
                        tile_nnz, stream)


def noalloc_workspace_bytes():
    return int(lib().cpd_mttkrp_noalloc_workspace_bytes())


def set_alloc_limit(nbytes):
    """Test hook: device allocation requests above nbytes fail with
    CPD_ENOMEM (None or a negative value: no limit)."""
    lib().cpd_set_alloc_limit(-1 if nbytes is None else int(nbytes))


def gram(A, stream=None):
    _need_cuda(A, "A", torch.float32)
    R = A.shape[1]
    G = torch.empty((R, R), dtype=torch.float64, device="cuda")
    _check(lib().cpd_gram(A.data_ptr(), A.shape[0], R, A.stride(0), G.data_ptr(), _stream(stream)))
    return G


def solve_normalize(grams, mode, Y, A=None, want_bf16=False, want_gram=True, stream=None):
    """cpd_solve_normalize -> dict(A, lam, G, used_pinv, A_bf16)."""
    _need_cuda(Y, "Y", torch.float32)
    rows, R = Y.shape
    if A is None:
        A = torch.empty((rows, R), dtype=torch.float32, device="cuda")
    Ab = torch.empty((rows, R), dtype=torch.bfloat16, device="cuda") if want_bf16 else None
    lam = torch.empty(R, dtype=torch.float64, device="cuda")
    G = torch.empty((R, R), dtype=torch.float64, device="cuda") if want_gram else None
    used = torch.zeros(1, dtype=torch.int32, device="cuda")
    _check(lib().cpd_solve_normalize(_ptrs(grams), len(grams), int(mode), Y.data_ptr(), rows, R,
                                     Y.stride(0), A.data_ptr(), A.stride(0),
                                     None if Ab is None else Ab.data_ptr(),
                                     R if Ab is None else Ab.stride(0), lam.data_ptr(),
                                     None if G is None else G.data_ptr(), used.data_ptr(),
                                     _stream(stream)))
    return dict(A=A, lam=lam, G=G, used_pinv=used, A_bf16=Ab)


def fit(normX2, lam, A_last, Y_last, grams, stream=None):
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    rows, R = A_last.shape
    _check(lib().cpd_fit(float(normX2), lam.data_ptr(), A_last.data_ptr(), A_last.stride(0),
                         Y_last.data_ptr(), Y_last.stride(0), rows, R, _ptrs(grams), len(grams),
                         out.data_ptr(), _stream(stream)))
    return out


def sumsq(vals, stream=None):
    _need_cuda(vals, "vals", torch.float32)
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    _check(lib().cpd_sumsq(vals.data_ptr(), vals.numel(), out.data_ptr(), _stream(stream)))
    return out


def row_gram(csf: Csf, factors, mode: int, rank=None, stream=None):
    """cpd_row_gram: (dims[mode], rank, rank) float64 row Grams (upper triangle)."""
    facs = [None if f is None else _need_cuda(f, "factor") for f in factors]
    f0 = next(f for f in facs if f is not None)
    ld = f0.stride(0)
    rank = rank or f0.shape[1]
    G = torch.empty((csf.dims[mode], rank, rank), dtype=torch.float64, device=f0.device)
    _check(lib().cpd_row_gram(csf.handle, _ptrs([None if m == mode else f for m, f in enumerate(facs)]), ld, rank,
                              mode, G.data_ptr(), _stream(stream)))
    return G


def row_solve(G, Y, reg, rank=None, out=None, stream=None):
    """cpd_row_solve: rows of (G_i + reg I)^{-1} y_i; returns (A, (cross, quad))."""
    G = _need_cuda(G, "G")
    Y = _need_cuda(Y, "Y")
    rows = Y.shape[0]
    rank = rank or G.shape[1]
    A = out if out is not None else torch.zeros((rows, rank), dtype=torch.float32, device=Y.device)
    terms = torch.zeros(2, dtype=torch.float64, device=Y.device)
    _check(lib().cpd_row_solve(G.data_ptr(), Y.data_ptr(), Y.stride(0), rows, rank, float(reg), A.data_ptr(),
                               A.stride(0), terms.data_ptr(), _stream(stream)))
    t = terms.cpu().tolist()
    return A, (t[0], t[1])


def complete(inds, vals, dims, rank, iters, reg, init, tol=0.0, stream=None):
    """cpd_complete: completion ALS; init is a list of N (I_m x rank) device
    tensors (copied, not modified).  Returns dict(factors, rmses, rmse, iters)."""
    inds, vals, dims = _coo_args(inds, vals, dims)
    facs = [_need_cuda(a, "init").to(torch.float32).contiguous().clone() for a in init]
    for m, f in enumerate(facs):
        if tuple(f.shape) != (dims[m], rank):
            raise ValueError("init factor %d has shape %s" % (m, tuple(f.shape)))
    rm = (_F64 * iters)()
    it = _I32()
    _check(lib().cpd_complete(len(dims), _i64s(dims), vals.numel(), _ptrs(inds), vals.data_ptr(), rank, iters,
                              float(tol), float(reg), _ptrs(facs), rm, ctypes.byref(it), _stream(stream)))
    rmses = [rm[i] for i in range(it.value)]
    return dict(factors=facs, rmses=rmses, rmse=rmses[-1] if rmses else 0.0, iters=it.value)


def als(inds, vals, dims, rank, iters, tol=0.0, init=None, precision="fp32", variant="auto",
        kernel="auto", tile_nnz=0, single_csf=False, order=None, seed=0, timing=False,
        select="none", selector=None, fast_fit=False, stream=None):
    """cpd_als -> dict(factors, lam, fit, iters, fits, timing_ms).

    select: "none", "network" (selector = (params CUDA tensor, hidden)) or
    "heuristic".  fast_fit: skip the FP64 evaluation of the returned model's fit."""
    inds, vals, dims = _coo_args(inds, vals, dims)
    nm = len(dims)
    outs = [torch.empty((d, rank), dtype=torch.float32, device="cuda") for d in dims]
    if init is not None:
        init = [_need_cuda(a, "init").to(torch.float32).contiguous() for a in init]
        for a, d in zip(init, dims):
            if tuple(a.shape) != (d, rank):
                raise ValueError("init factor shape %s, expected %s" % (tuple(a.shape), (d, rank)))
    trace = (ctypes.c_double * iters)()
    tms = (ctypes.c_double * (4 + iters * (nm + 1)))() if timing else None
    ordarr = None if order is None else (_I32 * nm)(*[int(m) for m in order])
    initarr = None if init is None else _ptrs(init)
    opts = AlsOpts(PRECISION[precision], VARIANT[variant], KERNEL[kernel], int(tile_nnz),
                   int(bool(single_csf)), int(bool(fast_fit)),
                   ctypes.cast(ordarr, ctypes.c_void_p) if ordarr is not None else None,
                   ctypes.cast(initarr, ctypes.c_void_p) if initarr is not None else None,
                   int(seed), ctypes.cast(trace, ctypes.c_void_p),
                   ctypes.cast(tms, ctypes.c_void_p) if tms is not None else None,
                   SELECT[select], 0, None)
    if select == "network":
        params, hidden = selector
        _need_cuda(params, "selector params", torch.float32)
        opts.selector_hidden = int(hidden)
        opts.selector_params = params.data_ptr()
    lam = (ctypes.c_double * rank)()
    fit_out = ctypes.c_double()
    it_out = ctypes.c_int32()
    _check(lib().cpd_als(nm, _i64s(dims), vals.numel(), _ptrs(inds), vals.data_ptr(), int(rank),
                         int(iters), float(tol), ctypes.byref(opts), _ptrs(outs), lam,
                         ctypes.byref(fit_out), ctypes.byref(it_out), _stream(stream)))
    n_it = it_out.value
    res = dict(factors=outs, lam=list(lam), fit=fit_out.value, iters=n_it,
               fits=[trace[i] for i in range(n_it)])
    if timing:
        t = list(tms)
        res["timing_ms"] = dict(csf_build=t[0], iterations=t[1], final_fit=t[2], total=t[3],
                                per_iter=[t[4 + i * (nm + 1): 4 + (i + 1) * (nm + 1)]
                                          for i in range(n_it)])
    return res


# ---------------------------------------------------------------------------
# Variant selector and its network


def tensor_stats(inds, dims, stream=None) -> Stats:
    """cpd_tensor_stats of a COO tensor (inds: N int tensors or (N, nnz))."""
    if isinstance(inds, torch.Tensor):
        inds = [inds[m] for m in range(inds.shape[0])]
    inds = [_need_cuda(i, "inds").to(torch.int32).contiguous() for i in inds]
    st = Stats()
    _check(lib().cpd_tensor_stats(len(dims), _i64s(dims), inds[0].numel(), _ptrs(inds),
                                  _stream(stream), ctypes.byref(st)))
    return st


def make_stats(dims, nnz, top1, distinct, alpha=None, sample=None) -> Stats:
    """A Stats record from given values (alpha from cpd_zipf_alpha if None)."""
    st = Stats()
    st.nmodes = len(dims)
    st.nnz = int(nnz)
    st.sample = int(sample if sample is not None else min(nnz, 1 << 20))
    for m, d in enumerate(dims):
        st.dims[m] = int(d)
        st.top1[m] = float(top1[m])
        st.distinct[m] = float(distinct[m])
        st.alpha[m] = float(alpha[m]) if alpha is not None else zipf_alpha(top1[m], d)
    return st


def make_choice(d) -> Choice:
    """A Choice record from its as_dict() form."""
    c = Choice()
    c.order_kind = ORDER_KINDS.index(d["order_kind"])
    c.depth = int(d["depth"])
    for l, m in enumerate(d["order"]):
        c.order[l] = int(m)
    c.opts = MttkrpOpts(FP32, VARIANT[d["variant"]], KERNEL[d["kernel"]], int(d["tile_nnz"]))
    return c


def zipf_alpha(top1, dim):
    return lib().cpd_zipf_alpha(float(top1), int(dim))


def select_candidates(st: Stats, rank, mode):
    out = (Choice * SEL_MAX_CAND)()
    n = _I32()
    _check(lib().cpd_select_candidates(ctypes.byref(st), int(rank), int(mode), out, ctypes.byref(n)))
    return [out[i] for i in range(n.value)]


def select_features(st: Stats, rank, mode, cands):
    import numpy as np
    arr = (Choice * max(1, len(cands)))(*cands)
    feat = np.zeros((len(cands), SEL_NFEAT), dtype=np.float32)
    _check(lib().cpd_select_features(ctypes.byref(st), int(rank), int(mode), arr, len(cands),
                                     feat.ctypes.data_as(ctypes.c_void_p)))
    return feat


def select_heuristic(st: Stats, rank, mode) -> Choice:
    out = Choice()
    _check(lib().cpd_select_heuristic(ctypes.byref(st), int(rank), int(mode), ctypes.byref(out)))
    return out


def select(st: Stats, rank, mode, params=None, hidden=64, stream=None):
    """cpd_select -> (Choice, predictions list)."""
    out = Choice()
    pred = (ctypes.c_float * SEL_MAX_CAND)()
    n = _I32()
    if params is not None:
        _need_cuda(params, "params", torch.float32)
    _check(lib().cpd_select(ctypes.byref(st), int(rank), int(mode),
                            None if params is None else params.data_ptr(), int(hidden),
                            ctypes.byref(out), pred, ctypes.byref(n),
                            None if params is None else _stream(stream)))
    return out, [pred[i] for i in range(n.value)]


def mlp_param_count(n_in, hidden):
    return int(lib().cpd_mlp_param_count(int(n_in), int(hidden)))


def mlp_init(n_in, hidden, seed, stream=None):
    p = torch.empty(mlp_param_count(n_in, hidden), dtype=torch.float32, device="cuda")
    _check(lib().cpd_mlp_init(p.data_ptr(), int(n_in), int(hidden), int(seed), _stream(stream)))
    return p


def mlp_forward(params, n_in, hidden, X, stream=None):
    _need_cuda(params, "params", torch.float32)
    X = _need_cuda(X, "X", torch.float32).contiguous()
    out = torch.empty(X.shape[0], dtype=torch.float32, device="cuda")
    _check(lib().cpd_mlp_forward(params.data_ptr(), int(n_in), int(hidden), X.data_ptr(),
                                 X.shape[0], out.data_ptr(), _stream(stream)))
    return out


def mlp_loss_grad(params, n_in, hidden, X, y, stream=None):
    _need_cuda(params, "params", torch.float32)
    X = _need_cuda(X, "X", torch.float32).contiguous()
    y = _need_cuda(y, "y", torch.float32).contiguous()
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    grad = torch.empty_like(params)
    _check(lib().cpd_mlp_loss_grad(params.data_ptr(), int(n_in), int(hidden), X.data_ptr(),
                                   y.data_ptr(), X.shape[0], loss.data_ptr(), grad.data_ptr(),
                                   _stream(stream)))
    return loss, grad


def mlp_adam(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    for t, nm in ((params, "params"), (grad, "grad"), (m, "m"), (v, "v")):
        _need_cuda(t, nm, torch.float32)
    _check(lib().cpd_mlp_adam(params.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(),
                              params.numel(), lr, beta1, beta2, eps, int(step), _stream(stream)))


def mlp_train(params, n_in, hidden, X, y, epochs, batch, lr, seed, stream=None):
    """cpd_mlp_train in place on params; returns the per-epoch mean loss."""
    _need_cuda(params, "params", torch.float32)
    X = _need_cuda(X, "X", torch.float32).contiguous()
    y = _need_cuda(y, "y", torch.float32).contiguous()
    trace = (ctypes.c_float * int(epochs))()
    _check(lib().cpd_mlp_train(params.data_ptr(), int(n_in), int(hidden), X.data_ptr(),
                               y.data_ptr(), X.shape[0], int(epochs), int(batch), float(lr),
                               int(seed), trace, _stream(stream)))
    return list(trace)
