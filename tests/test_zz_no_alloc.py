"""The allocation-free MTTKRP entry point (cpd_mttkrp_noalloc) against
cpd_mttkrp on the same trees and factors: every level and kernel family, two
calls in a row with the second on a smaller tensor, and a request whose
temporaries exceed the fixed workspace refused with a message."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1812_05961_amd import synth

pytestmark = pytest.mark.gpu


def _cpd():
    from paper_1812_05961_amd import cpd
    return cpd, cpd.lib()


def _noalloc(cpd, L, c, facs, mode, R, ld, kernel="auto", variant="auto", precision="fp32"):
    """cpd_mttkrp_noalloc into an output with two spare columns (set to 5.0,
    which must stay untouched); returns (status, output)."""
    out = torch.full((c.dims[mode], R + 2), 5.0, device="cuda")
    try:
        cpd.mttkrp_noalloc(c, facs, mode, out[:, :R], rank=R, precision=precision, variant=variant,
                           kernel=kernel)
        st = cpd.CPD_OK
    except cpd.CpdError as e:
        st = e.status
    return st, out


def _relerr(a, b):
    a = a.double().cpu().numpy()
    b = b.double().cpu().numpy()
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _factors(dims, R, ld, seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    out = []
    for d in dims:
        f = torch.zeros((d, ld), dtype=torch.float32, device="cuda")
        f[:, :R] = torch.rand((d, R), device="cuda", generator=g)
        out.append(f)
    return out


def _check_tree(cpd, L, t, R, ld, seed):
    c = cpd.csf_build(t.inds.cuda(), t.vals.cuda(), t.dims)
    facs = _factors(t.dims, R, ld, seed)
    for depth, mode in enumerate(c.order):
        kernels = ["auto", "lane"] + (["row"] if depth < t.nmodes - 1 else [])
        variants = ["auto"] + (["atomic", "private"] if depth > 0 else [])
        for kernel in kernels:
            for variant in (variants if kernel != "row" else ["auto"]):
                for prec in ("fp32", "bf16"):
                    fk = facs if prec == "fp32" else [f.to(torch.bfloat16) for f in facs]
                    # the allocation-free call first: on a fresh tree its tile tables and
                    # leaf-factor copy come from the workspace, not from the handle's cache
                    st, out = _noalloc(cpd, L, c, fk, mode, R, ld, kernel, variant, prec)
                    ref = torch.empty((t.dims[mode], R), device="cuda")
                    cpd.mttkrp(c, fk, mode, out=ref, rank=R, precision=prec, kernel=kernel, variant=variant)
                    torch.cuda.synchronize()
                    assert st == cpd.CPD_OK, (mode, kernel, variant, prec, L.cpd_last_error())
                    assert (out[:, R:] == 5.0).all()
                    err = _relerr(out[:, :R], ref)
                    assert err <= 1e-5, (t.dims, mode, kernel, variant, prec, err)
    c.free()


def test_noalloc_matches_mttkrp_twice_second_smaller():
    cpd, L = _cpd()
    assert cpd.noalloc_workspace_bytes() == 64 << 20
    big = synth.gen_sparse((900, 700, 1300), 300_000, (1.1, 1.1, 1.1), "lognormal:1.0", 5, topup=True)
    small = synth.gen_sparse((60, 50, 40, 30), 20_000, (0.5, 0.8, 0.0, 1.2), "lognormal:1.0", 7, topup=True)
    _check_tree(cpd, L, big, 35, 40, 1)
    _check_tree(cpd, L, small, 16, 16, 2)


def test_noalloc_refuses_temporaries_beyond_the_workspace():
    cpd, L = _cpd()
    # the per-XCD copies of a 70,000-row output at rank 32: 8 x 70,000 x 32 x 4 B > 64 MiB
    t = synth.gen_sparse((70_000, 50, 40), 100_000, (0.5, 0.5, 0.5), "lognormal:1.0", 9, topup=True)
    c = cpd.csf_build(t.inds.cuda(), t.vals.cuda(), t.dims)
    assert c.order[-1] == 0
    facs = _factors(t.dims, 32, 32, 3)
    st, _ = _noalloc(cpd, L, c, facs, 0, 32, 32, "lane", "private")
    assert st == cpd.CPD_EUNSUPPORTED
    assert b"workspace" in L.cpd_last_error()
    # the same call with atomics needs only the tile table: it runs
    st, out = _noalloc(cpd, L, c, facs, 0, 32, 32, "lane", "atomic")
    ref = cpd.mttkrp(c, facs, 0, rank=32)
    torch.cuda.synchronize()
    assert st == cpd.CPD_OK and _relerr(out[:, :32], ref) <= 1e-5
    c.free()
