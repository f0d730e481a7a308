"""Allocation failures (cpd_set_alloc_limit makes every device allocation
above a limit fail as if the device were out of memory): each entry point
returns CPD_ENOMEM with a message, leaks nothing it can be asked to free, and
the library works again once the limit is lifted (the results then match the
oracle)."""
import numpy as np
import pytest
import torch

from oracle import coo as ocoo
from paper_1812_05961_amd import synth

pytestmark = pytest.mark.gpu


def _cpd():
    from paper_1812_05961_amd import cpd
    cpd.lib()
    return cpd


@pytest.fixture
def limit():
    cpd = _cpd()
    yield cpd.set_alloc_limit
    cpd.set_alloc_limit(None)


def _tensor():
    return synth.gen_sparse((300, 400, 500), 200_000, (0.8, 0.5, 1.0), "lognormal:1.0", 61, device="cpu",
                            topup=True, fp32=True)


def _relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_csf_build_fails_cleanly_and_recovers(limit):
    cpd = _cpd()
    t = _tensor()
    inds, vals = t.inds.cuda(), t.vals.cuda()
    limit(4 << 10)
    with pytest.raises(cpd.CpdError) as e:
        cpd.csf_build(inds, vals, t.dims)
    assert e.value.status == cpd.CPD_ENOMEM
    assert "allocation" in str(e.value)
    limit(None)
    c = cpd.csf_build(inds, vals, t.dims)
    facs = [torch.rand((d, 16), device="cuda") for d in t.dims]
    ih, vh = t.numpy()
    for mode in range(3):
        y = cpd.mttkrp(c, facs, mode, rank=16).cpu().numpy()
        ref = ocoo.mttkrp(t.dims, ih, vh, [f.cpu().double().numpy() for f in facs], mode)
        assert _relerr(y, ref) <= 1e-5
    c.free()


def test_mttkrp_tables_fail_cleanly_and_recover(limit):
    """The tables an MTTKRP builds on first use (the leaf level's mode tiling,
    the tile table of a new width) are refused under the limit; the call then
    succeeds once it is lifted."""
    cpd = _cpd()
    t = _tensor()
    c = cpd.csf_build(t.inds.cuda(), t.vals.cuda(), t.dims)
    facs = [torch.rand((d, 16), device="cuda") for d in t.dims]
    leaf = c.order[-1]
    limit(4 << 10)
    for kernel, tile in (("tiled", 0), ("row", 96)):
        mode = leaf if kernel == "tiled" else c.order[0]
        with pytest.raises(cpd.CpdError) as e:
            cpd.mttkrp(c, facs, mode, rank=16, kernel=kernel, tile_nnz=tile)
        assert e.value.status == cpd.CPD_ENOMEM
    limit(None)
    ih, vh = t.numpy()
    for kernel, tile in (("tiled", 0), ("row", 96)):
        mode = leaf if kernel == "tiled" else c.order[0]
        y = cpd.mttkrp(c, facs, mode, rank=16, kernel=kernel, tile_nnz=tile).cpu().numpy()
        ref = ocoo.mttkrp(t.dims, ih, vh, [f.cpu().double().numpy() for f in facs], mode)
        assert _relerr(y, ref) <= 1e-5, kernel
    c.free()


def test_als_fails_cleanly_and_recovers(limit):
    cpd = _cpd()
    t = _tensor()
    inds, vals = t.inds.cuda(), t.vals.cuda()
    limit(4 << 10)
    with pytest.raises(cpd.CpdError) as e:
        cpd.als(inds, vals, t.dims, rank=8, iters=2, seed=3)
    assert e.value.status == cpd.CPD_ENOMEM
    limit(None)
    got = cpd.als(inds, vals, t.dims, rank=8, iters=2, seed=3)
    assert np.isfinite(got["fit"])


def test_auto_runs_without_the_tiling_when_it_does_not_fit(limit):
    """AUTO takes TILED at an internal level; when the level's mode tiling
    cannot be allocated it runs the shape rule's kernel instead (ROW here),
    while TILED asked for explicitly fails with CPD_ENOMEM.  A 1 MiB limit
    refuses the tiling (16 bytes per nonzero) and admits ROW's tables (the
    leaf factor in rank order: 5,000 rows of 64 bytes)."""
    cpd = _cpd()
    t = synth.gen_sparse((30, 40, 5000), 200_000, (0.5, 0.5, 1.0), "lognormal:1.0", 67, device="cpu",
                         topup=True, fp32=True)
    c = cpd.csf_build(t.inds.cuda(), t.vals.cuda(), t.dims, [0, 1, 2])
    facs = [torch.rand((d, 16), device="cuda") for d in t.dims]
    ih, vh = t.numpy()
    ref = ocoo.mttkrp(t.dims, ih, vh, [f.cpu().double().numpy() for f in facs], 1)
    limit(1 << 20)
    with pytest.raises(cpd.CpdError) as e:
        cpd.mttkrp(c, facs, 1, rank=16, kernel="tiled")
    assert e.value.status == cpd.CPD_ENOMEM
    y = cpd.mttkrp(c, facs, 1, rank=16).cpu().numpy()
    assert _relerr(y, ref) <= 1e-5
    limit(None)
    y = cpd.mttkrp(c, facs, 1, rank=16).cpu().numpy()  # TILED, the tiling built now
    assert _relerr(y, ref) <= 1e-5
    c.free()
