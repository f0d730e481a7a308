"""GPU parity at the benchmark's full sizes, in the launch configuration that
bench.py times (one CSF rooted at each mode, the root-level kernel, default
tile width): sampled output rows against the oracle's row-by-row COO MTTKRP,
and the fit reported by cpd_als against the oracle's fit of the returned model.

The oracle loops over every nonzero once per checked mode (single-threaded C),
so each workload costs a few seconds of host time.
"""
import numpy as np
import pytest
import torch

from oracle import als as oals
from oracle import coo as ocoo
from paper_1812_05961_amd import synth

pytestmark = pytest.mark.gpu


def _cpd():
    from paper_1812_05961_amd import cpd
    cpd.lib()
    return cpd


def _root_order(dims, m):
    # as cpd_als builds its trees: the mode first, the others by descending length
    return [m] + sorted([q for q in range(len(dims)) if q != m], key=lambda q: (-dims[q], q))


def _sample_rows(inds_mode, dim, rng, k=6):
    """The three fullest rows plus random non-empty ones."""
    counts = np.bincount(inds_mode, minlength=dim)
    hot = np.argsort(-counts, kind="stable")[:3]
    nonempty = np.flatnonzero(counts)
    rand = rng.choice(nonempty, size=min(k, nonempty.size), replace=False)
    return np.unique(np.concatenate([hot, rand]))


@pytest.mark.parametrize("name,precision", [("nell2", "fp32"), ("nell2", "bf16"), ("netflix", "fp32"),
                                            ("fourmode", "fp32")])
def test_full_size_mttkrp_sampled_rows(name, precision):
    cpd = _cpd()
    x = synth.make_config(name, device="cuda")
    R = synth.CONFIGS[name]["rank"]
    inds_h = x.inds.cpu().numpy()
    vals_h = x.vals.cpu().double().numpy()
    rng = np.random.default_rng(7)
    g = torch.Generator().manual_seed(3)
    dt = torch.float32 if precision == "fp32" else torch.bfloat16
    width = next(w for w in ((8, 16, 32, 36, 64) if precision == "fp32" else (16, 16, 32, 40, 64)) if w >= R)
    facs, facs_used = [], []
    for d in x.dims:
        a = torch.rand((d, R), generator=g, dtype=torch.float64)
        buf = torch.zeros((d, width), dtype=dt)
        buf[:, :R] = a.to(dt)
        facs.append(buf.cuda())
        facs_used.append(buf[:, :R].to(torch.float64).numpy())
    xi = x.inds.to(torch.int32)
    for m in range(x.nmodes):
        c = cpd.csf_build(xi, x.vals, x.dims, _root_order(x.dims, m))
        y = cpd.mttkrp(c, facs, m, rank=R, precision=precision)
        torch.cuda.synchronize()
        rows = _sample_rows(inds_h[m], x.dims[m], rng)
        ref = ocoo.mttkrp_rows(x.dims, inds_h, vals_h, facs_used, m, rows)
        got = y.cpu().numpy()[rows].astype(np.float64)
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        # the same rows, computed on the rows the kernel read: FP32 products and sums
        assert err <= 1e-5, (name, precision, m, err)
        c.free()
        del y


def test_full_size_als_fit_matches_oracle_fit_of_returned_model():
    cpd = _cpd()
    x = synth.make_config("nell2", device="cuda")
    R = synth.CONFIGS["nell2"]["rank"]
    got = cpd.als(x.inds.to(torch.int32), x.vals, x.dims, R, 3, 0.0, seed=5)
    inds_h = x.inds.cpu().numpy()
    vals_h = x.vals.cpu().double().numpy()
    A = [f.cpu().double().numpy() for f in got["factors"]]
    lam = np.array(got["lam"])
    nm = x.nmodes
    Y = ocoo.mttkrp(x.dims, inds_h, vals_h, A, nm - 1)
    ref = oals.fit_from(ocoo.sumsq(vals_h), lam, A[nm - 1], Y, [oals.gram(a) for a in A])
    assert abs(got["fit"] - ref) <= 1e-4, (got["fit"], ref)
    # unit-norm columns, finite factors
    for a in A:
        assert np.isfinite(a).all()
        np.testing.assert_allclose(np.linalg.norm(a, axis=0), 1.0, atol=1e-4)


def test_full_size_completion_kernels_sampled_rows():
    """CP with missing values at the benchmark size (NELL-2 shape, rank 35):
    the row Grams of sampled rows (the fullest three among them) against the
    oracle's, and the row solves of those rows against the oracle's solve of
    the same Gram and right side."""
    from oracle import complete as oc
    cpd = _cpd()
    x = synth.make_config("nell2", device="cuda")
    R = synth.CONFIGS["nell2"]["rank"]
    inds_h = x.inds.cpu().numpy()
    vals_h = x.vals.cpu().double().numpy()
    rng = np.random.default_rng(9)
    g = torch.Generator().manual_seed(4)
    facs, facs_used = [], []
    for d in x.dims:
        buf = torch.zeros((d, 36), dtype=torch.float32)
        buf[:, :R] = torch.rand((d, R), generator=g)
        facs.append(buf.cuda())
        facs_used.append(buf[:, :R].double().numpy())
    trees = cpd.csf_build_rooted(x.inds.to(torch.int32), x.vals, x.dims)
    reg = 0.1
    for m, c in enumerate(trees):
        rows = _sample_rows(inds_h[m], x.dims[m], rng, k=4)
        G = cpd.row_gram(c, facs, m, rank=R)
        y = cpd.mttkrp(c, facs, m, rank=R)
        A, _ = cpd.row_solve(G, y, reg, rank=R)
        torch.cuda.synchronize()
        got = G.cpu().numpy()[rows]
        ref = oc.row_grams(x.dims, inds_h, vals_h, facs_used, m, rows=rows)
        iu = np.triu_indices(R)
        scale = float(np.abs(ref).max())
        np.testing.assert_allclose(got[:, iu[0], iu[1]], ref[:, iu[0], iu[1]], rtol=0, atol=1e-12 * scale)
        # the solve of those rows from the same G and y, in the oracle
        ysel = y.cpu().numpy()[rows].astype(np.float64)
        full = np.stack([np.triu(gg) + np.triu(gg, 1).T for gg in got])
        want, _ = oc.solve_rows(full, ysel, reg, np.ones(rows.size, dtype=np.int64))
        err = np.linalg.norm(A.cpu().numpy()[rows] - want) / np.linalg.norm(want)
        assert err <= 1e-6, (m, err)
        del G, y, A
        c.free()
