"""GPU parity at the benchmark's full sizes (the 76M-nonzero NELL-2 shape, the
100M-nonzero NETFLIX shape and the 50M-nonzero 4-mode tensor), in the launch
configurations bench.py times:

  * the CSF trees bit-exact against the oracle's sort and run scans (the
    heuristic-order tree and the per-mode trees of CP-ALS);
  * every output row of every mode's MTTKRP, on the per-mode trees (the root
    kernel, FP32 and BF16 gathers) and at every level and conflict-handling
    variant of the single heuristic tree, against the oracle's COO loop on the
    same (rounded) factor rows: a relative Frobenius bound over the whole
    output and an element-wise bound per row;
  * the CP-ALS fit trajectory against the oracle's, from the same initial
    factors, and the final fits of FP32 and BF16 gathers.

Element-wise bound.  The factors here are U(0,1) and the values positive, so
every term of Y(i, r) = sum_k x_k prod_m A_m(i_m, r) is positive and the FP32
sums of the kernels (per-run FMA chains, scans, atomics in any order) carry a
rounding error that grows like a random walk over the n_i terms of row i:
about 2^-24 sqrt(n_i) |Y(i, r)|.  Each element must satisfy
|got - ref| <= max(1e-5, 4 * 2^-24 * sqrt(n_i)) * ref: 1e-5 for rows of up to
~1,700 nonzeros, where a dropped or repeated nonzero (an error of at least
ref / n_i) cannot hide, and four standard deviations of the random walk above
that.  The relative Frobenius error of the whole output stays <= 1e-5.

The oracle's MTTKRP loop runs on all the process's host cores (private
copies of Y per thread), its CP-ALS likewise.
"""
import os

import numpy as np
import pytest
import torch

from oracle import als as oals
from oracle import coo as ocoo
from oracle import csf as ocsf
from paper_1812_05961_amd import synth

pytestmark = pytest.mark.gpu

THREADS = min(16, len(os.sched_getaffinity(0)))
EPS32 = 2.0 ** -24


def _say(*what):
    """One progress line per finished step (these tests run minutes each)."""
    print("  [full-size]", *what, flush=True)


def _cpd():
    from paper_1812_05961_amd import cpd
    cpd.lib()
    return cpd


def _root_order(dims, m):
    # as cpd_als builds its trees: the mode first, the others by descending length
    return [m] + sorted([q for q in range(len(dims)) if q != m], key=lambda q: (-dims[q], q))


class Full:
    """A benchmark tensor on the device and on the host."""

    def __init__(self, name):
        self.name = name
        x = synth.make_config(name, device="cuda")
        self.dims = x.dims
        self.nm = x.nmodes
        self.R = synth.CONFIGS[name]["rank"]
        self.inds = x.inds.to(torch.int32)
        self.vals = x.vals
        self.inds_h = x.inds.cpu().numpy().astype(np.int64)
        self.vals_h = x.vals.cpu().double().numpy()
        self.row_nnz = [np.bincount(self.inds_h[m], minlength=self.dims[m]) for m in range(self.nm)]
        _say("generated", name, self.vals_h.size, "nonzeros")


_CACHE = {}


def _full(name):
    if name not in _CACHE:
        _CACHE.clear()
        torch.cuda.empty_cache()
        _CACHE[name] = Full(name)
    return _CACHE[name]


def _factors(t, precision, seed):
    """U(0,1) factors padded to the kernels' row widths; returns (device
    tensors, the FP64 values the kernels read)."""
    g = torch.Generator().manual_seed(seed)
    dt = torch.float32 if precision == "fp32" else torch.bfloat16
    width = next(w for w in ((8, 16, 32, 36, 64) if precision == "fp32" else (16, 16, 32, 40, 64)) if w >= t.R)
    dev, used = [], []
    for d in t.dims:
        buf = torch.zeros((d, width), dtype=dt)
        buf[:, :t.R] = torch.rand((d, t.R), generator=g, dtype=torch.float64).to(dt)
        dev.append(buf.cuda())
        used.append(buf[:, :t.R].to(torch.float64).numpy())
    return dev, used


def _check_all_rows(t, m, got, ref, what):
    """Relative Frobenius error <= 1e-5 and the per-row element-wise bound."""
    got = np.asarray(got, dtype=np.float64)
    fro = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert fro <= 1e-5, (what, "frobenius", fro)
    tol = np.maximum(1e-5, 4.0 * EPS32 * np.sqrt(t.row_nnz[m].astype(np.float64)))[:, None]
    bad = np.abs(got - ref) > tol * ref + 1e-30
    if bad.any():
        i, r = np.argwhere(bad)[0]
        pytest.fail("%s: %d elements beyond the bound; first row %d (%d nonzeros) col %d: got %r ref %r"
                    % (what, int(bad.sum()), i, t.row_nnz[m][i], r, got[i, r], ref[i, r]))


# ------------------------------------------------------------------ CSF trees

def test_full_size_csf_bit_exact():
    """The heuristic-order tree and the three per-mode trees of the NELL-2
    shape, level by level, against the oracle's stable sort and run scans."""
    cpd = _cpd()
    t = _full("nell2")
    vals32 = t.vals.cpu().numpy()
    orders = [None] + [_root_order(t.dims, m) for m in range(t.nm)]
    rooted = cpd.csf_build_rooted(t.inds, t.vals, t.dims)
    for k, order in enumerate(orders):
        c = cpd.csf_build(t.inds, t.vals, t.dims, order) if order is None else rooted[k - 1]
        ref = ocsf.build(t.dims, t.inds_h, vals32, order or ocsf.heuristic_order(t.dims))
        assert c.order == ref["order"] and c.counts == ref["counts"], (order, c.counts, ref["counts"])
        for l in range(t.nm):
            fids, fptr, v = c.export(l)
            np.testing.assert_array_equal(fids.cpu().numpy(), ref["fids"][l])
            if l < t.nm - 1:
                np.testing.assert_array_equal(fptr.cpu().numpy(), ref["fptr"][l])
            else:
                assert v.cpu().numpy().tobytes() == ref["vals"].tobytes()
            del fids, fptr, v
        _say("tree", order, "bit-exact")
        if k == 0:
            for T in (32, 128, 256):
                np.testing.assert_array_equal(c.tiles(T).cpu().numpy(), ocsf.tile_starts(ref, T))
        c.free()
        del ref


# ------------------------------------------------------------------ MTTKRP

@pytest.mark.parametrize("name,precision", [("nell2", "fp32"), ("nell2", "bf16"), ("netflix", "fp32"),
                                            ("netflix", "bf16"), ("fourmode", "fp32"), ("fourmode", "bf16")])
def test_full_size_mttkrp_all_rows_als_layout(name, precision):
    """Every row of every mode's MTTKRP on the tree rooted at the mode (the
    root kernel cpd_als runs)."""
    cpd = _cpd()
    t = _full(name)
    facs, used = _factors(t, precision, 3)
    for m in range(t.nm):
        c = cpd.csf_build(t.inds, t.vals, t.dims, _root_order(t.dims, m))
        y = cpd.mttkrp(c, facs, m, rank=t.R, precision=precision).cpu().numpy()
        c.free()
        ref = ocoo.mttkrp(t.dims, t.inds_h, t.vals_h, used, m, threads=THREADS)
        _check_all_rows(t, m, y, ref, (name, precision, "mode", m))
        _say(name, precision, "mode", m, "all rows checked")


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_full_size_single_tree_every_level(precision):
    """The heuristic tree of the NELL-2 shape, every kernel the single-tree
    timings run: the root (lane-group and LANE kernels), the internal level
    (lane-group without and with the hot-row table, TILED on the level's mode
    tiling, LANE atomic, LANE privatised into per-XCD copies) and the leaf
    level (TILED, ROUND, LANE atomic with the hot-row table, LANE
    privatised), every row."""
    cpd = _cpd()
    t = _full("nell2")
    facs, used = _factors(t, precision, 4)
    c = cpd.csf_build(t.inds, t.vals, t.dims, None)
    for depth, m in enumerate(c.order):
        ref = ocoo.mttkrp(t.dims, t.inds_h, t.vals_h, used, m, threads=THREADS)
        if depth == 0:
            runs = [("row", "auto")]
        elif depth < t.nm - 1:
            runs = [("row", "atomic"), ("row", "private"), ("tiled", "auto")]
        else:
            runs = [("tiled", "auto"), ("round", "auto")]
        runs += [("lane", "atomic")] + ([("lane", "private")] if depth > 0 else [])
        for kernel, variant in runs:
            y = cpd.mttkrp(c, facs, m, rank=t.R, precision=precision, kernel=kernel, variant=variant)
            _check_all_rows(t, m, y.cpu().numpy(), ref, ("single", precision, depth, kernel, variant))
            _say("single tree", precision, "depth", depth, kernel, variant, "all rows checked")
            del y
    c.free()


# ------------------------------------------------------------------ CP-ALS

def test_full_size_als_trajectory_nell2():
    """Ten sweeps at rank 35 from the same initial factors: every sweep's fit
    within 1e-5 of the oracle's, the reported final fit within 1e-4 of the
    oracle's and within 1e-6 of the oracle's fit of the returned model."""
    cpd = _cpd()
    t = _full("nell2")
    iters = synth.CONFIGS["nell2"]["iters"]
    init = synth.init_factors(t.dims, t.R, synth.CONFIGS["nell2"]["init_seed"])
    got = cpd.als(t.inds, t.vals, t.dims, t.R, iters, 0.0, init=[a.float().cuda() for a in init])
    _say("GPU CP-ALS done")
    init32 = [a.float().double().numpy() for a in init]
    ref = oals.cp_als(t.dims, t.inds_h, t.vals_h, t.R, iters, 0.0, init32, threads=THREADS)
    _say("oracle CP-ALS done")
    np.testing.assert_allclose(got["fits"], ref["fits"], rtol=0, atol=1e-5)
    assert abs(got["fit"] - ref["fit"]) <= 1e-4, (got["fit"], ref["fit"])
    A = [f.cpu().double().numpy() for f in got["factors"]]
    Y = ocoo.mttkrp(t.dims, t.inds_h, t.vals_h, A, t.nm - 1, threads=THREADS)
    own = oals.fit_from(ocoo.sumsq(t.vals_h), np.array(got["lam"]), A[t.nm - 1], Y, [oals.gram(a) for a in A])
    assert abs(got["fit"] - own) <= 1e-6, (got["fit"], own)
    for a in A:
        assert np.isfinite(a).all()
        np.testing.assert_allclose(np.linalg.norm(a, axis=0), 1.0, atol=1e-4)


_NETFLIX_REF = {}


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_full_size_als_final_fit_netflix(precision):
    """The NETFLIX shape, rank 16, 20 sweeps: the final fit with FP32 and with
    BF16 gathers within 1e-4 of the FP64 oracle's from the same start."""
    cpd = _cpd()
    t = _full("netflix")
    cfg = synth.CONFIGS["netflix"]
    init = synth.init_factors(t.dims, t.R, cfg["init_seed"])
    if "fit" not in _NETFLIX_REF:
        init32 = [a.float().double().numpy() for a in init]
        _NETFLIX_REF.update(oals.cp_als(t.dims, t.inds_h, t.vals_h, t.R, cfg["iters"], 0.0, init32,
                                        threads=THREADS))
        _say("oracle CP-ALS done")
    got = cpd.als(t.inds, t.vals, t.dims, t.R, cfg["iters"], 0.0, init=[a.float().cuda() for a in init],
                  precision=precision)
    assert abs(got["fit"] - _NETFLIX_REF["fit"]) <= 1e-4, (precision, got["fit"], _NETFLIX_REF["fit"])
    if precision == "fp32":
        np.testing.assert_allclose(got["fits"], _NETFLIX_REF["fits"], rtol=0, atol=1e-5)


# ------------------------------------------------------------------ completion

def test_full_size_completion_kernels_sampled_rows():
    """CP with missing values at the benchmark size (NELL-2 shape, rank 35):
    the row Grams of sampled rows (the fullest three among them) against the
    oracle's, and the row solves of those rows against the oracle's solve of
    the same Gram and right side."""
    from oracle import complete as oc
    cpd = _cpd()
    t = _full("nell2")
    R = t.R
    rng = np.random.default_rng(9)
    g = torch.Generator().manual_seed(4)
    facs, facs_used = [], []
    for d in t.dims:
        buf = torch.zeros((d, 36), dtype=torch.float32)
        buf[:, :R] = torch.rand((d, R), generator=g)
        facs.append(buf.cuda())
        facs_used.append(buf[:, :R].double().numpy())
    trees = cpd.csf_build_rooted(t.inds, t.vals, t.dims)
    reg = 0.1
    for m, c in enumerate(trees):
        counts = t.row_nnz[m]
        hot = np.argsort(-counts, kind="stable")[:3]
        rows = np.unique(np.concatenate([hot, rng.choice(np.flatnonzero(counts), size=4, replace=False)]))
        G = cpd.row_gram(c, facs, m, rank=R)
        y = cpd.mttkrp(c, facs, m, rank=R)
        A, _ = cpd.row_solve(G, y, reg, rank=R)
        torch.cuda.synchronize()
        got = G.cpu().numpy()[rows]
        ref = oc.row_grams(t.dims, t.inds_h, t.vals_h, facs_used, m, rows=rows)
        iu = np.triu_indices(R)
        scale = float(np.abs(ref).max())
        np.testing.assert_allclose(got[:, iu[0], iu[1]], ref[:, iu[0], iu[1]], rtol=0, atol=1e-12 * scale)
        ysel = y.cpu().numpy()[rows].astype(np.float64)
        full = np.stack([np.triu(gg) + np.triu(gg, 1).T for gg in got])
        want, _ = oc.solve_rows(full, ysel, reg, np.ones(rows.size, dtype=np.int64))
        err = np.linalg.norm(A.cpu().numpy()[rows] - want) / np.linalg.norm(want)
        assert err <= 1e-6, (m, err)
        _say("completion mode", m, "checked")
        del G, y, A
        c.free()
