"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a
hand-worked example, brute force on tiny tensors, closed forms, invariants or
a textbook/library routine for a special case.
"""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import als, coo, csf, dense_check
from paper_1812_05961_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_coo(rng, dims, nnz, dup=False):
    if dup:
        inds = np.stack([rng.integers(0, d, nnz) for d in dims])
    else:
        cells = rng.choice(int(np.prod(dims)), size=nnz, replace=False)
        inds = np.stack(np.unravel_index(cells, dims))
    vals = rng.standard_normal(nnz)
    return inds.astype(np.int64), vals


def _rand_factors(rng, dims, R):
    return [rng.standard_normal((d, R)) for d in dims]


# ---------------------------------------------------------------- MTTKRP pins

def test_mttkrp_hand_worked_example():
    g = json.load(open(os.path.join(GOLDEN, "mttkrp_2x2x2.json")))
    facs = [np.array(f, dtype=float) for f in g["factors"]]
    for n in range(3):
        Y = coo.mttkrp(g["dims"], g["inds"], g["vals"], facs, n)
        np.testing.assert_array_equal(Y, np.array(g["Y"][n], dtype=float))
        assert (facs[n] * Y).sum() == g["inner_product_all_modes"]


@pytest.mark.parametrize("dims", [(4, 3, 5), (3, 4, 2, 3), (2, 3, 2, 3, 2)])
@pytest.mark.parametrize("R", [1, 3])
@pytest.mark.parametrize("dup", [False, True])
def test_mttkrp_equals_unfolding_times_khatri_rao(dims, R, dup):
    rng = np.random.default_rng(7 + len(dims) + R + dup)
    nnz = int(np.prod(dims)) // 2
    inds, vals = _rand_coo(rng, dims, nnz, dup)
    facs = _rand_factors(rng, dims, R)
    X = dense_check.dense(dims, inds, vals)
    for n in range(len(dims)):
        Y = coo.mttkrp(dims, inds, vals, facs, n)
        Yd = dense_check.mttkrp_dense(X, facs, n)
        np.testing.assert_allclose(Y, Yd, rtol=1e-12, atol=1e-12)


def test_khatri_rao_kolda_column_order():
    # (A kr B)[i * I_B + j, r] = A[i, r] * B[j, r]
    A = np.arange(6.0).reshape(3, 2)
    B = np.arange(4.0).reshape(2, 2) + 10
    K = dense_check.khatri_rao([A, B])
    for i, j, r in itertools.product(range(3), range(2), range(2)):
        assert K[i * 2 + j, r] == A[i, r] * B[j, r]


def test_mttkrp_single_nonzero_is_scaled_hadamard():
    dims = (5, 6, 7, 4)
    rng = np.random.default_rng(3)
    facs = _rand_factors(rng, dims, 5)
    idx = np.array([[2], [5], [0], [3]])
    x = 1.75
    for n in range(4):
        Y = coo.mttkrp(dims, idx, [x], facs, n)
        expect = np.full(5, x)
        for m in range(4):
            if m != n:
                expect = expect * facs[m][idx[m, 0]]
        assert np.count_nonzero(np.abs(Y).sum(1)) == 1
        np.testing.assert_allclose(Y[idx[n, 0]], expect, rtol=1e-15)


def test_mttkrp_all_ones_factors_give_slice_sums():
    dims = (6, 5, 4)
    rng = np.random.default_rng(4)
    inds, vals = _rand_coo(rng, dims, 50)
    facs = [np.ones((d, 3)) for d in dims]
    for n in range(3):
        Y = coo.mttkrp(dims, inds, vals, facs, n)
        sums = np.bincount(inds[n], weights=vals, minlength=dims[n])
        for r in range(3):
            np.testing.assert_allclose(Y[:, r], sums, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("dims", [(30, 20, 10), (8, 7, 6, 5)])
def test_mttkrp_cross_mode_invariant(dims):
    rng = np.random.default_rng(5)
    inds, vals = _rand_coo(rng, dims, 400)
    facs = _rand_factors(rng, dims, 4)
    # <X, [[A]]> computed straight from the nonzeros
    model = np.ones((inds.shape[1], 4))
    for m in range(len(dims)):
        model = model * facs[m][inds[m]]
    ref = float(vals @ model.sum(1))
    for n in range(len(dims)):
        Y = coo.mttkrp(dims, inds, vals, facs, n)
        assert abs((facs[n] * Y).sum() - ref) <= 1e-11 * max(1.0, abs(ref))


def test_mttkrp_rows_matches_full_rows():
    dims = (40, 30, 20)
    rng = np.random.default_rng(6)
    inds, vals = _rand_coo(rng, dims, 3000)
    facs = _rand_factors(rng, dims, 6)
    Y = coo.mttkrp(dims, inds, vals, facs, 1)
    rows = np.array([0, 29, 7, 13])
    np.testing.assert_array_equal(coo.mttkrp_rows(dims, inds, vals, facs, 1, rows), Y[rows])
    with pytest.raises(ValueError):
        coo.mttkrp_rows(dims, inds, vals, facs, 1, [3, 3])


def test_mttkrp_rejects_out_of_range_index():
    with pytest.raises(ValueError):
        coo.mttkrp((3, 3, 3), [[0], [3], [0]], [1.0], [np.ones((3, 2))] * 3, 0)


# ------------------------------------------------------------------- CSF pins

def _csf_brute(dims, inds, vals, order):
    """Tree built from Python tuples and dicts (a different algorithm)."""
    entries = {}
    for k in range(inds.shape[1]):
        key = tuple(int(inds[m, k]) for m in order)
        entries[key] = np.float32(entries[key] + np.float32(vals[k])) if key in entries \
            else np.float32(vals[k])
    keys = sorted(entries)
    nm = len(order)
    levels = []
    for l in range(nm):
        levels.append(sorted({k[: l + 1] for k in keys}))
    fids = [[p[-1] for p in lv] for lv in levels]
    fptr = []
    for l in range(nm - 1):
        pos = {p: j for j, p in enumerate(levels[l + 1])}
        ptr = [pos[next(c for c in levels[l + 1] if c[: l + 1] == p)] for p in levels[l]]
        fptr.append(ptr + [len(levels[l + 1])])
    return dict(counts=[len(lv) for lv in levels], fids=fids, fptr=fptr,
                vals=[entries[k] for k in keys])


def test_csf_hand_worked_example():
    g = json.load(open(os.path.join(GOLDEN, "mttkrp_2x2x2.json")))
    for key, ref in g["csf"].items():
        order = [int(c) for c in key.split(",")]
        c = csf.build(g["dims"], g["inds"], g["vals"], order)
        assert c["counts"] == ref["counts"]
        for l in range(3):
            assert c["fids"][l].tolist() == ref["fids"][l]
        for l in range(2):
            assert c["fptr"][l].tolist() == ref["fptr"][l]
        assert c["vals"].tolist() == ref["vals"]


@pytest.mark.parametrize("dims,order", [((5, 4, 6), (0, 1, 2)), ((5, 4, 6), (2, 0, 1)),
                                        ((3, 4, 2, 3), (3, 1, 0, 2)),
                                        ((2, 3, 2, 3, 2), (4, 0, 3, 1, 2))])
@pytest.mark.parametrize("dup", [False, True])
def test_csf_matches_brute_force_tree(dims, order, dup):
    rng = np.random.default_rng(11)
    nnz = max(3, int(np.prod(dims)) // 3)
    inds, vals = _rand_coo(rng, dims, nnz, dup)
    vals = vals.astype(np.float32)
    c = csf.build(dims, inds, vals, order)
    b = _csf_brute(dims, inds, vals, order)
    assert c["counts"] == b["counts"]
    for l in range(len(dims)):
        assert c["fids"][l].tolist() == b["fids"][l]
    for l in range(len(dims) - 1):
        assert c["fptr"][l].tolist() == b["fptr"][l]
    assert c["vals"].tobytes() == np.array(b["vals"], dtype=np.float32).tobytes()


def test_csf_duplicates_sum_in_input_order():
    # float32 sums that depend on the order: 1e8 + 1 - 1e8 ...
    inds = np.array([[0, 0, 0, 1], [0, 0, 0, 0], [0, 0, 0, 0]])
    vals = np.array([1e8, 1.0, -1e8, 2.0], dtype=np.float32)
    c = csf.build((2, 1, 1), inds, vals, (0, 1, 2))
    expect = np.float32(np.float32(np.float32(1e8) + np.float32(1.0)) + np.float32(-1e8))
    assert c["vals"][0] == expect and c["vals"][1] == np.float32(2.0)
    assert c["counts"] == [2, 2, 2]


def test_csf_invariants_and_expand_roundtrip():
    t = synth.make_config("small3")
    inds, vals = t.numpy()
    for order in [csf.heuristic_order(t.dims), (0, 1, 2), (1, 2, 0)]:
        c = csf.build(t.dims, inds, vals, order)
        for l in range(2):
            p = c["fptr"][l]
            assert p[0] == 0 and p[-1] == c["counts"][l + 1]
            assert (np.diff(p) > 0).all()
        rows, v = csf.expand(c)
        perm = np.lexsort(inds[list(order)][::-1])
        np.testing.assert_array_equal(rows, inds[list(order)][:, perm])
        np.testing.assert_array_equal(v, vals.astype(np.float32)[perm])


def test_csf_tile_starts_by_walking():
    t = synth.make_config("small3")
    inds, vals = t.numpy()
    c = csf.build(t.dims, inds, vals, csf.heuristic_order(t.dims))
    rows, _ = csf.expand(c)
    for T in (1, 7, 256, 4096, 50000):
        ts = csf.tile_starts(c, T)
        # walk: the node of leaf k at level l is its ordinal among distinct prefixes
        for l in range(2):
            prefix_change = np.r_[True, (rows[: l + 1, 1:] != rows[: l + 1, :-1]).any(0)]
            node = np.cumsum(prefix_change) - 1
            np.testing.assert_array_equal(ts[l], node[np.arange(ts.shape[1]) * T])


def test_heuristic_order_ascending_ties_low_mode():
    assert csf.heuristic_order((12000, 9000, 29000)) == [1, 0, 2]
    assert csf.heuristic_order((480000, 18000, 2000)) == [2, 1, 0]
    assert csf.heuristic_order((5, 3, 5, 3)) == [1, 3, 0, 2]


# ------------------------------------------------------ Gram / solve / normalise

def test_gram_brute_force_and_symmetry():
    rng = np.random.default_rng(8)
    A = rng.standard_normal((37, 6))
    G = als.gram(A)
    B = np.zeros((6, 6))
    for i in range(37):
        for r in range(6):
            for s in range(6):
                B[r, s] += A[i, r] * A[i, s]
    np.testing.assert_allclose(G, B, rtol=1e-13, atol=1e-13)
    assert (G == G.T).all()


def test_cholesky_matches_library_factor_and_solve_residual():
    rng = np.random.default_rng(9)
    for R in (1, 5, 35, 64):
        M = rng.standard_normal((3 * R, R))
        V = M.T @ M
        L = als.cholesky(V)
        np.testing.assert_allclose(L, np.linalg.cholesky(V), rtol=1e-10, atol=1e-12)
        Y = rng.standard_normal((50, R))
        A, used = als.normal_solve(V, Y)
        assert not used
        assert np.linalg.norm(A @ V - Y) <= 1e-12 * np.linalg.norm(Y) * np.linalg.cond(V)


def test_disjoint_support_factors_give_identity_v():
    # factors with orthonormal columns (disjoint row supports) -> V = I -> A = Y
    dims = (6, 4, 5)
    facs = []
    for d in dims:
        F = np.zeros((d, 3))
        F[0, 0] = F[1, 1] = F[2, 2] = 1.0
        facs.append(F)
    grams = [als.gram(F) for F in facs]
    V = als.hadamard_v(grams, 0)
    np.testing.assert_array_equal(V, np.eye(3))
    Y = np.arange(18.0).reshape(6, 3)
    A, used = als.normal_solve(V, Y)
    assert not used
    np.testing.assert_allclose(A, Y, rtol=0, atol=1e-14)


def test_singular_v_uses_pseudo_inverse():
    rng = np.random.default_rng(10)
    M = rng.standard_normal((20, 4))
    M[:, 3] = M[:, 1]                       # duplicated column: rank 3
    V = M.T @ M
    Y = rng.standard_normal((7, 4))
    A, used = als.normal_solve(V, Y)
    assert used
    np.testing.assert_allclose(A, Y @ np.linalg.pinv(V, rcond=4 * np.finfo(float).eps),
                               rtol=1e-8, atol=1e-10)
    Z = np.zeros((3, 3))
    A0, used0 = als.normal_solve(Z, np.ones((2, 3)))
    assert used0 and (A0 == 0).all()


def test_normalize_zero_column_stays_zero():
    A = np.array([[3.0, 0.0], [4.0, 0.0]])
    B, lam = als.normalize_columns(A)
    np.testing.assert_allclose(lam, [5.0, 0.0])
    np.testing.assert_allclose(B, [[0.6, 0.0], [0.8, 0.0]])
    assert np.isfinite(B).all()


# ------------------------------------------------------------------- Fit pins

@pytest.mark.parametrize("dims", [(4, 5, 3), (3, 2, 4, 3)])
def test_fit_identity_matches_dense_residual(dims):
    rng = np.random.default_rng(12)
    inds, vals = _rand_coo(rng, dims, int(np.prod(dims)) // 2)
    R = 3
    facs = _rand_factors(rng, dims, R)
    lam = rng.uniform(0.5, 2.0, R)
    nm = len(dims)
    Y = coo.mttkrp(dims, inds, vals, facs, nm - 1)
    fit = als.fit_from(coo.sumsq(vals), lam, facs[-1], Y, [als.gram(f) for f in facs])
    X = dense_check.dense(dims, inds, vals)
    K = dense_check.full(lam, facs)
    ref = 1 - np.linalg.norm(X - K) / np.linalg.norm(X)
    assert abs(fit - ref) < 1e-11


def test_rank1_block_planted_fit_one_after_one_sweep():
    # X = a o b o c on a block: after the first mode update A_0 is exactly
    # proportional to a (X_(0)(C kr B) = a (c^T C)(b^T B) scaled), and so on.
    t, facs = synth.block_planted(dims=(30, 20, 10), rank=1, block=(9, 7, 5), seed=21)
    inds, vals = t.numpy()
    init = synth.init_factors(t.dims, 1, 5)
    out = als.cp_als(t.dims, inds, vals, 1, 1, 0.0, [a.numpy() for a in init])
    assert out["fit"] > 1 - 1e-7
    # the factor directions are the planted ones
    for m in range(3):
        a = facs[m][:, 0].numpy()
        np.testing.assert_allclose(np.abs(out["factors"][m][:, 0]), a / np.linalg.norm(a),
                                   atol=1e-10)


def test_block_sparse_rank8_recovery():
    t, _ = synth.block_planted()
    inds, vals = t.numpy()
    best = 0.0
    for s in range(3):
        init = [a.numpy() for a in synth.init_factors(t.dims, 8, 100 + s)]
        out = als.cp_als(t.dims, inds, vals, 8, 500, 1e-12, init)
        best = max(best, out["fit"])
        if best >= 1 - 1e-6:
            break
    assert best >= 1 - 1e-6


def test_fit_invariant_to_norm_convention():
    t = synth.make_config("small3")
    inds, vals = t.numpy()
    init = [a.numpy() for a in synth.init_factors(t.dims, 8, 11)]
    a = als.cp_als(t.dims, inds, vals, 8, 6, 0.0, init, norm="2")
    b = als.cp_als(t.dims, inds, vals, 8, 6, 0.0, init, norm="max")
    np.testing.assert_allclose(a["fits"], b["fits"], rtol=0, atol=1e-10)


def test_convergence_rule_and_zero_column():
    t = synth.make_config("small3")
    inds, vals = t.numpy()
    init = [a.numpy() for a in synth.init_factors(t.dims, 4, 11)]
    out = als.cp_als(t.dims, inds, vals, 4, 50, 1.0, init)
    assert out["iters"] == 2                 # |dfit| < 1 at the first check
    init[1][:, 2] = 0.0                       # a zero column: V singular in mode 0
    out = als.cp_als(t.dims, inds, vals, 4, 2, 0.0, init)
    assert out["pinv_used"] >= 1
    assert all(np.isfinite(f).all() for f in out["factors"])
    assert np.isfinite(out["fit"])


def test_splitmix64_published_first_output():
    # SplitMix64 seeded with 0: first output 0xE220A8397B1DCDAF
    assert synth.splitmix64_int(0) == 0xE220A8397B1DCDAF
    import torch
    assert synth.splitmix64(torch.tensor([0]))[0].item() == synth._s64(0xE220A8397B1DCDAF)


def test_threaded_mttkrp_equals_the_sequential_loop():
    """The multi-threaded oracle loop (private copies summed in range order)
    gives the sequential loop's sums up to FP64 addition order, for thread
    counts that do and do not divide the nonzeros, and more threads than
    nonzeros."""
    import numpy as np

    from oracle import coo
    rng = np.random.default_rng(41)
    dims = (30, 20, 10, 7)
    nnz = 5003
    inds = np.stack([rng.integers(0, d, nnz) for d in dims])
    vals = rng.standard_normal(nnz)
    F = [rng.standard_normal((d, 5)) for d in dims]
    for mode in range(4):
        ref = coo.mttkrp(dims, inds, vals, F, mode)
        for th in (2, 3, 16):
            got = coo.mttkrp(dims, inds, vals, F, mode, threads=th)
            np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    few = coo.mttkrp(dims, inds[:, :3], vals[:3], F, 1, threads=8)
    np.testing.assert_allclose(few, coo.mttkrp(dims, inds[:, :3], vals[:3], F, 1), rtol=0, atol=1e-15)


def test_csf_packed_sort_equals_lexsort():
    """The packed-integer sort of the CSF oracle orders the nonzeros exactly as
    numpy.lexsort on the index rows (stable, duplicates in input order), for
    every mode order of 3- and 4-mode tensors with repeated coordinates."""
    import itertools

    import numpy as np

    from oracle import csf
    rng = np.random.default_rng(5)
    for dims in ((7, 5, 9), (4, 6, 3, 5)):
        n = 400
        inds = np.stack([rng.integers(0, d, n) for d in dims])
        inds[:, 300:] = inds[:, :100]                    # duplicates
        vals = rng.standard_normal(n).astype(np.float32)
        for order in itertools.permutations(range(len(dims))):
            a = csf.sort_perm(dims, inds, list(order), "lexsort")
            b = csf.sort_perm(dims, inds, list(order), "packed")
            np.testing.assert_array_equal(a, b)
            ta = csf.build(dims, inds, vals, list(order), "lexsort")
            tb = csf.build(dims, inds, vals, list(order), "packed")
            assert ta["counts"] == tb["counts"]
            for l in range(len(dims)):
                np.testing.assert_array_equal(ta["fids"][l], tb["fids"][l])
            assert ta["vals"].tobytes() == tb["vals"].tobytes()
