"""Pins of the completion oracle (oracle/complete.py) against what the
mathematics fixes: plain loops, the dense least-squares update, closed forms,
the explicit model, and exact recovery."""
import itertools

import numpy as np
import pytest

from oracle import complete as oc
from oracle import dense_check as dc


def _observed(dims, frac, seed):
    """A random subset of all coordinates (distinct), as an (N, nnz) array."""
    rng = np.random.default_rng(seed)
    allc = np.array(list(itertools.product(*[range(d) for d in dims]))).T
    keep = rng.random(allc.shape[1]) < frac
    return allc[:, keep]


def _factors(dims, R, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return [rng.random((d, R)) * scale + 0.1 for d in dims]


def _model(inds, factors):
    P = np.ones((inds.shape[1], factors[0].shape[1]))
    for m, A in enumerate(factors):
        P = P * A[inds[m]]
    return P.sum(1)


def test_row_grams_match_a_plain_loop():
    dims, R = (5, 4, 6), 3
    inds = _observed(dims, 0.4, 1)
    vals = np.random.default_rng(2).random(inds.shape[1])
    A = _factors(dims, R, 3)
    for mode in range(3):
        G = oc.row_grams(dims, inds, vals, A, mode)
        ref = np.zeros((dims[mode], R, R))
        for k in range(inds.shape[1]):
            h = [1.0] * R
            for m in range(3):
                if m != mode:
                    h = [h[r] * A[m][inds[m, k], r] for r in range(R)]
            i = inds[mode, k]
            for r in range(R):
                for c in range(R):
                    ref[i, r, c] += h[r] * h[c]
        np.testing.assert_allclose(G, ref, rtol=1e-13, atol=1e-13)
        sub = oc.row_grams(dims, inds, vals, A, mode, rows=[dims[mode] - 1, 0])
        np.testing.assert_allclose(sub, ref[[dims[mode] - 1, 0]], rtol=1e-13, atol=1e-13)


def test_fully_observed_sweep_is_the_dense_least_squares_update():
    """Every entry observed and reg = 0: G_i = KR^T KR for every row and y_i is
    row i of X_(n) KR, so each update is A_n = X_(n) KR (KR^T KR)^{-1} with
    KR the Khatri-Rao product of the other factors (explicit unfolding)."""
    dims, R = (4, 5, 3), 2
    inds = _observed(dims, 1.1, 0)
    rng = np.random.default_rng(4)
    vals = rng.random(inds.shape[1]) + 0.5
    init = _factors(dims, R, 5)
    got = oc.cp_complete(dims, inds, vals, R, 2, 0.0, 0.0, init)
    X = dc.dense(dims, inds, vals)
    A = [a.copy() for a in init]
    for _ in range(2):
        for n in range(3):
            KR = dc.khatri_rao([A[m] for m in range(2, -1, -1) if m != n])
            A[n] = dc.unfold(X, n) @ KR @ np.linalg.inv(KR.T @ KR)
    for m in range(3):
        np.testing.assert_allclose(got["factors"][m], A[m], rtol=1e-9, atol=1e-12)
    # and the RMSE then is that of the dense residual
    resid = X - dc.full(np.ones(R), A)
    assert abs(got["rmse"] - np.sqrt(np.mean(resid ** 2))) < 1e-10


def test_single_observation_row_closed_form():
    """One observation x with row product h: (h h^T + reg I) a = x h gives
    a = x h / (h.h + reg) (Sherman-Morrison)."""
    dims, R, reg = (3, 4, 5), 3, 0.25
    inds = np.array([[0, 1, 1, 2], [1, 2, 3, 0], [4, 0, 2, 3]])
    vals = np.array([1.5, -2.0, 0.75, 3.0])
    A = _factors(dims, R, 7)
    counts = oc.row_counts(dims, inds, 0)
    from oracle import coo
    Y = coo.mttkrp(dims, inds, vals, A, 0)
    G = oc.row_grams(dims, inds, vals, A, 0)
    A0, pinv = oc.solve_rows(G, Y, reg, counts)
    h = A[1][1] * A[2][4]
    np.testing.assert_allclose(A0[0], 1.5 * h / (h @ h + reg), rtol=1e-12)
    assert pinv == 0


def test_rows_without_observations_become_zero():
    dims, R = (6, 3, 3), 2
    inds = np.array([[0, 0, 2], [0, 1, 2], [1, 2, 0]])
    vals = np.array([1.0, 2.0, 3.0])
    got = oc.cp_complete(dims, inds, vals, R, 1, 0.0, 0.1, _factors(dims, R, 1))
    A0 = got["factors"][0]
    assert (A0[[1, 3, 4, 5]] == 0).all() and np.abs(A0[[0, 2]]).sum() > 0


def test_rmse_identity_matches_the_explicit_model():
    dims, R = (7, 6, 5), 3
    inds = _observed(dims, 0.5, 8)
    vals = np.random.default_rng(9).random(inds.shape[1])
    for reg in (0.0, 0.3):
        got = oc.cp_complete(dims, inds, vals, R, 3, 0.0, reg, _factors(dims, R, 10))
        assert abs(got["rmse"] - oc.rmse_direct(inds, vals, got["factors"])) < 1e-10


def test_planted_low_rank_is_recovered_from_part_of_its_entries():
    """A rank-2 tensor observed at half of its entries: the unobserved entries
    are predicted too (the model, not only the fit, is recovered)."""
    dims, R = (12, 11, 10), 2
    truth = _factors(dims, R, 20)
    inds = _observed(dims, 0.5, 21)
    vals = _model(inds, truth)
    best = None
    for seed in range(3):
        got = oc.cp_complete(dims, inds, vals, R, 400, 0.0, 0.0, _factors(dims, R, 30 + seed))
        if best is None or got["rmse"] < best["rmse"]:
            best = got
    assert best["rmse"] < 1e-9
    held = _observed(dims, 1.1, 0)
    np.testing.assert_allclose(_model(held, best["factors"]), _model(held, truth), rtol=1e-6, atol=1e-8)


def test_solved_rows_satisfy_their_regularised_normal_equations():
    """Each row from solve_rows (own Cholesky) solves (G_i + reg I) a = y_i as
    LAPACK's general solver does; reg shrinks the factor."""
    from oracle import coo
    dims, R = (6, 5, 4), 3
    inds = _observed(dims, 0.7, 40)
    vals = np.random.default_rng(41).random(inds.shape[1])
    A = _factors(dims, R, 42)
    counts = oc.row_counts(dims, inds, 1)
    Y = coo.mttkrp(dims, inds, vals, A, 1)
    G = oc.row_grams(dims, inds, vals, A, 1)
    norms = []
    for reg in (0.0, 1.0):
        X, _ = oc.solve_rows(G, Y, reg, counts)
        for i in range(dims[1]):
            ref = np.linalg.solve(G[i] + reg * np.eye(R), Y[i])
            np.testing.assert_allclose(X[i], ref, rtol=1e-9, atol=1e-12)
        norms.append(np.linalg.norm(X))
    assert norms[1] < norms[0]


def test_rank_deficient_row_at_zero_reg_takes_the_minimum_norm_solution():
    """Reading C4: one observation and reg = 0 give G_i = h h^T (rank one), so
    the pseudo-inverse path must return the minimum-norm solution of
    h h^T a = x h, which is a = x h / (h.h)."""
    from oracle import coo
    dims, R = (3, 4, 5), 3
    inds = np.array([[0, 1, 1, 2], [1, 2, 3, 0], [4, 0, 2, 3]])
    vals = np.array([1.5, -2.0, 0.75, 3.0])
    A = _factors(dims, R, 7)
    counts = oc.row_counts(dims, inds, 0)
    Y = coo.mttkrp(dims, inds, vals, A, 0)
    G = oc.row_grams(dims, inds, vals, A, 0)
    A0, pinv = oc.solve_rows(G, Y, 0.0, counts)
    h = A[1][1] * A[2][4]
    np.testing.assert_allclose(A0[0], 1.5 * h / (h @ h), rtol=1e-10)
    # row 2 (one observation too) and row 1 (two: rank two, still below R = 3)
    assert pinv == 3
    h2 = A[1][0] * A[2][3]
    np.testing.assert_allclose(A0[2], 3.0 * h2 / (h2 @ h2), rtol=1e-10)
    np.testing.assert_allclose(A0[1], np.linalg.pinv(G[1]) @ Y[1], rtol=1e-8, atol=1e-12)


def test_stopping_rule():
    """Reading C6: with tol > 0 the sweeps stop once the RMSE changes by less
    than tol, checked from the second sweep; tol = 0 runs every sweep."""
    dims, R = (6, 5, 4), 2
    inds = _observed(dims, 0.6, 50)
    vals = np.random.default_rng(51).random(inds.shape[1])
    init = _factors(dims, R, 52)
    full = oc.cp_complete(dims, inds, vals, R, 6, 0.0, 0.1, init)
    assert full["iters"] == 6 and len(full["rmses"]) == 6
    early = oc.cp_complete(dims, inds, vals, R, 6, 1e9, 0.1, init)
    assert early["iters"] == 2 and early["rmses"] == full["rmses"][:2]
    # a tolerance between two consecutive changes stops right after the first change below it
    d = np.abs(np.diff(full["rmses"]))
    k = int(np.argmax(d < d[0])) if (d < d[0]).any() else None
    if k is not None:
        mid = oc.cp_complete(dims, inds, vals, R, 6, float(d[0]), 0.1, init)
        assert mid["iters"] == k + 2
