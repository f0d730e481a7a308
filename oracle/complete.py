"""CP with missing values (tensor completion) by alternating least squares,
in FP64 (oracle; test infrastructure only).

The paper lists CP with missing values among the decompositions of the CPD
library it starts from (Section III) but gives no algorithm; this oracle
takes the row-wise least-squares form of CP-ALS restricted to the observed
entries.  Readings (each listed in the design notes):
  C1  the observed entries are the tensor's stored nonzeros (coordinates and
      values); every other entry is unknown, not zero.
  C2  the loss is sum over observed entries of (x - K(i_0..i_{N-1}))^2 plus
      reg * sum_m ||A_m||_F^2, with K(i..) = sum_r prod_m A_m(i_m, r) (no
      column weights lambda).
  C3  modes are updated in order 0..N-1.  Row i of A_n solves
          (G_i + reg I) a = y_i,  G_i = sum_{k in O_i} h_k h_k^T,
                                  y_i = sum_{k in O_i} x_k h_k,
      O_i the observations with i_n = i and h_k the Hadamard product of the
      other modes' rows of observation k: y_i is row i of the MTTKRP of the
      observed entries (Algorithm 1's MTTKRP step), G_i a Gram
      restricted to the row's observations.
  C4  a row with no observation becomes zero; a system whose Cholesky pivot
      falls below R*eps*max diag (reg = 0, rank-deficient rows) uses the
      pseudo-inverse, as CP-ALS does (R3).
  C5  after each sweep, the RMSE over the observed entries,
      sqrt(max(0, sum x^2 - 2 sum_i a_i.y_i + sum_i a_i^T G_i a_i) / |O|),
      from the last mode's Grams and MTTKRP (its rows just solved, the other
      factors unchanged since that MTTKRP).
  C6  stop at the iteration limit, or when tol > 0 and the RMSE changes by
      less than tol (checked from the second sweep).

Pinned by (tests/test_oracle_complete.py): the row Grams against a plain
loop over observations; a fully observed tensor with reg = 0 against the
unnormalised dense ALS update A_n = X_(n) KR (KR^T KR)^{-1} built from an
explicit unfolding and Khatri-Rao product; the closed form of a row with one
observation, with reg > 0 and (the pseudo-inverse path, C4) at reg = 0; the RMSE identity against residuals of the explicit model; exact
recovery of a planted low-rank tensor from a subset of its entries.
"""
from __future__ import annotations

import numpy as np

from . import als
from . import coo


def _hadamard_rows(inds, factors, mode):
    """h_k for every observation k: product of the other modes' rows (nnz x R)."""
    nnz = inds.shape[1]
    R = factors[0].shape[1]
    H = np.ones((nnz, R))
    for m, A in enumerate(factors):
        if m != mode:
            H = H * np.asarray(A, dtype=np.float64)[inds[m]]
    return H


def row_grams(dims, inds, vals, factors, mode, rows=None):
    """G_i = sum over observations in row i of h h^T (reading C3), FP64,
    shape (len(rows), R, R); rows defaults to every row of the mode."""
    inds = np.asarray(inds, dtype=np.int64)
    if rows is None:
        rows = np.arange(int(dims[mode]))
    rows = np.asarray(rows, dtype=np.int64)
    R = factors[0].shape[1]
    pos = np.full(int(dims[mode]), -1, dtype=np.int64)
    pos[rows] = np.arange(rows.size)
    take = np.flatnonzero(pos[inds[mode]] >= 0)
    # group the observations by output row; G_i = H_i^T H_i over row i's h's
    take = take[np.argsort(pos[inds[mode][take]], kind="stable")]
    H = _hadamard_rows(inds[:, take], factors, mode)
    owner = pos[inds[mode][take]]
    G = np.zeros((rows.size, R, R))
    bounds = np.flatnonzero(np.diff(owner)) + 1
    for a, b in zip(np.r_[0, bounds], np.r_[bounds, owner.size]):
        if b > a:
            G[owner[a]] = H[a:b].T @ H[a:b]
    return G


def row_counts(dims, inds, mode):
    """Observations per row of the mode."""
    return np.bincount(np.asarray(inds[mode], dtype=np.int64), minlength=int(dims[mode]))


def solve_rows(G, Y, reg, counts):
    """Row i: (G_i + reg I)^{-1} y_i by Cholesky, the pseudo-inverse when a
    pivot is too small (C4), zero for a row without observations."""
    n, R = Y.shape
    A = np.zeros((n, R))
    pinv = 0
    for i in range(n):
        if counts[i] == 0:
            continue
        M = G[i] + reg * np.eye(R)
        a, used = als.normal_solve(M, Y[i:i + 1])
        A[i] = a[0]
        pinv += int(used)
    return A, pinv


def loss_terms(A_n, Y, G):
    """sum_i a_i.y_i and sum_i a_i^T G_i a_i (reading C5)."""
    cross = float(np.sum(A_n * Y))
    quad = float(np.einsum("ir,irs,is->", A_n, G, A_n))
    return cross, quad


def rmse_direct(inds, vals, factors):
    """RMSE over the observed entries from the explicit model value of each."""
    inds = np.asarray(inds, dtype=np.int64)
    R = factors[0].shape[1]
    P = np.ones((inds.shape[1], R))
    for m, A in enumerate(factors):
        P = P * np.asarray(A, dtype=np.float64)[inds[m]]
    r = np.asarray(vals, dtype=np.float64) - P.sum(1)
    return float(np.sqrt(np.mean(r * r)))


def cp_complete(dims, inds, vals, rank, iters, tol, reg, init):
    """Completion ALS (C1-C6); init is a list of N (I_m x R) arrays (A_0 is
    not read: mode 0 is solved first).  Returns dict(factors, rmse, rmses,
    iters, pinv_used)."""
    nm = len(dims)
    inds = np.asarray(inds, dtype=np.int64)
    A = [np.array(a, dtype=np.float64, copy=True) for a in init]
    for m in range(nm):
        if A[m].shape != (int(dims[m]), rank):
            raise ValueError("init factor %d has shape %s" % (m, A[m].shape))
    nobs = inds.shape[1]
    normX2 = coo.sumsq(vals)
    counts = [row_counts(dims, inds, m) for m in range(nm)]
    rmses, prev, pinv = [], None, 0
    it = 0
    for it in range(1, iters + 1):
        for n in range(nm):
            Y = coo.mttkrp(dims, inds, vals, A, n)
            G = row_grams(dims, inds, vals, A, n)
            A[n], p = solve_rows(G, Y, reg, counts[n])
            pinv += p
        cross, quad = loss_terms(A[nm - 1], Y, G)
        rmse = float(np.sqrt(max(0.0, normX2 - 2.0 * cross + quad) / nobs))
        rmses.append(rmse)
        if tol > 0 and prev is not None and abs(rmse - prev) < tol:
            break
        prev = rmse
    return dict(factors=A, rmse=rmses[-1] if rmses else 0.0, rmses=rmses, iters=it, pinv_used=pinv)
