"""Dense brute force for tiny tensors (oracle; test infrastructure only).

Builds the dense tensor, its mode-n unfolding and the explicit Khatri-Rao
product that the MTTKRP avoids (Section III), so the COO oracle can be checked
against the matrix form X_(n) (A_{N-1} kr ... kr A_{n+1} kr A_{n-1} kr ... kr A_0).

Unfolding convention (Kolda and Bader): column j of X_(n) is
j = sum_{k != n} i_k J_k with J_k = prod_{m < k, m != n} I_m, so the lowest
remaining mode varies fastest; the Khatri-Rao product lists the factors from
the highest mode down, whose Kronecker columns also put the lowest mode
fastest.  The Khatri-Rao product (A kr B) has column r = kron(a_r, b_r).
"""
from __future__ import annotations

import numpy as np


def dense(dims, inds, vals):
    X = np.zeros([int(d) for d in dims])
    np.add.at(X, tuple(np.asarray(inds, dtype=np.int64)), np.asarray(vals, dtype=np.float64))
    return X


def unfold(X, n):
    """Mode-n matricization X_(n), I_n x prod_{m != n} I_m."""
    return np.reshape(np.moveaxis(X, n, 0), (X.shape[n], -1), order="F")


def khatri_rao(mats):
    """Column-wise Kronecker product of the list, first matrix slowest."""
    R = mats[0].shape[1]
    cols = []
    for r in range(R):
        c = np.ones(1)
        for M in mats:
            c = np.kron(c, M[:, r])
        cols.append(c)
    return np.stack(cols, axis=1)


def mttkrp_dense(X, factors, n):
    """X_(n) times the explicit Khatri-Rao product of the other factors."""
    others = [factors[m] for m in range(X.ndim - 1, -1, -1) if m != n]
    return unfold(X, n) @ khatri_rao(others)


def full(lam, factors):
    """Dense K = sum_r lambda_r a_r^(0) o ... o a_r^(N-1)."""
    R = factors[0].shape[1]
    K = np.zeros([f.shape[0] for f in factors])
    for r in range(R):
        t = np.array(lam[r])
        for f in factors:
            t = np.multiply.outer(t, f[:, r])
        K += t
    return K
