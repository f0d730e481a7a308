"""CP-ALS driver in FP64 (oracle; test infrastructure only).

Algorithm 1 (Section III), generalised from three to N modes, in the paper's
update order: for each mode n in turn,
  V   <- Hadamard product of the Grams A_m^T A_m of the other modes,
  A_n <- MTTKRP_n(X; other factors) V^+,
  normalise the columns of A_n, keeping the norms as lambda,
and after each sweep the fit of the model; stop when the fit stops improving
or at the iteration limit.

Readings where the paper is silent (each listed in the design notes):
  R2  column norm: the 2-norm, every iteration.
  R3  V^+: Cholesky (the paper's code calls potrf/potrs, Section V-A); when a
      pivot is <= R*eps*max(diag V) the Moore-Penrose inverse is used instead,
      from a symmetric eigendecomposition that drops eigenvalues
      <= R*eps*max eigenvalue.
  R4  initial factors are supplied by the caller; A_0 is never read.
  R5  fit = 1 - ||X - K||_F / ||X||_F with K = [[lambda; A_0..A_{N-1}]], by
      ||X - K||^2 = ||X||^2 - 2<X, K> + ||K||^2, where
      <X, K> = sum_r lambda_r sum_i A_{N-1}(i, r) Y_{N-1}(i, r) and
      ||K||^2 = lambda^T (Hadamard of all Grams) lambda.
  R6  stop when tol > 0, from the second iteration on, if |fit - fit_prev| < tol.
  R7  a zero column keeps lambda_r = 0 and stays zero.

Pinned by: the fit identity against a dense residual; rank-1 block-planted
data reaching fit 1 after one sweep; block-sparse rank-8 recovery; the
Cholesky solve against numpy's factorisation and a residual bound; the
fallback against a constructed singular V; invariance of the fit under the
max-norm normalisation convention.
"""
from __future__ import annotations

import numpy as np

from . import coo

EPS = np.finfo(np.float64).eps


def gram(A):
    """A^T A (Algorithm 1's A^T A terms), FP64."""
    A = np.asarray(A, dtype=np.float64)
    return A.T @ A


def hadamard_v(grams, n):
    """V for mode n: element-wise product of the Grams of every other mode."""
    R = grams[0].shape[0]
    V = np.ones((R, R))
    for m, G in enumerate(grams):
        if m != n:
            V = V * G
    return V


def cholesky(V):
    """Lower L with L L^T = V (Cholesky-Banachiewicz), or None when a pivot is
    <= R*eps*max(diag V) (reading R3)."""
    R = V.shape[0]
    thresh = R * EPS * float(np.max(np.diag(V))) if R else 0.0
    L = np.zeros_like(V)
    for j in range(R):
        d = V[j, j] - L[j, :j] @ L[j, :j]
        if not d > thresh:
            return None
        L[j, j] = np.sqrt(d)
        L[j + 1:, j] = (V[j + 1:, j] - L[j + 1:, :j] @ L[j, :j]) / L[j, j]
    return L


def pinv_sym(V):
    """Moore-Penrose inverse of symmetric V by eigendecomposition, dropping
    eigenvalues <= R*eps*max eigenvalue (reading R3)."""
    R = V.shape[0]
    w, Q = np.linalg.eigh(V)
    wmax = float(w.max()) if R else 0.0
    keep = w > R * EPS * wmax
    return (Q[:, keep] / w[keep]) @ Q[:, keep].T


def forward_sub(L, B):
    """Solve L Z = B for lower-triangular L, column by column of B (FP64)."""
    R = L.shape[0]
    Z = np.zeros_like(B)
    for i in range(R):
        Z[i] = (B[i] - L[i, :i] @ Z[:i]) / L[i, i]
    return Z


def back_sub(U, B):
    """Solve U Z = B for upper-triangular U."""
    R = U.shape[0]
    Z = np.zeros_like(B)
    for i in range(R - 1, -1, -1):
        Z[i] = (B[i] - U[i, i + 1:] @ Z[i + 1:]) / U[i, i]
    return Z


def normal_solve(V, Y):
    """A = Y V^+ (Algorithm 1's V-dagger): Cholesky when it succeeds, else the
    pseudo-inverse.  Returns (A, used_pinv)."""
    Y = np.asarray(Y, dtype=np.float64)
    L = cholesky(V)
    if L is not None:
        Z = forward_sub(L, Y.T)            # L Z = Y^T
        return back_sub(L.T, Z).T, False   # L^T A^T = Z
    return Y @ pinv_sym(V), True


def normalize_columns(A, kind="2"):
    """Column norms lambda and A with unit columns (zero columns stay zero).
    kind "2" is the 2-norm (R2); "max" is the max-abs norm."""
    A = np.asarray(A, dtype=np.float64)
    lam = np.sqrt((A * A).sum(0)) if kind == "2" else np.abs(A).max(0)
    out = A.copy()
    nz = lam > 0
    out[:, nz] = A[:, nz] / lam[nz]
    return out, lam


def fit_from(normX2, lam, A_last, Y_last, grams):
    """Fit of K = [[lambda; A]] to X (reading R5)."""
    inner = float(lam @ (A_last * Y_last).sum(0))
    H = np.ones_like(grams[0])
    for G in grams:
        H = H * G
    normK2 = float(lam @ H @ lam)
    resid2 = max(0.0, normX2 - 2.0 * inner + normK2)
    return 1.0 - np.sqrt(resid2) / np.sqrt(normX2)


def cp_als(dims, inds, vals, rank, iters, tol, init, norm="2", threads=1):
    """Run CP-ALS; init is a list of N (I_m x R) arrays (A_0 is not read);
    threads: host threads of the MTTKRP loop (1: the sequential loop).

    Returns dict(lam, factors, fit, iters, fits, pinv_used)."""
    nm = len(dims)
    A = [np.array(a, dtype=np.float64, copy=True) for a in init]
    for m in range(nm):
        if A[m].shape != (int(dims[m]), rank):
            raise ValueError("init factor %d has shape %s" % (m, A[m].shape))
    normX2 = coo.sumsq(vals)
    grams = [gram(a) for a in A]
    fits, fit_prev, pinv_used = [], None, 0
    lam = np.zeros(rank)
    Y = None
    it = 0
    for it in range(1, iters + 1):
        for n in range(nm):
            V = hadamard_v(grams, n)
            Y = coo.mttkrp(dims, inds, vals, A, n, threads=threads)
            An, used = normal_solve(V, Y)
            pinv_used += int(used)
            A[n], lam = normalize_columns(An, norm)
            grams[n] = gram(A[n])
        fit = fit_from(normX2, lam, A[nm - 1], Y, grams)
        fits.append(fit)
        if tol > 0 and fit_prev is not None and abs(fit - fit_prev) < tol:
            break
        fit_prev = fit
    return dict(lam=lam, factors=A, fit=fits[-1] if fits else 0.0, iters=it, fits=fits,
                pinv_used=pinv_used)
