"""Householder QR and triangular solves of the oracle, float64.

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this module.

Step 3 of the sketch-and-solve paradigm (Sec. 1.2) solves the reduced problem
min ||SA x - Sb|| of Sec. 1.3 "using existing algorithms"; the classical one
is Householder QR of SA followed by back substitution.  The QR is applied to
the augmented matrix [SA | Sb] so that c = (Q^T Sb)[:n] and the sketched
residual norm come out of the same factorisation.

Householder convention (Golub and Van Loan, Householder vector of a column,
LAPACK sign choice): for the column x = M[k:, k], alpha = x[0],
beta = -sign(alpha) ||x|| with sign(0) = +1, tau = (beta - alpha) / beta,
v = x / (alpha - beta) with v[0] = 1, and H = I - tau v v^T maps x to
beta e_1.  A zero column (||x|| = 0) gets tau = 0 (H = I).
"""
from __future__ import annotations

import numpy as np


def householder_qr_augmented(SA: np.ndarray, Sb: np.ndarray | None = None):
    """Householder QR of [SA | Sb] (d x (n+1)), one column at a time.

    Returns (R, c, rho, V, tau): R the n x n upper factor, c the first n
    entries of Q^T Sb, rho = ||(Q^T Sb)[n:]|| (the sketched residual norm),
    V the d x n Householder vectors (unit lower trapezoidal) and tau.
    With Sb None, c and rho are None.
    """
    SA = np.asarray(SA, dtype=np.float64)
    d, n = SA.shape
    M = SA.copy() if Sb is None else np.column_stack([SA, np.asarray(Sb, dtype=np.float64)])
    V = np.zeros((d, n))
    tau = np.zeros(n)
    for k in range(min(n, d)):
        x = M[k:, k].copy()
        alpha = x[0]
        nu = np.sqrt(np.sum(x * x))
        if nu == 0.0:
            V[k, k] = 1.0
            continue
        beta = -nu if alpha >= 0.0 else nu
        t = (beta - alpha) / beta
        v = x / (alpha - beta)
        v[0] = 1.0
        # apply H = I - t v v^T to the trailing columns k..end
        w = v @ M[k:, k:]
        M[k:, k:] -= t * np.outer(v, w)
        M[k, k] = beta
        M[k + 1:, k] = 0.0
        V[k:, k] = v
        tau[k] = t
    R = np.triu(M[:n, :n])
    if Sb is None:
        return R, None, None, V, tau
    c = M[:n, n].copy()
    rho = float(np.sqrt(np.sum(M[n:, n] ** 2)))
    return R, c, rho, V, tau


def apply_qt(V: np.ndarray, tau: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Q^T y from the Householder vectors (H_{n-1} ... H_0 y)."""
    y = np.array(y, dtype=np.float64)
    for k in range(V.shape[1]):
        v = V[k:, k]
        y[k:] -= tau[k] * v * (v @ y[k:])
    return y


def back_substitution(R: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Solve R x = c for upper-triangular R, last unknown first."""
    n = R.shape[0]
    x = np.zeros(n)
    for j in range(n - 1, -1, -1):
        x[j] = (c[j] - R[j, j + 1:] @ x[j + 1:]) / R[j, j]
    return x


def forward_substitution_transposed(R: np.ndarray, z: np.ndarray) -> np.ndarray:
    """Solve R^T y = z for upper-triangular R, first unknown first."""
    n = R.shape[0]
    y = np.zeros(n)
    for j in range(n):
        y[j] = (z[j] - R[:j, j] @ y[:j]) / R[j, j]
    return y


def rank_deficient(R: np.ndarray, n_factor: float = 10.0) -> bool:
    """|R_jj| <= 10 n u64 max|R_ii| for some j: SA is numerically rank deficient."""
    dg = np.abs(np.diag(R))
    if dg.size == 0:
        return True
    return bool(np.any(dg <= n_factor * R.shape[0] * np.finfo(np.float64).eps / 2 * dg.max()))
