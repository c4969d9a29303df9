"""Sketch-and-solve and sketch-and-precondition least squares, float64.

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this module.

* sketch_and_solve: the three steps of Sec. 1.2 for the problem of Sec. 1.3:
  draw S, form SA and Sb, and solve min ||SA x - Sb|| by Householder QR of
  [SA | Sb] and back substitution.  This is the plain (SAS) answer x_0.
* sap_sas: the sketch-and-precondition solver named in Sec. 2.1 (SAP-SAS):
  start from the sketch-and-solve x_0, then run LSQR on A R^{-1} (applied as
  v -> A (R^{-1} v) and u -> R^{-T} (A^T u), never formed) against the
  residual r_0 = b - A x_0, and return x = x_0 + R^{-1} dy.
* saa_sas: the sketch-and-apply solver named beside it (SAA-SAS): the same
  start, but the preconditioned matrix Y = A R^{-1} is formed explicitly
  (column by column from Y R = A) and LSQR runs on Y itself.  In exact
  arithmetic its iterates are those of SAP-SAS.  `y_dtype` rounds Y to a
  storage precision before the iterations (float32 for float32 inputs).

Stop rule (reading C-8): with sigma_hat = 1 - sqrt(n / d), the lower edge of
the Marchenko-Pastur law for the singular values of the preconditioned
operator, stop when ||Abar^T r_k|| / ||r_k|| <= rtol * sigma_hat; this bounds
the residual error ||A (x_k - x*)|| / ||b - A x*|| by about rtol.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .lsqr import lsqr
from .qr import (back_substitution, forward_substitution_transposed,
                 householder_qr_augmented, rank_deficient)
from .sketch import countsketch_apply, gaussian_apply, hadamard_apply, sparse_sign_apply


@dataclass
class SolveResult:
    x: np.ndarray
    x0: np.ndarray
    R: np.ndarray
    c: np.ndarray
    rho: float
    iters: int
    rank_deficient: bool
    rnorm: float = float("nan")
    arnorm: float = float("nan")


def sketch(A, b, kind: str, seed: int, d: int, zeta: int = 1):
    if kind == "count":
        return countsketch_apply(A, b, seed, d)
    if kind == "sparse":
        return sparse_sign_apply(A, b, seed, d, zeta)
    if kind == "hadamard":
        return hadamard_apply(A, b, seed, d)
    if kind == "gaussian":
        return gaussian_apply(A, b, seed, d)
    raise ValueError(kind)


def _matvec(A, x):
    return np.asarray(A @ x, dtype=np.float64).ravel()


def _rmatvec(A, u):
    if sp.issparse(A):
        return np.asarray(A.T @ u, dtype=np.float64).ravel()
    return np.asarray(A, dtype=np.float64).T @ u


def sigma_hat(n: int, d: int) -> float:
    return 1.0 - math.sqrt(n / d)


def sketch_and_solve(A, b, kind: str, seed: int, d: int, SA=None, Sb=None,
                     zeta: int = 1) -> SolveResult:
    if SA is None:
        SA, Sb = sketch(A, b, kind, seed, d, zeta)
    R, c, rho, _, _ = householder_qr_augmented(SA, Sb)
    rd = rank_deficient(R)
    x0 = back_substitution(R, c)
    return SolveResult(x0, x0, R, c, rho, 0, rd)


def sap_sas(A, b, kind: str, seed: int, d: int, max_iters: int, rtol: float = 0.0,
            SA=None, Sb=None, zeta: int = 1) -> SolveResult:
    """SAP-SAS; rtol = 0 runs exactly max_iters LSQR iterations."""
    base = sketch_and_solve(A, b, kind, seed, d, SA, Sb, zeta)
    R = base.R
    n = R.shape[0]
    if sp.issparse(A):
        Af = A.astype(np.float64)
    else:
        Af = np.asarray(A, dtype=np.float64)
    bf = np.asarray(b, dtype=np.float64)
    r0 = bf - _matvec(Af, base.x0)
    res = lsqr(lambda v: _matvec(Af, back_substitution(R, v)),
               lambda u: forward_substitution_transposed(R, _rmatvec(Af, u)),
               r0, n, max_iters, stop_ratio=rtol * sigma_hat(n, d))
    x = base.x0 + back_substitution(R, res.x)
    return SolveResult(x, base.x0, R, base.c, base.rho, res.iters, base.rank_deficient,
                       res.rnorm, res.arnorm)


def form_y(A, R: np.ndarray) -> np.ndarray:
    """Y = A R^{-1} for upper-triangular R, one column at a time from Y R = A:
    Y[:, j] = (A[:, j] - Y[:, :j] R[:j, j]) / R[j, j]."""
    Af = A.toarray() if sp.issparse(A) else np.asarray(A)
    Af = Af.astype(np.float64)
    m, n = Af.shape
    Y = np.empty((m, n))
    for j in range(n):
        Y[:, j] = (Af[:, j] - Y[:, :j] @ R[:j, j]) / R[j, j]
    return Y


def saa_sas(A, b, kind: str, seed: int, d: int, max_iters: int, rtol: float = 0.0,
            SA=None, Sb=None, y_dtype=None, zeta: int = 1) -> SolveResult:
    """SAA-SAS; rtol = 0 runs exactly max_iters LSQR iterations."""
    base = sketch_and_solve(A, b, kind, seed, d, SA, Sb, zeta)
    R = base.R
    n = R.shape[0]
    Y = form_y(A, R)
    if y_dtype is not None:
        Y = Y.astype(y_dtype).astype(np.float64)
    Af = A.astype(np.float64) if sp.issparse(A) else np.asarray(A, dtype=np.float64)
    bf = np.asarray(b, dtype=np.float64)
    r0 = bf - _matvec(Af, base.x0)
    res = lsqr(lambda v: Y @ v, lambda u: Y.T @ u, r0, n, max_iters,
               stop_ratio=rtol * sigma_hat(n, d))
    x = base.x0 + back_substitution(R, res.x)
    return SolveResult(x, base.x0, R, base.c, base.rho, res.iters, base.rank_deficient,
                       res.rnorm, res.arnorm)
