"""Accuracy metrics of the oracle, float64.

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this module.

Sec. 3.2 compares forward error and residual error (figure captions); the
definitions below are the ones of the sketch-and-precondition literature the
benchmark set-up of Sec. 3.1 follows (reading C-8):
  FE  = ||x - x*|| / ||x*||
  RE  = ||A (x - x*)|| / ||b - A x*||            (residual error)
  SUB = ||b - A x|| / ||b - A x*|| - 1           (suboptimality)
  eta = ||A^T (b - A x)|| / (||A||_F ||b - A x||) (backward-error proxy)
x* is the float64 least-squares solution from LAPACK (numpy.linalg.lstsq).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def lstsq_exact(A, b) -> np.ndarray:
    if sp.issparse(A):
        A = A.toarray()
    return np.linalg.lstsq(np.asarray(A, dtype=np.float64), np.asarray(b, dtype=np.float64), rcond=None)[0]


def _mv(A, x):
    return np.asarray(A @ x, dtype=np.float64).ravel()


def metrics(A, b, x, xstar) -> dict:
    if sp.issparse(A):
        A = A.astype(np.float64)
        fro = float(np.sqrt(A.multiply(A).sum()))
    else:
        A = np.asarray(A, dtype=np.float64)
        fro = float(np.linalg.norm(A))
    b = np.asarray(b, dtype=np.float64)
    rstar = b - _mv(A, xstar)
    r = b - _mv(A, x)
    nr, nrs = float(np.linalg.norm(r)), float(np.linalg.norm(rstar))
    atr = np.asarray(A.T @ r, dtype=np.float64).ravel()
    return {
        "FE": float(np.linalg.norm(x - xstar) / np.linalg.norm(xstar)),
        "RE": float(np.linalg.norm(_mv(A, x - xstar)) / nrs),
        "SUB": nr / nrs - 1.0,
        "eta": float(np.linalg.norm(atr) / (fro * nr)) if nr > 0 else 0.0,
    }
