"""LSQR (Paige and Saunders, ACM TOMS 8(1), 1982, Sec. 4) in float64.

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this module.

The sketch-and-precondition solver the paper offers (Sec. 2.1, SAP-SAS after
Meier, Nakatsukasa, Townsend and Webb) runs LSQR on the right-preconditioned
operator A R^{-1}, where R comes from the QR of the sketch SA, starting from
the sketch-and-solve answer.  This module is the plain LSQR iteration in the
1982 paper's notation: Golub-Kahan bidiagonalisation

    beta_1 u_1 = b,           alpha_1 v_1 = A^T u_1,
    beta_{i+1} u_{i+1} = A v_i - alpha_i u_i,
    alpha_{i+1} v_{i+1} = A^T u_{i+1} - beta_{i+1} v_i,

followed by the plane rotations that update the QR of the lower bidiagonal
matrix and the solution:

    rho_i = (rhobar_i^2 + beta_{i+1}^2)^{1/2},  c_i = rhobar_i / rho_i,
    s_i = beta_{i+1} / rho_i,  theta_{i+1} = s_i alpha_{i+1},
    rhobar_{i+1} = -c_i alpha_{i+1},  phi_i = c_i phibar_i,
    phibar_{i+1} = s_i phibar_i,
    x_i = x_{i-1} + (phi_i / rho_i) w_i,
    w_{i+1} = v_{i+1} - (theta_{i+1} / rho_i) w_i.

||r_i|| is estimated by phibar_{i+1} and ||A^T r_i|| by
phibar_{i+1} alpha_{i+1} |c_i| (1982 paper, Sec. 5.1).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class LsqrResult:
    x: np.ndarray
    iters: int
    rnorm: float            # phibar_{k+1}
    arnorm: float           # phibar_{k+1} alpha_{k+1} |c_k|
    history: list = field(default_factory=list)  # (rnorm, arnorm) per iteration


def lsqr(apply_A, apply_At, b: np.ndarray, n: int, max_iters: int,
         stop_ratio: float = 0.0) -> LsqrResult:
    """Run LSQR from x_0 = 0 for at most max_iters iterations.

    Stops early when ||A^T r_k|| / ||r_k|| (= alpha_{k+1} |c_k|) falls to
    stop_ratio or below; stop_ratio = 0 runs exactly max_iters iterations
    (unless the bidiagonalisation terminates with beta or alpha = 0).
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros(n)
    beta = float(np.linalg.norm(b))
    if beta == 0.0:
        return LsqrResult(x, 0, 0.0, 0.0)
    u = b / beta
    v = apply_At(u)
    alpha = float(np.linalg.norm(v))
    if alpha == 0.0:
        return LsqrResult(x, 0, beta, 0.0)
    v = v / alpha
    w = v.copy()
    phibar = beta
    rhobar = alpha
    hist = []
    rnorm, arnorm = beta, beta * alpha
    k = 0
    for k in range(1, max_iters + 1):
        # bidiagonalisation step
        u = apply_A(v) - alpha * u
        beta = float(np.linalg.norm(u))
        if beta > 0.0:
            u = u / beta
            v = apply_At(u) - beta * v
            alpha = float(np.linalg.norm(v))
            if alpha > 0.0:
                v = v / alpha
        else:
            alpha = 0.0
        # plane rotation eliminating beta_{k+1}
        rho = float(np.hypot(rhobar, beta))
        c = rhobar / rho
        s = beta / rho
        theta = s * alpha
        rhobar = -c * alpha
        phi = c * phibar
        phibar = s * phibar
        # solution and search-direction updates
        x = x + (phi / rho) * w
        w = v - (theta / rho) * w
        rnorm = phibar
        arnorm = phibar * alpha * abs(c)
        hist.append((rnorm, arnorm))
        if beta == 0.0 or alpha == 0.0:
            break
        if stop_ratio > 0.0 and alpha * abs(c) <= stop_ratio:
            break
    return LsqrResult(x, k, rnorm, arnorm, hist)
