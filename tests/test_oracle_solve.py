"""Pins of the oracle's QR, triangular solves, LSQR, SAS/SAP-SAS and metrics.

QR: R equals LAPACK's (numpy.linalg.qr, same Householder sign convention)
entry for entry, Q rebuilt from the Householder vectors is orthogonal with
QR = SA, x_0 equals numpy.linalg.lstsq on the sketched problem and satisfies
the normal equations, rho is the sketched residual norm, and b = A x_true is
recovered exactly.  Triangular solves equal scipy.linalg.solve_triangular.
LSQR: iterates equal scipy.sparse.linalg.lsqr's for the same iteration count
and its residual-norm estimates equal the true norms.  SAS: the closed form
E||b - A x_0||^2 = ||r*||^2 (1 + n / (d - n - 1)) for a Gaussian sketch.
SAP-SAS: the preconditioned spectrum lies near the Marchenko-Pastur edges and
the stop rule delivers RE <= 1e-6.  SAA-SAS: the explicit Y = A R^{-1}
equals scipy's triangular solve and satisfies Y R = A; its iterates agree
with SAP-SAS (the same method in exact arithmetic) and it reaches the same
target, also with Y stored in float32.  The paper's benchmark generator
(Sec. 3.1) has the requested singular values and optimal residual norm beta.
Metrics: (1 + SUB)^2 = 1 + RE^2.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
from scipy.sparse.linalg import LinearOperator, lsqr as scipy_lsqr

from oracle import lsqr as L
from oracle import metrics as MT
from oracle import qr as Q
from oracle import sketch as S
from oracle import solve as SV
from workloads import dense_gaussian, dense_ill_conditioned, dense_scaled_columns, paper_benchmark


def test_qr_matches_lapack_r_exactly_in_sign():
    rng = np.random.default_rng(0)
    M = rng.standard_normal((120, 30))
    R, _, _, V, tau = Q.householder_qr_augmented(M)
    Rn = np.linalg.qr(M, mode="r")
    np.testing.assert_allclose(R, Rn, rtol=1e-12, atol=1e-12)
    # rebuild Q from the reflectors
    Qm = np.eye(120)
    for k in range(29, -1, -1):
        v = V[k:, k]
        Qm[k:, :] -= tau[k] * np.outer(v, v @ Qm[k:, :])
    np.testing.assert_allclose(Qm.T @ Qm, np.eye(120), atol=1e-13)
    np.testing.assert_allclose(Qm[:, :30] @ R, M, atol=1e-12)


def test_qr_augmented_solution_and_residual():
    rng = np.random.default_rng(1)
    SA, Sb = rng.standard_normal((80, 12)), rng.standard_normal(80)
    R, c, rho, V, tau = Q.householder_qr_augmented(SA, Sb)
    x = Q.back_substitution(R, c)
    xl = np.linalg.lstsq(SA, Sb, rcond=None)[0]
    np.testing.assert_allclose(x, xl, rtol=1e-12)
    np.testing.assert_allclose(SA.T @ SA @ x, SA.T @ Sb, rtol=1e-10, atol=1e-10)
    assert abs(rho - np.linalg.norm(SA @ x - Sb)) < 1e-12
    np.testing.assert_allclose(Q.apply_qt(V, tau, Sb)[:12], c, atol=1e-13)


def test_qr_zero_column_and_rank_deficiency():
    rng = np.random.default_rng(2)
    SA = rng.standard_normal((40, 6))
    SA[:, 2] = 0.0
    R, *_ = Q.householder_qr_augmented(SA)
    assert R[2, 2] == 0.0 and Q.rank_deficient(R)
    SA = rng.standard_normal((40, 6))
    SA[:, 4] = SA[:, 1]
    R, *_ = Q.householder_qr_augmented(SA)
    assert Q.rank_deficient(R)
    R, *_ = Q.householder_qr_augmented(rng.standard_normal((40, 6)))
    assert not Q.rank_deficient(R)


def test_triangular_solves_match_scipy():
    rng = np.random.default_rng(3)
    R = np.triu(rng.standard_normal((25, 25))) + 5 * np.eye(25)
    c = rng.standard_normal(25)
    np.testing.assert_allclose(Q.back_substitution(R, c), sla.solve_triangular(R, c), rtol=1e-13)
    np.testing.assert_allclose(Q.forward_substitution_transposed(R, c),
                               sla.solve_triangular(R, c, trans="T"), rtol=1e-13)


def test_exact_recovery_when_b_in_range():
    p = dense_gaussian(3000, 20, seed=4)
    b = p.A @ p.x_true
    r = SV.sketch_and_solve(p.A, b, "count", 42, 80)
    np.testing.assert_allclose(r.x, p.x_true, rtol=0, atol=1e-12 * np.linalg.norm(p.x_true))
    rg = SV.sketch_and_solve(p.A, b, "gaussian", 42, 80)
    # the Gaussian sketch sees bf16(A): recovery only up to the bf16 rounding of A
    A16 = S.bf16_round(p.A)
    xg = np.linalg.lstsq(A16, S.bf16_round(b), rcond=None)[0]
    assert np.linalg.norm(rg.x - p.x_true) < 0.05 * np.linalg.norm(p.x_true)
    assert np.isfinite(xg).all()


def test_lsqr_matches_scipy_iterates():
    rng = np.random.default_rng(5)
    # a well-conditioned operator, like the preconditioned A R^{-1} LSQR sees;
    # on ill-conditioned ones the two codes' rounding differences grow with k
    A = rng.standard_normal((200, 15)) @ np.diag(np.logspace(0, -0.5, 15))
    b = rng.standard_normal(200)
    for k in (1, 2, 5, 9, 14):
        mine = L.lsqr(lambda v: A @ v, lambda u: A.T @ u, b, 15, k)
        ref = scipy_lsqr(A, b, atol=0, btol=0, conlim=0, iter_lim=k)[0]
        np.testing.assert_allclose(mine.x, ref, rtol=1e-10, atol=1e-12)
        assert mine.iters == k
        r = b - A @ mine.x
        assert abs(mine.rnorm - np.linalg.norm(r)) < 1e-9 * np.linalg.norm(b)
        assert abs(mine.arnorm - np.linalg.norm(A.T @ r)) < 1e-8 * np.linalg.norm(A.T @ b)


def test_lsqr_converges_to_lstsq():
    rng = np.random.default_rng(6)
    A = rng.standard_normal((300, 10))
    b = rng.standard_normal(300)
    res = L.lsqr(lambda v: A @ v, lambda u: A.T @ u, b, 10, 200, stop_ratio=1e-13)
    np.testing.assert_allclose(res.x, np.linalg.lstsq(A, b, rcond=None)[0], rtol=1e-10)
    assert res.iters < 200


def test_metrics_pythagoras_identity():
    p = dense_gaussian(2000, 10, seed=7)
    xs = MT.lstsq_exact(p.A, p.b)
    x = xs + 0.01 * np.random.default_rng(0).standard_normal(10)
    m = MT.metrics(p.A, p.b, x, xs)
    assert abs((1 + m["SUB"]) ** 2 - (1 + m["RE"] ** 2)) < 1e-10
    m0 = MT.metrics(p.A, p.b, xs, xs)
    assert m0["FE"] == 0.0 and m0["RE"] == 0.0 and m0["eta"] < 1e-12


def test_metrics_closed_form_on_embedded_identity():
    # A = [I_n; 0], b = [c; r]: then x* = c, A^T (b - A x) = c - x,
    # ||A||_F = sqrt(n) and ||b - A x||^2 = ||c - x||^2 + ||r||^2, so every
    # metric has a closed form at any x.
    rng = np.random.default_rng(31)
    m, n = 40, 6
    A = np.zeros((m, n))
    A[:n, :n] = np.eye(n)
    c = rng.standard_normal(n)
    r = rng.standard_normal(m - n)
    b = np.concatenate([c, r])
    x = c + 0.3 * rng.standard_normal(n)
    xs = MT.lstsq_exact(A, b)
    np.testing.assert_allclose(xs, c, rtol=0, atol=1e-14)
    met = MT.metrics(A, b, x, c)
    e, nr = np.linalg.norm(c - x), np.linalg.norm(r)
    res = math.sqrt(e * e + nr * nr)
    assert abs(met["FE"] - e / np.linalg.norm(c)) < 1e-14
    assert abs(met["RE"] - e / nr) < 1e-14
    assert abs(met["SUB"] - (res / nr - 1.0)) < 1e-14
    assert abs(met["eta"] - e / (math.sqrt(n) * res)) < 1e-14
    # the same through a sparse A
    mets = MT.metrics(sp.csr_matrix(A), b, x, c)
    for k in met:
        assert abs(mets[k] - met[k]) < 1e-14


def test_gaussian_sas_closed_form_suboptimality():
    # data exactly representable in bf16 so the sketch sees the problem itself
    m, n, d = 1500, 8, 40
    rng = np.random.default_rng(8)
    A = S.bf16_round(rng.standard_normal((m, n)))
    b = S.bf16_round(A @ rng.standard_normal(n) + rng.standard_normal(m))
    xs = MT.lstsq_exact(A, b)
    rs2 = float(np.sum((b - A @ xs) ** 2))
    vals = []
    for seed in range(300):
        x0 = SV.sketch_and_solve(A, b, "gaussian", seed, d).x
        vals.append(float(np.sum((b - A @ x0) ** 2)) / rs2)
    vals = np.array(vals)
    expect = 1.0 + n / (d - n - 1)
    assert abs(vals.mean() - expect) < 4 * vals.std() / math.sqrt(len(vals)) + 0.01


def test_preconditioned_spectrum_marchenko_pastur():
    p = dense_gaussian(20000, 32, seed=9)
    for kind in ("gaussian", "count"):
        r = SV.sketch_and_solve(p.A, p.b, kind, 42, 128)
        sv = np.linalg.svd(p.A @ np.linalg.inv(r.R), compute_uv=False)
        kappa_mp = (1 + math.sqrt(32 / 128)) / (1 - math.sqrt(32 / 128))
        assert sv.max() / sv.min() < 1.5 * kappa_mp


@pytest.mark.parametrize("kind,gen", [("count", "illcond"), ("gaussian", "scaled"), ("count", "scaled")])
def test_sap_sas_stop_rule_reaches_target(kind, gen):
    if gen == "illcond":
        p = dense_ill_conditioned(60000, 48, seed=10)
    else:
        p = dense_scaled_columns(30000, 48, seed=11)
    xs = MT.lstsq_exact(p.A, p.b)
    r = SV.sap_sas(p.A, p.b, kind, 42, 192, 100, rtol=1e-6)
    m = MT.metrics(p.A, p.b, r.x, xs)
    assert m["RE"] <= 1e-6
    assert r.iters < 40


def test_sap_sas_exact_recovery_and_fixed_iterations():
    p = dense_ill_conditioned(20000, 24, seed=12, rel_noise=0.0)
    r = SV.sap_sas(p.A, p.b, "count", 42, 96, 6)
    assert r.iters == 6
    xs = MT.lstsq_exact(p.A, p.b)
    r2 = SV.sap_sas(p.A, p.b, "count", 42, 96, 60, rtol=1e-12)
    assert np.linalg.norm(p.A.astype(np.float64) @ (r2.x - xs)) <= 1e-9 * np.linalg.norm(p.b)


def test_form_y_matches_triangular_solve_and_reconstructs_a():
    p = dense_ill_conditioned(3000, 40, seed=13, cond=1e4)
    r = SV.sketch_and_solve(p.A, p.b, "count", 42, 160)
    Y = SV.form_y(p.A, r.R)
    Af = p.A.astype(np.float64)
    ref = sla.solve_triangular(r.R, Af.T, trans="T", lower=False).T
    assert np.linalg.norm(Y - ref) <= 1e-10 * np.linalg.norm(ref)
    assert np.linalg.norm(Y @ r.R - Af) <= 1e-13 * np.linalg.norm(Af)
    # the explicit preconditioned matrix is well conditioned (d = 4n)
    sv = np.linalg.svd(Y, compute_uv=False)
    assert sv.max() / sv.min() < 6.0


def test_saa_sas_iterates_equal_sap_sas():
    p = dense_scaled_columns(20000, 32, seed=14)
    a = SV.sap_sas(p.A, p.b, "count", 42, 128, 8)
    c = SV.saa_sas(p.A, p.b, "count", 42, 128, 8)
    assert a.iters == c.iters == 8
    assert np.linalg.norm(a.x - c.x) <= 1e-10 * np.linalg.norm(a.x)
    assert abs(a.rnorm - c.rnorm) <= 1e-10 * a.rnorm


@pytest.mark.parametrize("y_dtype", [None, np.float32])
def test_saa_sas_stop_rule_reaches_target(y_dtype):
    p = dense_ill_conditioned(60000, 48, seed=10)
    xs = MT.lstsq_exact(p.A, p.b)
    r = SV.saa_sas(p.A, p.b, "count", 42, 192, 100, rtol=1e-6, y_dtype=y_dtype)
    m = MT.metrics(p.A, p.b, r.x, xs)
    assert m["RE"] <= 1e-6
    assert r.iters < 40


def test_paper_benchmark_generator():
    p = paper_benchmark(3000, 60, seed=15, cond=1e10, beta=1e-10)
    sv = np.linalg.svd(p.A, compute_uv=False)
    sigma = np.logspace(0.0, -10.0, 60)
    # large singular values to relative rounding; the small ones to ||A|| u
    assert np.all(np.abs(sv - sigma) <= 1e-12 * sigma + 1e-14)
    # x is the least-squares solution and the optimal residual norm is beta
    r = p.b - p.A @ p.x_true
    assert abs(np.linalg.norm(r) - 1e-10) <= 1e-12
    assert np.linalg.norm(p.A.T @ r) <= 1e-14 * np.linalg.norm(r) * 10 + 1e-16


def test_paper_benchmark_device_generator_on_cpu():
    import torch
    from workloads import paper_benchmark_device
    A, b, x = paper_benchmark_device(4000, 80, seed=16, device="cpu")
    A, b, x = A.numpy(), b.numpy(), x.numpy()
    sv = np.linalg.svd(A, compute_uv=False)
    assert np.all(np.abs(sv - np.logspace(0.0, -10.0, 80)) <= 1e-12 * sv + 1e-14)
    r = b - A @ x
    assert abs(np.linalg.norm(r) - 1e-10) <= 1e-12
    assert np.linalg.norm(A.T @ r) <= 1e-15
    assert abs(np.linalg.norm(x) - 1.0) <= 1e-14


def test_sparse_sign_sap_sas_and_embedding_quality():
    p = dense_ill_conditioned(40000, 32, seed=17, cond=1e5)
    xs = MT.lstsq_exact(p.A, p.b)
    r = SV.sap_sas(p.A, p.b, "sparse", 42, 128, 100, rtol=1e-6, zeta=4)
    assert MT.metrics(p.A, p.b, r.x, xs)["RE"] <= 1e-6
    # at d = 2n the zeta = 8 embedding preconditions better than one nonzero per column
    q = dense_gaussian(20000, 32, seed=18)
    k1, k8 = [], []
    for seed in range(5):
        for zeta, out in ((1, k1), (8, k8)):
            R = SV.sketch_and_solve(q.A, q.b, "sparse", seed, 64, zeta=zeta).R
            sv = np.linalg.svd(q.A @ np.linalg.inv(R), compute_uv=False)
            out.append(sv.max() / sv.min())
    assert np.mean(k8) < np.mean(k1)


def test_hadamard_sketch_solves():
    p = dense_ill_conditioned(8192, 24, seed=19, cond=1e4)
    xs = MT.lstsq_exact(p.A, p.b)
    r = SV.sap_sas(p.A, p.b, "hadamard", 42, 96, 100, rtol=1e-6)
    assert MT.metrics(p.A, p.b, r.x, xs)["RE"] <= 1e-6
    # the SRHT is a subspace embedding: A R^-1 is well conditioned at d = 4n
    sv = np.linalg.svd(p.A @ np.linalg.inv(r.R), compute_uv=False)
    assert sv.max() / sv.min() < 6.0
