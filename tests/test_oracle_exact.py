"""Pins for the plain definitions of the optima (LP of Sec. III-A, the
(QP_lambda) optimality condition of Sec. III-B, FISTA of Sec. IV-A)."""
import numpy as np

from oracle import p1_lp, brute_force_p1, brute_force_qp, qp_fista, kkt_report
from workloads import tiny_dense, dense_p1


def test_lp_equals_bfs_enumeration_tiny():
    for key in range(4):
        P = tiny_dense(4, 9, key=key)
        x_lp, y = p1_lp(P.A, P.b[:, 0])
        x_bf = brute_force_p1(P.A, P.b[:, 0])
        np.testing.assert_allclose(x_lp, x_bf, atol=1e-8)
        # strong LP duality
        assert abs(np.abs(x_lp).sum() - P.b[:, 0].astype(float) @ y) < 1e-8
        rep = kkt_report(P.A, P.b[:, 0], x_lp, y)
        assert max(rep.values()) < 1e-7


def test_lp_recovers_planted_sparse_signal():
    # k/m = 0.1 at m/n = 0.2: inside the l1 exact-recovery region for Gaussian A
    P = dense_p1(trial=0)
    x, _ = p1_lp(P.A, P.b[:, 0])
    x0 = P.x0[:, 0].astype(float)
    assert np.linalg.norm(x - x0) / np.linalg.norm(x0) < 1e-6


def test_qp_bruteforce_vs_fista_tiny():
    for key in range(3):
        P = tiny_dense(5, 8, key=10 + key)
        A, b = P.A.astype(float), P.b[:, 0].astype(float)
        lam = 0.2 * np.max(np.abs(A.T @ b))
        xb = brute_force_qp(A, b, lam)
        xf = qp_fista(A, b, lam, iters=50000)
        np.testing.assert_allclose(xb, xf, atol=1e-8)
        assert max(kkt_report(A, b, xb, problem="qp", lam=lam).values()) < 1e-9


def test_qp_zero_solution_closed_form():
    P = tiny_dense(6, 10, key=20)
    A, b = P.A.astype(float), P.b[:, 0].astype(float)
    lam = 1.0001 * np.max(np.abs(A.T @ b))
    assert np.all(brute_force_qp(A, b, lam) == 0)
    assert np.allclose(qp_fista(A, b, lam, iters=200), 0)


def test_qp_small_lambda_reaches_p1():
    # For lambda below a problem-dependent threshold QP_lambda's solution is P1's (Sec. VI)
    P = tiny_dense(5, 9, key=30, k=2)
    A, b = P.A.astype(float), P.b[:, 0].astype(float)
    x_p1 = brute_force_p1(A, b)
    x_qp = brute_force_qp(A, b, 1e-7)
    np.testing.assert_allclose(x_qp, x_p1, atol=1e-5)
