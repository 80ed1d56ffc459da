"""Pins for the PALM oracle (Sec. V-A, eq. (alm), Algorithm 1)."""
import numpy as np

from oracle import palm, p1_lp, brute_force_qp, qp_fista, soft, full_matrix, dalm
from workloads import tiny_dense, dense_p1, cab_problem


def test_first_e_step_closed_form():
    # x_1 = 0, theta_1 = 0: e_2 = shrink(b, 1/xi) with xi = 2m/||b||_1
    P = cab_problem(m=40, classes=4, per_class=5, N=1, cfg=104)
    b = P.b[:, 0].astype(float)
    r = palm(P.A, b, structure="cab", fixed_outer=1, fixed_inner=3)
    np.testing.assert_allclose(r.e[:, 0], soft(b, np.abs(b).sum() / (2 * 40)), atol=1e-15)


def test_inner_fista_solves_the_x_subproblem():
    # One outer step with a long inner loop: x_2 = argmin ||x||_1 + xi/2 ||c - A x||^2
    # with c = b - e_2 (theta = 0), i.e. QP_lambda with lambda = 1/xi.
    P = cab_problem(m=30, classes=3, per_class=3, N=1, cfg=105)
    B, b = P.A.astype(float), P.b[:, 0].astype(float)
    xi = 2 * 30 / np.abs(b).sum()
    r = palm(B, b, structure="cab", fixed_outer=1, fixed_inner=20000)
    c = b - soft(b, 1.0 / xi)
    np.testing.assert_allclose(r.x[:, 0], brute_force_qp(B, c, 1.0 / xi), atol=1e-7)


def test_palm_dense_p1_matches_lp():
    P = dense_p1(trial=2)
    A, b = P.A.astype(float), P.b[:, 0].astype(float)
    r = palm(A, b, tol=1e-8, max_iter=2000, max_inner=200, xi_growth=1.2)
    assert r.status[0] == 0
    x_lp, _ = p1_lp(A, b)
    assert np.linalg.norm(r.x[:, 0] - x_lp) / np.linalg.norm(x_lp) < 1e-6


def test_palm_cab_matches_lp_and_dalm():
    P = cab_problem(m=60, classes=6, per_class=7, N=1, frac=0.3, cfg=103)
    b = P.b[:, 0].astype(float)
    r = palm(P.A, b, structure="cab", tol=1e-9, max_iter=20000, max_inner=300, xi_growth=1.1)
    assert r.status[0] == 0
    w = np.concatenate([r.x[:, 0], r.e[:, 0]])
    w_lp, _ = p1_lp(full_matrix(P.A, "cab"), b)
    assert np.linalg.norm(w - w_lp) / np.linalg.norm(w_lp) < 1e-5
    d = dalm(P.A, b, structure="cab", tol=1e-8, max_iter=100000)
    assert np.linalg.norm(w - d.w[:, 0]) / np.linalg.norm(w_lp) < 1e-5


def test_palm_qp_matches_bruteforce():
    P = tiny_dense(6, 8, key=60)
    A, b = P.A.astype(float), P.b[:, 0].astype(float)
    lam = 0.15 * np.max(np.abs(A.T @ b))
    r = palm(A, b, problem="qp", lam=lam, tol=1e-12, max_iter=5000, max_inner=500)
    assert r.status[0] == 0
    np.testing.assert_allclose(r.x[:, 0], brute_force_qp(A, b, lam), atol=1e-7)
    # the r-block is the residual at the optimum
    np.testing.assert_allclose(r.e[:, 0], b - A @ r.x[:, 0], atol=1e-7)


def test_palm_p12_matches_qp_at_matching_radius():
    P = tiny_dense(20, 50, key=61)
    A, b = P.A.astype(float), P.b[:, 0].astype(float)
    lam = 0.05 * np.max(np.abs(A.T @ b))
    x_lam = qp_fista(A, b, lam, iters=60000)
    eps = np.linalg.norm(b - A @ x_lam)
    r = palm(A, b, problem="p12", eps=eps, tol=1e-11, max_iter=5000, max_inner=1000)
    assert r.status[0] == 0
    np.testing.assert_allclose(r.x[:, 0], x_lam, atol=1e-6)
    assert np.linalg.norm(r.e[:, 0]) <= eps * (1 + 1e-12)


def test_adm_one_inner_step_converges():
    # ADM = PALM with a single FISTA step per outer step (Sec. V-A): slower, same optimum
    P = tiny_dense(20, 50, key=62, k=3)
    A, b = P.A.astype(float), P.b[:, 0].astype(float)
    r = palm(A, b, tol=1e-7, max_iter=100000, max_inner=1)
    x_lp, _ = p1_lp(A, b)
    assert r.status[0] == 0
    assert np.linalg.norm(r.x[:, 0] - x_lp) / np.linalg.norm(x_lp) < 1e-5
    assert np.all(r.inner == r.iters)


def test_zero_rhs():
    P = tiny_dense(6, 12, key=63)
    r = palm(P.A, np.zeros(6), structure="cab", tol=1e-6)
    assert r.status[0] == 0 and np.all(r.x == 0) and np.all(r.e == 0)
