"""Pins for the DALM oracle (Sec. V-B, Algorithm 2).

Closed forms derived from the three steps: from w = y = 0 the first iterate is
the minimum-l2-norm solution A^T (A A^T)^{-1} b for any beta, and while no
clamp is active the iterates stay on an exact plateau.  Converged results are
pinned to the LP optimum, brute force and KKT certificates."""
import numpy as np
import pytest

from oracle import dalm, p1_lp, brute_force_p1, brute_force_qp, qp_fista, kkt_report, full_matrix
from workloads import tiny_dense, dense_p1, cab_problem


def test_first_iterate_is_min_norm_solution():
    P = tiny_dense(20, 60, key=1)
    A, b = P.A.astype(float), P.b[:, 0].astype(float)
    w_mn = np.linalg.lstsq(A, b, rcond=None)[0]
    for beta in (0.05, 1.0, 30.0):
        r = dalm(A, b, beta=beta, fixed_iters=1)
        np.testing.assert_allclose(r.w[:, 0], w_mn, atol=1e-12)
        np.testing.assert_allclose(r.y[:, 0], np.linalg.solve(A @ A.T, b) / beta, atol=1e-12)


def test_first_iterate_qp_is_ridge_solution():
    P = tiny_dense(15, 40, key=2)
    A, b = P.A.astype(float), P.b[:, 0].astype(float)
    lam, beta = 0.3, 0.7
    r = dalm(A, b, problem="qp", lam=lam, beta=beta, fixed_iters=1)
    ridge = A.T @ np.linalg.solve(A @ A.T + (lam / beta) * np.eye(15), b)
    np.testing.assert_allclose(r.w[:, 0], ridge, atol=1e-12)


def test_plateau_closed_form():
    P = tiny_dense(20, 60, key=3)
    A, b = P.A.astype(float), P.b[:, 0].astype(float)
    w_mn = np.linalg.lstsq(A, b, rcond=None)[0]
    beta = 40.0 * np.max(np.abs(w_mn))
    kmax = int(np.ceil(beta / np.max(np.abs(w_mn)))) - 1   # (k+1)|A^+ b|_inf < beta
    assert kmax >= 5
    for k in (1, 2, kmax):
        r = dalm(A, b, beta=beta, fixed_iters=k)
        np.testing.assert_allclose(r.w[:, 0], w_mn, atol=1e-11)
        np.testing.assert_allclose(r.y[:, 0], k * np.linalg.solve(A @ A.T, b) / beta, rtol=1e-10)
    # and the stopping rule does not fire on it
    r = dalm(A, b, beta=beta, tol=1e-6, max_iter=kmax)
    assert r.status[0] == 1


def test_dalm_matches_bruteforce_tiny():
    for key in range(3):
        P = tiny_dense(5, 11, key=40 + key)
        A, b = P.A.astype(float), P.b[:, 0].astype(float)
        r = dalm(A, b, tol=1e-13, max_iter=200000)
        assert r.status[0] == 0
        np.testing.assert_allclose(r.w[:, 0], brute_force_p1(A, b), atol=1e-8)


def test_dalm_dense_p1_matches_lp_and_planted():
    P = dense_p1(trial=1)
    A, b = P.A.astype(float), P.b[:, 0].astype(float)
    # DALM ends on a slow final plateau (tiny off-support entries of w stay
    # put while A^T y drifts towards the box), so certify at gap 1e-7.
    r = dalm(A, b, tol=1e-7, max_iter=20000)
    assert r.status[0] == 0
    x_lp, _ = p1_lp(A, b)
    assert np.linalg.norm(r.w[:, 0] - x_lp) / np.linalg.norm(x_lp) < 1e-6
    x0 = P.x0[:, 0].astype(float)
    assert np.linalg.norm(r.w[:, 0] - x0) / np.linalg.norm(x0) < 1e-6
    rep = kkt_report(A, b, r.w[:, 0], r.y[:, 0])
    assert rep["primal"] < 1e-10 and rep["dual_inf"] < 1e-5 and rep["gap"] < 1e-6


def test_dalm_beta_independent_optimum():
    P = tiny_dense(12, 30, key=5, k=3)
    A, b = P.A.astype(float), P.b[:, 0].astype(float)
    ws = [dalm(A, b, beta=bt, tol=1e-13, max_iter=100000).w[:, 0] for bt in (0.05, 0.5, 3.0)]
    np.testing.assert_allclose(ws[0], ws[1], atol=1e-9)
    np.testing.assert_allclose(ws[0], ws[2], atol=1e-9)


def test_dalm_cab_small_matches_lp():
    P = cab_problem(m=60, classes=6, per_class=7, N=2, frac=0.3, cfg=103)
    Af = full_matrix(P.A, "cab")
    for j in range(P.N):
        b = P.b[:, j].astype(float)
        r = dalm(P.A, b, structure="cab", tol=1e-7, max_iter=200000)
        assert r.status[0] == 0
        w_lp, y_lp = p1_lp(Af, b)
        assert np.linalg.norm(r.w[:, 0] - w_lp) / np.linalg.norm(w_lp) < 1e-5
        rep = kkt_report(Af, b, r.w[:, 0], r.y[:, 0])
        assert rep["dual_inf"] < 1e-5 and rep["gap"] < 1e-6
        # the e-block of A^T y is y itself for A = [B, I]
        np.testing.assert_allclose(r.v[P.n_dict:, 0], r.y[:, 0], atol=1e-14)


def test_cab_without_dictionary_columns():
    # B with no columns: A = I, the unique optimum is e = b, and y = sign(b)
    rng = np.random.default_rng(7)
    b = rng.normal(size=8)
    r = dalm(np.zeros((8, 0)), b, structure="cab", tol=1e-13, max_iter=10000)
    np.testing.assert_allclose(r.w[:, 0], b, atol=1e-10)
    np.testing.assert_allclose(r.y[:, 0], np.sign(b), atol=1e-8)


def test_zero_rhs_converges_at_once():
    P = tiny_dense(6, 12, key=8)
    r = dalm(P.A, np.zeros(6), tol=1e-6)
    assert r.status[0] == 0 and r.iters[0] == 1 and np.all(r.w == 0)


def test_dalm_qp_matches_fista_and_bruteforce():
    P = tiny_dense(6, 8, key=50)
    A, b = P.A.astype(float), P.b[:, 0].astype(float)
    lam = 0.15 * np.max(np.abs(A.T @ b))
    r = dalm(A, b, problem="qp", lam=lam, beta=0.5, tol=1e-13, max_iter=200000)
    assert r.status[0] == 0
    np.testing.assert_allclose(r.w[:, 0], brute_force_qp(A, b, lam), atol=1e-8)
    P2 = tiny_dense(30, 80, key=51)
    A2, b2 = P2.A.astype(float), P2.b[:, 0].astype(float)
    lam2 = 0.05 * np.max(np.abs(A2.T @ b2))
    r2 = dalm(A2, b2, problem="qp", lam=lam2, beta=0.3, tol=1e-13, max_iter=200000)
    np.testing.assert_allclose(r2.w[:, 0], qp_fista(A2, b2, lam2, iters=60000), atol=1e-8)
    assert max(kkt_report(A2, b2, r2.w[:, 0], problem="qp", lam=lam2).values()) < 1e-8
    # the dual iterate is the scaled residual at the optimum: y = (b - A x)/lam
    np.testing.assert_allclose(r2.y[:, 0], (b2 - A2 @ r2.w[:, 0]) / lam2, atol=1e-7)


def test_dalm_p12_matches_qp_at_matching_radius():
    # Lagrangian equivalence: x_lam solves P12 with eps = ||b - A x_lam||
    P = tiny_dense(30, 80, key=52)
    A, b = P.A.astype(float), P.b[:, 0].astype(float)
    lam = 0.05 * np.max(np.abs(A.T @ b))
    x_lam = qp_fista(A, b, lam, iters=60000)
    eps = np.linalg.norm(b - A @ x_lam)
    r = dalm(A, b, problem="p12", eps=eps, tol=1e-13, max_iter=400000)
    assert r.status[0] == 0
    x = r.w[:80, 0]
    np.testing.assert_allclose(x, x_lam, atol=1e-7)
    rep = kkt_report(A, b, x, r.y[:, 0], problem="p12", eps=eps)
    assert max(rep.values()) < 1e-7
    # eps >= ||b|| makes x = 0 optimal
    r0 = dalm(A, b, problem="p12", eps=1.01 * np.linalg.norm(b), tol=1e-12, max_iter=100000)
    assert np.linalg.norm(r0.w[:80, 0]) < 1e-9


def test_a_planted_sign_mistake_is_caught():
    # A mistake anywhere in the y-step (here: the sign of b) breaks the
    # first-iterate pin: that pin is what guards the oracle's algebra.
    P = tiny_dense(10, 25, key=9)
    A, b = P.A.astype(float), P.b[:, 0].astype(float)
    w_mn = np.linalg.lstsq(A, b, rcond=None)[0]
    wrong = dalm(A, -b, beta=1.0, fixed_iters=1).w[:, 0]
    assert np.linalg.norm(wrong - w_mn) > 1e-3


def test_synthetic_recipe_recovers_planted():
    # the paper's noise-free recipe (Gaussian unit columns, U[-10, 10] nonzeros)
    # at a small size: the planted x0 is the l1 optimum up to the FP32 rounding
    # of b (the LP agrees), and both oracles reach the LP optimum
    from oracle import palm
    P = dense_p1(m=80, n=100, k=10, N=2, cfg=7, values="uniform10")
    A = P.A.astype(float)
    for j in range(2):
        b = P.b[:, j].astype(float)
        x0 = P.x0[:, j].astype(float)
        w_lp, _ = p1_lp(A, b)
        assert np.linalg.norm(w_lp - x0) < 1e-6 * np.linalg.norm(x0)
        rd = dalm(A, b, tol=1e-12, max_iter=20000)
        assert np.linalg.norm(rd.w[:, 0] - w_lp) < 1e-7 * np.linalg.norm(w_lp)
        rp = palm(A, b, tol=1e-10, max_iter=2000, max_inner=500)
        assert np.linalg.norm(rp.x[:, 0] - w_lp) < 1e-7 * np.linalg.norm(w_lp)


# ---- the one-CG-step y-step (the heuristic of Sec. V-B)

def test_cg1_is_exact_when_rows_are_orthogonal():
    # A A^T = c I: the y-subproblem is spherical, one steepest-descent step with
    # the exact step length solves it, so the iterates are Algorithm 2's
    rng = np.random.default_rng(41)
    Q, _ = np.linalg.qr(rng.standard_normal((90, 90)))
    A = 1.7 * Q[:30, :]
    x0 = np.zeros(90)
    x0[rng.choice(90, 5, replace=False)] = rng.standard_normal(5)
    b = A @ x0
    beta = np.abs(b).sum() / 30.0
    oc = dalm(A, b[:, None], fixed_iters=40, y_step="cg1", beta=beta)
    oe = dalm(A, b[:, None], fixed_iters=40, beta=beta)
    np.testing.assert_allclose(oc.w, oe.w, rtol=0, atol=1e-12 * np.abs(oe.w).max())
    np.testing.assert_allclose(oc.y, oe.y, rtol=0, atol=1e-12 * np.abs(oe.y).max())


def test_cg1_step_minimises_the_y_subproblem_along_the_gradient():
    # one iteration from a given (w, y): the new y is the minimiser of the
    # y-subproblem's quadratic on the line through y along its gradient
    from scipy.optimize import minimize_scalar
    rng = np.random.default_rng(42)
    A = rng.standard_normal((12, 30))
    b = rng.standard_normal(12)
    w0 = rng.standard_normal(30)
    y0 = rng.standard_normal(12)
    beta = 0.7
    o = dalm(A, b[:, None], beta=beta, fixed_iters=1, w0=w0[:, None], y0=y0[:, None], y_step="cg1")
    z = np.clip(A.T @ y0 + w0 / beta, -1.0, 1.0)
    G = A @ A.T

    def lagr(y):   # the augmented Lagrangian's y-dependent part (Sec. V-B)
        return -b @ y - w0 @ (z - A.T @ y) + 0.5 * beta * np.sum((z - A.T @ y) ** 2)

    h = 1e-6
    grad = np.array([(lagr(y0 + h * e) - lagr(y0 - h * e)) / (2 * h) for e in np.eye(12)])
    t = minimize_scalar(lambda t: lagr(y0 - t * grad), bracket=(0.0, 1e-3), tol=1e-14).x
    np.testing.assert_allclose(o.y[:, 0], y0 - t * grad, rtol=1e-6, atol=1e-9)
    del G


def test_cg1_converges_on_gaussian_data_and_not_on_face_shaped_data():
    # Sec. V-B: the heuristic works on random Gaussian dictionaries but not on
    # face dictionaries
    P = dense_p1(m=200, n=600, k=20, N=1, cfg=43)
    x_lp, _ = p1_lp(P.A, P.b[:, 0])
    o = dalm(P.A, P.b, tol=1e-6, max_iter=5000, y_step="cg1")
    assert o.status[0] == 0
    assert np.linalg.norm(o.w[:, 0] - x_lp) < 1e-5 * np.linalg.norm(x_lp)
    o = dalm(P.A, P.b, fixed_iters=2000, y_step="cg1")   # to the LP solver's own accuracy
    assert np.linalg.norm(o.w[:, 0] - x_lp) < 1e-7 * np.linalg.norm(x_lp)
    C = cab_problem(m=300, classes=20, per_class=7, N=1, frac=0.3, cfg=212)
    Af = full_matrix(C.A, "cab")
    w_lp, _ = p1_lp(Af, C.b[:, 0])
    oc = dalm(C.A, C.b, structure="cab", fixed_iters=3000, y_step="cg1")
    oe = dalm(C.A, C.b, structure="cab", fixed_iters=3000)
    err_c = np.linalg.norm(oc.w[:, 0] - w_lp) / np.linalg.norm(w_lp)
    err_e = np.linalg.norm(oe.w[:, 0] - w_lp) / np.linalg.norm(w_lp)
    assert err_e < 1e-3 and err_c > 10 * err_e
