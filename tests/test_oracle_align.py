"""Pins for the alignment l1 problem (Sec. II-B, eq. (align-simple)) and its
PALM (Sec. V-A / Algorithm 1 with the unpenalised block, as Sec. VI-C runs it)."""
import numpy as np

from oracle import align_lp, align_brute, align_palm
from workloads import align_problem


def test_lp_matches_brute_force_tiny():
    rng = np.random.default_rng(21)
    for _ in range(4):
        B = rng.standard_normal((7, 2))
        b = rng.standard_normal(7)
        w_lp, e_lp = align_lp(B, b)
        w_bf, f_bf = align_brute(B, b)
        assert abs(np.abs(e_lp).sum() - f_bf) < 1e-9
        np.testing.assert_allclose(B @ w_lp + e_lp, b, atol=1e-12)


def test_palm_reaches_the_lp_optimum_with_a_dual_certificate():
    P = align_problem(N=3, h=10, wd=8, n_img=3, cfg=61)
    r = align_palm(P.B, P.b, tol=1e-12, max_iter=20000)
    for j in range(P.N):
        B, b = P.B[j].astype(float), P.b[:, j].astype(float)
        w_lp, e_lp = align_lp(B, b)
        assert abs(np.abs(r.e[:, j]).sum() - np.abs(e_lp).sum()) < 1e-6 * np.abs(b).sum()
        assert np.linalg.norm(b - B @ r.w[:, j] - r.e[:, j]) < 1e-6 * np.linalg.norm(b)
        # optimality of min ||e||_1 s.t. b = Bw + e: a multiplier with
        # B^T theta = 0, |theta| <= 1, theta = sign(e) on the support
        th = r.theta[:, j]
        assert np.linalg.norm(B.T @ th) < 1e-6 * np.linalg.norm(th)
        assert np.max(np.abs(th)) < 1 + 1e-6
        supp = np.abs(r.e[:, j]) > 1e-6 * np.abs(r.e[:, j]).max()
        np.testing.assert_allclose(th[supp], np.sign(r.e[supp, j]), atol=1e-6)


def test_planted_block_error_is_recovered():
    # a 10 % occluding block is a sparse enough error: the optimum is the planted w0
    P = align_problem(N=2, cfg=62)
    for j in range(P.N):
        w_lp, _ = align_lp(P.B[j], P.b[:, j])
        w0 = P.w0[:, j].astype(float)
        assert np.linalg.norm(w_lp - w0) < 1e-5 * np.linalg.norm(w0)
    r = align_palm(P.B, P.b, tol=1e-9, max_iter=20000)
    assert np.all(r.status == 0)
    for j in range(P.N):
        w0 = P.w0[:, j].astype(float)
        assert np.linalg.norm(r.w[:, j] - w0) < 1e-5 * np.linalg.norm(w0)


def test_stopping_rule_is_the_relative_change_of_w():
    P = align_problem(N=1, h=10, wd=8, n_img=3, cfg=63)
    r = align_palm(P.B, P.b, tol=1e-3, max_iter=20000)
    k = int(r.iters[0])
    a = align_palm(P.B, P.b, fixed_iters=k - 1).w[:, 0]
    c = align_palm(P.B, P.b, fixed_iters=k).w[:, 0]
    assert np.linalg.norm(c - a) < 1e-3 * np.linalg.norm(a)
    if k > 2:
        z = align_palm(P.B, P.b, fixed_iters=k - 2).w[:, 0]
        assert np.linalg.norm(a - z) >= 1e-3 * np.linalg.norm(z)
