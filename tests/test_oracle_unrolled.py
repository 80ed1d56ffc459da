"""Pins for the unrolled-DALM gradient oracle: K = 1 closed form and central
finite differences of the FP64 forward map (h = 1e-3), kept only where the
clamp pattern is the same at both ends of the difference."""
import numpy as np

from oracle import unrolled_dalm, unrolled_vjp, unrolled_grad, unrolled_loss, clamp_pattern
from workloads import cab_problem


def _small(N=4, seed_cfg=110):
    P = cab_problem(m=24, classes=4, per_class=3, N=N, frac=0.3, cfg=seed_cfg)
    B = P.A.astype(float)
    b = P.b.astype(float)
    beta = np.abs(b).sum(axis=0) / b.shape[0]
    return P, B, b, beta


def test_k1_closed_form():
    P, B, b, beta = _small()
    A = np.hstack([B, np.eye(B.shape[0])])
    x, e, _ = unrolled_dalm(B, b, beta, 1)
    w1 = A.T @ np.linalg.solve(A @ A.T, b)       # minimum-norm solution, any beta
    np.testing.assert_allclose(np.vstack([x, e]), w1, atol=1e-12)
    rng = np.random.default_rng(0)
    gx = rng.normal(size=x.shape)
    ge = rng.normal(size=e.shape)
    gb, _ = unrolled_vjp(B, b, beta, 1, gx, ge)
    np.testing.assert_allclose(gb, np.linalg.solve(A @ A.T, A @ np.vstack([gx, ge])), atol=1e-12)


def _fd_check(K, n_dir=10, h=1e-3):
    P, B, b, beta = _small()
    loss, gb, gB = unrolled_grad(B, b, beta, K, P.labels, P.per_class)
    assert abs(loss - unrolled_loss(B, b, beta, K, P.labels, P.per_class)) < 1e-14
    rng = np.random.default_rng(K)
    kept = 0
    for d in range(2 * n_dir):
        on_b = d % 2 == 0
        D = rng.normal(size=b.shape if on_b else B.shape)
        D /= np.linalg.norm(D)
        if on_b:
            args_p, args_m = (B, b + h * D), (B, b - h * D)
            exact = np.sum(gb * D)
        else:
            args_p, args_m = (B + h * D, b), (B - h * D, b)
            exact = np.sum(gB * D)
        if not np.array_equal(clamp_pattern(*args_p, beta, K), clamp_pattern(*args_m, beta, K)):
            continue
        fd = (unrolled_loss(*args_p, beta, K, P.labels, P.per_class)
              - unrolled_loss(*args_m, beta, K, P.labels, P.per_class)) / (2 * h)
        assert abs(fd - exact) <= 2e-5 * max(1.0, abs(exact)), (d, fd, exact)
        kept += 1
    assert kept >= n_dir // 2
    return kept


def test_fd_few_iterations():
    _fd_check(3)


def test_fd_twenty_iterations():
    # h = 1e-3 moves some clamp argument across +-1 in most directions over
    # 20 iterations; a smaller step keeps enough kink-free samples.
    _fd_check(20, h=1e-5)
