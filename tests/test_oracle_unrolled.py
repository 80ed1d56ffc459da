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


def test_forward_is_algorithm2_iterates():
    # the unrolled forward map is exactly K iterations of Algorithm 2: the
    # independently pinned DALM oracle (Cholesky y-step, first iterate = the
    # minimum-norm solution, exact plateau) after K fixed iterations, with the
    # same per-instance beta, for K beyond the closed-form first iterate
    P = cab_problem(m=40, classes=5, per_class=4, N=3, frac=0.3, cfg=112)
    B = P.A.astype(float)
    b = P.b.astype(float)
    beta = np.abs(b).sum(axis=0) / b.shape[0] * np.array([0.6, 1.0, 1.7])
    from oracle import dalm
    for K in (2, 7, 50):
        x, e, _ = unrolled_dalm(B, b, beta, K)
        o = dalm(B, b, structure="cab", beta=beta, fixed_iters=K)
        np.testing.assert_allclose(np.vstack([x, e]), o.w, rtol=1e-9, atol=1e-11 * np.abs(o.w).max())


def test_fd_at_unrolled_workload_setting():
    # the setting of the differentiable unrolled-DALM workload: the 1200 x 700
    # face-shaped dictionary, 50 iterations, beta held constant (an input of
    # the map), central differences.  A sample is kept only when no clamp
    # argument crosses +-1 between the two ends of the difference (the map is
    # piecewise linear in the clamp pattern); kept and skipped counts are
    # printed for each step.  At h = 1e-3 over 50 iterations every direction
    # tried moves some of the 95 000 clamp arguments per instance across +-1
    # (counted, not asserted); at h = 1e-6 the pattern holds and the
    # differences must match the reverse-mode gradient.  Three unit
    # directions each for b (one instance's column) and for B, two instances.
    from oracle.unrolled import class_residual_loss
    from workloads import cab_instances, cab_dictionary
    B = cab_dictionary(1200, 100, 7, cfg=5).astype(float)
    b32, labels, _, _ = cab_instances(B.astype(np.float32), 2, 7, frac=0.3, cfg=5)
    b = b32.astype(float)
    beta = np.abs(b).sum(axis=0) / b.shape[0]
    K = 50
    loss, gb, gB = unrolled_grad(B, b, beta, K, labels, 7)

    def point(Bp, bp):
        x, e, (tape, *_r) = unrolled_dalm(Bp, bp, beta, K, keep_tape=True)
        pat = np.concatenate([np.sign(np.abs(t[2]) - 1.0).ravel() for t in tape])
        return class_residual_loss(Bp, bp, x, e, labels, 7)[0], pat

    rng = np.random.default_rng(5050)
    dirs = []
    for d in range(6):
        if d % 2 == 0:
            D = np.zeros_like(b)
            D[:, (d // 2) % 2] = rng.normal(size=b.shape[0])
        else:
            D = rng.normal(size=B.shape)
        dirs.append((d % 2 == 0, D / np.linalg.norm(D)))
    counts = {}
    for h in (1e-3, 1e-6):
        kept = skipped = 0
        for on_b, D in dirs:
            if on_b:
                (lp, pp), (lm, pm), exact = point(B, b + h * D), point(B, b - h * D), np.sum(gb * D)
            else:
                (lp, pp), (lm, pm), exact = point(B + h * D, b), point(B - h * D, b), np.sum(gB * D)
            if not np.array_equal(pp, pm):
                skipped += 1
                continue
            fd = (lp - lm) / (2 * h)
            assert abs(fd - exact) <= 1e-4 * abs(exact) + 1e-9, (h, on_b, fd, exact)
            kept += 1
        counts[h] = (kept, skipped)
    print(f"unrolled FD (K={K}): kept/skipped by step {counts}")
    assert counts[1e-6][0] >= 4, counts
