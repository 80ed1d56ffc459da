"""Pins for the proximal maps: each closed form against the minimisation
that defines it (Sec. IV prox definition; Sec. V-B projection)."""
import numpy as np
import scipy.optimize as so

from oracle import soft, proj_box, block_soft, proj_ball


def _prox_l1_brute(v, alpha):
    # argmin_u alpha|u| + (u - v)^2 / 2 on a fine grid, refined by bounded search
    grid = np.linspace(v - 3 * abs(alpha) - 1, v + 3 * abs(alpha) + 1, 200001)
    f = alpha * np.abs(grid) + 0.5 * (grid - v) ** 2
    u0 = grid[np.argmin(f)]
    h = grid[1] - grid[0]
    r = so.minimize_scalar(lambda u: alpha * abs(u) + 0.5 * (u - v) ** 2,
                           bounds=(u0 - 2 * h, u0 + 2 * h), method="bounded",
                           options={"xatol": 1e-13})
    return r.x


def test_soft_matches_prox_definition():
    rng = np.random.default_rng(0)
    for v, a in zip(rng.uniform(-5, 5, 40), rng.uniform(0.01, 2, 40)):
        assert abs(soft(v, a) - _prox_l1_brute(v, a)) < 1e-7


def test_soft_ties_and_sign():
    assert soft(0.7, 0.7) == 0.0 and soft(-0.7, 0.7) == 0.0
    assert soft(0.0, 0.1) == 0.0
    np.testing.assert_array_equal(soft(np.array([3.0, -3.0]), 1.0), [2.0, -2.0])


def test_moreau_identity_box():
    # v = prox_{a|.|}(v) + a * P_box(v / a): the conjugate of a|.| is the box indicator
    rng = np.random.default_rng(1)
    v = rng.normal(0, 3, 1000)
    for a in (0.1, 1.0, 2.5):
        np.testing.assert_allclose(soft(v, a) + a * proj_box(v / a), v, rtol=0, atol=1e-13)


def test_proj_box_is_projection():
    rng = np.random.default_rng(2)
    v = rng.normal(0, 2, 500)
    p = proj_box(v)
    assert np.all(np.abs(p) <= 1)
    # optimality of a projection onto a convex set: (v - p)^T (q - p) <= 0 for q in the set
    for _ in range(20):
        q = rng.uniform(-1, 1, 500)
        assert (v - p) @ (q - p) <= 1e-12
    np.testing.assert_array_equal(proj_box(np.array([1.0, -1.0, 0.3])), [1.0, -1.0, 0.3])


def test_block_soft_matches_definition_and_moreau():
    rng = np.random.default_rng(3)
    for tau in (0.1, 1.0, 5.0):
        v = rng.normal(0, 1, 6)
        r = so.minimize(lambda u: tau * np.linalg.norm(u) + 0.5 * np.sum((u - v) ** 2),
                        np.zeros(6) + 1e-3, method="Nelder-Mead",
                        options={"xatol": 1e-11, "fatol": 1e-14, "maxiter": 40000})
        np.testing.assert_allclose(block_soft(v, tau), r.x, atol=1e-5)
        # Moreau: v = prox_{tau||.||}(v) + P_{tau-ball}(v)
        np.testing.assert_allclose(block_soft(v, tau) + proj_ball(v, tau), v, atol=1e-14)
    assert np.all(block_soft(np.zeros(4), 1.0) == 0)
