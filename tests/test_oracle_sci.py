"""Pins for the recognition criterion of the face experiments (Sec. VI-B)."""
import numpy as np

from oracle import sci


def test_one_subject_support_scores_one():
    ptr = np.array([0, 3, 7, 10])
    x = np.zeros(10)
    x[3:7] = [0.5, -2.0, 0.0, 1.0]
    mass, label, score = sci(x, ptr)
    assert label[0] == 1 and score[0] == 1.0
    np.testing.assert_allclose(mass[:, 0], [0.0, 3.5, 0.0])


def test_equal_masses_score_zero_and_first_label():
    ptr = np.array([0, 2, 4, 6, 8])
    x = np.array([1.0, -1.0, 0.5, 1.5, -2.0, 0.0, 0.25, 1.75])
    mass, label, score = sci(x, ptr)
    np.testing.assert_allclose(mass[:, 0], [2.0, 2.0, 2.0, 2.0])
    assert label[0] == 0 and abs(score[0]) < 1e-15


def test_zero_vector_has_no_label():
    mass, label, score = sci(np.zeros((6, 2)), np.array([0, 3, 6]))
    assert list(label) == [-1, -1] and list(score) == [0.0, 0.0]


def test_matches_explicit_projections():
    # the criterion written with the projection delta_i as a masking matrix
    rng = np.random.default_rng(5)
    ptr = np.array([0, 4, 5, 11, 16])
    C, n = 4, 16
    X = rng.standard_normal((n, 7))
    mass, label, score = sci(X, ptr)
    for j in range(7):
        crit = []
        for i in range(C):
            D = np.zeros((n, n))
            D[ptr[i]:ptr[i + 1], ptr[i]:ptr[i + 1]] = np.eye(ptr[i + 1] - ptr[i])
            crit.append((C * np.abs(D @ X[:, j]).sum() / np.abs(X[:, j]).sum() - 1) / (C - 1))
        assert label[j] == int(np.argmax(crit))
        np.testing.assert_allclose(score[j], max(crit), rtol=1e-13)


# ---- per-subject residuals (the residual rule of the classifier the paper builds on)

from oracle import class_residuals  # noqa: E402


def test_residuals_worked_example():
    # A = [[1, 0], [0, 1], [1, 1]], one column per subject, x = (1, 2), b = (1, 2, 3):
    # subject 0 leaves b - 1*(1, 0, 1) = (0, 2, 2), subject 1 leaves b - 2*(0, 1, 1) = (1, 0, 1)
    A = np.array([[1.0, 0.0], [0.0, 1.0], [1.0, 1.0]])
    res, label = class_residuals(A, np.array([1.0, 2.0]), np.array([1.0, 2.0, 3.0]), [0, 1, 2])
    np.testing.assert_allclose(res[:, 0], [np.sqrt(8.0), np.sqrt(2.0)], rtol=1e-15)
    assert label[0] == 1
    # with an error block e = (1, 0, 0) the target is (0, 2, 3): subject 0 leaves
    # (-1, 2, 2), subject 1 leaves (0, 0, 1): residuals (3, 1)
    res, label = class_residuals(A, np.array([1.0, 2.0]), np.array([1.0, 2.0, 3.0]), [0, 1, 2],
                                 e=np.array([1.0, 0.0, 0.0]))
    np.testing.assert_allclose(res[:, 0], [3.0, 1.0], rtol=1e-15)
    assert label[0] == 1


def test_residuals_one_subject_support():
    rng = np.random.default_rng(31)
    ptr = np.array([0, 3, 7, 7, 12])                  # subject 2 owns no column
    A = rng.standard_normal((20, 12))
    x = np.zeros(12)
    x[3:7] = rng.standard_normal(4)
    e = np.zeros(20)
    e[[2, 9]] = [4.0, -1.5]
    b = A @ x + e
    res, label = class_residuals(A, x, b, ptr, e=e)
    assert res[1, 0] < 1e-12 and label[0] == 1
    for i in (0, 2, 3):                               # nothing of b - e is explained
        np.testing.assert_allclose(res[i, 0], np.linalg.norm(A @ x), rtol=1e-13)


def test_residuals_match_explicit_projections():
    # the rule written with delta_i as a masking matrix, several columns at once
    rng = np.random.default_rng(32)
    ptr = np.array([0, 4, 5, 11, 16])
    A = rng.standard_normal((9, 16))
    X = rng.standard_normal((16, 5))
    B = rng.standard_normal((9, 5))
    E = rng.standard_normal((9, 5))
    res, label = class_residuals(A, X, B, ptr, e=E)
    for j in range(5):
        r = []
        for i in range(4):
            D = np.zeros((16, 16))
            D[ptr[i]:ptr[i + 1], ptr[i]:ptr[i + 1]] = np.eye(ptr[i + 1] - ptr[i])
            r.append(np.sqrt(np.sum((B[:, j] - E[:, j] - A @ (D @ X[:, j])) ** 2)))
        np.testing.assert_allclose(res[:, j], r, rtol=1e-13)
        assert label[j] == int(np.argmin(r))
