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
