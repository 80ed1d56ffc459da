"""The recognition criterion of the face experiments (Sec. VI-B): a test
vector is assigned to the subject whose coefficients carry the largest share
of the l1 norm of the representation x, scored by the sparsity concentration
index (the quantity maximised over subjects in the criterion of Sec. VI-B).

For a dictionary whose columns are grouped by subject (subject i owns the
columns ``class_ptr[i] : class_ptr[i + 1]``), with C subjects:

    mass_i  = ||delta_i(x)||_1          (delta_i keeps subject i's entries)
    score_i = (C * mass_i / ||x||_1 - 1) / (C - 1)
    label   = argmax_i score_i          (the lowest i among equal scores)

x = 0 has no label (-1) and score 0.

The residual rule of the sparse-representation classifier the paper builds
on (Sec. I and Fig. src; the cross-and-bouquet model b = A x + e of
Sec. II-A) assigns b to the subject whose coefficients alone explain b - e
best:

    res_i = ||b - e - A delta_i(x)||_2,   label = argmin_i res_i
    (the lowest i among equal residuals; e = 0 without an error block).

TEST INFRASTRUCTURE ONLY.  Pins: tests/test_oracle_sci.py (one-subject
support -> score 1; equal masses over all subjects -> score 0; a brute-force
argmax over explicit projections; residuals: a hand-worked example,
one-subject support -> residual 0 for it and ||b - e|| for the others, an
empty subject, explicit projection matrices)."""
import numpy as np


def sci(x, class_ptr):
    """Per column of ``x`` (n_dict, N): subject masses (C, N), label (N,)
    and the winning score (N,), in float64."""
    x = np.asarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    ptr = np.asarray(class_ptr, dtype=np.int64)
    C = len(ptr) - 1
    N = x.shape[1]
    mass = np.zeros((C, N))
    for i in range(C):
        mass[i] = np.abs(x[ptr[i]:ptr[i + 1]]).sum(axis=0)
    total = mass.sum(axis=0)
    label = np.full(N, -1, dtype=np.int64)
    score = np.zeros(N)
    for j in range(N):
        if total[j] > 0:
            label[j] = int(np.argmax(mass[:, j]))   # first maximum
            score[j] = (C * mass[label[j], j] / total[j] - 1.0) / (C - 1)
    return mass, label, score


def class_residuals(A, x, b, class_ptr, e=None):
    """Per column of ``x`` (n_dict, N) with ``b`` (m, N) and optional ``e``
    (m, N): the residual of every subject (C, N) and the label (N,), in
    float64."""
    A = np.asarray(A, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    if b.ndim == 1:
        b = b[:, None]
    target = b if e is None else b - np.asarray(e, dtype=np.float64).reshape(b.shape)
    ptr = np.asarray(class_ptr, dtype=np.int64)
    C = len(ptr) - 1
    N = x.shape[1]
    res = np.zeros((C, N))
    for i in range(C):
        cols = slice(ptr[i], ptr[i + 1])
        res[i] = np.linalg.norm(target - A[:, cols] @ x[cols], axis=0)
    label = np.argmin(res, axis=0).astype(np.int64)   # first minimum
    return res, label
