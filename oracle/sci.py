"""The recognition criterion of the face experiments (Sec. VI-B): a test
vector is assigned to the subject whose coefficients carry the largest share
of the l1 norm of the representation x, scored by the sparsity concentration
index (the quantity maximised over subjects in the criterion of Sec. VI-B).

For a dictionary whose columns are grouped by subject (subject i owns the
columns ``class_ptr[i] : class_ptr[i + 1]``), with C subjects:

    mass_i  = ||delta_i(x)||_1          (delta_i keeps subject i's entries)
    score_i = (C * mass_i / ||x||_1 - 1) / (C - 1)
    label   = argmax_i score_i          (the lowest i among equal scores)

x = 0 has no label (-1) and score 0.  TEST INFRASTRUCTURE ONLY.  Pins:
tests/test_oracle_sci.py (one-subject support -> score 1; equal masses over
all subjects -> score 0; a brute-force argmax over explicit projections)."""
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
