"""GPU parity for the recognition criterion of the face experiments (Sec. VI-B)
through the C ABI: subject masses, label and sparsity concentration index
against the FP64 oracle on the same FP32 representations."""
import numpy as np
import pytest

from oracle import sci
from workloads import cab_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _classify(x, ptr):
    from paper_1007_3753_amd import classify
    mass, label, score = classify(torch.as_tensor(x, device="cuda"), np.asarray(ptr))
    return mass.cpu().numpy().astype(np.float64), label.cpu().numpy(), score.cpu().numpy().astype(np.float64)


def _check(x, ptr):
    mg, lg, sg = _classify(x, ptr)
    mo, lo, so = sci(x.astype(np.float64), ptr)
    np.testing.assert_allclose(mg, mo, rtol=1e-6, atol=1e-30)
    np.testing.assert_array_equal(lg, lo)
    np.testing.assert_allclose(sg, so, rtol=1e-6, atol=1e-7)


def test_after_a_batched_solve():
    # 1200 x 700 cross-and-bouquet, 64 instances at 30 % corruption
    from paper_1007_3753_amd import Plan
    P = cab_problem(N=64)
    pl = Plan(torch.as_tensor(P.A, device="cuda"), structure="cab", precision="bf16_refine", max_batch=64)
    r = pl.solve(torch.as_tensor(P.b, device="cuda"), tol=4e-6, max_iter=40000)
    x = r.x.cpu().numpy()
    ptr = np.arange(0, P.n_dict + 1, P.per_class)
    _check(x, ptr)
    _, label, _ = _classify(x, ptr)
    # every test vector is drawn from one subject's columns
    assert np.mean(label == P.labels) >= 0.95


def test_ragged_subjects_and_edge_cases():
    rng = np.random.default_rng(11)
    ptr = np.array([0, 1, 4, 4, 9, 30, 31, 40])           # an empty subject and single columns
    X = rng.standard_normal((40, 9)).astype(np.float32)
    X[:, 0] = 0.0                                          # no label
    X[:, 1] = 0.0
    X[4:9, 1] = [1.0, -2.0, 0.5, 0.0, 3.0]                 # one subject: score 1
    X[:, 2] = 0.0
    X[0, 2], X[1, 2] = 2.0, -2.0                           # equal masses: the lower subject
    _check(X, ptr)
    mg, lg, sg = _classify(X, ptr)
    assert lg[0] == -1 and sg[0] == 0.0
    assert lg[1] == 3 and abs(sg[1] - 1.0) < 1e-7
    assert lg[2] == 0


def test_two_subjects_and_wide_batch():
    rng = np.random.default_rng(12)
    X = rng.standard_normal((500, 700)).astype(np.float32)
    _check(X, np.array([0, 250, 500]))
    ptr = np.concatenate([np.arange(0, 500, 3), [500]])    # 167 subjects, the last one short
    _check(X, ptr)


def test_bad_arguments_are_rejected():
    from paper_1007_3753_amd import classify, L1Error
    x = torch.zeros(10, 2, device="cuda")
    with pytest.raises(L1Error):
        classify(x, np.array([0, 10]))                     # C = 1


# ---- per-subject residuals (the residual rule of the classifier the paper builds on)

from oracle import class_residuals as oracle_residuals  # noqa: E402


def _residuals(A, x, b, ptr, e=None):
    from paper_1007_3753_amd import class_residuals
    dev = "cuda"
    res, label = class_residuals(torch.as_tensor(A, device=dev), torch.as_tensor(x, device=dev),
                                 torch.as_tensor(b, device=dev), np.asarray(ptr),
                                 e=None if e is None else torch.as_tensor(e, device=dev))
    return res.cpu().numpy().astype(np.float64), label.cpu().numpy()


def _check_res(A, x, b, ptr, e=None):
    rg, lg = _residuals(A, x, b, ptr, e)
    ro, lo = oracle_residuals(A.astype(np.float64), x.astype(np.float64), b.astype(np.float64), ptr,
                              e=None if e is None else e.astype(np.float64))
    # both sides sum in FP64 from the same FP32 inputs; the GPU returns FP32 residuals
    scale = np.linalg.norm(b.astype(np.float64), axis=0)
    np.testing.assert_allclose(rg, ro, rtol=1e-6, atol=0)
    assert np.all(np.abs(rg - ro) <= 1e-6 * ro + 1e-12 * scale)
    # the label is the oracle's wherever the two smallest residuals differ
    srt = np.sort(ro, axis=0)
    clear = srt[1] - srt[0] > 1e-12 * scale
    np.testing.assert_array_equal(lg[clear], lo[clear])
    # elsewhere it is a valid argmin
    for j in np.where(~clear)[0]:
        assert ro[lg[j], j] <= srt[0, j] + 1e-12 * scale[j]
    return rg, lg


def test_residuals_after_a_batched_solve():
    from paper_1007_3753_amd import Plan
    P = cab_problem(N=64)
    pl = Plan(torch.as_tensor(P.A, device="cuda"), structure="cab", precision="bf16_refine", max_batch=64)
    r = pl.solve(torch.as_tensor(P.b, device="cuda"), tol=4e-6, max_iter=40000)
    x, e = r.x.cpu().numpy(), r.e.cpu().numpy()
    ptr = np.arange(0, P.n_dict + 1, P.per_class)
    _, label = _check_res(P.A, x, P.b, ptr, e)
    assert np.mean(label == P.labels) >= 0.95


def test_residuals_ragged_subjects_and_ties():
    rng = np.random.default_rng(13)
    m, n, N = 45, 40, 9
    A = rng.standard_normal((m, n)).astype(np.float32)
    X = rng.standard_normal((n, N)).astype(np.float32)
    B = rng.standard_normal((m, N)).astype(np.float32)
    E = rng.standard_normal((m, N)).astype(np.float32)
    ptr = np.array([0, 1, 4, 4, 9, 30, 31, 40])           # an empty subject and single columns
    _check_res(A, X, B, ptr, E)
    _check_res(A, X, B, ptr)                               # e = 0
    # x = 0: every residual is ||b - e||, the first subject wins
    rg, lg = _check_res(A, np.zeros((n, N), np.float32), B, ptr, E)
    assert np.all(lg == 0)
    # subject 3 explains b - e exactly: residual 0 (to FP32 rounding of b)
    x1 = np.zeros((n, 1), np.float32)
    x1[4:9, 0] = rng.standard_normal(5)
    b1 = (A.astype(np.float64) @ x1.astype(np.float64) + E[:, :1]).astype(np.float32)
    rg, lg = _check_res(A, x1, b1, ptr, E[:, :1])
    assert lg[0] == 3


def test_residuals_wide_batch():
    rng = np.random.default_rng(14)
    m, n, N = 300, 500, 700
    A = rng.standard_normal((m, n)).astype(np.float32)
    X = (rng.standard_normal((n, N)) * (rng.random((n, N)) < 0.05)).astype(np.float32)
    B = (A.astype(np.float64) @ X + 0.1 * rng.standard_normal((m, N))).astype(np.float32)
    ptr = np.concatenate([np.arange(0, n, 7), [n]])        # 72 subjects, the last one short
    _check_res(A, X, B, ptr)


def test_residuals_bad_arguments_are_rejected():
    from paper_1007_3753_amd import class_residuals, L1Error
    from paper_1007_3753_amd import _lib
    lib = _lib.load()
    assert lib.l1_alm_class_residuals(None, 10, 4, 10, None, 4, None, 10, None, 10, 0, None, 2, None, None,
                                      None) == 0
    A = torch.zeros(10, 4, device="cuda")
    x = torch.zeros(4, 2, device="cuda")
    b = torch.zeros(10, 2, device="cuda")
    with pytest.raises(L1Error):
        class_residuals(A, x, b, np.array([0, 4]))          # C = 1
