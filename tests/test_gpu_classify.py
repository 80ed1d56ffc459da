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
