"""The KKT report is zero at certified optima and flags planted defects."""
import numpy as np

from oracle import kkt_report, p1_lp, qp_fista
from workloads import tiny_dense, dense_p1


def test_p1_certificate_zero_at_optimum_and_flags_defects():
    P = dense_p1(m=40, n=120, k=5, trial=3)
    A, b = P.A.astype(float), P.b[:, 0].astype(float)
    x, y = p1_lp(A, b)
    rep = kkt_report(A, b, x, y)
    assert max(rep.values()) < 1e-8
    # a feasible but non-optimal point: add a null-space direction
    d = np.linalg.svd(A)[2][-1]
    rep2 = kkt_report(A, b, x + 0.1 * d, y)
    assert rep2["primal"] < 1e-12 and rep2["gap"] > 1e-3
    # a dual point scaled out of the box
    assert kkt_report(A, b, x, 1.5 * y)["dual_inf"] > 0.4


def test_qp_certificate():
    P = tiny_dense(20, 50, key=70)
    A, b = P.A.astype(float), P.b[:, 0].astype(float)
    lam = 0.1 * np.max(np.abs(A.T @ b))
    x = qp_fista(A, b, lam, iters=50000)
    assert max(kkt_report(A, b, x, problem="qp", lam=lam).values()) < 1e-9
    assert kkt_report(A, b, 1.1 * x, problem="qp", lam=lam)["gap"] > 1e-4
