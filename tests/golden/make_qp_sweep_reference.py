"""Writes qp_sweep_instance0.npy: the (QP_lambda) optimum of instance 0 of the
2000 x 8000 compressive-sensing sweep (lambda = 1e-3, beta = the batch mean of
||b_j||_1 / m), computed by the FP64 oracle only (dual ALM run to tol 1e-9,
then checked by the FP64 optimality report).  Run from the repository root:
python tests/golden/make_qp_sweep_reference.py"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import dalm, kkt_report  # noqa: E402
from workloads import dense_qp  # noqa: E402


def main():
    P = dense_qp(N=64)
    b = P.b.astype(np.float64)
    beta = float(np.mean(np.abs(b).sum(0) / P.m))
    r = dalm(P.A, b[:, 0], problem="qp", lam=P.lam, beta=beta, tol=1e-9, max_iter=100000)
    rep = kkt_report(P.A, b[:, 0], r.w[:, 0], problem="qp", lam=P.lam)
    assert r.status[0] == 0 and rep["dual_inf"] < 1e-7 and rep["gap"] < 1e-7, rep
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "qp_sweep_instance0.npy")
    np.save(out, r.w[:, 0])
    print(out, r.iters, rep)


if __name__ == "__main__":
    main()
