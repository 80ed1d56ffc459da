"""GPU parity on the paper's noise-free synthetic benchmark (Sec. VI-A): m = 800,
Gaussian dictionary with unit columns, x0 d-sparse with U[-10, 10] entries,
b = A x0.  At these sparsity levels l1-minimisation recovers x0 exactly, so
every instance is checked against its planted x0; instance 0 is also checked
iterate by iterate against the FP64 oracle."""
import numpy as np
import pytest

from oracle import dalm as oracle_dalm, palm as oracle_palm
from workloads import dense_p1

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _plan(A, **kw):
    from paper_1007_3753_amd import Plan
    return Plan(torch.as_tensor(A, device="cuda"), **kw)


def _rel_cols(X, X0):
    return np.linalg.norm(X - X0, axis=0) / np.linalg.norm(X0, axis=0)


@pytest.mark.parametrize("n,d", [(1000, 100), (1000, 200), (2000, 100)])
def test_dalm_recovers_planted(n, d):
    P = dense_p1(m=800, n=n, k=d, N=20, cfg=5, values="uniform10")
    pl = _plan(P.A, structure="dense", method="dalm", precision="fp32", max_batch=20)
    r = pl.solve(torch.as_tensor(P.b, device="cuda"), tol=1e-6, max_iter=20000)
    assert np.all(r.status.cpu().numpy() == 0)
    err = _rel_cols(r.x.cpu().numpy().astype(np.float64), P.x0.astype(np.float64))
    assert err.max() < 1e-5


def test_palm_recovers_planted():
    P = dense_p1(m=800, n=1000, k=100, N=20, cfg=5, values="uniform10")
    pl = _plan(P.A, structure="dense", method="palm", precision="fp32", max_batch=20)
    r = pl.solve(torch.as_tensor(P.b, device="cuda"), tol=1e-6, max_iter=2000)
    assert np.all(r.status.cpu().numpy() == 0)
    err = _rel_cols(r.x.cpu().numpy().astype(np.float64), P.x0.astype(np.float64))
    assert err.max() < 1e-5


def test_dalm_iterates_match_oracle():
    # 40 iterations of Algorithm 2 on instance 0 of the batch, GPU FP32 against the FP64 oracle
    P = dense_p1(m=800, n=1000, k=100, N=20, cfg=5, values="uniform10")
    pl = _plan(P.A, structure="dense", method="dalm", precision="fp32", max_batch=20)
    r = pl.solve(torch.as_tensor(P.b, device="cuda"), max_iter=-40)
    o = oracle_dalm(P.A, P.b[:, :1], structure="dense", fixed_iters=40)
    x = r.x.cpu().numpy()[:, 0].astype(np.float64)
    assert np.linalg.norm(x - o.w[:, 0]) / np.linalg.norm(o.w[:, 0]) < 2e-5


def test_palm_iterates_match_oracle():
    # 3 outer steps of Algorithm 1 with 100 FISTA steps each, instance 0
    P = dense_p1(m=800, n=1000, k=100, N=20, cfg=5, values="uniform10")
    pl = _plan(P.A, structure="dense", method="palm", precision="fp32", max_batch=20)
    r = pl.solve(torch.as_tensor(P.b, device="cuda"), max_iter=-3)
    o = oracle_palm(P.A, P.b[:, :1], structure="dense", fixed_outer=3, fixed_inner=100)
    x = r.x.cpu().numpy()[:, 0].astype(np.float64)
    # FP32 over 300 FISTA steps
    assert np.linalg.norm(x - o.x[:, 0]) / np.linalg.norm(o.x[:, 0]) < 1e-4


def test_adm_recovers_planted():
    # ADM: PALM with one FISTA step per outer step (Sec. V-A); on Gaussian data
    # it converges (the oracle stops after ~180 outer steps at this tolerance)
    P = dense_p1(m=800, n=1000, k=100, N=20, cfg=5, values="uniform10")
    pl = _plan(P.A, structure="dense", method="palm", precision="fp32", max_batch=20, max_inner=1)
    r = pl.solve(torch.as_tensor(P.b, device="cuda"), tol=1e-6, max_iter=20000)
    assert np.all(r.status.cpu().numpy() == 0)
    assert r.iters.cpu().numpy().max() < 1000
    err = _rel_cols(r.x.cpu().numpy().astype(np.float64), P.x0.astype(np.float64))
    assert err.max() < 1e-5


def test_adm_iterates_match_oracle():
    # 60 outer steps of one FISTA step each, instance 0
    P = dense_p1(m=800, n=1000, k=100, N=20, cfg=5, values="uniform10")
    pl = _plan(P.A, structure="dense", method="palm", precision="fp32", max_batch=20, max_inner=1)
    r = pl.solve(torch.as_tensor(P.b, device="cuda"), max_iter=-60)
    o = oracle_palm(P.A, P.b[:, :1], structure="dense", fixed_outer=60, fixed_inner=1)
    x = r.x.cpu().numpy()[:, 0].astype(np.float64)
    assert np.linalg.norm(x - o.x[:, 0]) / np.linalg.norm(o.x[:, 0]) < 2e-5
