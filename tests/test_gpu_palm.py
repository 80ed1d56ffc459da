"""GPU parity of the PALM path (Sec. V-A, Algorithm 1; C ABI via the Python
binding) against the FP64 oracle, on seeded synthetic inputs.

Iterate-level parity: with a fixed number of outer and inner steps the GPU
state equals the oracle's iterate to FP32 accuracy.  Converged parity: the
GPU result matches the LP optimum (P1), FISTA on QP_lambda, or the oracle's
converged PALM (P_{1,2}).
"""
import numpy as np
import pytest

from oracle import palm as oracle_palm, p1_lp, full_matrix, qp_fista
from workloads import tiny_dense, dense_p1, cab_problem

from _parity import assert_cols_close, assert_all_close, rel_err_cols, assert_solution_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _plan(A, **kw):
    from paper_1007_3753_amd import Plan
    return Plan(torch.as_tensor(A, device="cuda"), method="palm", **kw)


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("outer,inner", [(1, 1), (1, 7), (3, 10), (6, 25)])
def test_dense_fixed_steps_match_oracle(outer, inner):
    P = tiny_dense(20, 60, N=3, key=21)
    pl = _plan(P.A, max_batch=3, max_inner=inner)
    r = pl.solve(torch.as_tensor(P.b, device="cuda"), max_iter=-outer)
    o = oracle_palm(P.A, P.b, fixed_outer=outer, fixed_inner=inner)
    assert_cols_close(_np(r.x), o.x, 5e-5, what="_np(r.x)")
    assert np.all(_np(r.iters) == outer) and np.all(_np(r.status) == 0)


def test_dense_fixed_steps_with_growth():
    P = tiny_dense(40, 130, N=5, key=22)
    pl = _plan(P.A, max_batch=5, max_inner=12, xi_growth=1.5)
    r = pl.solve(torch.as_tensor(P.b, device="cuda"), max_iter=-5)
    o = oracle_palm(P.A, P.b, fixed_outer=5, fixed_inner=12, xi_growth=1.5)
    assert_cols_close(_np(r.x), o.x, 5e-5, what="_np(r.x)")


@pytest.mark.parametrize("precision,bound", [("fp32", 5e-5), ("bf16x3", 2e-4)])
def test_cab_fixed_steps_match_oracle(precision, bound):
    # 130 rows / 49 columns, 70 instances: ragged tiles in every dimension
    P = cab_problem(m=130, classes=7, per_class=7, N=70, cfg=211)
    pl = _plan(P.A, structure="cab", precision=precision, max_batch=70, max_inner=10)
    r = pl.solve(torch.as_tensor(P.b, device="cuda"), max_iter=-3)
    cols = [0, 1, 33, 64, 69]
    o = oracle_palm(P.A, P.b[:, cols], structure="cab", fixed_outer=3, fixed_inner=10)
    assert_cols_close(_np(r.x)[:, cols], o.x, bound, what="x")
    assert_cols_close(_np(r.e)[:, cols], o.e, bound, what="e")


def test_qp_fixed_steps_match_oracle():
    P = tiny_dense(30, 90, N=4, key=23)
    lam = 0.05
    pl = _plan(P.A, problem="qp", lam=lam, max_batch=4, max_inner=15)
    r = pl.solve(torch.as_tensor(P.b, device="cuda"), max_iter=-4)
    o = oracle_palm(P.A, P.b, problem="qp", lam=lam, fixed_outer=4, fixed_inner=15)
    assert_cols_close(_np(r.x), o.x, 5e-5, what="_np(r.x)")
    assert_cols_close(_np(r.e), o.e, 5e-5, what="_np(r.e)")


def test_p12_fixed_steps_match_oracle():
    P = tiny_dense(30, 90, N=4, key=24)
    eps = 0.3 * np.linalg.norm(P.b, axis=0)
    pl = _plan(P.A, problem="p12", max_batch=4, max_inner=15)
    r = pl.solve(torch.as_tensor(P.b, device="cuda"), max_iter=-4,
                 eps=torch.as_tensor(eps, dtype=torch.float32, device="cuda"))
    o = oracle_palm(P.A, P.b, problem="p12", eps=eps, fixed_outer=4, fixed_inner=15)
    assert_cols_close(_np(r.x), o.x, 5e-5, what="_np(r.x)")
    assert_cols_close(_np(r.e), o.e, 5e-5, what="_np(r.e)")


def test_cab_adm_fixed_steps_match_oracle():
    # ADM (one FISTA step per outer step) on a cross-and-bouquet dictionary:
    # iterate parity; on such data it converges far more slowly than PALM
    # (the oracle is still short of tol 1e-5 after 50000 outer steps here)
    P = cab_problem(m=300, classes=20, per_class=7, N=6, frac=0.3, cfg=213)
    pl = _plan(P.A, structure="cab", precision="fp32", max_batch=6, max_inner=1)
    r = pl.solve(torch.as_tensor(P.b, device="cuda"), max_iter=-50)
    o = oracle_palm(P.A, P.b, structure="cab", fixed_outer=50, fixed_inner=1)
    assert_cols_close(_np(r.x), o.x, 5e-5, what="_np(r.x)")
    assert_cols_close(_np(r.e), o.e, 5e-5, what="_np(r.e)")


def test_dense_p1_converged_matches_lp():
    P = dense_p1(trial=2, N=2)
    pl = _plan(P.A, max_batch=2, max_inner=200, xi_growth=1.2)
    r = pl.solve(torch.as_tensor(P.b, device="cuda"), tol=1e-5, max_iter=3000)
    assert np.all(_np(r.status) == 0)
    for j in range(2):
        x_lp, _ = p1_lp(P.A, P.b[:, j])
        assert_solution_close(_np(r.x)[:, j], x_lp, 1e-3, what=f"x of instance {j}")


@pytest.mark.parametrize("precision,tol", [("fp32", 3e-6), ("bf16x3", 1e-5)])
def test_cab_converged_matches_lp(precision, tol):
    # PALM's stopping rule (relative change and residual) leaves an error to
    # the LP optimum of the order of the oracle's own at the same settings
    P = cab_problem(m=300, classes=20, per_class=7, N=24, frac=0.3, cfg=212)
    pl = _plan(P.A, structure="cab", precision=precision, max_batch=24, max_inner=300,
               xi_growth=1.1)
    r = pl.solve(torch.as_tensor(P.b, device="cuda"), tol=tol, max_iter=20000)
    assert np.all(_np(r.status) == 0)
    Afull = full_matrix(P.A, "cab")
    w = np.vstack([_np(r.x), _np(r.e)])
    cols = [0, 11, 23]
    o = oracle_palm(P.A, P.b[:, cols], structure="cab", tol=tol, max_iter=20000, max_inner=300,
                    xi_growth=1.1)
    for k, j in enumerate(cols):
        w_lp, _ = p1_lp(Afull, P.b[:, j])
        err_o = _rel(np.concatenate([o.x[:, k], o.e[:, k]]), w_lp)
        assert_solution_close(w[:, j], w_lp, 1.5 * err_o + 2e-4, what=f"w of instance {j}")


def test_qp_converged_matches_fista():
    # fixed xi = 50: with the default xi the QP splitting converges too slowly
    # for a test (the oracle needs thousands of outer steps as well)
    P = tiny_dense(60, 200, N=3, key=25)
    lam = 0.02
    pl = _plan(P.A, problem="qp", lam=lam, xi=50.0, max_batch=3, max_inner=500)
    r = pl.solve(torch.as_tensor(P.b, device="cuda"), tol=2e-6, max_iter=3000)
    assert np.all(_np(r.status) == 0)
    o = oracle_palm(P.A, P.b, problem="qp", lam=lam, xi=50.0, tol=2e-6, max_iter=3000,
                    max_inner=500)
    for j in range(3):
        x_ref = qp_fista(P.A, P.b[:, j], lam, iters=30000)
        err_o = _rel(o.x[:, j], x_ref)
        assert_solution_close(_np(r.x)[:, j], x_ref, 1.5 * err_o + 2e-4, what=f"x of instance {j}")


def test_p12_converged_matches_oracle():
    P = tiny_dense(40, 120, N=2, key=26)
    eps = 0.2 * np.linalg.norm(P.b, axis=0)
    pl = _plan(P.A, problem="p12", max_batch=2, max_inner=500)
    r = pl.solve(torch.as_tensor(P.b, device="cuda"), tol=2e-6, max_iter=5000,
                 eps=torch.as_tensor(eps, dtype=torch.float32, device="cuda"))
    assert np.all(_np(r.status) == 0)
    o = oracle_palm(P.A, P.b, problem="p12", eps=eps, tol=1e-10, max_iter=20000, max_inner=2000)
    assert_cols_close(_np(r.x), o.x, 1e-3, what="_np(r.x)")
    assert np.all(np.linalg.norm(_np(r.e), axis=0) <= eps * (1 + 1e-5))


def test_batched_equals_single():
    P = cab_problem(m=130, classes=7, per_class=7, N=9, cfg=213)
    pl = _plan(P.A, structure="cab", max_batch=9, max_inner=40)
    b = torch.as_tensor(P.b, device="cuda")
    rb = pl.solve(b, tol=1e-4, max_iter=300)
    r1 = pl.solve(b[:, 4:5].contiguous(), tol=1e-4, max_iter=300)
    assert np.array_equal(_np(rb.x)[:, 4], _np(r1.x)[:, 0])
    assert np.array_equal(_np(rb.e)[:, 4], _np(r1.e)[:, 0])
    assert int(rb.iters[4]) == int(r1.iters[0])


def test_zero_rhs_and_nonfinite():
    P = cab_problem(m=130, classes=7, per_class=7, N=3, cfg=214)
    b = P.b.copy()
    b[:, 0] = 0.0
    b[5, 2] = np.nan
    pl = _plan(P.A, structure="cab", max_batch=3, max_inner=50)
    r = pl.solve(torch.as_tensor(b, device="cuda"), tol=1e-4, max_iter=200)
    st = _np(r.status)
    assert st[0] == 0 and np.all(_np(r.x)[:, 0] == 0) and np.all(_np(r.e)[:, 0] == 0)
    assert st[2] == 2
    assert st[1] in (0, 1)


def test_maxiter_status():
    P = tiny_dense(20, 60, N=2, key=27)
    pl = _plan(P.A, max_batch=2, max_inner=3)
    r = pl.solve(torch.as_tensor(P.b, device="cuda"), tol=1e-9, max_iter=2)
    assert np.all(_np(r.status) == 1) and np.all(_np(r.iters) == 2)
