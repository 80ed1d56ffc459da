"""GPU parity of the DALM path (C ABI via the Python binding) against the FP64
oracle, on seeded synthetic inputs.

Iterate-level parity: after exactly k iterations the GPU state equals the
oracle's Algorithm-2 iterate to FP32 accuracy.  Converged parity: the GPU
result matches the exact LP optimum (HiGHS on the split LP) to the bound the
precision mode promises (FP32 1e-4, split-BF16 1e-4, BF16 + refinement 1e-3).
"""
import numpy as np
import pytest

from oracle import dalm as oracle_dalm, p1_lp, full_matrix, kkt_report, qp_fista
from workloads import tiny_dense, dense_p1, cab_problem, dense_qp

from _parity import assert_cols_close, assert_all_close, rel_err_cols, assert_solution_close, oracle_pen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _plan(A, **kw):
    from paper_1007_3753_amd import Plan
    return Plan(torch.as_tensor(A, device="cuda"), **kw)


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def test_library_loads_on_gpu():
    import paper_1007_3753_amd as pkg
    lib = pkg.load()
    assert lib is not None and torch.cuda.is_available()


@pytest.mark.parametrize("k", [1, 3, 40])
def test_dense_fixed_iterations_match_oracle(k):
    P = tiny_dense(20, 60, N=3, key=11)
    pl = _plan(P.A, max_batch=3)
    r = pl.solve(torch.as_tensor(P.b, device="cuda"), max_iter=-k)
    o = oracle_dalm(P.A, P.b, fixed_iters=k)
    assert_cols_close(_np(r.x), o.w, 2e-5, what="_np(r.x)")
    assert_cols_close(_np(r.y), o.y, 2e-5, what="_np(r.y)")
    assert np.all(_np(r.iters) == k) and np.all(_np(r.status) == 0)


@pytest.mark.parametrize("form", ["dense", "structured"])
@pytest.mark.parametrize("k,r", [(1, 5e-5), (5, 5e-5), (60, 2e-4)])
def test_cab_fixed_iterations_match_oracle(k, r, form):
    # 130 rows / 49 columns: several tiles with ragged edges in both dimensions.
    # Per-element bound r (x column rms): FP32 products (unit 6e-8) over
    # ~200-term sums, growing with the iterations; with the oracle's
    # face-shaped penalty beta0/8 (passed to the solve) the operand before
    # the first refresh is O(||w||/beta), eight times that of beta0, whose
    # rounding the later iterations carry (2e-4 at 60 iterations).  The structured form (the x
    # rows of P u, q = u_x - (P u)_x, then u_e + B q; the x block ends inside
    # the first row tile, so that tile's e rows come from P u) runs the same
    # Algorithm 2 steps with other rounding.
    P = cab_problem(m=130, classes=7, per_class=7, N=70, cfg=201)
    pl = _plan(P.A, structure="cab", max_batch=70, iteration_form=form)
    pen = torch.as_tensor(oracle_pen(P.b), device="cuda")
    r_ = pl.solve(torch.as_tensor(P.b, device="cuda"), max_iter=-k, pen=pen)
    o = oracle_dalm(P.A, P.b[:, :6], structure="cab", fixed_iters=k)
    w = np.vstack([_np(r_.x), _np(r_.e)])[:, :6]
    assert_cols_close(w, o.w, r, what="w")
    assert_cols_close(_np(r_.y)[:, :6], o.y, r, what="y")


def test_dense_p1_converged_matches_lp_and_planted():
    P = dense_p1(trial=3)
    pl = _plan(P.A, max_batch=1)
    b = torch.as_tensor(P.b, device="cuda")
    r = pl.solve(b, tol=1e-6, max_iter=20000)
    x_lp, _ = p1_lp(P.A, P.b[:, 0])
    assert int(r.status[0]) == 0
    assert_cols_close(_np(r.x)[:, 0], x_lp, 1e-4, what="_np(r.x)[:, 0]")
    assert_cols_close(_np(r.x)[:, 0], P.x0[:, 0].astype(float), 1e-4, what="_np(r.x)[:, 0]")
    rep = pl.kkt(b, r.x, y=r.y).cpu().numpy()[0]
    ref = kkt_report(P.A, P.b[:, 0], _np(r.x)[:, 0], _np(r.y)[:, 0])
    np.testing.assert_allclose(rep, [ref["primal"], ref["dual_inf"], ref["sign"], ref["gap"]],
                               rtol=1e-6, atol=1e-12)


@pytest.mark.parametrize("precision,bound", [("fp32", 1e-4), ("bf16x3", 1e-4), ("bf16_refine", 1e-3)])
def test_cab_converged_matches_lp(precision, bound):
    P = cab_problem(m=300, classes=20, per_class=7, N=96, frac=0.3, cfg=202)
    pl = _plan(P.A, structure="cab", precision=precision, max_batch=96)
    b = torch.as_tensor(P.b, device="cuda")
    r = pl.solve(b, tol=5e-6, max_iter=30000)
    st = _np(r.status)
    assert np.all(st == 0), np.unique(st, return_counts=True)
    Af = full_matrix(P.A, "cab")
    for j in (0, 37, 95):
        w_lp, _ = p1_lp(Af, P.b[:, j])
        x = _np(r.x)[:, j]
        assert_solution_close(x, w_lp[:P.n_dict], bound, what=f"x of instance {j}")
    rep = pl.kkt(b, r.x, e=r.e, y=r.y).cpu().numpy()
    assert rep[:, 0].max() < 1e-5 and rep[:, 3].max() < 1e-4


@pytest.mark.parametrize("precision,bound", [("fp32", 1e-4), ("bf16_refine", 1e-4)])
def test_structured_form_converges_to_the_lp_optimum(precision, bound):
    # the structured iteration (forced on a batch the automatic rule would
    # run densely): converged, within the bound of the exact LP optimum, and
    # the solve reports its instance-iterations as structured, but for the
    # last few instances' iterations, which the tail kernel runs densely, and
    # the split-BF16 phase of BF16 + refinement, which stays dense
    P = cab_problem(m=300, classes=20, per_class=7, N=96, frac=0.3, cfg=202)
    pl = _plan(P.A, structure="cab", precision=precision, max_batch=96, iteration_form="structured")
    b = torch.as_tensor(P.b, device="cuda")
    r = pl.solve(b, tol=4e-6, max_iter=30000)
    st = pl.last_stats()
    assert np.all(_np(r.status) == 0), np.unique(_np(r.status), return_counts=True)
    assert 0.9 * (st["cols_fp32"] + st["cols_bf16"]) < st["cols_structured"] <= st["cols_fp32"] + st["cols_bf16"]
    Af = full_matrix(P.A, "cab")
    for j in (0, 37, 95):
        w_lp, _ = p1_lp(Af, P.b[:, j])
        assert_solution_close(_np(r.x)[:, j], w_lp[:P.n_dict], bound, what=f"x of instance {j}")
        assert_solution_close(np.concatenate([_np(r.x)[:, j], _np(r.e)[:, j]]), w_lp, bound,
                              what=f"w of instance {j}")
    # the automatic rule keeps this batch (2 column tiles) on the dense operator
    pa = _plan(P.A, structure="cab", precision=precision, max_batch=96)
    pa.solve(b, tol=4e-6, max_iter=30000)
    assert pa.last_stats()["cols_structured"] == 0


@pytest.mark.parametrize("problem", ["p1", "qp"])
@pytest.mark.parametrize("k,r", [(1, 5e-5), (5, 5e-5), (40, 2e-4)])
def test_dense_structured_form_matches_oracle(problem, k, r):
    # Gaussian 100 x 400 (m < n_dict, so t = (A A^T + shift I)^{-1} A u then
    # v = A^T t + c): Algorithm 2's iterates, element by element, forced
    # structured and in the automatic mode (dense for a batch of one tile)
    rng = np.random.default_rng(31)
    A = rng.standard_normal((100, 400))
    A = (A / np.linalg.norm(A, axis=0)).astype(np.float32).astype(np.float64)
    x0 = np.zeros((400, 5))
    for j in range(5):
        x0[rng.choice(400, 15, replace=False), j] = rng.uniform(-1, 1, 15)
    b = (A @ x0).astype(np.float32).astype(np.float64)
    kw = dict(problem="qp", lam=1e-2, beta=0.5) if problem == "qp" else {}
    o = oracle_dalm(A, b, fixed_iters=k, **({"problem": "qp", "lam": 1e-2, "beta": 0.5} if problem == "qp" else {}))
    for form in ("structured", "auto"):
        pl = _plan(A.astype(np.float32), max_batch=5, iteration_form=form, **kw)
        res = pl.solve(torch.as_tensor(b.astype(np.float32), device="cuda"), max_iter=-k)
        assert (pl.last_stats()["cols_structured"] > 0) == (form == "structured")
        assert_cols_close(_np(res.x), o.w, r, what=f"x ({form})")


def test_structured_and_dense_forms_agree():
    # FP32, 150 fixed iterations on 70 instances at penalty beta0/8: the two
    # forms differ only in rounding (per-element bound 2e-4 of the column
    # rms, as for the oracle comparison at 60 iterations)
    P = cab_problem(m=130, classes=7, per_class=7, N=70, cfg=201)
    b = torch.as_tensor(P.b, device="cuda")
    pen = torch.as_tensor(oracle_pen(P.b), device="cuda")
    out = {}
    for form in ("dense", "structured"):
        pl = _plan(P.A, structure="cab", max_batch=70, iteration_form=form)
        r = pl.solve(b, max_iter=-150, pen=pen)
        out[form] = np.vstack([_np(r.x), _np(r.e)])
        assert (pl.last_stats()["cols_structured"] > 0) == (form == "structured")
    assert_cols_close(out["structured"], out["dense"], 2e-4, what="w")


def test_batched_equals_single_instance():
    P = cab_problem(m=130, classes=7, per_class=7, N=20, cfg=203)
    pl = _plan(P.A, structure="cab", max_batch=20)
    b = torch.as_tensor(P.b, device="cuda")
    rb = pl.solve(b, tol=1e-6, max_iter=20000)
    for j in (0, 7, 19):
        r1 = pl.solve(b[:, j:j + 1], tol=1e-6, max_iter=20000)
        # same per-column arithmetic in the same order: bitwise equal
        assert torch.equal(r1.x[:, 0], rb.x[:, j])
        assert int(r1.iters[0]) == int(rb.iters[j])


def test_zero_rhs_and_mixed_batch():
    P = cab_problem(m=130, classes=7, per_class=7, N=5, cfg=204)
    b = P.b.copy()
    b[:, 2] = 0.0
    pl = _plan(P.A, structure="cab", max_batch=8)
    r = pl.solve(torch.as_tensor(b, device="cuda"), tol=1e-6, max_iter=20000)
    assert int(r.status[2]) == 0 and int(r.iters[2]) == 1
    assert float(r.x[:, 2].abs().max()) == 0.0 and float(r.e[:, 2].abs().max()) == 0.0
    assert np.all(_np(r.status) == 0)


def test_nonfinite_input_reported_per_instance():
    P = cab_problem(m=130, classes=7, per_class=7, N=3, cfg=205)
    b = P.b.copy()
    b[5, 1] = np.nan
    pl = _plan(P.A, structure="cab", max_batch=3)
    r = pl.solve(torch.as_tensor(b, device="cuda"), tol=1e-6, max_iter=30000)
    st = _np(r.status)
    assert st[1] == 2 and st[0] == 0 and st[2] == 0


def test_maxiter_status():
    P = cab_problem(m=130, classes=7, per_class=7, N=2, cfg=206)
    pl = _plan(P.A, structure="cab", max_batch=2)
    r = pl.solve(torch.as_tensor(P.b, device="cuda"), tol=1e-9, max_iter=3)
    assert np.all(_np(r.status) == 1) and np.all(_np(r.iters) == 3)


def test_error_paths():
    from paper_1007_3753_amd import L1Error
    P = tiny_dense(10, 30, key=12)
    pl = _plan(P.A, max_batch=2)
    with pytest.raises(L1Error) as ei:
        pl.solve(torch.zeros(10, 3, device="cuda"))
    assert ei.value.code == -1
    A = P.A.copy()
    A[3] = A[2]  # dependent rows: A A^T singular
    with pytest.raises(L1Error) as ei:
        _plan(A, max_batch=1)
    assert ei.value.code == -2
    with pytest.raises(L1Error) as ei:
        _plan(P.A, problem="qp", lam=0.1, max_batch=1)   # DALM-QP needs beta
    assert ei.value.code == -1


def test_qp_dalm_matches_fista():
    P = tiny_dense(40, 120, N=4, key=13)
    lam = 0.05
    beta = float(np.mean(np.abs(P.b).sum(axis=0) / 40))
    pl = _plan(P.A, problem="qp", lam=lam, beta=beta, max_batch=4)
    r = pl.solve(torch.as_tensor(P.b, device="cuda"), tol=1e-7, max_iter=50000)
    assert np.all(_np(r.status) == 0)
    for j in range(4):
        xf = qp_fista(P.A, P.b[:, j], lam, iters=40000)
        assert_cols_close(_np(r.x)[:, j], xf, 1e-4, what="_np(r.x)[:, j]")


def test_p12_dalm_matches_oracle():
    P = tiny_dense(40, 120, N=3, key=14)
    A, b = P.A.astype(float), P.b.astype(float)
    eps = np.array([0.3, 0.5, 0.8]) * np.linalg.norm(b, axis=0)
    o = oracle_dalm(A, b, problem="p12", eps=eps, tol=1e-10, max_iter=200000)
    pl = _plan(P.A, problem="p12", max_batch=3)
    r = pl.solve(torch.as_tensor(P.b, device="cuda"), eps=torch.as_tensor(eps, dtype=torch.float32),
                 tol=1e-6, max_iter=100000)
    assert np.all(_np(r.status) == 0)
    assert_cols_close(_np(r.x), o.w[:120], 1e-4, what="_np(r.x)")
    # fixed-iteration parity of the block prox
    r5 = pl.solve(torch.as_tensor(P.b, device="cuda"), eps=torch.as_tensor(eps, dtype=torch.float32),
                  max_iter=-7)
    o5 = oracle_dalm(A, b, problem="p12", eps=eps, fixed_iters=7)
    assert_cols_close(np.vstack([_np(r5.x), _np(r5.e)]), o5.w, 5e-5, what="np.vstack([_np(r5.x), _np(r5.e)])")


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_tail_kernel_reproduces_launch_path(precision, monkeypatch):
    # at most 6 instances: after the first block the tail kernel runs the rest
    # of the solve; with it switched off the same iterations run one launch
    # each.  Same K split and summation order: the same bits.
    P = cab_problem(m=130, classes=7, per_class=7, N=4, cfg=207)
    pl = _plan(P.A, structure="cab", precision=precision, max_batch=4)
    b = torch.as_tensor(P.b, device="cuda")
    fixed_tail = pl.solve(b, max_iter=-200)
    tol_tail = pl.solve(b, tol=5e-6, max_iter=20000)
    monkeypatch.setenv("L1ALM_TAIL", "0")
    fixed_loop = pl.solve(b, max_iter=-200)
    tol_loop = pl.solve(b, tol=5e-6, max_iter=20000)
    assert torch.equal(fixed_tail.x, fixed_loop.x) and torch.equal(fixed_tail.e, fixed_loop.e)
    assert torch.equal(tol_tail.x, tol_loop.x)
    assert torch.equal(tol_tail.iters, tol_loop.iters) and torch.equal(tol_tail.status, tol_loop.status)


@pytest.mark.parametrize("N", [12, 16])
def test_tail_kernel_at_full_operator_size(N, monkeypatch):
    # 1200 x 700 cross-and-bouquet (n_pad 1920): the instances run one launch
    # per iteration until at most 6 are left, then the tail kernel runs the
    # rest; it reproduces the launch-per-iteration path bit for bit
    P = cab_problem(m=1200, classes=100, per_class=7, N=N, frac=0.3, cfg=208)
    pl = _plan(P.A, structure="cab", precision="bf16_refine", max_batch=N)
    b = torch.as_tensor(P.b, device="cuda")
    fixed_tail = pl.solve(b, max_iter=-300)
    tol_tail = pl.solve(b, tol=4e-6, max_iter=40000)
    monkeypatch.setenv("L1ALM_TAIL", "0")
    fixed_loop = pl.solve(b, max_iter=-300)
    tol_loop = pl.solve(b, tol=4e-6, max_iter=40000)
    assert torch.equal(fixed_tail.x, fixed_loop.x) and torch.equal(fixed_tail.e, fixed_loop.e)
    assert torch.equal(tol_tail.x, tol_loop.x)
    assert torch.equal(tol_tail.iters, tol_loop.iters) and torch.equal(tol_tail.status, tol_loop.status)
    assert np.all(tol_tail.status.cpu().numpy() == 0)


@pytest.mark.parametrize("structure", ["dense", "cab"])
def test_warm_start_continues_the_iteration(structure):
    # Algorithm 2 from a given (w, y): 12 iterations from the oracle's state
    # after 8 equal 20 iterations from zero
    if structure == "dense":
        P = tiny_dense(40, 130, N=4, key=31)
    else:
        P = cab_problem(m=130, classes=7, per_class=7, N=4, cfg=209)
    pl = _plan(P.A, structure=structure, max_batch=4)
    o8 = oracle_dalm(P.A, P.b, structure=structure, fixed_iters=8)
    o20 = oracle_dalm(P.A, P.b, structure=structure, fixed_iters=20)
    dev = "cuda"
    r = pl.solve(torch.as_tensor(P.b, device=dev), max_iter=-12,
                 w0=torch.as_tensor(o8.w.astype(np.float32), device=dev),
                 y0=torch.as_tensor(o8.y.astype(np.float32), device=dev))
    nd = P.A.shape[1]
    assert_cols_close(_np(r.x), o20.w[:nd], 5e-5, what="_np(r.x)")
    if structure == "cab":
        assert_cols_close(_np(r.e), o20.w[nd:], 5e-5, what="_np(r.e)")
    assert_cols_close(_np(r.y), o20.y, 5e-5, what="_np(r.y)")


def test_empty_batch():
    P = tiny_dense(20, 50, N=1, key=32)
    pl = _plan(P.A, max_batch=4)
    r = pl.solve(torch.zeros(20, 0, device="cuda"), tol=1e-6, max_iter=100)
    assert r.x.shape == (50, 0) and r.iters.numel() == 0


def test_p12_kkt_report_matches_oracle():
    # the FP64 certificate of the (P_{1,2}) branch against the oracle's report
    P = tiny_dense(40, 120, N=3, key=15)
    eps = np.array([0.2, 0.4, 0.7]) * np.linalg.norm(P.b.astype(float), axis=0)
    pl = _plan(P.A, problem="p12", max_batch=3)
    b = torch.as_tensor(P.b, device="cuda")
    epst = torch.as_tensor(eps, dtype=torch.float32)
    r = pl.solve(b, eps=epst, tol=1e-6, max_iter=100000)
    assert np.all(_np(r.status) == 0)
    rep = pl.kkt(b, r.x, y=r.y, eps=epst).cpu().numpy()
    X, Y = _np(r.x), _np(r.y)
    for j in range(3):
        ref = kkt_report(P.A, P.b[:, j], X[:, j], Y[:, j], problem="p12",
                         eps=float(np.float32(eps[j])))
        np.testing.assert_allclose(rep[j], [ref["primal"], ref["dual_inf"], ref["sign"], ref["gap"]],
                                   rtol=1e-6, atol=1e-12)
    # a converged pair is (nearly) optimal
    assert rep[:, 0].max() < 1e-5 and rep[:, 3].max() < 1e-3


@pytest.mark.parametrize("method", ["dalm", "dalm_cg1", "palm"])
def test_diverged_status(method):
    # L1_DIVERGED fires when ||w||_2 exceeds div_factor sqrt(m) ||b||_2; a
    # tiny factor forces it from the host for every instance with b != 0,
    # while b = 0 (w stays 0) converges and fixed-count solves never test it
    P = cab_problem(m=130, classes=7, per_class=7, N=3, cfg=210)
    b = P.b.copy()
    b[:, 1] = 0.0
    kw = {} if method == "dalm_cg1" else {}
    pl = _plan(P.A, structure="cab", method=method, max_batch=3, div_factor=1e-6, **kw)
    bt = torch.as_tensor(b, device="cuda")
    r = pl.solve(bt, tol=1e-6, max_iter=2000)
    st = _np(r.status).astype(int)
    assert st[0] == 3 and st[2] == 3 and st[1] == 0, st
    rf = pl.solve(bt, max_iter=-5)
    assert np.all(_np(rf.status) == 0)
    # the default factor never fires on this (convergent) problem
    pl2 = _plan(P.A, structure="cab", method=method, max_batch=3)
    r2 = pl2.solve(bt, tol=1e-5, max_iter=20000 if method != "palm" else 3000)
    assert not np.any(_np(r2.status) == 3)
