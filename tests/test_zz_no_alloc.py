"""l1_alm_kkt_noalloc (the FP64 report without a plan and without any
allocation; its scratch is a static device array) against l1_alm_kkt on the
same inputs.  The no-alloc path forms each instance's residual and A^T u in
one workgroup, l1_alm_kkt as FP64 matrix-core GEMMs over the batch: the same
FP64 products of the same FP32 inputs, added in another order.  The sums
differ by FP64 rounding, about 1e-16 sqrt(K) of the terms' scale; the
inputs here are 40- and 5-iteration iterates and random points, whose
residuals and gaps are at least 1e-4 of that scale, so the reports agree to
rtol 1e-9 (atol 1e-13 for entries that are exactly 0 on one side).  Two calls
in a row, the second with a smaller input; a batch large enough that the
scratch is used in several launches; the size limit."""
import ctypes

import numpy as np
import pytest

from workloads import cab_problem, dense_qp, tiny_dense

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _cm(a):
    """(rows, N) numpy -> column-major float32 device buffer (as a (N, rows) tensor)."""
    return torch.as_tensor(np.ascontiguousarray(np.asarray(a, np.float32).T), device="cuda")


def _noalloc(A, problem, structure, lam, b, x, e, y, eps=None):
    from paper_1007_3753_amd import _lib
    lib = _lib.load()
    m, nd = A.shape
    N = b.shape[1]
    Ac, bc, xc = _cm(A), _cm(b), _cm(x)
    ec = _cm(e) if e is not None else None
    yc = _cm(y) if y is not None else None
    epsc = None if eps is None else torch.as_tensor(np.asarray(eps, np.float32), device="cuda")
    rep = torch.full((N, 4), -1.0, dtype=torch.float64, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    _lib.check(lib.l1_alm_kkt_noalloc(_p(Ac), m, nd, m, problem, structure, ctypes.c_double(lam), _p(bc), m, N,
                                      _p(epsc), _p(xc), nd, _p(ec), m, _p(yc), m, _p(rep), s))
    torch.cuda.synchronize()
    return rep.cpu().numpy()


def _with_plan(A, b, x, e, y, **kw):
    from paper_1007_3753_amd import Plan
    with Plan(torch.as_tensor(A, device="cuda"), max_batch=b.shape[1], **kw) as pl:
        bt = torch.as_tensor(b, device="cuda")
        f = lambda a: None if a is None else torch.as_tensor(np.asarray(a, np.float32), device="cuda")
        rep = pl.kkt(bt, f(x), e=f(e), y=f(y)).cpu().numpy()
    return rep


def _cab_case(m, classes, N, cfg, iters):
    from paper_1007_3753_amd import Plan
    P = cab_problem(m=m, classes=classes, per_class=7, N=N, cfg=cfg)
    with Plan(torch.as_tensor(P.A, device="cuda"), structure="cab", max_batch=N) as pl:
        r = pl.solve(torch.as_tensor(P.b, device="cuda"), max_iter=-iters)
        return P, r.x.cpu().numpy(), r.e.cpu().numpy(), r.y.cpu().numpy()


def _same(got, ref):
    np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-13)


def test_noalloc_report_equals_plan_report_twice():
    # first call: 1200 x 700 face-shaped, 96 instances; second: 300 x 140, 9
    for (m, classes, N, cfg) in ((1200, 100, 96, 261), (300, 20, 9, 262)):
        P, x, e, y = _cab_case(m, classes, N, cfg, 40)
        ref = _with_plan(P.A, P.b, x, e, y, structure="cab")
        got = _noalloc(P.A, 0, 1, 0.0, P.b, x, e, y)
        _same(got, ref)


def test_noalloc_in_several_launches_and_qp():
    # m = 4800 rows: 218 instances per launch of the scratch, so 300
    # instances take two launches
    P, x, e, y = _cab_case(4800, 10, 300, 263, 5)
    ref = _with_plan(P.A, P.b, x, e, y, structure="cab")
    got = _noalloc(P.A, 0, 1, 0.0, P.b, x, e, y)
    _same(got, ref)
    # dense QP_lambda (no y), then a smaller dense P1 call
    Q = tiny_dense(40, 120, N=5, key=264)
    xq = np.random.default_rng(1).standard_normal((120, 5)).astype(np.float32) * 0.1
    ref = _with_plan(Q.A, Q.b, xq, None, None, problem="qp", lam=0.05, beta=0.3)
    got = _noalloc(Q.A, 2, 0, 0.05, Q.b, xq, None, None)
    _same(got, ref)
    yq = np.random.default_rng(2).standard_normal((40, 2)).astype(np.float32) * 0.1
    ref = _with_plan(Q.A, Q.b[:, :2], xq[:, :2], None, yq)
    got = _noalloc(Q.A, 0, 0, 0.0, Q.b[:, :2], xq[:, :2], None, yq)
    _same(got, ref)


def test_noalloc_rejects_sizes_beyond_the_scratch():
    from paper_1007_3753_amd import _lib
    lib = _lib.load()
    big = (1 << 20) + 1
    dummy = torch.zeros(8, device="cuda")
    rc = lib.l1_alm_kkt_noalloc(_p(dummy), big, 1, big, 0, 0, ctypes.c_double(0.0), _p(dummy), big, 1,
                                None, _p(dummy), 1, None, big, _p(dummy), big, _p(dummy), None)
    assert rc == _lib.L1_EINVAL
    assert b"scratch" in lib.l1_alm_last_error()
