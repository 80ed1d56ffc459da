"""GPU parity for the l1 problem of the alignment step (Sec. II-B, the
linearised registration problem; the PALM of Sec. V-A as Sec. VI-C runs it)
through the C ABI, against the FP64 oracle on the same FP32 instances.

Tolerances.  The kernel runs the e- and theta-steps in FP32 and the normal
equations in FP64 from an FP32 right-hand side, so one iteration perturbs w
by about cond(B) * u32 * ||w|| (u32 = 6e-8; cond(B) of the 1200 x 11
alignment dictionaries is below 100) and e by u32 * ||b||.  Over a few tens
of iterations this stays below 1e-4 relative; a flipped shrink decision at
the threshold moves one entry of e by about one FP32 ulp of it, which the
same bound covers."""
import numpy as np
import pytest

from oracle import align_palm
from workloads import align_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

L1_CONVERGED, L1_MAXITER, L1_NONFINITE = 0, 1, 2


def _align(B, b, **kw):
    from paper_1007_3753_amd import align
    w, e, it, st = align(torch.as_tensor(B, device="cuda"), torch.as_tensor(b, device="cuda"), **kw)
    return (w.cpu().numpy().astype(np.float64), e.cpu().numpy().astype(np.float64),
            it.cpu().numpy(), st.cpu().numpy())


def _rel(a, b, axis=0):
    return np.linalg.norm(a - b, axis=axis) / np.maximum(np.linalg.norm(b, axis=axis), 1e-30)


def test_fixed_iterations_match_the_oracle():
    # the alignment shape: 40 x 30 images, 7 training images + 4 Jacobian columns
    P = align_problem(N=24, cfg=71)
    for K in (1, 3, 12):
        w, e, it, st = _align(P.B, P.b, fixed_iters=K)
        r = align_palm(P.B, P.b, fixed_iters=K)
        assert np.all(it == K) and np.all(st == L1_MAXITER)
        assert _rel(w, r.w).max() < 1e-4, K
        assert (np.linalg.norm(e - r.e, axis=0) / np.linalg.norm(P.b.astype(float), axis=0)).max() < 1e-4, K


def test_converged_solves_recover_the_planted_transform():
    P = align_problem(N=32, cfg=72)
    w, e, it, st = _align(P.B, P.b, tol=1e-5, max_iter=2000)
    r = align_palm(P.B, P.b, tol=1e-5, max_iter=2000)
    assert np.all(st == L1_CONVERGED)
    assert _rel(w, r.w).max() < 1e-4
    # the stopping rule is the oracle's.  At tol 1e-5 the FP32 rounding of
    # the iterate (about cond(B) * u32 = 2.4e-6 of ||w||) is a quarter of the
    # threshold and the change shrinks by a few per cent an iteration, so the
    # stopping iteration may move by a few
    assert np.abs(it.astype(int) - r.iters.astype(int)).max() <= 4
    assert np.mean(it == r.iters) >= 0.6
    # with a fixed xi the relative change of w can fall below tol while w is
    # still about 1e-3 from the optimum (the oracle stops there too), so the
    # planted w0 and the occluding block's difference e0 are recovered by
    # most instances, and by every instance no worse than by the oracle
    w0, e0 = P.w0.astype(np.float64), P.e0.astype(np.float64)
    assert np.median(_rel(w, w0)) < 1e-4
    assert np.all(_rel(w, w0) < _rel(r.w, w0) + 1e-4)
    assert np.median(np.linalg.norm(e - e0, axis=0) / np.linalg.norm(e0, axis=0)) < 1e-4


@pytest.mark.parametrize("tol", [1e-2, 1e-3, 1e-4])
def test_table_tolerances_stop_where_the_oracle_stops(tol):
    P = align_problem(N=40, cfg=73)
    w, e, it, st = _align(P.B, P.b, tol=tol, max_iter=1000)
    r = align_palm(P.B, P.b, tol=tol, max_iter=1000)
    assert np.all(st == L1_CONVERGED)
    assert np.mean(it == r.iters) >= 0.9
    same = it == r.iters
    assert _rel(w[:, same], r.w[:, same]).max() < 1e-4


def test_ragged_rows_and_small_dictionaries():
    # m not a multiple of the 256 threads; k = 5, 7 and 12
    for (h, wd, n_img, cfg) in [(37, 29, 3, 74), (2, 5, 1, 75), (45, 45, 8, 76)]:
        P = align_problem(N=5, h=h, wd=wd, n_img=n_img, cfg=cfg)
        w, e, it, st = _align(P.B, P.b, fixed_iters=6)
        r = align_palm(P.B, P.b, fixed_iters=6)
        assert _rel(w, r.w).max() < 1e-4, (h, wd, n_img)
        assert (np.linalg.norm(e - r.e, axis=0) / np.linalg.norm(P.b.astype(float), axis=0)).max() < 1e-4


def test_single_column_and_widest_dictionary():
    rng = np.random.default_rng(80)
    for (m, k) in [(300, 1), (64, 16)]:
        B = rng.standard_normal((4, m, k)).astype(np.float32)
        b = rng.standard_normal((m, 4)).astype(np.float32)
        w, e, it, st = _align(B, b, fixed_iters=9)
        r = align_palm(B, b, fixed_iters=9)
        assert _rel(w, r.w).max() < 1e-4, (m, k)
        assert (np.linalg.norm(e - r.e, axis=0) / np.linalg.norm(b.astype(float), axis=0)).max() < 1e-4


def test_largest_dictionary_fits():
    # the largest sizes: m = 2048 (8 rows a thread), k = 16
    rng = np.random.default_rng(77)
    N, m, k = 3, 2048, 16
    B = rng.standard_normal((N, m, k)).astype(np.float32)
    w0 = rng.standard_normal((k, N))
    b = np.einsum("jmk,kj->mj", B.astype(np.float64), w0)
    b[rng.random((m, N)) < 0.1] += 5.0
    b = b.astype(np.float32)
    w, e, it, st = _align(B, b, fixed_iters=8)
    r = align_palm(B, b, fixed_iters=8)
    assert _rel(w, r.w).max() < 1e-4
    w, e, it, st = _align(B, b, tol=1e-5, max_iter=500)
    assert np.all(st == L1_CONVERGED)
    assert _rel(w, w0).max() < 1e-4


def test_degenerate_instances():
    P = align_problem(N=4, h=20, wd=15, n_img=3, cfg=79)
    B, b = P.B.copy(), P.b.copy()
    b[:, 1] = 0.0                    # b = 0: w stays 0, the strict test never holds
    B[2, :, 1] = B[2, :, 0]          # a repeated column: B^T B is singular
    B[3, :, 4] = 0.0                 # a zero column
    w, e, it, st = _align(B, b, tol=1e-3, max_iter=7)
    assert st[1] == L1_MAXITER and it[1] == 7
    assert np.all(w[:, 1] == 0.0) and np.all(e[:, 1] == 0.0)
    for j in (2, 3):
        assert st[j] == L1_NONFINITE and it[j] == 0
        assert np.all(w[:, j] == 0.0)
        np.testing.assert_array_equal(e[:, j], b[:, j])
    r = align_palm(B[:1], b[:, :1], tol=1e-3, max_iter=7)
    assert st[0] == r.status[0] and it[0] == r.iters[0]


def test_empty_batch_and_bad_sizes():
    from paper_1007_3753_amd import _lib
    from paper_1007_3753_amd.api import align
    from paper_1007_3753_amd._lib import L1Error
    lib = _lib.load()
    assert lib.l1_alm_align(None, 100, 4, 0, None, 100, 1e-3, 10, None, None, 100, None, None, None) == 0
    dev = torch.device("cuda")
    for (m, k) in [(2049, 1), (100, 17), (100, 0)]:
        with pytest.raises(L1Error):
            align(torch.zeros(1, m, k, device=dev), torch.ones(m, 1, device=dev), max_iter=5)
    with pytest.raises(L1Error):
        align(torch.zeros(1, 10, 2, device=dev), torch.ones(10, 1, device=dev), tol=0.0)
    with pytest.raises(L1Error):
        align(torch.zeros(1, 10, 2, device=dev), torch.ones(10, 1, device=dev), max_iter=0)


def test_full_batch_sampled_against_the_oracle():
    # the bench workload (1000 instances of 1200 x 11), checked on a sample
    P = align_problem(N=1000, cfg=6)
    w, e, it, st = _align(P.B, P.b, tol=1e-3, max_iter=1000)
    assert np.all(st == L1_CONVERGED)
    idx = np.array([0, 1, 137, 500, 998, 999])
    r = align_palm(P.B[idx], P.b[:, idx], tol=1e-3, max_iter=1000)
    assert np.mean(it[idx] == r.iters) >= 0.8
    same = it[idx] == r.iters
    assert _rel(w[:, idx][:, same], r.w[:, same]).max() < 1e-4
    wf, _, _, _ = _align(P.B[idx], P.b[:, idx], fixed_iters=10)
    rf = align_palm(P.B[idx], P.b[:, idx], fixed_iters=10)
    assert _rel(wf, rf.w).max() < 1e-4
