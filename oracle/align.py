"""The l1 problem of the alignment step (Sec. II-B, eq. (align-simple)):

    min_{w, e} ||e||_1   s.t.   b = B w + e,

B m x k with k = n_i + q_i small (the subject's training images and the
Jacobian of the transformation), w not penalised.  TEST INFRASTRUCTURE ONLY.

``align_lp``: the plain definition as a linear program (w free, e = u - v,
u, v >= 0), HiGHS.  ``align_brute``: for tiny m, the optimum is attained with
at least k zero residuals (a vertex of the LP), so it is the best of the
interpolants w = B_S^{-1} b_S over the k-row subsets S.

``align_palm``: the primal ALM of Sec. V-A / Algorithm 1 for this problem, as
the alignment experiment of Sec. VI-C runs it ("the l1 norm of w is no longer
penalised"):

    e_{k+1} = shrink(b - B w_k + theta_k/xi, 1/xi)
    w_{k+1} = argmin_w ||b - B w - e_{k+1} + theta_k/xi||^2
            = (B^T B)^{-1} B^T (b - e_{k+1} + theta_k/xi)
    theta_{k+1} = theta_k + xi (b - B w_{k+1} - e_{k+1})

from w_1 = 0, e_1 = b, theta_1 = 0, xi = 2m/||b||_1 (as in Algorithm 1).
Reading: Algorithm 1's inner loop minimises the augmented Lagrangian over the
primal block; without the l1 term that minimiser is the least-squares
solution above, taken exactly.  Stopping rule of Sec. VI-C: the relative
change ||w_{k+1} - w_k|| / ||w_k|| < tol.

Pins: tests/test_oracle_align.py (LP against brute force on tiny problems, the
PALM fixed point against the LP, exact recovery of the planted w0 when the
error is a small block, the first iterate in closed form).
"""
import itertools
from dataclasses import dataclass

import numpy as np
from scipy.optimize import linprog

from .prox import soft

CONVERGED, MAXITER, NONFINITE = 0, 1, 2


def align_lp(B, b):
    """Exact optimum (w, e) of min ||e||_1 s.t. b = B w + e."""
    B = np.asarray(B, np.float64)
    b = np.asarray(b, np.float64)
    m, k = B.shape
    c = np.concatenate([np.zeros(k), np.ones(2 * m)])
    A_eq = np.hstack([B, np.eye(m), -np.eye(m)])
    bounds = [(None, None)] * k + [(0, None)] * (2 * m)
    res = linprog(c, A_eq=A_eq, b_eq=b, bounds=bounds, method="highs",
                  options={"primal_feasibility_tolerance": 1e-10, "dual_feasibility_tolerance": 1e-10})
    if res.status != 0:
        raise RuntimeError(res.message)
    w = res.x[:k]
    return w, b - B @ w


def align_brute(B, b):
    """Best interpolant over all k-row subsets (tiny m only)."""
    B = np.asarray(B, np.float64)
    b = np.asarray(b, np.float64)
    m, k = B.shape
    best, arg = np.inf, None
    for S in itertools.combinations(range(m), k):
        BS = B[list(S)]
        if abs(np.linalg.det(BS)) < 1e-12:
            continue
        w = np.linalg.solve(BS, b[list(S)])
        f = np.abs(b - B @ w).sum()
        if f < best:
            best, arg = f, w
    return arg, best


@dataclass
class AlignResult:
    w: np.ndarray        # (k, N)
    e: np.ndarray        # (m, N)
    theta: np.ndarray    # (m, N)
    iters: np.ndarray    # (N,)
    status: np.ndarray   # (N,)
    xi: np.ndarray       # (N,)


def align_palm(Bs, b, *, xi=None, tol=1e-12, max_iter=100000, fixed_iters=None) -> AlignResult:
    """PALM on every instance: ``Bs`` (N, m, k) or one (m, k) shared by all
    columns of ``b`` (m, N)."""
    b = np.asarray(b, np.float64)
    if b.ndim == 1:
        b = b[:, None]
    m, N = b.shape
    Bs = np.asarray(Bs, np.float64)
    if Bs.ndim == 2:
        Bs = np.broadcast_to(Bs, (N,) + Bs.shape)
    k = Bs.shape[2]
    W = np.zeros((k, N)); E = np.zeros((m, N)); T = np.zeros((m, N))
    its = np.zeros(N, np.int64); st = np.zeros(N, np.int64); xis = np.zeros(N)
    for j in range(N):
        B, bj = Bs[j], b[:, j]
        n1 = np.abs(bj).sum()
        xij = (2.0 * m / n1 if n1 > 0 else 1.0) if xi is None else float(xi)
        xis[j] = xij
        G = B.T @ B
        w, e, th = np.zeros(k), bj.copy(), np.zeros(m)
        cap = fixed_iters if fixed_iters is not None else max_iter
        status, it = MAXITER, 0
        for it in range(1, cap + 1):
            e = soft(bj - B @ w + th / xij, 1.0 / xij)
            w_new = np.linalg.solve(G, B.T @ (bj - e + th / xij))
            th = th + xij * (bj - B @ w_new - e)
            if not np.all(np.isfinite(w_new)):
                status = NONFINITE
                w = w_new
                break
            done = fixed_iters is None and np.linalg.norm(w_new - w) < tol * np.linalg.norm(w)
            w = w_new
            if done:
                status = CONVERGED
                break
        W[:, j], E[:, j], T[:, j], its[j], st[j] = w, e, th, it, status
    return AlignResult(W, E, T, its, st, xis)
