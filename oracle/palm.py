"""Primal augmented Lagrangian method (PALM), FP64, one instance at a time.

Sec. V-A: the method of multipliers on the augmented Lagrangian
``L_xi(x, theta) = ||x||_1 + xi/2 ||b - A x||^2 + theta^T (b - A x)``
(eq. (alm)), with the x-subproblem solved by FISTA (Sec. IV-A).  For the
cross-and-bouquet problem the e-subproblem has a closed form and x and e are
updated separately (eq. (alm-CAB), Algorithm 1):

    e_{k+1} = shrink(b - A x_k + theta_k/xi, 1/xi)
    FISTA from z_1 = w_1 = x_k, t_1 = 1:
        w_{l+1} = shrink(z_l + (1/L) A^T (b - A z_l - e_{k+1} + theta_k/xi), 1/(xi L))
        t_{l+1} = (1 + sqrt(1 + 4 t_l^2)) / 2
        z_{l+1} = w_{l+1} + ((t_l - 1)/t_{l+1}) (w_{l+1} - w_l)
    x_{k+1} = last w;  theta_{k+1} = theta_k + xi (b - A x_{k+1} - e_{k+1})

with inputs x_1 = 0, e_1 = b, theta_1 = 0 and ``xi = 2m/||b||_1``.

Readings of points the paper leaves open:

* L, used but not defined in Algorithm 1, is the Lipschitz constant of the
  FISTA gradient, ``||A^T A||_2`` for the dictionary the x-block multiplies.
* "while not converged": inner -- ``||w_{l+1} - w_l|| <= tol_inner ||w_{l+1}||``
  or ``max_inner`` steps; outer -- ``||[x;e]_{k+1} - [x;e]_k|| <= tol ||[x;e]_{k+1}||``
  and the primal residual ``||b - A x - e|| <= tol ||b||``.
* ``xi`` fixed by default (the paper's face-data setting); ``xi_growth > 1``
  multiplies it after every outer step (the synthetic-data setting xi_k -> inf).
* Dense (P1): no e-block (eq. (alm) as written).  (QP_lambda) and (P_{1,2}) have
  no PALM derivation in the paper; both split ``b = A x + r`` as the
  cross-and-bouquet case does, and replace the e-step by the prox of the
  r-term: for ``||x||_1 + 1/(2 lam) ||r||^2`` it is the scaling
  ``r = (xi lam / (1 + xi lam)) v``; for the eps-ball indicator it is the
  projection of v onto the ball; v = b - A x + theta/xi in both cases.
* b = 0: xi is undefined; 1 is used, and the iterate stays at 0.

Parity pins: tests/test_oracle_palm.py (first e-step closed form, agreement
with the LP optimum / DALM / brute force, ADM = one inner step runs).
"""
from dataclasses import dataclass

import numpy as np

from .prox import soft, proj_ball

CONVERGED, MAXITER, NONFINITE = 0, 1, 2


@dataclass
class PalmResult:
    x: np.ndarray        # (n_dict, N)
    e: np.ndarray        # (m, N) error / residual block (zeros for dense P1)
    theta: np.ndarray    # (m, N) multiplier
    iters: np.ndarray    # (N,) outer iterations
    inner: np.ndarray    # (N,) total inner FISTA iterations
    status: np.ndarray
    xi: np.ndarray       # (N,) initial xi used
    L: float


def default_xi(b):
    """xi = 2 m / ||b||_1 (Sec. V-A), 1 when b = 0."""
    b = np.asarray(b, dtype=np.float64)
    s = np.abs(b).sum()
    return 2.0 * b.shape[0] / s if s > 0 else 1.0


def _e_step(v, xi, problem, has_e, lam, eps):
    if not has_e:
        return np.zeros_like(v)
    if problem == "p1":
        return soft(v, 1.0 / xi)
    if problem == "qp":
        return (xi * lam / (1.0 + xi * lam)) * v
    return proj_ball(v, eps)


def _palm_one(A, b, xi, L, problem, has_e, lam, eps, tol, tol_in, max_iter,
              max_inner, xi_growth, fixed_outer, fixed_inner):
    m, n = A.shape
    x = np.zeros(n)
    e = b.copy() if has_e else np.zeros(m)
    theta = np.zeros(m)
    status, k, inner_total = MAXITER, 0, 0
    outer_cap = fixed_outer if fixed_outer is not None else max_iter
    inner_cap = fixed_inner if fixed_inner is not None else max_inner
    while k < outer_cap:
        e_new = _e_step(b - A @ x + theta / xi, xi, problem, has_e, lam, eps)
        c = b - e_new + theta / xi
        z = x.copy()
        w = x.copy()
        t = 1.0
        for _ in range(inner_cap):
            w_new = soft(z + (A.T @ (c - A @ z)) / L, 1.0 / (xi * L))
            t_new = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * t * t))
            z = w_new + ((t - 1.0) / t_new) * (w_new - w)
            inner_total += 1
            d, nw = np.linalg.norm(w_new - w), np.linalg.norm(w_new)
            w, t = w_new, t_new
            if fixed_inner is None and d <= tol_in * nw:
                break
        x_new = w
        theta = theta + xi * (b - A @ x_new - e_new)
        k += 1
        dw = np.sqrt(np.sum((x_new - x) ** 2) + np.sum((e_new - e) ** 2))
        nw = np.sqrt(np.sum(x_new ** 2) + np.sum(e_new ** 2))
        res = np.linalg.norm(b - A @ x_new - e_new)
        x, e = x_new, e_new
        if not (np.isfinite(nw) and np.isfinite(res)):
            status = NONFINITE
            break
        if fixed_outer is None and dw <= tol * nw and res <= tol * np.linalg.norm(b):
            status = CONVERGED
            break
        xi = xi * xi_growth
    if fixed_outer is not None and status != NONFINITE:
        status = CONVERGED if k == fixed_outer else MAXITER
    return x, e, theta, k, inner_total, status


def palm(A, b, *, structure="dense", problem="p1", xi=None, L=None, lam=None, eps=None,
         tol=1e-12, tol_inner=None, max_iter=100000, max_inner=100, xi_growth=1.0,
         fixed_outer=None, fixed_inner=None) -> PalmResult:
    """Run PALM on every column of ``b``.  ``A`` is the dictionary (B for the
    cross-and-bouquet structure, where the e-block is the identity part)."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if b.ndim == 1:
        b = b[:, None]
    m, n = A.shape
    N = b.shape[1]
    if problem in ("qp", "p12") and structure == "cab":
        raise ValueError("QP_lambda / P_{1,2} are defined on a dense dictionary")
    if problem == "qp" and (lam is None or lam <= 0):
        raise ValueError("QP_lambda needs lam > 0")
    if problem == "p12" and eps is None:
        raise ValueError("P_{1,2} needs eps")
    has_e = structure == "cab" or problem in ("qp", "p12")
    Lc = float(np.linalg.norm(A, 2) ** 2) if L is None else float(L)
    tol_in = tol if tol_inner is None else tol_inner
    eps_arr = None if eps is None else np.broadcast_to(np.asarray(eps, np.float64), (N,))
    X = np.zeros((n, N)); E = np.zeros((m, N)); T = np.zeros((m, N))
    its = np.zeros(N, np.int64); inn = np.zeros(N, np.int64); st = np.zeros(N, np.int64)
    xis = np.empty(N)
    for j in range(N):
        xij = default_xi(b[:, j]) if xi is None else float(
            np.broadcast_to(np.asarray(xi, np.float64), (N,))[j])
        xis[j] = xij
        x, e, th, k, ni, s = _palm_one(
            A, b[:, j], xij, Lc, problem, has_e, lam,
            None if eps_arr is None else eps_arr[j], tol, tol_in, max_iter,
            max_inner, xi_growth, fixed_outer, fixed_inner)
        X[:, j], E[:, j], T[:, j], its[j], inn[j], st[j] = x, e, th, k, ni, s
    return PalmResult(X, E, T, its, inn, st, xis, Lc)
