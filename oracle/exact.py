"""Plain definitions of the optima, computed without any ALM arithmetic.

* ``p1_lp``          -- (P1) ``min ||x||_1 s.t. Ax = b`` as the linear program
  of Sec. III-A: split ``x = x+ - x-`` with ``x+-, >= 0`` and solve
  ``min 1^T(x+ + x-)  s.t. [A, -A][x+; x-] = b`` with HiGHS (a library LP
  solver used as one step).  Also returns the LP dual (the ``y`` of the dual
  problem in Sec. V-B) from HiGHS's equality marginals.
* ``brute_force_p1`` -- for tiny A: the LP optimum is attained at a basic
  feasible solution, i.e. ``x_S = A_S^{-1} b`` for some m-column basis S;
  enumerate them all and keep the smallest l1 norm.
* ``brute_force_qp`` -- for tiny A: enumerate supports and sign patterns of
  the (QP_lambda) optimality condition (Sec. III-B): on the support
  ``A_S^T(b - A x) = lambda*s``, off it ``|A_i^T(b - A x)| <= lambda``.
* ``qp_fista``       -- FISTA (Sec. IV-A, eq. (fista_iteration)) for
  (QP_lambda), an iteration independent of the ALM methods.
"""
import itertools

import numpy as np
import scipy.optimize as so

from .prox import soft


def p1_lp(A, b):
    """Exact (P1) optimum of ``min ||x||_1 s.t. A x = b`` via the split LP.

    Returns ``(x, y)`` with y the dual solution (``max b^T y`` subject to
    ``||A^T y||_inf <= 1``).  Raises if HiGHS does not report optimality."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    m, n = A.shape
    res = so.linprog(np.ones(2 * n), A_eq=np.hstack([A, -A]), b_eq=b,
                     bounds=(0, None), method="highs",
                     options={"primal_feasibility_tolerance": 1e-10,
                              "dual_feasibility_tolerance": 1e-10})
    if res.status != 0:
        raise RuntimeError(f"HiGHS failed: {res.message}")
    x = res.x[:n] - res.x[n:]
    y = np.asarray(res.eqlin.marginals, dtype=np.float64)
    return x, y


def brute_force_p1(A, b, rcond=1e-10):
    """Enumerate all m-column bases of A (tiny problems only: the count is
    C(n, m)); return the basic solution of least l1 norm."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    m, n = A.shape
    best, best_val = None, np.inf
    for S in itertools.combinations(range(n), m):
        AS = A[:, S]
        s = np.linalg.svd(AS, compute_uv=False)
        if s[-1] <= rcond * s[0]:
            continue
        xS = np.linalg.solve(AS, b)
        val = np.abs(xS).sum()
        if val < best_val - 1e-12:
            best_val = val
            best = np.zeros(n)
            best[list(S)] = xS
    return best


def brute_force_qp(A, b, lam):
    """Enumerate supports S and signs s of (QP_lambda); return the unique
    candidate satisfying the optimality condition (n <= ~10 only)."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    m, n = A.shape
    best, best_val = np.zeros(n), 0.5 * b @ b
    if np.max(np.abs(A.T @ b)) <= lam:
        return best
    for k in range(1, n + 1):
        for S in itertools.combinations(range(n), k):
            AS = A[:, S]
            Gs = AS.T @ AS
            if np.linalg.matrix_rank(Gs) < k:
                continue
            for signs in itertools.product((-1.0, 1.0), repeat=k):
                s = np.array(signs)
                xS = np.linalg.solve(Gs, AS.T @ b - lam * s)
                if np.any(np.sign(xS) != s):
                    continue
                x = np.zeros(n)
                x[list(S)] = xS
                corr = A.T @ (b - A @ x)
                if np.max(np.abs(corr)) > lam * (1 + 1e-9):
                    continue
                val = 0.5 * np.sum((b - A @ x) ** 2) + lam * np.abs(x).sum()
                if val < best_val:
                    best, best_val = x, val
    return best


def qp_fista(A, b, lam, iters=20000, x0=None):
    """FISTA for ``min 1/2 ||b - A x||^2 + lam ||x||_1`` with the constant
    step 1/L_f, ``L_f = ||A^T A||_2`` (Sec. IV-A)."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    Lf = np.linalg.norm(A, 2) ** 2
    x_prev = np.zeros(A.shape[1]) if x0 is None else np.asarray(x0, np.float64)
    yk = x_prev.copy()
    t = 1.0
    for _ in range(iters):
        grad = A.T @ (A @ yk - b)
        x = soft(yk - grad / Lf, lam / Lf)
        t_next = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * t * t))
        yk = x + ((t - 1.0) / t_next) * (x - x_prev)
        x_prev, t = x, t_next
    return x_prev
