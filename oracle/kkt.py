"""Optimality certificates, FP64.

(P1) ``min ||w||_1 s.t. A w = b``: LP strong duality (Sec. III-A) with the
dual ``max b^T y s.t. ||A^T y||_inf <= 1`` (Sec. V-B).  A pair (w, y) is
optimal iff it is primal feasible, dual feasible, ``A^T y = sign(w)`` on the
support of w, and the gap ``||w||_1 - b^T y`` vanishes.

(QP_lambda): the optimality condition used by Homotopy (Sec. III-B),
``A^T (b - A x) in lambda d||x||_1``; with ``u = (b - A x)/lambda`` this is
``||A^T u||_inf <= 1`` and ``A^T u = sign(x)`` on the support.  The gap is
primal minus dual objective with ``theta = b - A x`` scaled to feasibility.

(P_{1,2}): ``||b - A x|| <= eps`` and, with the dual y, ``A^T y`` a
subgradient of ``||x||_1`` and gap ``||x||_1 - (b^T y - eps ||y||)``.

All residuals are relative; a report is a dict of floats.
"""
import numpy as np


def _support_sign_err(w, g, rel=1e-6):
    aw = np.abs(w)
    if aw.max() == 0:
        return 0.0
    S = aw > rel * aw.max()
    return float(np.max(np.abs(g[S] - np.sign(w[S]))))


def kkt_report(A, b, w, y=None, problem="p1", lam=None, eps=None):
    """Certificate for one instance.  ``A`` is the full matrix the problem
    is posed on ([B, I] for the cross-and-bouquet form)."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    nb = max(np.linalg.norm(b), 1e-300)
    r = b - A @ w
    l1 = np.abs(w).sum()
    if problem == "p1":
        y = np.asarray(y, dtype=np.float64)
        g = A.T @ y
        return {
            "primal": float(np.linalg.norm(r) / nb),
            "dual_inf": float(max(np.max(np.abs(g)) - 1.0, 0.0)),
            "sign": _support_sign_err(w, g),
            "gap": float(abs(l1 - b @ y) / max(l1, 1e-300)),
        }
    if problem == "qp":
        g = A.T @ r / lam
        gmax = np.max(np.abs(g))
        theta = r / max(gmax, 1.0)
        pobj = 0.5 * r @ r + lam * l1
        dobj = b @ theta - 0.5 * theta @ theta
        return {
            "primal": 0.0,
            "dual_inf": float(max(gmax - 1.0, 0.0)),
            "sign": _support_sign_err(w, g),
            "gap": float(abs(pobj - dobj) / max(abs(pobj), 1e-300)),
        }
    if problem == "p12":
        y = np.asarray(y, dtype=np.float64)
        g = A.T @ y
        dobj = b @ y - eps * np.linalg.norm(y)
        return {
            "primal": float(max(np.linalg.norm(r) - eps, 0.0) / nb),
            "dual_inf": float(max(np.max(np.abs(g)) - 1.0, 0.0)),
            "sign": _support_sign_err(w, g),
            "gap": float(abs(l1 - dobj) / max(l1, 1e-300)),
        }
    raise ValueError(problem)
