"""Dual augmented Lagrangian method (DALM), FP64, one instance at a time.

Follows Sec. V-B of the paper: the dual of (P1) is
``max b^T y  s.t.  A^T y in B_inf`` (B_inf the unit l-inf ball), and the
augmented Lagrangian in (y, z) with multiplier x is minimised alternately:

    z_{k+1} = P_Binf(A^T y_k + x_k / beta)                        (z-step)
    beta A A^T y_{k+1} = beta A z_{k+1} - (A x_k - b)              (y-step)
    x_{k+1} = x_k - beta (z_{k+1} - A^T y_{k+1})                   (x-step)

For the cross-and-bouquet problem (Algorithm 2) the same steps run with the
full matrix [B, I] and w = [x; e].  The y-step uses a Cholesky factor of the
Gram matrix (``scipy.linalg.cho_factor``/``cho_solve``); the paper applies
the inverse directly, which is the same solve.

Readings of points the paper leaves open:

* Algorithm 2 writes the face dictionary in steps 4 and 5; the dimensions only
  agree with the full matrix [B, I], which is what runs here.
* beta is not given; default per instance ``beta = beta0 / 8`` for the
  cross-and-bouquet form and ``beta = beta0`` otherwise, with
  ``beta0 = ||b||_1 / m`` (1 if b = 0), the scale of x: on face-shaped
  problems the penalty at beta0 leaves the slowest instances several times
  as many iterations to a given error as beta0 / 8 does (typical instances
  need about as many), while on Gaussian dictionaries beta0 is the faster
  one.  The one-CG-step variant keeps beta0.
* "while not converged": stop after iteration k >= 1 when both
  ``(beta0 / beta) ||w_k - w_{k-1}|| <= tol ||w_k||`` and the complementarity
  gap of the l1 block ``| ||w||_1 - w^T v | <= tol ||w||_1`` with
  ``v = A^T y``.  Since ``w_k - w_{k-1} = -beta (z_k - A^T y_k)``, the first
  test is ``beta0 ||z_k - A^T y_k|| <= tol ||w_k||``: the relative-change
  rule the paper uses in Sec. VI-C, measured at the penalty beta0 whatever
  penalty runs, so the stopping point does not move with beta.  For the
  cross-and-bouquet form the gap is measured against
  ``max(||w||_1, ||b||_1 / 4)``: every optimum has ``||w*||_1 <= ||b||_1``
  (``[0; b]`` is feasible), and the floor holds an instance with little
  corruption (small ||w||_1) to an absolute gap no smaller than the
  rounding of finite-precision iterates leaves in it: each off-support
  entry of w carries beta times the rounding of v, and with beta a fixed
  fraction of ||b||_1 / m their sum is a fixed fraction of ||b||_1.  The
  second test
  keeps the iteration from stopping on the initial plateau where no clamp is
  active: there w stays at the minimum-norm solution while y grows linearly,
  so the relative change of w is zero but the gap is ``||w||_1``.  For (P1)
  every iterate satisfies ``A w = b``, so the gap is the LP duality gap
  ``||w||_1 - b^T y``.  For (P_{1,2}) the sums run over the x-block only.
* (QP_lambda), no derivation in the paper: the dual is
  ``max b^T y - (lambda/2)||y||^2 s.t. ||A^T y||_inf <= 1``; the same three
  steps apply with the y-step matrix ``A A^T + (lambda/beta) I``.
* (P_{1,2}), no derivation in the paper: split ``b = A x + r`` with
  ``||r|| <= eps``, i.e. the matrix [A, I] with w = [x; r]; the z-step on the
  r-block is the prox of ``(eps/beta)||.||_2`` (block soft-threshold), the
  conjugate of the eps-ball indicator.

Parity pins: tests/test_oracle_dalm.py (the first iterate equals the
minimum-norm solution, the exact plateau formula, LP optimum, brute force,
KKT certificates, QP_lambda -> P1 as lambda -> 0, P_{1,2} <-> QP_lambda;
the one-CG-step y-step: Algorithm 2's iterates when A A^T = cI, its step is
the line minimiser of the augmented Lagrangian, LP optimum on Gaussian data
and no convergence in 3000 iterations on face-shaped data).
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import scipy.linalg as sl

from .prox import proj_box, block_soft

CONVERGED, MAXITER, NONFINITE = 0, 1, 2


def full_matrix(A, structure="dense", problem="p1"):
    """The matrix the iteration runs on: A itself, or [A, I] for the
    cross-and-bouquet structure and for the (P_{1,2}) splitting."""
    A = np.asarray(A, dtype=np.float64)
    if structure == "cab" or problem == "p12":
        return np.hstack([A, np.eye(A.shape[0])])
    return A


def beta_scale(b):
    """beta0 = ||b||_1 / m (1 when b = 0): the scale of x, which sets the
    default penalty and the unit of the stopping test."""
    b = np.asarray(b, dtype=np.float64)
    s = np.abs(b).sum() / b.shape[0]
    return s if s > 0 else 1.0


def default_beta(b, structure="dense", y_step="exact"):
    """Reading of the unspecified DALM penalty: beta0 / 8 for the
    cross-and-bouquet form, beta0 otherwise and for the one-CG-step
    variant."""
    if structure == "cab" and y_step == "exact":
        return beta_scale(b) / 8.0
    return beta_scale(b)


@dataclass
class DalmResult:
    w: np.ndarray            # (n_full, N) primal iterate [x; e]
    y: np.ndarray            # (m, N) dual iterate
    v: np.ndarray            # (n_full, N) A^T y
    iters: np.ndarray        # (N,) iterations run
    status: np.ndarray       # (N,) 0 converged, 1 max-iter, 2 non-finite
    beta: np.ndarray         # (N,) penalty used
    history: list = field(default_factory=list)


def _dalm_one(Af, b, beta, tol, max_iter, lam, eps, n_dict, problem,
              w0, y0, fixed, record, y_step="exact", gap_floor=0.0):
    m, n = Af.shape
    dscale = beta_scale(b) / beta if y_step == "exact" else 1.0
    if y_step == "exact":
        G = Af @ Af.T
        if problem == "qp":
            G = G + (lam / beta) * np.eye(m)
        cf = sl.cho_factor(G, lower=True)
    w = np.zeros(n) if w0 is None else np.array(w0, dtype=np.float64)
    y = np.zeros(m) if y0 is None else np.array(y0, dtype=np.float64)
    v = Af.T @ y
    hist = []
    status = MAXITER
    k = 0
    while k < max_iter:
        # z-step: projection of A^T y + w/beta (clamp; block prox on r-block)
        s = v + w / beta
        z = proj_box(s)
        if problem == "p12":
            z[n_dict:] = block_soft(s[n_dict:], eps / beta)
        # y-step: (A A^T [+ lam/beta I]) y = A z - (A w - b)/beta
        rhs = Af @ z - (Af @ w - b) / beta
        if y_step == "exact":
            y = sl.cho_solve(cf, rhs)
        else:
            # one conjugate-gradient step from y_k on the same system (the
            # heuristic of Sec. V-B): the first CG step is steepest descent
            # on q(y) = y^T G y / 2 - rhs^T y with the exact step length
            g = Af @ v + (lam / beta) * y - rhs if problem == "qp" else Af @ v - rhs
            Atg = Af.T @ g
            den = Atg @ Atg + ((lam / beta) * (g @ g) if problem == "qp" else 0.0)
            if den > 0:
                y = y - (g @ g) / den * g
        v_new = Af.T @ y
        # w-step
        w_new = w - beta * (z - v_new)
        k += 1
        dw, nw = np.linalg.norm(w_new - w), np.linalg.norm(w_new)
        l1blk = slice(0, n_dict) if problem == "p12" else slice(0, n)
        wl1 = np.abs(w_new[l1blk]).sum()
        gap = abs(wl1 - w_new[l1blk] @ v_new[l1blk])
        w, v = w_new, v_new
        if record:
            hist.append((dw, nw, gap, wl1))
        if not (np.isfinite(nw) and np.isfinite(gap)):
            status = NONFINITE
            break
        if fixed is None and dscale * dw <= tol * nw and gap <= tol * max(wl1, gap_floor):
            status = CONVERGED
            break
    if fixed is not None and status != NONFINITE:
        status = CONVERGED if k == fixed else MAXITER
    return w, y, v, k, status, hist


def dalm(A, b, *, structure="dense", problem="p1", beta=None, lam=None, eps=None,
         tol=1e-12, max_iter=100000, fixed_iters: Optional[int] = None,
         w0=None, y0=None, record=False, y_step="exact") -> DalmResult:
    """Run DALM on every column of ``b``.

    ``y_step="cg1"`` replaces the exact y-step by one conjugate-gradient step
    from the current y (the cheaper heuristic mentioned in Sec. V-B).

    ``A`` is the dictionary (B for ``structure="cab"``).  ``beta`` is a scalar
    or a per-instance array (default ``default_beta(b_j)``).  ``fixed_iters`` runs
    exactly that many iterations with no stopping test.  Returns a
    :class:`DalmResult` whose ``w`` rows are ``[x; e]`` for the split forms.
    """
    b = np.asarray(b, dtype=np.float64)
    if b.ndim == 1:
        b = b[:, None]
    Af = full_matrix(A, structure, problem)
    m, n = Af.shape
    n_dict = np.asarray(A).shape[1]
    N = b.shape[1]
    if problem == "qp" and (lam is None or lam <= 0):
        raise ValueError("QP_lambda needs lam > 0")
    if problem == "p12" and eps is None:
        raise ValueError("P_{1,2} needs eps")
    if problem == "qp" and structure == "cab":
        raise ValueError("QP_lambda is defined on a dense dictionary")
    if problem == "p12" and structure == "cab":
        raise ValueError("P_{1,2} is defined on a dense dictionary")
    if y_step not in ("exact", "cg1"):
        raise ValueError("y_step must be 'exact' or 'cg1'")
    betas = np.empty(N)
    for j in range(N):
        if beta is None:
            betas[j] = default_beta(b[:, j], structure, y_step)
        else:
            betas[j] = float(np.broadcast_to(np.asarray(beta, np.float64), (N,))[j])
    eps_arr = None if eps is None else np.broadcast_to(np.asarray(eps, np.float64), (N,))
    W = np.zeros((n, N)); Y = np.zeros((m, N)); V = np.zeros((n, N))
    its = np.zeros(N, dtype=np.int64); st = np.zeros(N, dtype=np.int64)
    hist = []
    for j in range(N):
        w, y, v, k, s, h = _dalm_one(
            Af, b[:, j], betas[j], tol,
            fixed_iters if fixed_iters is not None else max_iter,
            lam, None if eps_arr is None else eps_arr[j], n_dict, problem,
            None if w0 is None else np.asarray(w0)[:, j],
            None if y0 is None else np.asarray(y0)[:, j],
            fixed_iters, record, y_step,
            0.25 * np.abs(b[:, j]).sum() if (structure == "cab" and problem == "p1") else 0.0)
        W[:, j], Y[:, j], V[:, j], its[j], st[j] = w, y, v, k, s
        hist.append(h)
    return DalmResult(W, Y, V, its, st, betas, hist)
