"""A fixed number of Algorithm-2 iterations as a differentiable map, FP64.

Forward: exactly K iterations of the cross-and-bouquet DALM (Sec. V-B,
Algorithm 2) from w = 0, y = 0, with no stopping test, for every column of b:

    s_k     = A^T y_k + w_k / beta
    z_{k+1} = clamp(s_k)
    y_{k+1} = G^{-1} (A z_{k+1} - (A w_k - b)/beta),   G = A A^T = B B^T + I
    w_{k+1} = w_k - beta (z_{k+1} - A^T y_{k+1})

with A = [B, I].  beta is a per-instance constant (not differentiated).

Loss (a reading: the paper prints only the SCI classifier; the residual rule
comes from the sparse-representation classifier it builds on): per instance
j and class c, ``res_{jc} = ||b_j - e_j - B_c x_{j,c}||_2`` over the class's
columns, logits ``-res_{jc}``, and the mean softmax cross-entropy against the
generating class.

Gradient: plain reverse mode over the full stored tape (no checkpointing),
written out step by step.  The clamp derivative is 1 where |s| < 1 and 0
elsewhere (a.e. derivative).

Parity pins: tests/test_oracle_unrolled.py (central finite differences on the
forward map at points where the clamp pattern is unchanged, and the K = 1
closed form dw_1/db = A^T (A A^T)^{-1}).
"""
import numpy as np


def _full(B):
    m = B.shape[0]
    return np.hstack([B, np.eye(m)])


def unrolled_dalm(B, b, beta, K, keep_tape=False):
    """K iterations for all columns of b (m x N).  Returns (x, e, tape)."""
    B = np.asarray(B, np.float64)
    b = np.asarray(b, np.float64)
    beta = np.broadcast_to(np.asarray(beta, np.float64), (b.shape[1],))
    A = _full(B)
    m, n = A.shape
    Ginv = np.linalg.inv(A @ A.T)
    N = b.shape[1]
    w = np.zeros((n, N))
    y = np.zeros((m, N))
    tape = []
    for _ in range(K):
        s = A.T @ y + w / beta
        z = np.clip(s, -1.0, 1.0)
        y_new = Ginv @ (A @ z - (A @ w - b) / beta)
        w_new = w - beta * (z - A.T @ y_new)
        if keep_tape:
            tape.append((w, y, s, z, y_new))
        w, y = w_new, y_new
    nB = B.shape[1]
    return w[:nB], w[nB:], (tape, Ginv, A, w, y)


def class_residual_loss(B, b, x, e, labels, per_class):
    """Mean softmax cross-entropy of logits -res_{jc}.  Returns (loss, aux)
    where aux holds what the gradient needs."""
    B = np.asarray(B, np.float64)
    b = np.asarray(b, np.float64)
    m, nB = B.shape
    C = nB // per_class
    N = b.shape[1]
    D = np.empty((C, m, N))
    res = np.empty((C, N))
    for c in range(C):
        sl = slice(c * per_class, (c + 1) * per_class)
        D[c] = b - e - B[:, sl] @ x[sl]
        res[c] = np.linalg.norm(D[c], axis=0)
    logits = -res
    mx = logits.max(axis=0, keepdims=True)
    p = np.exp(logits - mx)
    p /= p.sum(axis=0, keepdims=True)
    lab = np.asarray(labels)
    loss = float(-np.mean(np.log(p[lab, np.arange(N)])))
    return loss, (D, res, p)


def unrolled_loss(B, b, beta, K, labels, per_class):
    x, e, _ = unrolled_dalm(B, b, beta, K)
    return class_residual_loss(B, b, x, e, labels, per_class)[0]


def unrolled_vjp(B, b, beta, K, gx, ge):
    """Vector-Jacobian product of (x_K, e_K) with respect to (b, B): given
    output adjoints ``gx`` (n_B x N) and ``ge`` (m x N), return (gb, gB)."""
    B = np.asarray(B, np.float64)
    b = np.asarray(b, np.float64)
    beta = np.broadcast_to(np.asarray(beta, np.float64), (b.shape[1],))
    m, nB = B.shape
    N = b.shape[1]
    _, _, (tape, Ginv, A, wK, yK) = unrolled_dalm(B, b, beta, K, keep_tape=True)
    gb = np.zeros((m, N))
    gA = np.zeros_like(A)
    gG = np.zeros((m, m))
    gw = np.vstack([np.asarray(gx, np.float64), np.asarray(ge, np.float64)])
    gy = np.zeros((m, N))
    for (w, y, s, z, y_new) in reversed(tape):
        # w_new = w - beta z + beta A^T y_new
        gw_k = gw.copy()
        gz = -beta * gw
        gy_tot = gy + beta * (A @ gw)
        gA += (y_new * beta) @ gw.T
        # y_new = G^{-1} r
        gr = Ginv @ gy_tot
        gG -= gr @ y_new.T
        # r = A z - A w / beta + b / beta
        gz += A.T @ gr
        gw_k -= (A.T @ gr) / beta
        gb += gr / beta
        gA += gr @ (z - w / beta).T
        # z = clamp(s)
        gs = gz * (np.abs(s) < 1.0)
        # s = A^T y + w / beta
        gy = A @ gs
        gw_k += gs / beta
        gA += y @ gs.T
        gw = gw_k
    # G = B B^T + I ;  A = [B, I]
    gB = gA[:, :nB] + (gG + gG.T) @ B
    return gb, gB


def unrolled_grad(B, b, beta, K, labels, per_class):
    """Returns (loss, d loss/d b (m x N), d loss/d B (m x n_B))."""
    B = np.asarray(B, np.float64)
    b = np.asarray(b, np.float64)
    m, nB = B.shape
    N = b.shape[1]
    x, e, _ = unrolled_dalm(B, b, beta, K)
    loss, (D, res, p) = class_residual_loss(B, b, x, e, labels, per_class)
    C = nB // per_class
    lab = np.asarray(labels)
    # loss -> (x, e, b, B) directly
    gb = np.zeros((m, N))
    gB = np.zeros((m, nB))
    gx = np.zeros((nB, N))
    ge = np.zeros((m, N))
    onehot = np.zeros((C, N))
    onehot[lab, np.arange(N)] = 1.0
    gres = -(p - onehot) / N                      # d loss / d res
    for c in range(C):
        sl = slice(c * per_class, (c + 1) * per_class)
        gD = gres[c] * D[c] / np.maximum(res[c], 1e-300)   # d loss / d D_c
        gb += gD
        ge -= gD
        gx[sl] -= B[:, sl].T @ gD
        gB[:, sl] -= gD @ x[sl].T
    vb, vB = unrolled_vjp(B, b, beta, K, gx, ge)
    return loss, gb + vb, gB + vB


def clamp_pattern(B, b, beta, K):
    """Sign pattern of every clamp argument over the K iterations (used to
    keep finite-difference samples away from kinks)."""
    _, _, (tape, *_rest) = unrolled_dalm(B, b, beta, K, keep_tape=True)
    return np.concatenate([np.sign(np.abs(t[2]) - 1.0).ravel() for t in tape])
