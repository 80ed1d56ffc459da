"""Proximal maps used by the ALM iterations (FP64, elementwise NumPy).

Pins (tests/test_oracle_prox.py): the closed forms are checked against a
brute-force 1-D minimisation of the defining prox problem and against the
Moreau decomposition; the block maps against their defining minimisation.
"""
import numpy as np


def soft(v, alpha):
    """Soft-thresholding, the prox of ``alpha*||.||_1`` (Sec. IV, the
    shrinkage operator): ``sign(v_i) * max(|v_i| - alpha, 0)``.

    ``alpha`` may be a scalar or broadcast against ``v``.  sign(0) = 0, so
    ``soft(+-alpha, alpha) = 0`` exactly."""
    v = np.asarray(v, dtype=np.float64)
    return np.sign(v) * np.maximum(np.abs(v) - alpha, 0.0)


def proj_box(v):
    """Projection onto the unit l-infinity ball {z : ||z||_inf <= 1}
    (Sec. V-B, the z-update of the dual ALM): clamp every entry to [-1, 1]."""
    v = np.asarray(v, dtype=np.float64)
    return np.minimum(np.maximum(v, -1.0), 1.0)


def block_soft(v, tau):
    """Prox of ``tau*||.||_2`` (block soft-threshold):
    ``v * max(0, 1 - tau/||v||_2)``, and 0 for v = 0.

    Used for the error block of the dual ALM for (P_{1,2}): the conjugate of
    the indicator of the eps-ball is ``eps*||.||_2``, and its prox with step
    1/beta is this map with ``tau = eps/beta``."""
    v = np.asarray(v, dtype=np.float64)
    nv = np.linalg.norm(v)
    if nv <= tau:
        return np.zeros_like(v)
    return v * (1.0 - tau / nv)


def proj_ball(v, eps):
    """Projection onto the l2 ball of radius eps: ``v * min(1, eps/||v||)``.

    Used for the error block of the primal ALM for (P_{1,2})."""
    v = np.asarray(v, dtype=np.float64)
    nv = np.linalg.norm(v)
    if nv <= eps:
        return v.copy()
    return v * (eps / nv)
