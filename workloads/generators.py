"""Seeded generators for the synthetic l1 workloads.

Shapes and value distributions follow the paper's experiments:

* Gaussian compressive-sensing problems (Sec. VI-A): i.i.d. Gaussian ``A`` with
  unit-norm columns, a sparse ``x0`` with random support, ``b = A x0``
  (optionally plus Gaussian noise).
* Cross-and-bouquet face-shaped problems (Sec. II-A, Sec. VI-B): a tight
  "bouquet" dictionary ``B`` whose columns come in classes of highly
  correlated nonnegative vectors, and test vectors ``b = B_c w`` of one class
  with a fraction of the entries replaced by large random values (dense
  corruption).  The face images of the paper are not used; these are
  synthetic stand-ins with the same geometry (m pixels, 7 images per class).

Every array is generated in FP64 and rounded to FP32 once; the returned
arrays are float32.  Both the oracle and the GPU path solve exactly these
FP32 numbers.  Random streams are ``numpy.random.default_rng`` seeded with
``[SEED_ROOT, cfg, stream, index...]`` so any instance can be regenerated on
its own.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

SEED_ROOT = 10073753


def _rng(*key: int) -> np.random.Generator:
    return np.random.default_rng([SEED_ROOT, *key])


def _unit_columns(M: np.ndarray) -> np.ndarray:
    return M / np.linalg.norm(M, axis=0, keepdims=True)


@dataclass
class Problem:
    """A batch of l1 instances sharing one dictionary.

    ``A`` is the dictionary as the caller passes it: the full matrix for a
    dense problem, or ``B`` for a cross-and-bouquet problem (the solver
    appends the identity).  ``b`` is (m, N): one column per instance.
    """

    A: np.ndarray                      # (m, n_dict) float32
    b: np.ndarray                      # (m, N) float32
    structure: str                     # "dense" or "cab"
    problem: str = "p1"                # "p1", "qp", "p12"
    lam: Optional[float] = None        # QP_lambda weight
    eps: Optional[np.ndarray] = None   # P_{1,2} radius per instance
    x0: Optional[np.ndarray] = None    # planted coefficients (n_dict, N)
    e0: Optional[np.ndarray] = None    # planted corruption (m, N)
    labels: Optional[np.ndarray] = None  # class of each instance (cab)
    per_class: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return self.A.shape[0]

    @property
    def n_dict(self) -> int:
        return self.A.shape[1]

    @property
    def N(self) -> int:
        return self.b.shape[1]


def gaussian_dictionary(m: int, n: int, *key: int) -> np.ndarray:
    """i.i.d. N(0, 1/m) entries, then every column scaled to unit l2 norm."""
    A = _rng(*key).standard_normal((m, n)) / np.sqrt(m)
    return _unit_columns(A).astype(np.float32)


def dense_p1(m: int = 200, n: int = 1000, k: int = 20, trial: int = 0,
             N: int = 1, cfg: int = 1, values: str = "normal") -> Problem:
    """Noise-free (P1) with a planted k-sparse x0 (Sec. VI-A shape).

    Default sizes are the 200x1000, 20-nonzero workload; ``values`` is
    "normal" (N(0,1)) or "uniform10" (U[-10, 10] as in the paper's own
    synthetic benchmark).
    """
    A = gaussian_dictionary(m, n, cfg, 0, trial)
    X = np.zeros((n, N))
    for j in range(N):
        r = _rng(cfg, 1, trial, j)
        idx = r.choice(n, k, replace=False)
        if values == "uniform10":
            X[idx, j] = r.uniform(-10.0, 10.0, k)
        else:
            X[idx, j] = r.standard_normal(k)
    X = X.astype(np.float32)
    b = (A.astype(np.float64) @ X.astype(np.float64)).astype(np.float32)
    return Problem(A=A, b=b, structure="dense", problem="p1", x0=X,
                   meta={"cfg": cfg, "trial": trial})


def dense_qp(m: int = 2000, n: int = 8000, k: int = 200, N: int = 64,
             sigma: float = 0.01, lam: float = 1e-3, cfg: int = 2) -> Problem:
    """(QP_lambda) compressive-sensing sweep: +-1 spikes plus Gaussian noise."""
    A = gaussian_dictionary(m, n, cfg, 0)
    X = np.zeros((n, N))
    noise = np.zeros((m, N))
    for j in range(N):
        r = _rng(cfg, 1, j)
        idx = r.choice(n, k, replace=False)
        X[idx, j] = r.choice(np.array([-1.0, 1.0]), k)
        noise[:, j] = sigma * r.standard_normal(m)
    X = X.astype(np.float32)
    b = (A.astype(np.float64) @ X.astype(np.float64) + noise).astype(np.float32)
    return Problem(A=A, b=b, structure="dense", problem="qp", lam=lam, x0=X,
                   meta={"cfg": cfg, "sigma": sigma})


def cab_dictionary(m: int = 1200, classes: int = 100, per_class: int = 7,
                   spread: float = 0.05, cfg: int = 3) -> np.ndarray:
    """Bouquet dictionary: per class a nonnegative U[0,1] mean image, and
    ``per_class`` columns ``max(mean + spread*N(0,1), 0)``, unit l2 norm."""
    r = _rng(cfg, 0)
    B = np.empty((m, classes * per_class))
    for c in range(classes):
        mu = r.uniform(0.0, 1.0, m)
        cols = np.maximum(mu[:, None] + spread * r.standard_normal((m, per_class)), 0.0)
        B[:, c * per_class:(c + 1) * per_class] = cols
    return _unit_columns(B).astype(np.float32)


def cab_instances(B: np.ndarray, N: int, per_class: int, frac=0.3,
                  cfg: int = 3, first: int = 0):
    """Test vectors ``b = B_c w`` (w ~ Dirichlet(1) over one class's columns)
    with ``round(p*m)`` entries, chosen without replacement, replaced by
    ``U[0,1] * max(b_clean)``.  ``frac`` is a number, or ``"uneven"`` for a
    per-instance fraction p ~ U[0, 0.5].  Returns (b, labels, x0, e0)."""
    m, nB = B.shape
    classes = nB // per_class
    b = np.empty((m, N))
    x0 = np.zeros((nB, N))
    e0 = np.zeros((m, N))
    labels = np.empty(N, dtype=np.int64)
    B64 = B.astype(np.float64)
    for jj in range(N):
        j = first + jj
        r = _rng(cfg, 1, j)
        c = int(r.integers(classes))
        w = r.dirichlet(np.ones(per_class))
        clean = B64[:, c * per_class:(c + 1) * per_class] @ w
        p = r.uniform(0.0, 0.5) if frac == "uneven" else float(frac)
        k = int(round(p * m))
        idx = r.choice(m, k, replace=False)
        vec = clean.copy()
        vec[idx] = r.uniform(0.0, 1.0, k) * clean.max()
        b[:, jj] = vec
        x0[c * per_class:(c + 1) * per_class, jj] = w
        e0[:, jj] = vec - clean
        labels[jj] = c
    return b.astype(np.float32), labels, x0.astype(np.float32), e0.astype(np.float32)


def cab_problem(m: int = 1200, classes: int = 100, per_class: int = 7, N: int = 512,
                frac=0.3, cfg: int = 3, first: int = 0) -> Problem:
    """Cross-and-bouquet (P1) batch: ``min ||w||_1 s.t. b = [B, I] w``."""
    B = cab_dictionary(m, classes, per_class, cfg=cfg)
    b, labels, x0, e0 = cab_instances(B, N, per_class, frac=frac, cfg=cfg, first=first)
    return Problem(A=B, b=b, structure="cab", problem="p1", x0=x0, e0=e0,
                   labels=labels, per_class=per_class,
                   meta={"cfg": cfg, "frac": frac, "classes": classes})


def tiny_dense(m: int, n: int, N: int = 1, key: int = 0, k: Optional[int] = None) -> Problem:
    """Small Gaussian problems for brute-force checks (b from a sparse x0 when
    ``k`` is given, else a Gaussian b)."""
    r = _rng(99, key)
    A = _unit_columns(r.standard_normal((m, n))).astype(np.float32)
    if k is None:
        b = r.standard_normal((m, N)).astype(np.float32)
        X = None
    else:
        X = np.zeros((n, N))
        for j in range(N):
            idx = r.choice(n, k, replace=False)
            X[idx, j] = r.standard_normal(k)
        X = X.astype(np.float32)
        b = (A.astype(np.float64) @ X.astype(np.float64)).astype(np.float32)
    return Problem(A=A, b=b, structure="dense", problem="p1", x0=X, meta={"key": key})


@dataclass
class AlignProblem:
    """A batch of alignment l1 problems ``min ||e||_1 s.t. b = B_j w + e``,
    each instance with its own m x k dictionary (eq. (align-simple))."""
    B: np.ndarray        # (N, m, k) float32: B[j] is instance j's dictionary
    b: np.ndarray        # (m, N) float32
    w0: np.ndarray       # (k, N) planted coefficients
    e0: np.ndarray       # (m, N) planted sparse error (the occluding block)
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return self.b.shape[0]

    @property
    def k(self) -> int:
        return self.B.shape[2]

    @property
    def N(self) -> int:
        return self.b.shape[1]


def align_problem(N: int = 1000, h: int = 40, wd: int = 30, n_img: int = 7,
                  occl: float = 0.10, cfg: int = 6, first: int = 0) -> AlignProblem:
    """Alignment-shaped instances (Sec. II-B, Sec. VI-C), a synthetic stand-in
    for the Multi-PIE alignment experiment: an h x wd image grid (m = h*wd),
    ``B_j = [A_j, -J_j]`` with ``n_img`` training images of one subject (a
    smooth nonnegative mean image plus small per-image variation, unit norm)
    and the four columns of a similarity transform's Jacobian of the mean
    image (x and y derivative, rotation, scale; unit norm); ``b = B_j w0 + e0``
    with w0 a convex combination of the images plus a small transform step,
    and e0 the difference made by a randomly placed block covering ``occl``
    of the image whose pixels are replaced by U[0, 1] values."""
    m = h * wd
    k = n_img + 4
    yy, xx = np.meshgrid(np.arange(h) - (h - 1) / 2.0, np.arange(wd) - (wd - 1) / 2.0, indexing="ij")
    Bs = np.empty((N, m, k))
    b = np.empty((m, N))
    w0 = np.zeros((k, N))
    e0 = np.zeros((m, N))
    bh = max(1, int(round(np.sqrt(occl * m * h / wd))))
    bw = max(1, int(round(occl * m / bh)))
    for jj in range(N):
        j = first + jj
        r = _rng(cfg, 0, j)
        # smooth mean image: a few random Gaussian bumps on a bright base
        img = 0.3 * np.ones((h, wd))
        for _ in range(6):
            cy, cx = r.uniform(-h / 2, h / 2), r.uniform(-wd / 2, wd / 2)
            s = r.uniform(3.0, 8.0)
            img += r.uniform(0.2, 0.7) * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2 * s * s))
        A = np.maximum(img.reshape(-1, 1) + 0.05 * r.standard_normal((m, n_img)), 0.0)
        gy, gx = np.gradient(img)
        J = np.stack([gx, gy, xx * gy - yy * gx, xx * gx + yy * gy], axis=-1).reshape(m, 4)
        B = np.concatenate([_unit_columns(A), -_unit_columns(J)], axis=1)
        w = np.concatenate([r.dirichlet(np.ones(n_img)), 0.05 * r.standard_normal(4)])
        clean = B @ w
        y0, x0 = int(r.integers(0, h - bh + 1)), int(r.integers(0, wd - bw + 1))
        vec = clean.reshape(h, wd).copy()
        vec[y0:y0 + bh, x0:x0 + bw] = r.uniform(0.0, 1.0, (bh, bw))
        vec = vec.reshape(-1)
        Bs[jj] = B
        b[:, jj] = vec
        w0[:, jj] = w
        e0[:, jj] = vec - clean
    return AlignProblem(B=Bs.astype(np.float32), b=b.astype(np.float32), w0=w0.astype(np.float32),
                        e0=e0.astype(np.float32), meta={"cfg": cfg, "occl": occl, "h": h, "w": wd})
