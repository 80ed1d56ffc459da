"""FP64 CPU oracle for the augmented-Lagrangian l1 solvers.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline
leg of ``bench.py`` use it.  It shares no code with the GPU library.

Everything here is plain NumPy/SciPy in float64, written to be checked by eye
against the paper (Yang, Zhou, Ganesh, Sastry, Ma, "Fast l1-minimization
algorithms for robust face recognition"):

* ``prox``    -- soft-thresholding (Sec. IV) and the projections used by the
  dual method (Sec. V-B);
* ``exact``   -- the plain definitions of the optima: the (P1) linear program
  (Sec. III-A), brute-force enumeration for tiny problems, and an independent
  FISTA (Sec. IV-A) for (QP_lambda);
* ``dalm``    -- the dual ALM iteration (Sec. V-B, Algorithm 2);
* ``palm``    -- the primal ALM iteration (Sec. V-A, eq. (alm) and
  Algorithm 1) with FISTA as the inner solver;
* ``kkt``     -- optimality certificates (LP duality, Sec. III-A / V-B; the
  Homotopy optimality condition of Sec. III-B for QP_lambda);
* ``unrolled``-- a fixed number of Algorithm-2 iterations and its exact
  reverse-mode gradient with respect to b and the dictionary;
* ``sci``     -- the recognition criterion of the face experiments
  (Sec. VI-B): subject l1 masses, the sparsity concentration index, label;
  and the per-subject residuals of the classifier the paper builds on;
* ``align``   -- the l1 problem of the alignment step (Sec. II-B, eq.
  (align-simple)): its LP, brute force, and PALM as Sec. VI-C runs it.

Parity status of each function is stated in its docstring; those without an
independent pin say "parity unpinned".
"""
from .prox import soft, proj_box, block_soft, proj_ball  # noqa: F401
from .exact import p1_lp, brute_force_p1, brute_force_qp, qp_fista  # noqa: F401
from .dalm import dalm, DalmResult, full_matrix  # noqa: F401
from .palm import palm, PalmResult  # noqa: F401
from .sci import sci, class_residuals  # noqa: F401
from .align import align_lp, align_brute, align_palm  # noqa: F401
from .kkt import kkt_report  # noqa: F401
from .unrolled import (  # noqa: F401
    unrolled_dalm, unrolled_loss, unrolled_grad, unrolled_vjp,
    class_residual_loss, clamp_pattern,
)
