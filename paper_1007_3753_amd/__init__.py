"""Batched augmented-Lagrangian l1 solvers (PALM / DALM) for AMD MI355X.

The solver runs in ``libl1alm.so`` (hand-written HIP for gfx950, C ABI in
``include/l1_alm.h``); this package is its Python binding.
"""
from ._lib import L1Error, LIB_PATH, load  # noqa: F401


def __getattr__(name):
    # the torch-facing binding is imported lazily so that the C-ABI checks can
    # run without initialising a GPU
    if name in ("Plan", "SolveResult", "DALMUnrolled", "classify", "class_residuals", "align"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
