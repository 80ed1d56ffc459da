"""Seeded synthetic workloads shaped like the paper's experiments.

This package only draws random numbers and assembles matrices and vectors;
it holds none of the solver arithmetic.  Both the FP64 oracle tests and the
GPU path take their inputs from here, so that the two sides solve the same
FP32-rounded problems.
"""
from .generators import (  # noqa: F401
    SEED_ROOT,
    Problem,
    gaussian_dictionary,
    dense_p1,
    dense_qp,
    cab_dictionary,
    cab_instances,
    cab_problem,
    tiny_dense,
    AlignProblem,
    align_problem,
)
