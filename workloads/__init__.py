"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package generates data only: feature matrices, labels, held-out sets and
problem descriptors. It holds none of the optimisation method's arithmetic
(no sampling of mini-batches, no gradients, no Gram matrices), so the oracle
and the GPU path can both draw on it without sharing any of the computation
they are compared on.
"""
from .generators import (  # noqa: F401
    DenseProblem,
    SparseProblem,
    dense_c1,
    dense_c2,
    dense_glm,
    dense_logreg,
    glm_labels,
    lambda_path_c4,
    normalize_rows,
    sparse_c4,
    sparse_zipf_glm,
    sparse_zipf_logreg,
    uneven_problem_specs,
    uneven_problem,
)
