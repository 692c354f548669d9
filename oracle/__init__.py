"""CPU float64 oracle of the hierarchical MAT SVD and its comparison metrics.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg; never by the library's execution path.
Parity status of each function is recorded in its docstring and in the pins
under tests/test_oracle.py.
"""
from .hsvd_oracle import (EPS, balanced_split, truncation_rank, leaf, randomised_leaf,  # noqa: F401
                          merge,
                          merge_complement, merge_tree, slab_nodes, col_slab_nodes, project, improve,
                          sign_normalise, hsvd, hsvd_gram, flop_model)
from . import metrics  # noqa: F401
