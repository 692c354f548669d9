"""MI355X-native hierarchical merge-and-truncate truncated SVD (arXiv:1710.02812).

The compute path is the HIP library ``libhsvd.so`` built from ``csrc/``; the
``hsvd`` module only marshals arguments to its C ABI.  ``synth`` holds the
seeded synthetic workloads.
"""
from .hsvd import (Plan, BatchPlan, svd, svd_batched, HsvdError, FP64, FP32, MIXED_BF16,  # noqa: F401
                   RULE_GAMMA, RULE_FROB, FLAG_NONFINITE, FLAG_NOCONV)
