"""MI355X-native hierarchical merge-and-truncate truncated SVD (arXiv:1710.02812).

The compute path is the HIP library ``libhsvd.so`` built from ``csrc/``; the
``hsvd`` module only marshals arguments to its C ABI.  ``synth`` holds the
seeded synthetic workloads.
"""
from .hsvd import (Plan, BatchPlan, RankModel, svd, svd_batched, learned_svd, block_features,  # noqa: F401
                   HsvdError, FP64, FP32, MIXED_BF16, RULE_GAMMA, RULE_FROB, FLAG_NONFINITE, FLAG_NOCONV,
                   FLAG_RANK_FALLBACK)
