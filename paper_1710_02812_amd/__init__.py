"""MI355X-native hierarchical merge-and-truncate truncated SVD (arXiv:1710.02812).

The compute path is the HIP library ``libhsvd.so`` built from ``csrc/``; this
package only marshals arguments to its C ABI (see ``hsvd.py``).
"""
