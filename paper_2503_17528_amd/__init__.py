"""MI355X-native block Cholesky (POBTAF) and selected inversion (POBTASI) of
symmetric positive-definite block-tridiagonal-arrowhead (BTA) matrices.

The compute path lives in a HIP shared library (``csrc/``) behind a C ABI
(``include/bta.h``).  ``paper_2503_17528_amd.bta`` is the thin ctypes binding
with the same entry-point names; ``paper_2503_17528_amd.synth`` holds the
seeded synthetic-input generators.  Importing this package loads nothing.
"""

__all__ = ["bta", "synth", "autograd"]
__version__ = "0.1.0"
