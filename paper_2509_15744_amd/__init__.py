"""fdwave for MI355X: memory-efficient superposition adjoint sensitivities of the
scalar acoustic wave equation (arXiv:2509.15744), as hand-written HIP kernels for
gfx950 behind a C-ABI library.

Importing the package loads nothing; ``paper_2509_15744_amd.fdwave`` binds the
built library (``libfdwave.so``) and raises if it is missing.
"""
__all__ = ["fdwave", "workloads"]
