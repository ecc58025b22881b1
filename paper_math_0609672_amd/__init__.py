"""Random-walk incomplete LDL^T preconditioning for R-matrices on MI355X (gfx950).

Importing the package loads nothing native; ``paper_math_0609672_amd.srw`` binds the
HIP library (``libsrw.so``) and raises if it is missing.
"""
__version__ = "0.1.0"
