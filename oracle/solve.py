"""Exact discrete solution (oracle side).

The system of eq. (3.3) is symmetric positive definite (Section 3.5), so its
solution is unique; the oracle obtains it by a sparse direct LU solve
(SuperLU via scipy) followed by one step of iterative refinement in FP64.
The GPU path reaches the same vector only approximately, with a multigrid
preconditioned conjugate gradient method stopped on a residual tolerance.
"""
import numpy as np
import scipy.sparse.linalg as spla


def direct_solve(A, b, refine=True):
    lu = spla.splu(A.tocsc())
    x = lu.solve(b)
    if refine:
        r = b - A @ x
        x = x + lu.solve(r)
    return x


def residual_norm(A, x, b):
    return float(np.linalg.norm(b - A @ x))
