"""Exact discrete solution (oracle side).

The system of eq. (3.3) is symmetric positive definite (Section 3.5), so its
solution is unique.  The oracle obtains it in one of two plain ways:

* direct_solve: a sparse direct LU solve (SuperLU via scipy) followed by one
  step of iterative refinement in FP64 -- for every 2-D grid and for 3-D grids
  up to 32^3, where the factor fits comfortably in memory;
* cg_solve: the conjugate gradient method of Section 3.5 with the simplest
  preconditioner there is (the diagonal of A, Jacobi), started from x0 = 0 and
  run until the recursively updated residual satisfies ||r|| / ||b|| < 1e-14 --
  for the 3-D grids 64^3 and 128^3, whose direct factors do not fit.  Its
  answer is checked by the recomputed true residual, which the caller gets
  back; for a QoI g^T x the error is g^T A^-1 (b - A x), so a residual at the
  FP64 rounding level fixes the QoI far below 1e-10 relative.

The GPU path reaches the same vector only approximately, with a multigrid
preconditioned conjugate gradient method stopped on a looser residual
tolerance.
"""
import numpy as np
import scipy.sparse.linalg as spla

# 3-D grids above this many cells per direction are solved by cg_solve
DIRECT_MAX_3D = 32


def direct_solve(A, b, refine=True):
    lu = spla.splu(A.tocsc())
    x = lu.solve(b)
    if refine:
        r = b - A @ x
        x = x + lu.solve(r)
    return x


def cg_solve(A, b, tol=1e-14, maxit=200000):
    """Jacobi-preconditioned conjugate gradients from x0 = 0.

    Stops when ||r_k|| / ||b|| < tol for the recursively updated residual r_k.
    Returns (x, iterations, ||b - A x|| / ||b|| recomputed from x).  Raises
    RuntimeError when maxit iterations do not reach tol.
    """
    A = A.tocsr()
    b = np.asarray(b, dtype=np.float64)
    dinv = 1.0 / A.diagonal()
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b)
    if bnorm == 0.0:
        return x, 0, 0.0
    r = b.copy()
    z = dinv * r
    p = z.copy()
    rz = r @ z
    for it in range(1, maxit + 1):
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        if np.linalg.norm(r) < tol * bnorm:
            return x, it, float(np.linalg.norm(b - A @ x) / bnorm)
        z = dinv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    raise RuntimeError("cg_solve: no convergence to %g in %d iterations" % (tol, maxit))


def uses_cg(dim, m):
    """The rule for choosing the solver: CG for 3-D grids above 32^3."""
    return dim == 3 and m > DIRECT_MAX_3D


def solve(A, b, dim, m, solver="auto"):
    """The discrete solution by the solver `solver` ("direct", "cg", or "auto":
    the rule of uses_cg)."""
    if solver == "auto":
        solver = "cg" if uses_cg(dim, m) else "direct"
    if solver == "direct":
        return direct_solve(A, b)
    if solver == "cg":
        return cg_solve(A, b)[0]
    raise ValueError(solver)


def residual_norm(A, x, b):
    return float(np.linalg.norm(b - A @ x))
