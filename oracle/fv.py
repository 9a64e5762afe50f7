"""Cell-centred finite volume system (oracle side).

Section 3.1 integrates the equation over each box of a uniform m^d mesh and
approximates each face flux by (face value of k) x (difference of the two
cell values) / (distance of the centres), eq. (3.3); Section 3.4 takes the
face value of k as the harmonic average of the two neighbouring cells.  On a
face between cells P and Q this gives the transmissibility

    T_PQ = h^(d-1) / h * 2 k_P k_Q / (k_P + k_Q) = h^(d-2) * harmonic(k_P, k_Q),

and row P of the system reads  sum_Q T_PQ (p_P - p_Q) + sum_bdry T_b (p_P - p_D) = b_P.

Boundary conditions:
* Model Problem 2, eq. (3.11): p = 1 on x1 = 0, p = 0 on x1 = 1, zero flux on
  the other faces, f = 0.  A Dirichlet face replaces the central difference
  by a one-sided difference over the half cell between the centre and the
  face (reading of Section 3.1 adopted here), so T_b = 2 k_P h^(d-2), and the
  known boundary value moves to the right-hand side, b_P = T_b p_D.
* Model Problem 1: f = 1 and p = 0 on the whole boundary; the right-hand side
  is the midpoint rule f h^d.

Arrays are indexed [..., x2, x1] (x1, the flow direction, is the last axis);
unknown P = (j, i) has linear index j*m + i (x1 fastest).
"""
import numpy as np
import scipy.sparse as sp

MP2 = "mp2"
MP1 = "mp1"


def harmonic(a, b):
    return 2.0 * a * b / (a + b)


def face_transmissibilities(k):
    """Interior face transmissibilities per axis and Dirichlet-face values.

    Returns (T, Tb) where T[ax] has the shape of k with axis `ax` shortened by
    one (face between index i and i+1 along that array axis), and Tb = 2 k
    h^(d-2) is the transmissibility of a cell's half-cell boundary face.
    """
    d = k.ndim
    m = k.shape[0]
    h = 1.0 / m
    scale = h ** (d - 2)
    T = []
    for ax in range(d):
        lo = np.take(k, np.arange(m - 1), axis=ax)
        hi = np.take(k, np.arange(1, m), axis=ax)
        T.append(scale * harmonic(lo, hi))
    return T, 2.0 * k * scale


def assemble(k, bc=MP2):
    """Sparse matrix A and right-hand side b of eq. (3.3) for the given problem."""
    d = k.ndim
    m = k.shape[0]
    n = k.size
    idx = np.arange(n).reshape(k.shape)
    T, Tb = face_transmissibilities(k)
    rows, cols, vals = [], [], []
    diag = np.zeros(k.shape)
    b = np.zeros(k.shape)
    for ax in range(d):
        p = np.take(idx, np.arange(m - 1), axis=ax).ravel()
        q = np.take(idx, np.arange(1, m), axis=ax).ravel()
        t = T[ax].ravel()
        rows += [p, q]
        cols += [q, p]
        vals += [-t, -t]
        np.add.at(diag.reshape(-1), p, t)
        np.add.at(diag.reshape(-1), q, t)
    x1_axis = d - 1
    first = [slice(None)] * d
    last = [slice(None)] * d
    if bc == MP2:
        first[x1_axis] = 0
        last[x1_axis] = m - 1
        first, last = tuple(first), tuple(last)
        diag[first] += Tb[first]
        diag[last] += Tb[last]
        b[first] += Tb[first] * 1.0      # p = 1 on x1 = 0
        # p = 0 on x1 = 1 adds nothing to b; other faces carry zero flux
    elif bc == MP1:
        for ax in range(d):
            for end in (0, m - 1):
                sl = [slice(None)] * d
                sl[ax] = end
                sl = tuple(sl)
                diag[sl] += Tb[sl]      # p = 0 on every boundary face
        b[...] = 1.0 / m ** d           # midpoint rule for f = 1
    else:
        raise ValueError(bc)
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    return A, b.ravel()
