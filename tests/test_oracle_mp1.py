"""Pins of the oracle's Model Problem 1 (Section 3.4): -div(k grad p) = 1 on the
unit cube, p = 0 on the whole boundary, QoI M^(1) = mean of p over D*.

* Constant k: the cell-centred operator with half-cell Dirichlet faces is
  k h^(d-2) times a sum over the axes of the 1-D matrix tridiag(-1, 2, -1)
  with end entries 3, whose eigenvectors are sin(pi a (i + 1/2) / m) with
  eigenvalues 4 sin^2(pi a / (2m)), a = 1..m (the discrete sine basis of the
  reflected ghost cell p_-1 = -p_0).  The discrete solution is therefore a
  finite sine series, written out here in 2-D and 3-D, independent of the
  sparse solver.
* The box functional against a brute-force midpoint integration of the
  cell-wise constant pressure over D* on a fine point grid, for grids whose
  cell edges do and do not meet the box edges.
* Invariants: M^(1)(c k) = M^(1)(k) / c; M^(1) is unchanged by mirroring k in
  any axis and (the problem being isotropic) by swapping axes, since D* is the
  centred cube.
* Conservation: the source h^d per cell leaves through the boundary faces.
"""
import numpy as np
import pytest

import workloads as W
from oracle import field, fv, mlmc, qoi, solve


def sine_series_solution(m, d, k):
    """Discrete solution of Model Problem 1 for constant k (see module doc)."""
    h = 1.0 / m
    i = np.arange(m)
    a = np.arange(1, m + 1)
    V = np.sin(np.pi * np.outer(a, i + 0.5) / m)          # V[a-1, i]
    lam = 4.0 * np.sin(np.pi * a / (2 * m)) ** 2
    c = V.sum(axis=1) / np.sum(V * V, axis=1)              # coefficient of 1 in the basis
    p = np.zeros((m,) * d)
    if d == 2:
        for x in range(m):
            for y in range(m):
                p += c[x] * c[y] / (lam[x] + lam[y]) * np.multiply.outer(V[x], V[y])
    else:
        for x in range(m):
            for y in range(m):
                for z in range(m):
                    w = c[x] * c[y] * c[z] / (lam[x] + lam[y] + lam[z])
                    p += w * np.multiply.outer(np.multiply.outer(V[x], V[y]), V[z])
    return p * h ** d / (k * h ** (d - 2))


@pytest.mark.parametrize("d,m,kval", [(2, 8, 1.0), (2, 12, 2.5), (3, 6, 0.7)])
def test_constant_k_matches_sine_series(d, m, kval):
    k = np.full((m,) * d, kval)
    A, b = fv.assemble(k, fv.MP1)
    p = solve.direct_solve(A, b).reshape(k.shape)
    ref = sine_series_solution(m, d, kval)
    assert np.max(np.abs(p - ref)) < 1e-13 * np.max(np.abs(ref))
    assert abs(qoi.box_average(p) - qoi.box_average(ref)) < 1e-13 * qoi.box_average(ref)


@pytest.mark.parametrize("m", [8, 16, 24, 40])
def test_box_average_brute_force(m):
    rng = np.random.default_rng(m)
    p = rng.standard_normal((m, m)) + 2.0
    lo, hi = qoi.MP1_BOX
    # midpoint rule on an N x N point grid over D*: every point lies inside one cell
    N = 2400
    x = lo + (np.arange(N) + 0.5) * (hi - lo) / N
    cell = np.floor(x * m).astype(int)
    brute = p[np.ix_(cell, cell)].mean()
    assert abs(qoi.box_average(p) - brute) < 1e-12 * abs(brute)


def test_box_average_of_linear_profile_is_centre_value():
    # cell values of a linear function; D* and every grid are symmetric about 1/2
    for m in (8, 24):
        x = (np.arange(m) + 0.5) / m
        p = 3.0 + 2.0 * x[:, None] - 5.0 * x[None, :]
        assert abs(qoi.box_average(p) - (3.0 + 1.0 - 2.5)) < 1e-13


def test_box_weights_partition_the_box():
    for m in (8, 10, 24, 64):
        w = qoi.axis_overlaps(m, *qoi.MP1_BOX)
        assert abs(w.sum() - (qoi.MP1_BOX[1] - qoi.MP1_BOX[0])) < 1e-15
        assert np.all(w >= 0.0)


def mp1_q(k):
    return mlmc.solve_qoi(k, fv.MP1)[0]


def test_invariants():
    rng = np.random.default_rng(3)
    k = np.exp(rng.standard_normal((16, 16)))
    q = mp1_q(k)
    assert abs(mp1_q(3.0 * k) - q / 3.0) < 1e-12 * q
    for kk in (k[::-1, :], k[:, ::-1], k.T, k[::-1, ::-1].T):
        assert abs(mp1_q(np.ascontiguousarray(kk)) - q) < 1e-12 * q
    k3 = np.exp(rng.standard_normal((6, 6, 6)))
    q3 = mp1_q(k3)
    for kk in (k3[::-1], k3[:, ::-1], k3[:, :, ::-1], np.transpose(k3, (2, 0, 1))):
        assert abs(mp1_q(np.ascontiguousarray(kk)) - q3) < 1e-12 * q3


def test_source_leaves_through_boundary():
    rng = np.random.default_rng(4)
    m = 12
    k = np.exp(rng.standard_normal((m, m)))
    A, b = fv.assemble(k, fv.MP1)
    p = solve.direct_solve(A, b).reshape(m, m)
    tb = 2.0 * k
    out = (tb[:, 0] * p[:, 0]).sum() + (tb[:, -1] * p[:, -1]).sum() + \
        (tb[0, :] * p[0, :]).sum() + (tb[-1, :] * p[-1, :]).sum()
    assert abs(out - 1.0) < 1e-12


def test_level_sample_uses_model_problem_1():
    model = W.MP1_CE2
    r = mlmc.level_sample(model, 1, 3, 16)
    k, kc = field.sample_k(model, 1, 3, 16, with_coarse=True)
    assert abs(r["Q_f"] - mp1_q(k)) < 1e-15 * r["Q_f"]
    assert abs(r["Q_c"] - mp1_q(kc)) < 1e-15 * r["Q_c"]
    assert r["Q_f"] > 0.0
