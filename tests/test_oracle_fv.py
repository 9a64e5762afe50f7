"""Pins of the oracle's finite volume system, direct solve and outflow QoI.

Closed forms of eq. (3.3) with harmonic faces and half-cell Dirichlet faces:
* homogeneous k: p is linear in x1 and Q = k (2D and 3D);
* k depending only on the transverse coordinates (layers parallel to the
  flow): Q = arithmetic mean of k over the cross-section;
* k depending only on x1 (layers across the flow): Q = harmonic mean.
Invariants: the matrix is symmetric positive definite with non-positive
off-diagonals and row sums equal to the boundary transmissibilities; inflow
equals outflow (local conservation); Q(c k) = c Q(k); Q is unchanged by
mirroring k in x1 or x2; Q equals the dissipated power sum T (dp)^2 (for a
unit pressure drop).  Brute force: the matrix and right-hand side recovered
from the dissipation energy evaluated at unit vectors; the direct solve
against numpy.linalg.solve and against a conjugate gradient solve.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fv, qoi, solve


def _solve_q(k, bc=fv.MP2):
    A, b = fv.assemble(k, bc)
    p = solve.direct_solve(A, b)
    return A, b, p, qoi.outflow(k, p), qoi.inflow(k, p)


@pytest.mark.parametrize("d,m", [(2, 8), (2, 16), (3, 6)])
def test_homogeneous_linear_pressure(d, m):
    k = np.full((m,) * d, 3.7)
    _, _, p, qo, qi = _solve_q(k)
    x1 = (np.arange(m) + 0.5) / m
    assert np.allclose(p.reshape(k.shape), 1.0 - x1, rtol=0, atol=1e-13)
    assert abs(qo - 3.7) < 1e-12 and abs(qi - 3.7) < 1e-12


def test_parallel_layers_arithmetic_mean():
    rng = np.random.default_rng(1)
    m = 16
    kr = np.exp(rng.standard_normal(m))
    k = np.repeat(kr[:, None], m, axis=1)        # depends on x2 only
    _, _, _, qo, _ = _solve_q(k)
    assert abs(qo - kr.mean()) < 1e-12 * kr.mean()
    k3v = np.exp(rng.standard_normal((6, 6)))     # depends on (x3, x2)
    k3 = np.repeat(k3v[:, :, None], 6, axis=2)
    _, _, _, qo3, _ = _solve_q(k3)
    assert abs(qo3 - k3v.mean()) < 1e-12 * k3v.mean()


def test_perpendicular_layers_harmonic_mean():
    rng = np.random.default_rng(2)
    m = 16
    kc = np.exp(2.0 * rng.standard_normal(m))
    k = np.repeat(kc[None, :], m, axis=0)         # depends on x1 only
    _, _, _, qo, _ = _solve_q(k)
    hm = m / np.sum(1.0 / kc)
    assert abs(qo - hm) < 1e-12 * hm


def test_matrix_structure_and_invariants():
    rng = np.random.default_rng(3)
    m = 8
    k = np.exp(rng.standard_normal((m, m)))
    A, b, p, qo, qi = _solve_q(k)
    Ad = A.toarray()
    assert np.allclose(Ad, Ad.T, rtol=0, atol=0)
    assert np.linalg.eigvalsh(Ad).min() > 0
    off = Ad - np.diag(np.diag(Ad))
    assert np.all(off <= 0)
    # row sums = boundary transmissibility 2k on the x1 = 0 and x1 = 1 faces
    rs = Ad.sum(axis=1).reshape(m, m)
    ref = np.zeros((m, m))
    ref[:, 0] += 2 * k[:, 0]
    ref[:, -1] += 2 * k[:, -1]
    assert np.allclose(rs, ref, rtol=1e-14, atol=1e-14)
    assert abs(qo - qi) < 1e-13 * qo
    assert abs(_solve_q(3.0 * k)[3] - 3.0 * qo) < 1e-13 * qo
    assert abs(_solve_q(k[:, ::-1].copy())[3] - qo) < 1e-13 * qo
    assert abs(_solve_q(k[::-1, :].copy())[3] - qo) < 1e-13 * qo


def _energy(k, p):
    """Dissipation sum_faces T (p_P - p_Q)^2 with p = 1 / 0 on the x1 faces, loops."""
    m = k.shape[0]
    e = 0.0
    for j in range(m):
        for i in range(m):
            if i + 1 < m:
                t = 2 * k[j, i] * k[j, i + 1] / (k[j, i] + k[j, i + 1])
                e += t * (p[j, i] - p[j, i + 1]) ** 2
            if j + 1 < m:
                t = 2 * k[j, i] * k[j + 1, i] / (k[j, i] + k[j + 1, i])
                e += t * (p[j, i] - p[j + 1, i]) ** 2
        e += 2 * k[j, 0] * (p[j, 0] - 1.0) ** 2
        e += 2 * k[j, m - 1] * (p[j, m - 1] - 0.0) ** 2
    return e


def test_brute_force_energy_matrix():
    rng = np.random.default_rng(4)
    m = 4
    n = m * m
    k = np.exp(rng.standard_normal((m, m)))
    A, b = fv.assemble(k)
    E = lambda v: _energy(k, v.reshape(m, m))
    e0 = E(np.zeros(n))
    Ab = np.zeros((n, n))
    bb = np.zeros(n)
    I = np.eye(n)
    Ei = [E(I[q]) for q in range(n)]
    for q in range(n):
        for r in range(n):
            Ab[q, r] = 0.5 * (E(I[q] + I[r]) - Ei[q] - Ei[r] + e0)
    for q in range(n):
        bb[q] = 0.5 * (Ab[q, q] - Ei[q] + e0)
    assert np.allclose(A.toarray(), Ab, rtol=1e-12, atol=1e-12)
    assert np.allclose(b, bb, rtol=1e-12, atol=1e-12)


def test_outflow_equals_dissipation():
    rng = np.random.default_rng(5)
    m = 12
    k = np.exp(1.5 * rng.standard_normal((m, m)))
    _, _, p, qo, _ = _solve_q(k)
    assert abs(_energy(k, p.reshape(m, m)) - qo) < 1e-12 * qo


def test_direct_solve_against_dense_and_cg():
    rng = np.random.default_rng(6)
    m = 16
    k = np.exp(rng.standard_normal((m, m)))
    A, b = fv.assemble(k)
    pd = np.linalg.solve(A.toarray(), b)
    p = solve.direct_solve(A, b)
    assert np.allclose(p, pd, rtol=0, atol=1e-13)
    m = 48
    k = np.exp(rng.standard_normal((m, m)))
    A, b = fv.assemble(k)
    p = solve.direct_solve(A, b)
    pc, info = spla.cg(A, b, rtol=1e-15, atol=0.0, maxiter=20000)
    qd, qc = qoi.outflow(k, p), qoi.outflow(k, pc)
    assert abs(qd - qc) < 1e-11 * qd
    # one refinement step changes the QoI negligibly
    p0 = solve.direct_solve(A, b, refine=False)
    assert abs(qoi.outflow(k, p0) - qd) < 1e-13 * qd


def test_model_problem_1_homogeneous_closed_form_1d_profile():
    # f = 1, p = 0 on the boundary, k = 1: with k depending on nothing, the
    # 2D solution is symmetric under mirroring in both axes and positive.
    m = 8
    k = np.ones((m, m))
    A, b = fv.assemble(k, fv.MP1)
    p = solve.direct_solve(A, b).reshape(m, m)
    assert np.all(p > 0)
    assert np.allclose(p, p[::-1, :]) and np.allclose(p, p[:, ::-1]) and np.allclose(p, p.T)
    # total source = total boundary flux
    flux = 2 * (p[:, 0].sum() + p[:, -1].sum() + p[0, :].sum() + p[-1, :].sum())
    assert abs(flux - 1.0) < 1e-13
