"""Pins of the oracle's conjugate gradient solve (the exact discrete solution
on the 3-D grids 64^3 and 128^3, where the direct factor does not fit).

* against the direct sparse solve on random log-normal 2-D and 3-D
  permeabilities small enough for it (solution and outflow);
* against the closed forms of the 3-D system at 64^3, a size only the CG
  path solves: homogeneous k (linear pressure, Q = k), layers parallel to the
  flow (Q = mean of k over the rows), layers across the flow (Q = 1 / the
  series resistance with half-cell Dirichlet faces);
* the returned true residual is recomputed from x and sits at the FP64
  rounding level; a sample of the served 3-D model at 64^3 conserves flux
  (Q_in = Q_out, which only the exact discrete solution does);
* the solver choice of the oracle's level samples: direct up to 32^3 in 3-D,
  CG above.
"""
import numpy as np
import pytest

import workloads as W
from oracle import field, fv, mlmc, qoi, solve


@pytest.mark.parametrize("shape", [(24, 24), (8, 8, 8), (16, 16, 16)])
def test_cg_matches_direct_solve(shape):
    rng = np.random.default_rng(len(shape) * 100 + shape[0])
    k = np.exp(1.5 * rng.standard_normal(shape))
    A, b = fv.assemble(k)
    pd = solve.direct_solve(A, b)
    pc, its, relres = solve.cg_solve(A, b)
    assert its > 1
    assert relres < 1e-13
    assert np.linalg.norm(pc - pd) <= 1e-11 * np.linalg.norm(pd)
    qd, qc = qoi.outflow(k, pd), qoi.outflow(k, pc)
    assert abs(qc - qd) <= 1e-12 * qd


def _cg_q(k):
    A, b = fv.assemble(k)
    p, its, relres = solve.cg_solve(A, b)
    assert relres < 1e-13
    return qoi.outflow(k, p), qoi.inflow(k, p), p


def test_cg_homogeneous_3d_closed_form():
    m = 64
    k = np.full((m, m, m), 3.7)
    q_out, q_in, p = _cg_q(k)
    assert abs(q_out - 3.7) <= 1e-12 * 3.7
    assert abs(q_in - 3.7) <= 1e-12 * 3.7
    x1 = (np.arange(m) + 0.5) / m
    lin = np.broadcast_to((1.0 - x1)[None, None, :], (m, m, m)).ravel()
    assert np.max(np.abs(p - lin)) <= 1e-12


def test_cg_parallel_and_series_layers_3d():
    m = 64
    rng = np.random.default_rng(64)
    kj = np.exp(1.2 * rng.standard_normal(m))
    k = np.broadcast_to(kj[None, :, None], (m, m, m)).copy()      # depends on x2 only
    q_out, q_in, _ = _cg_q(k)
    assert abs(q_out - kj.mean()) <= 1e-12 * kj.mean()
    assert abs(q_in - q_out) <= 1e-12 * q_out
    ki = np.exp(1.2 * rng.standard_normal(m))
    k = np.broadcast_to(ki[None, None, :], (m, m, m)).copy()      # depends on x1 only
    q_out, _, _ = _cg_q(k)
    h = 1.0 / m
    res = 0.5 * h / ki[0] + 0.5 * h / ki[-1] + sum(h / fv.harmonic(ki[i], ki[i + 1])
                                                   for i in range(m - 1))
    assert abs(q_out - 1.0 / res) <= 1e-12 / res


def test_cg_served_model_sample_conserves_flux():
    """A sample of the served 3-D layered model at 64^3: the recomputed true
    residual is at rounding level and inflow equals outflow."""
    k = field.sample_k(W.TILTED3, 1, 0, 64)
    q_out, q_in, _ = _cg_q(k)
    assert abs(q_in - q_out) <= 1e-11 * q_out


def test_cg_refuses_to_return_unconverged():
    k = np.exp(np.random.default_rng(1).standard_normal((8, 8, 8)))
    A, b = fv.assemble(k)
    with pytest.raises(RuntimeError):
        solve.cg_solve(A, b, maxit=3)


def test_solver_choice_of_level_samples():
    assert not solve.uses_cg(3, 32) and solve.uses_cg(3, 64) and solve.uses_cg(3, 128)
    assert not solve.uses_cg(2, 1024)
    # both solvers give the same level sample where both apply
    a = mlmc.level_sample(W.TILTED3, 1, 5, 16, solver="direct")
    b = mlmc.level_sample(W.TILTED3, 1, 5, 16, solver="cg")
    assert abs(a["Q_f"] - b["Q_f"]) <= 1e-12 * a["Q_f"]
    assert abs(a["Q_c"] - b["Q_c"]) <= 1e-12 * a["Q_c"]
