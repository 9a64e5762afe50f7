"""Multilevel and Coarse Grid Variates estimators (oracle side).

* eq. (3.5)/(3.6): E[Q_L] = E[Q_0] + sum_l E[Q_l - Q_{l-1}], each term estimated
  by an independent Monte Carlo mean over N_l samples; Q_{-1} = 0, and both
  terms of a difference come from the same omega (Section 3.2).
* eq. (3.7): MSE = sum_l V[Q_l - Q_{l-1}] / N_l + bias^2; the first sum is
  estimated with the unbiased sample variances.
* eq. (4.1): Q^cgv_{l-1} = 2^-d sum_j Q(k_l^(j)) over the 2^d sub-lattices of
  the fine sample; eq. (4.2): Y^cgv = mean of Q_l - Q^cgv_{l-1} (level l >= 1).

Grid sizes: level l uses m_l cells per direction with m_l = 2 m_{l-1}
(eq. (3.4) with s = 2, as Section 4.1 requires).
Level l draws from random streams with counter word c2 = l, so the levels
are independent, as eq. (3.7) assumes.
"""
import numpy as np

from . import field, fv, qoi, solve


def solve_qoi(k, bc=fv.MP2):
    """Exact discrete QoI for one permeability sample: Model Problem 2, the
    outflow and the inflow; Model Problem 1, M^(1) (box mean of the pressure)
    and None."""
    A, b = fv.assemble(k, bc)
    p = solve.direct_solve(A, b)
    if bc == fv.MP1:
        return qoi.box_average(p.reshape(k.shape)), None
    return qoi.outflow(k, p), qoi.inflow(k, p)


def problem_of(model):
    """Boundary value problem of a model record: problem 1 = Model Problem 1,
    anything else (default 0) = Model Problem 2."""
    return fv.MP1 if getattr(model, "problem", 0) == 1 else fv.MP2


def level_sample(model, level, sample, m_fine, cgv=False, lam_eig=None):
    """One term of eq. (3.6) (or eq. (4.2) when cgv) for sample `sample` of level `level`.

    Returns dict with Q_f (fine QoI), Q_c (coarse QoI; 0 on level 0), Y = Q_f - Q_c,
    and the individual companion QoIs.
    """
    bc = problem_of(model)
    if level == 0:
        k = field.sample_k(model, level, sample, m_fine, lam_eig=lam_eig)
        qf, _ = solve_qoi(k, bc)
        return {"Q_f": qf, "Q_c": 0.0, "Y": qf, "companions": []}
    if cgv:
        k = field.sample_k(model, level, sample, m_fine, lam_eig=lam_eig)
        qf, _ = solve_qoi(k, bc)
        comps = [solve_qoi(kc, bc)[0] for kc in field.cgv_sublattices(k)]
        qc = sum(comps) / len(comps)
    else:
        k, kc = field.sample_k(model, level, sample, m_fine, lam_eig=lam_eig, with_coarse=True)
        qf, _ = solve_qoi(k, bc)
        comps = [solve_qoi(kc, bc)[0]]
        qc = comps[0]
    return {"Q_f": qf, "Q_c": qc, "Y": qf - qc, "companions": comps}


def level_sums(Y, Qf, Qc):
    """Per-level sums N, sum Y, sum Y^2, sum Q_f, sum Q_c (summed in index order)."""
    Y = np.asarray(Y, dtype=np.float64)
    return {"n": len(Y), "sum_y": float(np.sum(Y)), "sum_y2": float(np.sum(Y * Y)),
            "sum_qf": float(np.sum(Qf)), "sum_qc": float(np.sum(Qc))}


def estimate(sums):
    """Estimator eq. (3.6) and the statistical part of eq. (3.7)."""
    q = 0.0
    var_sum = 0.0
    per_level = []
    for s in sums:
        n = s["n"]
        mean = s["sum_y"] / n
        var = (s["sum_y2"] - n * mean * mean) / (n - 1) if n > 1 else float("nan")
        q += mean
        var_sum += var / n
        per_level.append({"mean_y": mean, "var_y": var})
    return {"estimate": q, "variance_of_estimate": var_sum,
            "std_error": float(np.sqrt(var_sum)), "levels": per_level}
