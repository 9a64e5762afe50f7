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


def solve_qoi(k, bc=fv.MP2, solver="auto"):
    """Exact discrete QoI for one permeability sample: Model Problem 2, the
    outflow and the inflow; Model Problem 1, M^(1) (box mean of the pressure)
    and None.  solver: "direct", "cg" or "auto" (direct solve except for 3-D
    grids above 32^3, which take the conjugate gradient solve to 1e-14)."""
    A, b = fv.assemble(k, bc)
    p = solve.solve(A, b, k.ndim, k.shape[0], solver)
    if bc == fv.MP1:
        return qoi.box_average(p.reshape(k.shape)), None
    return qoi.outflow(k, p), qoi.inflow(k, p)


def problem_of(model):
    """Boundary value problem of a model record: problem 1 = Model Problem 1,
    anything else (default 0) = Model Problem 2."""
    return fv.MP1 if getattr(model, "problem", 0) == 1 else fv.MP2


def level_sample(model, level, sample, m_fine, cgv=False, lam_eig=None, solver="auto"):
    """One term of eq. (3.6) (or eq. (4.2) when cgv) for sample `sample` of level `level`.

    Returns dict with Q_f (fine QoI), Q_c (coarse QoI; 0 on level 0), Y = Q_f - Q_c,
    and the individual companion QoIs.
    """
    bc = problem_of(model)
    if level == 0:
        k = field.sample_k(model, level, sample, m_fine, lam_eig=lam_eig)
        qf, _ = solve_qoi(k, bc, solver)
        return {"Q_f": qf, "Q_c": 0.0, "Y": qf, "companions": []}
    if cgv:
        k = field.sample_k(model, level, sample, m_fine, lam_eig=lam_eig)
        qf, _ = solve_qoi(k, bc, solver)
        comps = [solve_qoi(kc, bc, solver)[0] for kc in field.cgv_sublattices(k)]
        qc = sum(comps) / len(comps)
    else:
        k, kc = field.sample_k(model, level, sample, m_fine, lam_eig=lam_eig, with_coarse=True)
        qf, _ = solve_qoi(k, bc, solver)
        comps = [solve_qoi(kc, bc, solver)[0]]
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


# ------------------------------------------------------- choosing L and N_l
# Section 3.2 splits the mean square error eq. (3.7) evenly: the variance
# sum_l V_l / N_l and the squared bias (E[Q_L - Q])^2 each get eps^2 / 2, and
# N_l is chosen so that the variance part is reached at the least total cost
# sum_l N_l C_l.  With a Lagrange multiplier for the constraint
# sum_l V_l / N_l = eps^2 / 2 the minimiser over real N_l is
#     N_l = 2 eps^-2 sqrt(V_l / C_l) sum_k sqrt(V_k C_k),
# rounded up here.  The rates of the complexity theorem (M1)-(M3),
# |E[Y_l]| ~ h_l^alpha, V[Y_l] ~ h_l^beta, C_l ~ h_l^-gamma, are the least
# squares slopes of log2 of the measured values against log2(1/h_l) over the
# levels l >= 1 (level 0 has no difference).  With h_l = h_{l-1} / 2 the
# remaining bias of the finest level L is estimated as |E[Y_L]| / (2^alpha - 1)
# (the geometric tail of the differences beyond L).

def optimal_samples(var, cost, eps):
    """Rounded-up minimiser of sum N_l C_l subject to sum V_l / N_l = eps^2 / 2."""
    var = np.asarray(var, dtype=np.float64)
    cost = np.asarray(cost, dtype=np.float64)
    total = np.sum(np.sqrt(var * cost))
    return np.ceil(2.0 / eps ** 2 * np.sqrt(var / cost) * total).astype(np.int64)


def fit_rate(h, values):
    """Least squares slope p of log2|value| = c + p log2(h) (values ~ h^p)."""
    x = np.log2(np.asarray(h, dtype=np.float64))
    y = np.log2(np.abs(np.asarray(values, dtype=np.float64)))
    A = np.stack([x, np.ones_like(x)], axis=1)
    return float(np.linalg.lstsq(A, y, rcond=None)[0][0])


def bias_estimate(mean_y_finest, alpha):
    """Bias of the finest level from its mean difference and the rate alpha."""
    return abs(mean_y_finest) / (2.0 ** alpha - 1.0)
