"""Pins of the oracle's sample-size rule and rate fits (Section 3.2, the
complexity theorem's (M1)-(M3)).

* optimal_samples: the rounded-up N meets the variance constraint
  sum V_l / N_l <= eps^2 / 2 (with equality before rounding), and its cost is
  within rounding of the least cost found by a general-purpose constrained
  minimiser (scipy SLSQP) started from a different point.
* fit_rate recovers exact power laws and is the slope of the least squares
  line through (log2 h, log2 value).
* bias_estimate: for differences E[Y_l] = c h_l^alpha the tail beyond L sums
  exactly to the estimate.
"""
import numpy as np
from scipy.optimize import minimize

from oracle import mlmc


def test_optimal_samples_meets_constraint_at_least_cost():
    rng = np.random.default_rng(5)
    for _ in range(5):
        L1 = rng.integers(2, 6)
        V = np.exp(rng.standard_normal(L1) * 2 - 4)
        C = np.exp(rng.standard_normal(L1) * 2)
        eps = 0.01
        N = mlmc.optimal_samples(V, C, eps)
        assert np.sum(V / N) <= eps ** 2 / 2 * (1 + 1e-12)
        # continuous minimiser by SLSQP on log N from a far start
        target = eps ** 2 / 2

        scale = np.sum(N * C)

        def cost(u):
            return np.sum(np.exp(u) * C) / scale

        cons = {"type": "eq", "fun": lambda u: (np.sum(V / np.exp(u)) - target) / target}
        # feasible start: every level takes an equal share of the variance budget
        u0 = np.log(2.0 * L1 * V / eps ** 2)
        res = minimize(cost, u0, constraints=[cons], method="SLSQP",
                       options={"ftol": 1e-14, "maxiter": 500})
        assert res.success
        # N costs at most the rounding (one sample per level) above the minimum
        assert 1.0 <= res.fun * (1 + 1e-6) + np.sum(C) / scale
        np.testing.assert_allclose(np.exp(res.x), N.astype(float), rtol=5e-3, atol=1.0)


def test_fit_rate_recovers_power_laws():
    h = 1.0 / np.array([8, 16, 32, 64])
    assert abs(mlmc.fit_rate(h, 3.0 * h ** 2) - 2.0) < 1e-12
    assert abs(mlmc.fit_rate(h, 0.5 * h ** -2.3) + 2.3) < 1e-12
    rng = np.random.default_rng(1)
    v = np.exp(rng.standard_normal(4))
    x, y = np.log2(h), np.log2(v)
    slope = np.polyfit(x, y, 1)[0]
    assert abs(mlmc.fit_rate(h, v) - slope) < 1e-12


def test_bias_estimate_is_the_geometric_tail():
    alpha, c, L = 1.3, 0.7, 5
    h = lambda l: 2.0 ** -(l + 3)            # noqa: E731
    tail = sum(c * h(l) ** alpha for l in range(L + 1, L + 200))
    mean_y_L = c * h(L) ** alpha
    assert abs(mlmc.bias_estimate(mean_y_L, alpha) - tail) < 1e-12 * tail
