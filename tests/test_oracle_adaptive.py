"""Pins of the oracle's sample-size rule and rate fits (Section 3.2, the
complexity theorem's (M1)-(M3)).

* optimal_samples: the rounded-up N meets the variance constraint
  sum V_l / N_l <= eps^2 / 2, and it is the ceiling of the exact minimiser of
  sum N_l C_l under sum V_l / N_l = eps^2 / 2.  That minimiser is fixed by the
  first-order (KKT) conditions of the problem, checked without the closed form:
  stationarity C_l = mu V_l / N_l^2 with one multiplier mu for every level
  (N_l = sqrt(mu V_l / C_l)), mu found by a scalar root-finder on the
  constraint; and every feasible move away from it costs more.
* fit_rate recovers exact power laws and is the slope of the least squares
  line through (log2 h, log2 value).
* bias_estimate: for differences E[Y_l] = c h_l^alpha the tail beyond L sums
  exactly to the estimate.
"""
import numpy as np
from scipy.optimize import brentq

from oracle import mlmc


def test_optimal_samples_is_the_ceiling_of_the_kkt_point():
    rng = np.random.default_rng(5)
    for _ in range(8):
        L1 = int(rng.integers(2, 7))
        V = np.exp(rng.standard_normal(L1) * 2 - 4)
        C = np.exp(rng.standard_normal(L1) * 2)
        eps = float(10.0 ** rng.uniform(-3, -1.5))
        target = eps ** 2 / 2
        N = mlmc.optimal_samples(V, C, eps)
        assert np.sum(V / N) <= target * (1 + 1e-12)
        # stationarity of the Lagrangian sum N C + mu (sum V / N - target):
        # C_l - mu V_l / N_l^2 = 0, i.e. N_l(mu) = sqrt(mu V_l / C_l); the
        # constraint fixes mu (monotone in mu, so a bracketing root-finder)
        def excess(log_mu):
            return np.sum(V / np.sqrt(np.exp(log_mu) * V / C)) / target - 1.0
        log_mu = brentq(excess, -200.0, 200.0, xtol=1e-14, rtol=1e-15)
        Nstar = np.sqrt(np.exp(log_mu) * V / C)
        assert np.all(N >= Nstar * (1 - 1e-9))
        assert np.all(N < Nstar + 1.0 + 1e-9 * Nstar)
        # every feasible direction away from N* raises the cost: move along
        # random directions u, then rescale all levels back onto the constraint
        base = np.sum(Nstar * C)
        for _ in range(20):
            u = rng.standard_normal(L1) * 0.05
            Nm = Nstar * np.exp(u)
            Nm *= np.sum(V / Nm) / target          # back onto sum V / N = target
            assert abs(np.sum(V / Nm) / target - 1.0) < 1e-12
            assert np.sum(Nm * C) >= base * (1 - 1e-12)


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
