"""Pins of the oracle's three-layer correlated model (Section 3.4): three layers
between two random lines, bottom and top with mean 0, lambda 0.3, middle with
mean 4, lambda 0.1, all sigma^2 = 1, 2-norm exponential covariance, no
correlation across layers.

* Layers share an embedding sample only when their covariance agrees: bottom
  and top take Re and Im of one sample, the middle layer its own.
* Each layer's field has its own covariance sigma^2 exp(-d / lambda_l):
  empirical covariances at lags 0, h, 3h, 6h along both axes within 4.5
  standard errors, over independent samples.
* Different layers are uncorrelated (empirical cross-covariance at lag 0 and
  h within 4.5 standard errors of 0), for the pair that shares an embedding
  sample and for the pairs that do not.
* The composite sample uses the middle layer's mean and field on the middle
  layer's cells only.
"""
import numpy as np

import workloads as W
from oracle import field, geometry

MODEL = W.PAPER3_CE


def test_pairs_follow_the_covariances():
    assert field.ce_pairs(MODEL) == [[1.0, 0.3, [0, 2]], [1.0, 0.1, [1, None]]]
    same = MODEL.with_(lam=(0.3,) * 4, mu=(0.0,) * 4)
    assert field.ce_pairs(same) == [[1.0, 0.3, [0, 1]], [1.0, 0.3, [2, None]]]


def lag_products(a, b, lag, axis):
    sl_a = [slice(None)] * 2
    sl_b = [slice(None)] * 2
    m = a.shape[0]
    sl_a[axis] = slice(0, m - lag)
    sl_b[axis] = slice(lag, m)
    return (a[tuple(sl_a)] * b[tuple(sl_b)]).mean()


def test_layer_covariances_and_independence():
    m, n_samples = 32, 400
    lam = [0.3, 0.1, 0.3]
    eig = {}
    for p, (s2, lm, _) in enumerate(field.ce_pairs(MODEL)):
        eig[p] = field.ce_eigenvalues(MODEL.n_ce[m], m, s2, lm, 2)
    # one statistic per sample: products at one point pair away from the
    # torus wrap (rows/columns 0..m-1 of the embedding are ordinary grid points)
    stats = {}
    for s in range(n_samples):
        g = field.gaussian_layers(MODEL, 0, s, m)
        for l in range(3):
            for lag in (0, 1, 3, 6):
                for axis in (0, 1):
                    stats.setdefault(("auto", l, lag, axis), []).append(
                        lag_products(g[l], g[l], lag, axis))
        for a, b in ((0, 1), (0, 2), (1, 2)):
            for lag in (0, 1):
                stats.setdefault(("cross", a, b, lag), []).append(lag_products(g[a], g[b], lag, 0))
    for key, vals in stats.items():
        vals = np.asarray(vals)
        mean, se = vals.mean(), vals.std(ddof=1) / np.sqrt(len(vals))
        if key[0] == "auto":
            _, l, lag, _ = key
            expect = np.exp(-lag / m / lam[l])
        else:
            expect = 0.0
        assert abs(mean - expect) < 4.5 * se + 1e-3, (key, mean, expect, se)


def test_composite_uses_each_layers_mean_and_field():
    m = 32
    for s in range(3):
        k = field.sample_k(MODEL, 1, s, m)
        g = field.gaussian_layers(MODEL, 1, s, m)
        lid = geometry.layer_ids(MODEL, 1, s, m)
        assert set(np.unique(lid)) == {0, 1, 2}
        for l in range(3):
            np.testing.assert_allclose(np.log(k[lid == l]), MODEL.mu[l] + g[l][lid == l],
                                       rtol=0, atol=1e-13)
