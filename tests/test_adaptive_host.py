"""Host arithmetic of the adaptive estimator through the C ABI (no GPU needed):
the sample-size rule and the rate fits against the oracle's (which are pinned
in test_oracle_adaptive.py), and argument checks."""
import numpy as np
import pytest

from oracle import mlmc as omlmc


@pytest.fixture(scope="module")
def lib():
    try:
        import paper_1506_04694_amd as lib
    except ImportError as e:
        pytest.skip("library not built: %s" % e)
    return lib


def test_optimal_samples_matches_oracle(lib):
    rng = np.random.default_rng(9)
    for _ in range(20):
        L1 = int(rng.integers(1, 8))
        V = np.exp(rng.standard_normal(L1) * 3 - 5)
        C = np.exp(rng.standard_normal(L1) * 2 - 6)
        eps = float(np.exp(rng.uniform(np.log(1e-4), np.log(1e-1))))
        got = np.array(lib.mlmc_optimal_samples(V, C, eps))
        ref = omlmc.optimal_samples(V, C, eps)
        # identical up to the rounding order of the sum (ceil may move by one)
        assert np.all(np.abs(got - ref) <= 1), (got, ref)


def test_optimal_samples_refuses_bad_input(lib):
    for V, C, eps in (([1.0], [0.0], 0.1), ([-1.0], [1.0], 0.1), ([1.0], [1.0], 0.0),
                      ([np.nan], [1.0], 0.1)):
        with pytest.raises(lib.MlmcError):
            lib.mlmc_optimal_samples(V, C, eps)


def sums_for(lib, ys):
    out = []
    for y in ys:
        s = lib.mlmc_level_sums()
        s.n = len(y)
        s.sum_y = float(np.sum(y))
        s.sum_y2 = float(np.sum(y * y))
        out.append(s)
    return out


def test_rates_match_oracle_fits(lib):
    rng = np.random.default_rng(2)
    m = [8, 16, 32, 64, 128]
    ys = [rng.standard_normal(200) * (0.3 * 2.0 ** -l) + 0.05 * 1.7 ** -l for l in range(5)]
    cost = [1e-4 * 3.9 ** l for l in range(5)]
    a, b, g = lib.mlmc_rates(sums_for(lib, ys), cost, m)
    h = 1.0 / np.array(m[1:])
    sums = omlmc.estimate([omlmc.level_sums(y, y, np.zeros_like(y)) for y in ys])["levels"]
    mean = [lv["mean_y"] for lv in sums[1:]]
    var = [lv["var_y"] for lv in sums[1:]]
    assert abs(a - omlmc.fit_rate(h, mean)) < 1e-10
    assert abs(b - omlmc.fit_rate(h, var)) < 1e-10
    assert abs(g + omlmc.fit_rate(h, cost[1:])) < 1e-10
    with pytest.raises(lib.MlmcError):
        lib.mlmc_rates(sums_for(lib, ys[:2]), cost[:2], m[:2])
