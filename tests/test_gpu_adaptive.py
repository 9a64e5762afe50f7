"""The adaptive MLMC driver on the GPU (Section 3.2: MSE split evenly, sample
sizes minimising the cost for the variance part, levels added while the
estimated bias exceeds eps/sqrt(2)).

* Two-layer piecewise constant model with a horizontal interface: every level
  has E[Q_l] = E[k] = e^(1/2) exactly (closed form, the layers are parallel to
  the flow), so the estimator is unbiased on any hierarchy: the estimate must
  lie within 4.5 standard errors of e^(1/2), the variance part must meet
  eps^2/2 (up to the last re-estimate of V_l), and per-level sums must equal
  those of plain level runs over the same sample numbers.
* The layered correlated model with CGV: converges on the 16^2..512^2
  hierarchy and reports rates with beta > 1 (V[Y_l] decays).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import workloads as W  # noqa: E402
from oracle import mlmc as omlmc  # noqa: E402


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1506_04694_amd as lib
    return lib


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.mlmc_ctx_create(0, torch.cuda.current_stream(0))
    yield c
    lib.mlmc_ctx_destroy(c)


def test_adaptive_unbiased_model(lib, ctx):
    eps = 0.01
    ms = [8, 16, 32, 64, 128, 256]
    print("adaptive PC2 eps=%g" % eps, flush=True)
    opts = lib.mlmc_adaptive_opts_default(eps=eps, n_initial=128)
    r = lib.mlmc_adaptive(ctx, W.PC2, ms, opts, lib.mlmc_solver_opts_default())
    L1 = r.n_levels
    assert 3 <= L1 <= len(ms)
    n = [r.n[l] for l in range(L1)]
    assert all(x >= 128 for x in n)
    # the variance part, with the final variance estimates
    assert r.variance <= eps ** 2 / 2 * 1.25, (r.variance, eps ** 2 / 2)
    # unbiased on every level: the estimate is e^(1/2) up to its statistical error
    assert abs(r.estimate - np.exp(0.5)) < 4.5 * np.sqrt(r.variance), (r.estimate, r.variance)
    # the sample sizes follow the rule for the reported variances and costs
    ref = omlmc.optimal_samples([r.var_y[l] for l in range(L1)], [r.cost[l] for l in range(L1)],
                                eps)
    # (the rule was applied with the estimates of the last round; later samples
    # move them, and samples are never taken back)
    for l in range(L1):
        assert n[l] >= 0.5 * ref[l] and n[l] <= 4.0 * ref[l] + 128, (l, n[l], ref[l])
    # per-level sums are those of plain level runs over samples 0..N_l-1
    for l in (0, L1 - 1):
        s = lib.mlmc_level_run(ctx, W.PC2, l, ms[l], 0, n[l], False,
                               lib.mlmc_solver_opts_default())
        assert s.n == n[l]
        assert abs(s.sum_y - r.sums[l].sum_y) <= 1e-12 * abs(s.sum_y) + 1e-12
        assert abs(s.sum_y2 - r.sums[l].sum_y2) <= 1e-12 * s.sum_y2


def test_adaptive_layered_cgv(lib, ctx):
    eps = 0.05
    ms = [16, 32, 64, 128, 256, 512]
    print("adaptive CE2 CGV eps=%g" % eps, flush=True)
    opts = lib.mlmc_adaptive_opts_default(eps=eps, n_initial=64, cgv=1)
    r = lib.mlmc_adaptive(ctx, W.CE2, ms, opts, lib.mlmc_solver_opts_default())
    print("levels %d bias %.3e alpha %.2f means %s n %s" % (
        r.n_levels, r.bias, r.alpha, [round(r.mean_y[l], 5) for l in range(r.n_levels)],
        [r.n[l] for l in range(r.n_levels)]), flush=True)
    assert r.converged == 1
    assert r.variance <= eps ** 2 / 2 * 1.25
    assert r.bias <= eps / np.sqrt(2)
    if r.n_levels >= 3:
        assert r.beta > 1.0


def test_adaptive_refuses_bad_hierarchy(lib, ctx):
    opts = lib.mlmc_adaptive_opts_default()
    with pytest.raises(lib.MlmcError):
        lib.mlmc_adaptive(ctx, W.PC2, [8, 12, 24], opts, lib.mlmc_solver_opts_default())


@pytest.mark.parametrize("key", ["2d_mp2", "2d_mp1", "3d_mp2"])
def test_reference_solution_rates_inputs(lib, ctx, key):
    """The reference-solution rates of the bench (Section 3.4) solve the same
    sample on every grid: for the paper's three piecewise constant layers the
    level-0 stream fixes the lines and the constants independently of the grid.
    Samples 0-2 on each grid (and on the 3-D reference grid's half) equal the
    oracle's exact discrete QoI of that sample on that grid (1e-10), and the
    paired weak errors against the reference grid shrink as h does."""
    spec = {k: (mdl, grids, ref, n) for k, mdl, grids, ref, n in W.RATES_REFERENCE}
    mdl, grids, ref, _ = spec[key]
    n = 16
    opts = lib.mlmc_solver_opts_default()
    q = {}
    for m in grids + [ref]:
        print("reference rates %s m=%d" % (key, m), flush=True)
        qt = torch.empty(n, dtype=torch.float64, device="cuda")
        sums = lib.mlmc_level_run(ctx, mdl, 0, m, 0, n, False, opts, q_f=qt)
        assert sums.n_failed == 0
        q[m] = qt.cpu().numpy()
    check = [g for g in grids if g <= (32 if mdl.dim == 3 else 256)][:3]
    for m in check:
        for s in range(3):
            ref_q = omlmc.level_sample(mdl, 0, s, m)["Q_f"]
            assert abs(q[m][s] - ref_q) <= 1e-10 * abs(ref_q), (m, s, q[m][s], ref_q)
    err = [abs(np.mean(q[m] - q[ref])) for m in grids]
    assert err[-1] < err[0], err
