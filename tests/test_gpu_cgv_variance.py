"""The variance experiment of Section 4.2 on the GPU, through the C ABI: the
stationary log-normal field with the 1-norm exponential covariance (lambda 0.3,
sigma^2 1, no layers), Model Problem 2, plain and Coarse Grid Variates level
differences Y_l on fine grids from h_l = 1/8, in 2-D and 3-D.

Per sample, Q_f, Q_c and Y match the oracle (1e-10 relative to Q_f); the
sample variance of Y over the first samples equals the oracle's variance of the
same samples; and averaging over the 2^d sub-lattices lowers the variance of Y
by more than an order of magnitude at h_l = 1/8.  The paper reports factors of
about 200 (2-D) and 100 (3-D) there, read off its figures, whose data are not
given: that value is not pinned, only the direction and size class.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import workloads as W  # noqa: E402
from oracle import mlmc as omlmc  # noqa: E402

QTOL = 1e-10
DEV = "cuda:0"


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


def f64(*shape):
    return torch.empty(*shape, dtype=torch.float64, device=DEV)


def level_run(lib, ctx, model, level, m, first, n, cgv):
    qf, qc, y = f64(n), f64(n), f64(n)
    sums = lib.mlmc_level_run(ctx, model, level, m, first, n, cgv,
                              lib.mlmc_solver_opts_default(), q_f=qf, q_c=qc, y=y)
    torch.cuda.synchronize()
    return sums, qf.cpu().numpy(), qc.cpu().numpy(), y.cpu().numpy()


def sample_var(y):
    return float(np.var(y, ddof=1))


@pytest.mark.parametrize("dim,m", [(2, 8), (2, 16), (3, 8)])
@pytest.mark.parametrize("cgv", [False, True])
def test_stationary_level_run_matches_oracle(lib, ctx, dim, m, cgv):
    model = W.STATIONARY_1NORM if dim == 2 else W.STATIONARY_1NORM_3D
    n = 6
    print("stationary level run dim=%d m=%d cgv=%d" % (dim, m, cgv), flush=True)
    sums, qf, qc, y = level_run(lib, ctx, model, 1, m, 5, n, cgv)
    assert sums.n == n and sums.n_failed == 0
    for s in range(n):
        ref = omlmc.level_sample(model, 1, 5 + s, m, cgv=cgv)
        assert abs(qf[s] - ref["Q_f"]) <= QTOL * ref["Q_f"], (s, qf[s], ref["Q_f"])
        assert abs(qc[s] - ref["Q_c"]) <= QTOL * ref["Q_c"], (s, qc[s], ref["Q_c"])
        assert abs(y[s] - ref["Y"]) <= QTOL * ref["Q_f"], (s, y[s], ref["Y"])


@pytest.mark.parametrize("dim,n", [(2, 64), (3, 24)])
def test_variance_of_y_matches_oracle(lib, ctx, dim, n):
    """The sample variances of plain and CGV Y at h_l = 1/8 over the same samples
    as the oracle; the GPU's Y differ from the oracle's by at most 1e-10 Q_f, so
    the variances agree far below their statistical error."""
    model = W.STATIONARY_1NORM if dim == 2 else W.STATIONARY_1NORM_3D
    m = 8
    print("variance of Y dim=%d n=%d" % (dim, n), flush=True)
    for cgv in (False, True):
        _, qf, _, y = level_run(lib, ctx, model, 1, m, 0, n, cgv)
        ref = np.array([omlmc.level_sample(model, 1, s, m, cgv=cgv)["Y"] for s in range(n)])
        assert np.max(np.abs(y - ref)) <= QTOL * np.max(qf)
        v, vr = sample_var(y), sample_var(ref)
        assert abs(v - vr) <= 1e-6 * vr, (cgv, v, vr)


@pytest.mark.parametrize("dim,n", [(2, 4096), (3, 2048)])
def test_cgv_lowers_variance_at_coarsest_level(lib, ctx, dim, n):
    model = W.STATIONARY_1NORM if dim == 2 else W.STATIONARY_1NORM_3D
    m = 8
    print("CGV variance reduction dim=%d n=%d" % (dim, n), flush=True)
    sp = lib.mlmc_level_run(ctx, model, 1, m, 0, n, False, lib.mlmc_solver_opts_default())
    sc = lib.mlmc_level_run(ctx, model, 1, m, 0, n, True, lib.mlmc_solver_opts_default())
    assert sp.n_failed == 0 and sc.n_failed == 0
    # the same fine samples on both runs
    assert sp.sum_qf == sc.sum_qf

    def var(s):
        mean = s.sum_y / s.n
        return (s.sum_y2 - s.n * mean * mean) / (s.n - 1)

    ratio = var(sp) / var(sc)
    print("variance ratio plain / CGV at h = 1/8 (%d-D): %.1f" % (dim, ratio), flush=True)
    assert ratio > 10.0
    # both estimators are unbiased for E[Q_l - Q_{l-1}]: their means agree
    # within the statistical error of the difference
    se = np.sqrt(var(sp) / n + var(sc) / n)
    assert abs(sp.sum_y / n - sc.sum_y / n) < 5 * se
