"""GPU parity of layered correlated models whose layers have different
covariances (Section 3.4's three layers between two random lines: bottom and
top lambda 0.3, middle lambda 0.1, means 0 / 4 / 0), against the CPU oracle
through the C ABI: the composite fields (1e-11 in log k, including the plain
coarse companion), the smallest common embedding size, level runs with both
model problems and with CGV (QoI 1e-10 relative), and a 3-D two-layer model
with different correlation lengths.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import workloads as W  # noqa: E402
from oracle import field as ofield  # noqa: E402
from oracle import mlmc as omlmc  # noqa: E402

QTOL = 1e-10
DEV = "cuda:0"
MODEL = W.PAPER3_CE
MODEL3D = W.TILTED3.with_(lam=(0.2, 0.1, 0.2, 0.2))


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


@pytest.mark.parametrize("model,m,level", [("paper3", 32, 1), ("paper3", 64, 2),
                                           ("paper3", 256, 1), ("tilted3d", 16, 1)])
def test_field_matches_oracle(lib, ctx, model, m, level):
    mdl = MODEL if model == "paper3" else MODEL3D
    d = mdl.dim
    batch = 3
    print("field %s m=%d level=%d" % (model, m, level), flush=True)
    k = f64(batch, *(m,) * d)
    kc = f64(batch, *(m // 2,) * d)
    lib.mlmc_sample_field(ctx, lib.model_for_grid(mdl, m), m, level, 5, batch, k, kc)
    torch.cuda.synchronize()
    k, kc = k.cpu().numpy(), kc.cpu().numpy()
    for s in range(batch):
        ref, refc = ofield.sample_k(mdl, level, 5 + s, m, with_coarse=True)
        assert np.max(np.abs(np.log(k[s]) - np.log(ref))) < 1e-11
        assert np.max(np.abs(np.log(kc[s]) - np.log(refc))) < 1e-11


@pytest.mark.parametrize("m", [32, 64])
def test_min_embedding_covers_every_layer(lib, ctx, m):
    got = lib.mlmc_ce_min_embedding(ctx, lib.make_model(MODEL), m)
    ref = None
    for n in ofield.smooth_sizes(2 * m, 12 * m):
        try:
            for s2, lam, _ in ofield.ce_pairs(MODEL):
                ofield.ce_eigenvalues(n, m, s2, lam, MODEL.norm_r)
        except ValueError:
            continue
        ref = n
        break
    assert got == ref


@pytest.mark.parametrize("problem,m,cgv", [(0, 32, False), (0, 32, True), (1, 32, False),
                                           (1, 64, True)])
def test_level_run_matches_oracle(lib, ctx, problem, m, cgv):
    mdl = MODEL.with_(problem=problem)
    n = 4
    print("three-layer level run problem=%d m=%d cgv=%d" % (problem, m, cgv), flush=True)
    qf, qc, y = f64(n), f64(n), f64(n)
    sums = lib.mlmc_level_run(ctx, mdl, 1, m, 3, n, cgv, lib.mlmc_solver_opts_default(),
                              q_f=qf, q_c=qc, y=y)
    torch.cuda.synchronize()
    assert sums.n == n and sums.n_failed == 0
    qf, qc = qf.cpu().numpy(), qc.cpu().numpy()
    for s in range(n):
        ref = omlmc.level_sample(mdl, 1, 3 + s, m, cgv=cgv)
        assert abs(qf[s] - ref["Q_f"]) <= QTOL * ref["Q_f"], (s, qf[s], ref["Q_f"])
        assert abs(qc[s] - ref["Q_c"]) <= QTOL * ref["Q_c"], (s, qc[s], ref["Q_c"])


def test_level_run_3d_matches_oracle(lib, ctx):
    m, n = 16, 3
    print("3-D two-covariance level run m=%d" % m, flush=True)
    qf = f64(n)
    sums = lib.mlmc_level_run(ctx, MODEL3D, 1, m, 0, n, False, lib.mlmc_solver_opts_default(),
                              q_f=qf)
    torch.cuda.synchronize()
    assert sums.n_failed == 0
    qf = qf.cpu().numpy()
    for s in range(n):
        ref = omlmc.level_sample(MODEL3D, 1, s, m)
        assert abs(qf[s] - ref["Q_f"]) <= QTOL * ref["Q_f"], (s, qf[s], ref["Q_f"])
