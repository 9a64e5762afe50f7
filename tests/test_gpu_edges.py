"""Degenerate calls through the C ABI on the GPU: empty batches leave their
outputs untouched and return MLMC_OK on every entry point (2-D and 3-D), a
level run of no samples adds nothing to the sums, all-levels runs accept
levels without samples, a server started and stopped without requests
shuts down cleanly, and a solve after a level run (which skips the true
residual) still reports it."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import workloads as W  # noqa: E402

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


def full(shape, v, dtype=torch.float64):
    return torch.full(shape, v, dtype=dtype, device=DEV)


@pytest.mark.parametrize("d", [2, 3])
def test_empty_batches(lib, ctx, d):
    m = 8
    cells = m ** d
    k, T, tb, b = full((1, cells), 7.0), full((1, d * cells), 7.0), full((1, d * m ** (d - 1)), 7.0), \
        full((1, cells), 7.0)
    p, q = full((1, cells), 7.0), full((1,), 7.0)
    st, it, rr = full((1,), 7, torch.int32), full((1,), 7, torch.int32), full((1,), 7.0)
    model = W.CE2 if d == 2 else W.TILTED3
    lib.mlmc_sample_field(ctx, lib.model_for_grid(model, m), m, 0, 0, 0, k)
    lib.mlmc_assemble(ctx, d, m, 0, k, T, tb, b)
    lib.mlmc_assemble_problem(ctx, 1, d, m, 0, k, T, tb, b)
    lib.mlmc_solve(ctx, d, m, 0, T, tb, b, p, lib.mlmc_solver_opts_default(), st, it, rr)
    lib.mlmc_qoi_outflow(ctx, d, m, 0, k, p, q)
    lib.mlmc_qoi_box_mean(ctx, d, m, 0, p, 0.25, 0.75, q)
    lib.mlmc_cgv_extract(ctx, d, m, 0, k, full((1, 2 ** d * (m // 2) ** d), 7.0))
    torch.cuda.synchronize()
    for t in (k, T, tb, b, p, q, rr):
        assert torch.all(t == 7.0)
    assert torch.all(st == 7) and torch.all(it == 7)


def test_level_runs_without_samples(lib, ctx):
    opts = lib.mlmc_solver_opts_default()
    s = lib.mlmc_level_run(ctx, W.CE2, 1, 32, 0, 0, False, opts)
    assert s.n == 0 and s.sum_y == 0.0 and s.sum_y2 == 0.0
    sums = lib.mlmc_run_levels(ctx, W.CE2, [16, 32, 64], [0, 0, 0], [4, 0, 2], False, opts)
    assert sums[1].n == 0 and sums[0].n == 4 and sums[2].n == 2
    ref = lib.mlmc_level_run(ctx, W.CE2, 2, 64, 0, 2, False, opts)
    assert sums[2].sum_y == ref.sum_y


def test_server_without_requests(lib):
    opts = lib.serve_opts_for_models([(W.CE2, [32])])
    srv = lib.mlmc_serve_start_models([W.CE2], opts)
    res, _ = lib.mlmc_serve_poll(srv)
    assert res == []
    lib.mlmc_serve_stop(srv)


@pytest.mark.parametrize("d,m", [(2, 32), (2, 128), (3, 16)])
def test_solve_reports_true_residual_after_level_run(lib, ctx, d, m):
    """Level runs skip the end-of-solve true residual (their samples' status
    comes from the recursive residual); a solve on the same context afterwards
    still reports ||b - A x|| / ||b||, recomputed here with the oracle's matrix."""
    from oracle import fv as ofv
    print("true residual after a level run: d=%d m=%d" % (d, m), flush=True)
    model = W.CE2 if d == 2 else W.TILTED3
    lib.mlmc_level_run(ctx, model, 1, m, 0, 4, False, lib.mlmc_solver_opts_default())
    rng = np.random.default_rng(50 + m)
    batch = 2
    kh = np.exp(rng.standard_normal((batch,) + (m,) * d))
    k = torch.from_numpy(kh).to(DEV)
    cells = m ** d
    T = torch.empty((batch, d * cells), dtype=torch.float64, device=DEV)
    tb = torch.empty((batch, d * m ** (d - 1)), dtype=torch.float64, device=DEV)
    b = torch.empty((batch, cells), dtype=torch.float64, device=DEV)
    p = torch.empty((batch, cells), dtype=torch.float64, device=DEV)
    st = torch.empty((batch,), dtype=torch.int32, device=DEV)
    it = torch.empty((batch,), dtype=torch.int32, device=DEV)
    rr = torch.full((batch,), -1.0, dtype=torch.float64, device=DEV)
    opts = lib.mlmc_solver_opts_default(tol=1e-6)   # loose: the true residual is well above 0
    lib.mlmc_assemble(ctx, d, m, batch, k, T, tb, b)
    lib.mlmc_solve(ctx, d, m, batch, T, tb, b, p, opts, st, it, rr)
    torch.cuda.synchronize()
    assert np.all(st.cpu().numpy() == 0)
    x = p.cpu().numpy()
    for s in range(batch):
        A, bb = ofv.assemble(kh[s])
        want = np.linalg.norm(bb - A @ x[s].ravel()) / np.linalg.norm(bb)
        got = rr[s].item()
        assert want < 1e-6 and abs(got - want) <= 1e-6 * want + 1e-15, (s, got, want)
