"""mlmc_solve_noalloc (every workspace in the library's static scratch array)
against mlmc_solve on the same operators, through the C ABI: two calls in a
row on each configuration, the second with a smaller batch (the array then
still holds the first call's contents), for the whole-on-chip 64 x 64 solve,
the tiled 2-D kernels (FP64 and FP32 hierarchies) and the 3-D solver.  The
solutions must be bitwise those of mlmc_solve (same kernels, same inputs);
the outflow of the first sample is also checked against the oracle (1e-10).
Oversize batches and graph mode are refused before any work is enqueued.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import fv as ofv  # noqa: E402
from oracle import qoi as oqoi  # noqa: E402
from oracle import solve as osolve  # noqa: E402

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


def i32(*shape):
    return torch.empty(*shape, dtype=torch.int32, device=DEV)


def operators(lib, ctx, dim, m, batch, seed):
    rng = np.random.default_rng(seed)
    kh = np.exp(1.3 * rng.standard_normal((batch,) + (m,) * dim))
    k = torch.from_numpy(kh).to(DEV)
    T = f64(batch, dim, *(m,) * dim)
    tb = f64(batch, dim, *(m,) * (dim - 1))
    b = f64(batch, *(m,) * dim)
    lib.mlmc_assemble(ctx, dim, m, batch, k, T, tb, b)
    return kh, k, T, tb, b


def run(lib, ctx, fn, dim, m, batch, T, tb, b, opts):
    p = torch.full((batch,) + (m,) * dim, float("nan"), dtype=torch.float64, device=DEV)
    st, it, rr = i32(batch), i32(batch), f64(batch)
    fn(ctx, dim, m, batch, T, tb, b, p, opts, st, it, rr)
    torch.cuda.synchronize()
    return p, st, it, rr


CASES = [
    (2, 64, (40, 7), "f64"),     # whole solve of a sample in one workgroup
    (2, 128, (12, 5), "f64"),    # tiled kernels with the on-chip 64^2 sub-cycle
    (2, 256, (6, 2), "f32"),     # tiled kernels, FP32 hierarchy, flexible CG
    (3, 32, (6, 3), "f64"),      # 3-D per-sweep levels and the in-LDS cycle
    (3, 16, (8, 3), "f32"),
]


@pytest.mark.parametrize("dim,m,batches,prec", CASES)
def test_noalloc_equals_solve(lib, ctx, dim, m, batches, prec):
    opts = lib.mlmc_solver_opts_default(
        precision=lib.MLMC_PREC_FP32 if prec == "f32" else lib.MLMC_PREC_FP64)
    for call, batch in enumerate(batches):
        print("noalloc dim=%d m=%d batch=%d %s call %d" % (dim, m, batch, prec, call), flush=True)
        kh, k, T, tb, b = operators(lib, ctx, dim, m, batch, 1000 * dim + m + call)
        ref = run(lib, ctx, lib.mlmc_solve, dim, m, batch, T, tb, b, opts)
        got = run(lib, ctx, lib.mlmc_solve_noalloc, dim, m, batch, T, tb, b, opts)
        assert torch.all(ref[1] == 0), ref[1]
        assert torch.equal(got[1], ref[1]) and torch.equal(got[2], ref[2])
        assert torch.equal(got[0], ref[0]), (dim, m, batch)
        assert torch.equal(got[3], ref[3])
        q = f64(batch)
        lib.mlmc_qoi_outflow(ctx, dim, m, batch, k, got[0], q)
        torch.cuda.synchronize()
        A, bb = ofv.assemble(kh[0])
        q_ref = oqoi.outflow(kh[0], osolve.direct_solve(A, bb))
        assert abs(q[0].item() - q_ref) <= 1e-10 * q_ref


def test_noalloc_then_solve_still_allocates_normally(lib, ctx):
    dim, m, batch = 2, 128, 3
    opts = lib.mlmc_solver_opts_default()
    _, _, T, tb, b = operators(lib, ctx, dim, m, batch, 7)
    a = run(lib, ctx, lib.mlmc_solve_noalloc, dim, m, batch, T, tb, b, opts)
    c = run(lib, ctx, lib.mlmc_solve, dim, m, batch, T, tb, b, opts)
    assert torch.equal(a[0], c[0]) and torch.equal(a[2], c[2])


def test_noalloc_refuses_oversize_batch_before_any_work(lib, ctx):
    dim, m, batch = 2, 64, 4000          # about 105 MB of workspaces > 64 MiB
    opts = lib.mlmc_solver_opts_default()
    T, tb, b = f64(batch, 2, m, m), f64(batch, 2, m), f64(batch, m, m)
    T.fill_(1.0)
    tb.fill_(1.0)
    b.fill_(1.0)
    p = torch.full((batch, m, m), 7.0, dtype=torch.float64, device=DEV)
    st, it, rr = i32(batch).fill_(-5), i32(batch).fill_(-5), f64(batch).fill_(-5.0)
    torch.cuda.synchronize()
    with pytest.raises(lib.MlmcError) as e:
        lib.mlmc_solve_noalloc(ctx, dim, m, batch, T, tb, b, p, opts, st, it, rr)
    torch.cuda.synchronize()
    assert e.value.code == lib.MLMC_EINVAL and "scratch" in str(e.value)
    assert torch.all(p == 7.0) and torch.all(st == -5) and torch.all(rr == -5.0)


def test_noalloc_refuses_graph_mode(lib, ctx):
    dim, m, batch = 2, 128, 2
    _, _, T, tb, b = operators(lib, ctx, dim, m, batch, 9)
    opts = lib.mlmc_solver_opts_default(graph=1)
    with pytest.raises(lib.MlmcError) as e:
        run(lib, ctx, lib.mlmc_solve_noalloc, dim, m, batch, T, tb, b, opts)
    assert e.value.code == lib.MLMC_EINVAL
