"""GPU parity: every stage of the HIP path against the CPU oracle, through the C ABI.

Tolerances:
* layer decisions and the CGV sub-lattice gather are exact;
* k from Example 1 layers: 1e-14 relative (device exp/log/sincos may differ
  from the host libm by an ulp);
* k from circulant embedding: |log k_gpu - log k_oracle| <= 1e-11 (two
  different FFTs of length n_ce <= 1875, errors ~ eps log n per value);
* assembly: 1e-14 relative;
* QoI: 1e-10 relative per sample -- the required parity; the solver
  tolerance (relative residual 1e-13) is chosen so that this holds.
"""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import workloads as W  # noqa: E402
from oracle import field as ofield  # noqa: E402
from oracle import fv as ofv  # noqa: E402
from oracle import geometry as ogeom  # noqa: E402
from oracle import mlmc as omlmc  # noqa: E402
from oracle import qoi as oqoi  # noqa: E402
from oracle import solve as osolve  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
QTOL = 1e-10


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


DEV = "cuda:0"


def f64(*shape):
    return torch.empty(*shape, dtype=torch.float64, device=DEV)


def i32(*shape):
    return torch.empty(*shape, dtype=torch.int32, device=DEV)


def run_field(lib, ctx, model, m, level, first, batch, coarse=False):
    k = f64(batch, m, m)
    kc = f64(batch, m // 2, m // 2) if coarse else None
    lib.mlmc_sample_field(ctx, model, m, level, first, batch, k, kc)
    torch.cuda.synchronize()
    return k.cpu().numpy(), (kc.cpu().numpy() if coarse else None)


# ------------------------------------------------------------------ fields
@pytest.mark.parametrize("m,level", [(16, 0), (32, 1), (24, 2)])
def test_field_piecewise_constant(lib, ctx, m, level):
    print("field pc m=%d level=%d" % (m, level), flush=True)
    batch = 40
    k, kc = run_field(lib, ctx, W.PC2, m, level, 5, batch, coarse=True)
    for s in range(batch):
        ref, refc = ofield.sample_k(W.PC2, level, 5 + s, m, with_coarse=True)
        np.testing.assert_allclose(k[s], ref, rtol=1e-14, atol=0)
        np.testing.assert_allclose(kc[s], refc, rtol=1e-14, atol=0)


def test_field_paper_two_lines_and_pw_linear(lib, ctx):
    print("field geometry kinds", flush=True)
    for model, m in ((W.PC2.with_(interface_kind=W.PAPER_TWO_LINES, n_layers=3), 24),
                     (W.PC2.with_(interface_kind=W.PIECEWISE_LINEAR, n_nodes=8), 40),
                     (W.PC2.with_(interface_kind=W.PIECEWISE_LINEAR, n_nodes=3), 16)):
        k, _ = run_field(lib, ctx, model, m, 1, 0, 16)
        for s in range(16):
            lid = ogeom.layer_ids(model, 1, s, m)
            z = ofield.layer_constants(model, 1, s)
            np.testing.assert_allclose(k[s], np.exp(z[lid]), rtol=1e-14, atol=0)


@pytest.mark.parametrize("m,level", [(16, 0), (32, 1), (64, 2)])
def test_field_circulant_embedding(lib, ctx, m, level):
    print("field ce m=%d level=%d" % (m, level), flush=True)
    batch = 6
    k, kc = run_field(lib, ctx, W.CE2, m, level, 3, batch, coarse=True)
    lam = ofield.ce_eigenvalues(W.CE2.n_ce[m], m, 1.0, 0.3, 2)
    for s in range(batch):
        ref, refc = ofield.sample_k(W.CE2, level, 3 + s, m, lam_eig=lam, with_coarse=True)
        assert np.max(np.abs(np.log(k[s]) - np.log(ref))) < 1e-11
        assert np.max(np.abs(np.log(kc[s]) - np.log(refc))) < 1e-11


def test_field_ce_stationary_one_norm(lib, ctx):
    print("field ce stationary 1-norm", flush=True)
    model = W.STATIONARY_1NORM
    m = 32
    k, _ = run_field(lib, ctx, model, m, 0, 0, 4)
    lam = ofield.ce_eigenvalues(model.n_ce[m], m, 1.0, 0.3, 1)
    for s in range(4):
        ref = ofield.sample_k(model, 0, s, m, lam_eig=lam)
        assert np.max(np.abs(np.log(k[s]) - np.log(ref))) < 1e-11


@pytest.mark.parametrize("m,sigma2,lam,r", [(16, 1.0, 0.3, 2), (64, 1.0, 0.3, 2), (32, 3.0, 0.1, 2),
                                            (32, 1.0, 0.3, 1)])
def test_min_embedding_matches_oracle(lib, ctx, m, sigma2, lam, r):
    model = W.CE2.with_(sigma2=(sigma2,) * 4, lam=(lam,) * 4, norm_r=r)
    got = lib.mlmc_ce_min_embedding(ctx, lib.make_model(model), m)
    assert got == ofield.min_embedding(m, sigma2, lam, r)


def test_embedding_refused(lib, ctx):
    mm = lib.make_model(W.CE2, n_ce=128)
    k = f64(1, 64, 64)
    with pytest.raises(lib.MlmcError) as e:
        lib.mlmc_sample_field(ctx, mm, 64, 0, 0, 1, k)
    assert e.value.code == lib.MLMC_EEMBED


def test_cgv_extract_exact(lib, ctx):
    m, batch = 12, 3
    kf = torch.arange(batch * m * m, dtype=torch.float64, device=DEV).reshape(batch, m, m)
    ks = f64(batch, 4, m // 2, m // 2)
    lib.mlmc_cgv_extract(ctx, 2, m, batch, kf, ks)
    torch.cuda.synchronize()
    kf_h = kf.cpu().numpy()
    ks_h = ks.cpu().numpy()
    for s in range(batch):
        for a, sub in enumerate(ofield.cgv_sublattices(kf_h[s])):
            assert np.array_equal(ks_h[s, a], sub)


# ------------------------------------------------------------------ assembly
def test_assemble_matches_oracle(lib, ctx):
    rng = np.random.default_rng(11)
    batch, m = 4, 10
    kh = np.exp(1.5 * rng.standard_normal((batch, m, m)))
    k = torch.from_numpy(kh).to(DEV)
    T, tb, b = f64(batch, 2, m, m), f64(batch, 2, m), f64(batch, m, m)
    lib.mlmc_assemble(ctx, 2, m, batch, k, T, tb, b)
    torch.cuda.synchronize()
    T, tb, b = T.cpu().numpy(), tb.cpu().numpy(), b.cpu().numpy()
    for s in range(batch):
        Tint, Tb = ofv.face_transmissibilities(kh[s])
        np.testing.assert_allclose(T[s, 0, :, :-1], Tint[1], rtol=1e-14)   # x1 faces
        np.testing.assert_allclose(T[s, 1, :-1, :], Tint[0], rtol=1e-14)   # x2 faces
        np.testing.assert_allclose(T[s, 0, :, -1], Tb[:, -1], rtol=1e-15)
        assert np.all(T[s, 1, -1, :] == 0) and np.all(tb[s, 1] == 0)
        np.testing.assert_allclose(tb[s, 0], Tb[:, 0], rtol=1e-15)
        _, bref = ofv.assemble(kh[s])
        np.testing.assert_allclose(b[s].ravel(), bref, rtol=1e-15)


# ------------------------------------------------------------------ solve + QoI
def solve_batch(lib, ctx, kh, opts=None):
    batch, m, _ = kh.shape
    k = torch.from_numpy(np.ascontiguousarray(kh)).to(DEV)
    T, tb, b = f64(batch, 2, m, m), f64(batch, 2, m), f64(batch, m, m)
    p = f64(batch, m, m)
    st, it, rr = i32(batch), i32(batch), f64(batch)
    qo, qi = f64(batch), f64(batch)
    opts = opts or lib.mlmc_solver_opts_default()
    lib.mlmc_assemble(ctx, 2, m, batch, k, T, tb, b)
    lib.mlmc_solve(ctx, 2, m, batch, T, tb, b, p, opts, st, it, rr)
    lib.mlmc_qoi_outflow(ctx, 2, m, batch, k, p, qo, qi)
    torch.cuda.synchronize()
    return {"p": p.cpu().numpy(), "status": st.cpu().numpy(), "iters": it.cpu().numpy(),
            "relres": rr.cpu().numpy(), "q_out": qo.cpu().numpy(), "q_in": qi.cpu().numpy()}


@pytest.mark.parametrize("m", [1, 2, 3, 5, 6, 8, 12, 16, 24, 40, 64, 96])
def test_solve_qoi_random_lognormal(lib, ctx, m):
    print("solve m=%d" % m, flush=True)
    rng = np.random.default_rng(100 + m)
    batch = 5
    kh = np.exp(1.5 * rng.standard_normal((batch, m, m)))
    out = solve_batch(lib, ctx, kh)
    assert np.all(out["status"] == 0), out["status"]
    assert np.all(out["relres"] < 1e-12), out["relres"]
    for s in range(batch):
        A, b = ofv.assemble(kh[s])
        pr = osolve.direct_solve(A, b)
        q = oqoi.outflow(kh[s], pr)
        assert abs(out["q_out"][s] - q) <= QTOL * q, (s, out["q_out"][s], q)
        assert abs(out["q_in"][s] - q) <= 1e-9 * q
        assert np.max(np.abs(out["p"][s].ravel() - pr)) < 1e-8


def test_solve_closed_forms(lib, ctx):
    m = 32
    rng = np.random.default_rng(5)
    rows = np.exp(rng.standard_normal(m))
    cols = np.exp(2.0 * rng.standard_normal(m))
    kh = np.stack([np.full((m, m), 3.7), np.repeat(rows[:, None], m, 1), np.repeat(cols[None, :], m, 0)])
    out = solve_batch(lib, ctx, kh)
    assert abs(out["q_out"][0] - 3.7) < 1e-11 * 3.7
    assert abs(out["q_out"][1] - rows.mean()) < 1e-11 * rows.mean()
    hm = m / np.sum(1.0 / cols)
    assert abs(out["q_out"][2] - hm) < 1e-11 * hm
    x1 = (np.arange(m) + 0.5) / m
    assert np.max(np.abs(out["p"][0] - (1 - x1)[None, :])) < 1e-11


def test_solve_failure_paths(lib, ctx):
    rng = np.random.default_rng(9)
    m, batch = 32, 3
    kh = np.exp(rng.standard_normal((batch, m, m)))
    kh[1, 5, 7] = np.nan
    out = solve_batch(lib, ctx, kh)
    assert out["status"][0] == lib.MLMC_SAMPLE_OK and out["status"][2] == lib.MLMC_SAMPLE_OK
    assert out["status"][1] == lib.MLMC_SAMPLE_BREAKDOWN
    out = solve_batch(lib, ctx, kh[[0, 2]], lib.mlmc_solver_opts_default(maxit=1))
    assert np.all(out["status"] == lib.MLMC_SAMPLE_NOCONV) and np.all(out["iters"] == 1)
    with pytest.raises(lib.MlmcError) as e:
        solve_batch(lib, ctx, kh[[0]], lib.mlmc_solver_opts_default(nu1=2, nu2=1))
    assert e.value.code == lib.MLMC_EINVAL
    with pytest.raises(lib.MlmcError):
        solve_batch(lib, ctx, kh[[0]], lib.mlmc_solver_opts_default(gamma=3))
    with pytest.raises(lib.MlmcError):
        solve_batch(lib, ctx, kh[[0]], lib.mlmc_solver_opts_default(gamma_levels=-1))
    with pytest.raises(lib.MlmcError):
        solve_batch(lib, ctx, np.ones((1, 88, 88)))     # 88 = 11 * 8: coarsest 11 > 8


# ------------------------------------------------------------------ initial guess
def solve_with_guess(lib, ctx, kh, x0, opts):
    batch, m, _ = kh.shape
    k = torch.from_numpy(np.ascontiguousarray(kh)).to(DEV)
    T, tb, b = f64(batch, 2, m, m), f64(batch, 2, m), f64(batch, m, m)
    p = torch.from_numpy(np.ascontiguousarray(x0)).to(DEV)
    st, it, rr, qo = i32(batch), i32(batch), f64(batch), f64(batch)
    lib.mlmc_assemble(ctx, 2, m, batch, k, T, tb, b)
    lib.mlmc_solve(ctx, 2, m, batch, T, tb, b, p, opts, st, it, rr)
    lib.mlmc_qoi_outflow(ctx, 2, m, batch, k, p, qo)
    torch.cuda.synchronize()
    return p.cpu().numpy(), st.cpu().numpy(), it.cpu().numpy(), qo.cpu().numpy()


@pytest.mark.parametrize("m", [32, 64, 128])
def test_initial_guess(lib, ctx, m):
    """A zero guess with initial_guess = 1 gives the zero-start solve bit for bit;
    a perturbed guess still reaches the oracle's QoI; the on-chip 64 x 64 path
    starts from zero whatever p holds."""
    print("initial guess m=%d" % m, flush=True)
    rng = np.random.default_rng(40 + m)
    batch = 3
    kh = np.exp(1.5 * rng.standard_normal((batch, m, m)))
    zero = np.zeros((batch, m, m))
    pa, sa, ia, qa = solve_with_guess(lib, ctx, kh, zero, lib.mlmc_solver_opts_default())
    pb, sb, ib, qb = solve_with_guess(lib, ctx, kh, zero,
                                      lib.mlmc_solver_opts_default(initial_guess=1))
    assert np.array_equal(pa, pb) and np.array_equal(ia, ib)
    x1 = (np.arange(m) + 0.5) / m
    guess = (1.0 - x1)[None, None, :] + 0.05 * rng.standard_normal((batch, m, m))
    pc, sc, ic, qc = solve_with_guess(lib, ctx, kh, guess,
                                      lib.mlmc_solver_opts_default(initial_guess=1))
    assert np.all(sc == 0)
    for s in range(batch):
        A, bb = ofv.assemble(kh[s])
        q = oqoi.outflow(kh[s], osolve.direct_solve(A, bb))
        assert abs(qc[s] - q) <= QTOL * q, (s, qc[s], q)
    if m == 64:
        assert np.array_equal(pc, pa)          # on chip: the guess is not used


def test_initial_guess_option_checked(lib, ctx):
    kh = np.ones((1, 16, 16))
    with pytest.raises(lib.MlmcError):
        solve_with_guess(lib, ctx, kh, np.zeros((1, 16, 16)),
                         lib.mlmc_solver_opts_default(initial_guess=2))


# ------------------------------------------------------------------ level runs
def level_run(lib, ctx, model, level, m, first, n, cgv, opts=None):
    qf, qc, y = f64(n), f64(n), f64(n)
    opts = opts or lib.mlmc_solver_opts_default()
    sums = lib.mlmc_level_run(ctx, model, level, m, first, n, cgv, opts, q_f=qf, q_c=qc, y=y)
    torch.cuda.synchronize()
    return sums, qf.cpu().numpy(), qc.cpu().numpy(), y.cpu().numpy()


@pytest.mark.parametrize("name", ["pc2_16_32_plain.json", "pc2_16_32_cgv.json",
                                  "ce2_16_32_plain.json", "ce2_16_32_cgv.json"])
def test_level_run_matches_golden(lib, ctx, name):
    print("level run golden %s" % name, flush=True)
    rec = json.load(open(os.path.join(GOLDEN, name)))
    model = {"pc2": W.PC2, "ce2": W.CE2}[name[:3]]
    for lv in rec["levels"]:
        rows = lv["samples"]
        n = len(rows)
        sums, qf, qc, y = level_run(lib, ctx, model, lv["level"], lv["m"], 0, n, rec["cgv"])
        assert sums.n == n and sums.n_failed == 0
        for s, row in enumerate(rows):
            assert abs(qf[s] - row["Q_f"]) <= QTOL * abs(row["Q_f"])
            if lv["level"] > 0:
                assert abs(qc[s] - row["Q_c"]) <= QTOL * abs(row["Q_c"])
                assert abs(y[s] - row["Y"]) <= QTOL * abs(row["Q_f"])
        assert abs(sums.sum_y - y.sum()) <= 1e-12 * np.abs(y).sum()


def test_level_run_config_small_estimator(lib, ctx):
    """Two-level plain MLMC of the 16/32 piecewise constant workload (200 samples per
    level): every sample against its closed form, and the estimate against e^(1/2)."""
    wl = W.SMALL_PC
    sums = []
    for level, (m, n) in enumerate(zip(wl.m_levels, wl.n_samples)):
        s, qf, qc, y = level_run(lib, ctx, wl.model, level, m, 0, n, False)
        sums.append(s)
        for i in range(0, n, 7):
            y0 = ogeom.interface_params(wl.model, level, i)["y0"]
            kl = np.exp(ofield.layer_constants(wl.model, level, i))
            ff = np.ceil(m * y0 - 0.5) / m
            ref = ff * kl[0] + (1 - ff) * kl[1]
            assert abs(qf[i] - ref) <= QTOL * ref
    est = lib.mlmc_estimate(sums)
    assert abs(est["estimate"] - np.exp(0.5)) < 5 * est["std_error"]


def test_batch_invariance_bitwise(lib, ctx):
    """A sample's result does not depend on the batch it is solved in."""
    model, m = W.CE2, 64
    _, qf_big, qc_big, _ = level_run(lib, ctx, model, 1, m, 10, 37, False)
    for s in (0, 17, 36):
        _, qf1, qc1, _ = level_run(lib, ctx, model, 1, m, 10 + s, 1, False)
        assert qf1[0] == qf_big[s] and qc1[0] == qc_big[s]


def test_level_run_noconv_is_reported(lib, ctx):
    opts = lib.mlmc_solver_opts_default(maxit=2)
    qf = f64(4)
    sums = lib.mlmc_level_run(ctx, W.CE2, 1, 32, 0, 4, False, opts, q_f=qf, allow_noconv=True)
    assert sums.n == 4 and sums.n_failed == 4
    with pytest.raises(lib.MlmcError) as e:
        lib.mlmc_level_run(ctx, W.CE2, 1, 32, 0, 4, False, opts)
    assert e.value.code == lib.MLMC_ENOCONV


# ------------------------------------------------------------------ full-size levels
FULL = W.LAYERED_CE


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_layered_ce_full_level_sampled(lib, ctx, level):
    """Each level of the layered correlated workload at its full size with the
    solver options the bench times it with, sampled samples checked against the
    oracle one by one."""
    m, n = FULL.m_levels[level], FULL.n_samples[level]
    print("full level %d: %d x %d^2" % (level, n, m), flush=True)
    opts = lib.mlmc_solver_opts_default(**W.LAYERED_CE_LEVEL_OPTS[level])
    sums, qf, qc, y = level_run(lib, ctx, FULL.model, level, m, 0, n, False, opts)
    assert sums.n == n and sums.n_failed == 0
    assert np.all(np.isfinite(qf)) and np.all(qf > 0)
    lam = ofield.ce_eigenvalues(FULL.model.n_ce[m], m, 1.0, 0.3, 2)
    picks = [0, n // 3, n - 1] if m >= 512 else [0, n // 3, 2 * n // 3, n - 1]
    for s in picks:
        k = ofield.sample_k(FULL.model, level, s, m, lam_eig=lam, with_coarse=level > 0)
        kf = k[0] if level > 0 else k
        q_ref = omlmc.solve_qoi(kf)[0]
        assert abs(qf[s] - q_ref) <= QTOL * q_ref, (s, qf[s], q_ref)
        if level > 0:
            qc_ref = omlmc.solve_qoi(k[1])[0]
            assert abs(qc[s] - qc_ref) <= QTOL * qc_ref, (s, qc[s], qc_ref)


# ------------------------------------------------------------------ fused vs per-sweep V-cycle
@pytest.mark.parametrize("gamma,glev", [(1, 2), (2, 2), (2, 1), (2, 0)])
@pytest.mark.parametrize("m", [8, 24, 40, 64, 96, 128, 256])
def test_fused_cycle_matches_unfused(lib, ctx, m, gamma, glev):
    """The fused tiled V-/W-cycle and the one-launch-per-sweep cycle are the same
    preconditioner: equal iteration counts (+-1 from rounding) and QoIs, both at
    the oracle's value.  W on the glev finest levels (0: all, including the
    levels held in LDS)."""
    print("fused vs unfused m=%d gamma=%d gamma_levels=%d" % (m, gamma, glev), flush=True)
    rng = np.random.default_rng(300 + m)
    batch = 3
    kh = np.exp(1.5 * rng.standard_normal((batch, m, m)))
    kw = dict(gamma=gamma, gamma_levels=glev)
    a = solve_batch(lib, ctx, kh, lib.mlmc_solver_opts_default(variant=0, **kw))
    b = solve_batch(lib, ctx, kh, lib.mlmc_solver_opts_default(variant=1, **kw))
    assert np.all(a["status"] == 0) and np.all(b["status"] == 0)
    assert np.all(np.abs(a["iters"] - b["iters"]) <= 1), (a["iters"], b["iters"])
    for s in range(batch):
        A, bb = ofv.assemble(kh[s])
        q = oqoi.outflow(kh[s], osolve.direct_solve(A, bb))
        assert abs(a["q_out"][s] - q) <= QTOL * q
        assert abs(b["q_out"][s] - q) <= QTOL * q


@pytest.mark.parametrize("gamma,bound,spread", [(1, 25, 5), (2, 12, 3)])
def test_iterations_flat_in_grid_size(lib, ctx, gamma, bound, spread):
    """Multigrid-preconditioned CG needs a bounded number of iterations on the
    layered correlated model from 64^2 to 512^2 (optimal solver, Section 3.5);
    the W-cycle needs fewer than the V-cycle."""
    its = []
    for level, m in enumerate([64, 128, 256, 512]):
        sums = lib.mlmc_level_run(ctx, W.CE2, level, m, 0, 8, False,
                                  lib.mlmc_solver_opts_default(gamma=gamma))
        its.append(sums.iters_fine / 8)
    print("gamma %d mean iterations %s" % (gamma, its), flush=True)
    assert max(its) <= bound and max(its) - min(its) <= spread, its


def test_w_cycle_breakdown_restarts_with_v(lib, ctx):
    """Samples of the layered workload on which the W-cycle preconditioner with
    omega = 2 is indefinite (its PCG breaks down in the first iterations) are solved again
    with the V-cycle: every status is OK, the restarted samples report both
    passes' iterations, and their QoIs match the V-cycle solve and the oracle."""
    model, m = FULL.model, 128
    ids = [31, 601, 672, 0, 1]
    kk = f64(len(ids), m, m)
    sid = torch.tensor(ids, dtype=torch.int32, device=DEV)
    lib.mlmc_sample_field_ids(ctx, model, m, 1, sid, len(ids), kk)
    kh = kk.cpu().numpy()
    w = solve_batch(lib, ctx, kh, lib.mlmc_solver_opts_default(omega=2.0))
    v = solve_batch(lib, ctx, kh, lib.mlmc_solver_opts_default(omega=2.0, gamma=1))
    print("W iterations", w["iters"], "V iterations", v["iters"], flush=True)
    assert np.all(w["status"] == 0) and np.all(w["relres"] < 1e-12)
    assert np.max(w["iters"][:3]) >= 15 and np.all(w["iters"][3:] <= 12)
    np.testing.assert_allclose(w["q_out"], v["q_out"], rtol=QTOL)
    q = omlmc.solve_qoi(kh[0])[0]
    assert abs(w["q_out"][0] - q) <= QTOL * q


# ------------------------------------------------------------------ reduced-precision multigrid
@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("m", [40, 64, 96, 256])
def test_mixed_precision_multigrid_qoi(lib, ctx, m, prec):
    """FP32 / bfloat16 multigrid inside the FP64 flexible CG: the outer residual is
    FP64, so the QoI reaches the same 1e-10 parity; iterations stay bounded."""
    print("mixed precision %d m=%d" % (prec, m), flush=True)
    rng = np.random.default_rng(500 + m)
    batch = 3
    kh = np.exp(1.5 * rng.standard_normal((batch, m, m)))
    ref = solve_batch(lib, ctx, kh, lib.mlmc_solver_opts_default())
    out = solve_batch(lib, ctx, kh, lib.mlmc_solver_opts_default(precision=prec))
    assert np.all(out["status"] == 0), out["status"]
    assert np.all(out["relres"] < 1e-12)
    slack = 3 if prec == 1 else 12
    assert np.all(out["iters"] <= ref["iters"] + slack), (out["iters"], ref["iters"])
    for s in range(batch):
        A, bb = ofv.assemble(kh[s])
        q = oqoi.outflow(kh[s], osolve.direct_solve(A, bb))
        assert abs(out["q_out"][s] - q) <= QTOL * q


def test_mixed_precision_level_run_golden(lib, ctx):
    rec = json.load(open(os.path.join(GOLDEN, "ce2_16_32_plain.json")))
    for prec in (1, 2):
        opts = lib.mlmc_solver_opts_default(precision=prec)
        for lv in rec["levels"]:
            n = len(lv["samples"])
            sums, qf, qc, y = level_run(lib, ctx, W.CE2, lv["level"], lv["m"], 0, n, False, opts)
            assert sums.n_failed == 0
            for s, row in enumerate(lv["samples"]):
                assert abs(qf[s] - row["Q_f"]) <= QTOL * abs(row["Q_f"])


def test_high_contrast_1024_all_precisions(lib, ctx):
    """The high-contrast workload at full size (256 samples on 1024^2, sigma^2 = 3,
    lambda = 0.1, means -2 / +2) with the multigrid in FP64, FP32 and bfloat16, at the
    workload's tolerance (relative residual 1e-15; the true residual stalls near
    5e-13 at this contrast while the QoI still converges): every solve converges,
    samples 0-15 and 200 match the oracle to 1e-10 in every precision, and
    all 256 reduced-precision QoIs stay within 1e-10 of the FP64 ones."""
    wl = W.HIGH_CONTRAST
    m, n = wl.m_levels[0], wl.n_samples[0]
    out = {}
    for prec in (0, 1, 2):
        print("high contrast %d x %d^2 precision %d" % (n, m, prec), flush=True)
        opts = lib.mlmc_solver_opts_default(precision=prec, tol=wl.tol)
        if prec == 2:
            opts.omega = wl.omega_bf16
        sums, qf, _, _ = level_run(lib, ctx, wl.model, 0, m, 0, n, False, opts)
        assert sums.n == n and sums.n_failed == 0
        out[prec] = qf
    for prec in (1, 2):
        assert np.max(np.abs(out[prec] - out[0]) / out[0]) <= QTOL
    lam = ofield.ce_eigenvalues(wl.model.n_ce[m], m, 3.0, 0.1, 2)
    for s in (200,):
        q_ref = omlmc.solve_qoi(ofield.sample_k(wl.model, 0, s, m, lam_eig=lam))[0]
        for prec in (0, 1, 2):
            assert abs(out[prec][s] - q_ref) <= QTOL * q_ref, (s, prec, out[prec][s], q_ref)
    # samples 0-15 against the oracle's values stored by tests/golden/make_golden.py
    rec = json.load(open(os.path.join(GOLDEN, "ce_hc_1024_fine.json")))
    for row in rec["levels"][0]["samples"]:
        s = row["sample"]
        for prec in (0, 1, 2):
            assert abs(out[prec][s] - row["Q_f"]) <= QTOL * row["Q_f"], (s, prec, out[prec][s])


@pytest.mark.parametrize("m,prec,variant", [(64, 0, 2), (128, 0, 0), (192, 0, 0), (256, 0, 0),
                                             (128, 1, 0), (256, 1, 0), (128, 2, 0)])
def test_tile_shapes_agree(lib, ctx, m, prec, variant):
    """The alternative tile shapes of the multigrid kernels (tile_shape = 1) do
    the same arithmetic per cell: same iterations (+-1: the r^T z tile sums add
    in another order) and QoIs to 1e-12 of the default shapes, and the oracle's
    QoI to 1e-10.  m = 192 takes the 64-wide fallback of the default up tile."""
    print("tile shapes m=%d prec=%d variant=%d" % (m, prec, variant), flush=True)
    rng = np.random.default_rng(1300 + m + prec)
    kh = np.exp(1.4 * rng.standard_normal((3, m, m)))
    a = solve_batch(lib, ctx, kh, lib.mlmc_solver_opts_default(precision=prec, variant=variant))
    b = solve_batch(lib, ctx, kh, lib.mlmc_solver_opts_default(precision=prec, variant=variant,
                                                             tile_shape=1))
    assert np.all(a["status"] == 0) and np.all(b["status"] == 0)
    assert np.all(np.abs(a["iters"] - b["iters"]) <= 1), (a["iters"], b["iters"])
    np.testing.assert_allclose(b["q_out"], a["q_out"], rtol=1e-12, atol=0)
    A, bb = ofv.assemble(kh[0])
    q = oqoi.outflow(kh[0], osolve.direct_solve(A, bb))
    assert abs(b["q_out"][0] - q) <= QTOL * q


def test_mixed_precision_requires_fused(lib, ctx):
    kh = np.ones((1, 16, 16))
    with pytest.raises(lib.MlmcError):
        solve_batch(lib, ctx, kh, lib.mlmc_solver_opts_default(precision=1, variant=1))


# ------------------------------------------------------------------ all levels in one call
@pytest.mark.parametrize("cgv", [False, True])
def test_run_levels_matches_level_runs(lib, ctx, cgv):
    """Running the levels concurrently in one call (a pipeline per level on its own
    stream) does not change any sample's numbers; formerly: merging level l's fine samples with level l+1's companions into one solve per
    grid does not change any sample's numbers, so the level sums are identical."""
    model, ms, ns = W.CE2, [32, 64, 128], [48, 24, 8]
    per = []
    for level, (m, n) in enumerate(zip(ms, ns)):
        per.append(lib.mlmc_level_run(ctx, model, level, m, 7, n, cgv,
                                      lib.mlmc_solver_opts_default()))
    allv = lib.mlmc_run_levels(ctx, model, ms, [7, 7, 7], ns, cgv, lib.mlmc_solver_opts_default())
    for a, b in zip(per, allv):
        assert a.n == b.n and a.n_failed == b.n_failed == 0
        assert (a.sum_y, a.sum_y2, a.sum_qf, a.sum_qc) == (b.sum_y, b.sum_y2, b.sum_qf, b.sum_qc)
        assert a.iters_fine == b.iters_fine and a.iters_coarse == b.iters_coarse


@pytest.mark.parametrize("cycle_max", [8, 16])
def test_coarse_cycle_threshold_same_preconditioner(lib, ctx, cycle_max):
    """Moving levels between the tiled kernels and the one-workgroup coarse cycle
    changes only rounding: iterations +-1, QoIs at the oracle."""
    rng = np.random.default_rng(700 + cycle_max)
    kh = np.exp(1.5 * rng.standard_normal((3, 128, 128)))
    a = solve_batch(lib, ctx, kh, lib.mlmc_solver_opts_default())
    b = solve_batch(lib, ctx, kh, lib.mlmc_solver_opts_default(cycle_max=cycle_max))
    assert np.all(b["status"] == 0) and np.all(np.abs(a["iters"] - b["iters"]) <= 1)
    for s in range(3):
        A, bb = ofv.assemble(kh[s])
        q = oqoi.outflow(kh[s], osolve.direct_solve(A, bb))
        assert abs(b["q_out"][s] - q) <= QTOL * q


# ------------------------------------------------------------------ graph-captured iterations
def test_graph_iterations_bitwise_equal_eager(lib, ctx):
    """PCG iterations replayed from a captured HIP graph give the eager results bit
    for bit.  Level runs alternate between the graph and the eager form and between
    grids, so cached graphs are replayed again after other eager work, and every
    replay is compared with the eager run of the same samples."""
    wl = FULL
    plan = [(1, 128, 64), (3, 512, 4), (1, 128, 64), (2, 256, 16), (3, 512, 4), (1, 128, 64)]
    for rep, (level, m, n) in enumerate(plan):
        print("graph vs eager: level %d m %d rep %d" % (level, m, rep), flush=True)
        first = 7 + 11 * rep
        se, qfe, qce, _ = level_run(lib, ctx, wl.model, level, m, first, n, False)
        sg, qfg, qcg, _ = level_run(lib, ctx, wl.model, level, m, first, n, False,
                                    lib.mlmc_solver_opts_default(graph=1))
        assert sg.n_failed == 0
        assert np.array_equal(qfe, qfg) and np.array_equal(qce, qcg), rep
        assert (se.iters_fine, se.iters_coarse) == (sg.iters_fine, sg.iters_coarse)
        level_run(lib, ctx, wl.model, 0, 64, 3 + rep, 32, False)       # eager work in between


@pytest.mark.parametrize("check,prec,omega", [(2, 0, 1.9), (6, 0, 1.9), (4, 1, 1.9), (4, 0, 2.0)])
def test_graph_solve_options(lib, ctx, check, prec, omega):
    """Graph form against the eager form for other check intervals, the FP32 hierarchy
    (flexible CG) and omega = 2, where some samples' W iterations break down and are
    restarted with the V-cycle: status, iterations, relres and the pressure bitwise."""
    model, m = FULL.model, 128
    ids = [31, 601, 672, 0, 1, 2]
    kk = f64(len(ids), m, m)
    sid = torch.tensor(ids, dtype=torch.int32, device=DEV)
    lib.mlmc_sample_field_ids(ctx, model, m, 1, sid, len(ids), kk)
    kh = kk.cpu().numpy()
    kw = dict(check_every=check, precision=prec, omega=omega)
    eager = solve_batch(lib, ctx, kh, lib.mlmc_solver_opts_default(**kw))
    for rep in range(3):
        graph = solve_batch(lib, ctx, kh, lib.mlmc_solver_opts_default(graph=1, **kw))
        for key in ("status", "iters", "relres", "p"):
            assert np.array_equal(eager[key], graph[key]), (rep, key)
    assert np.all(eager["status"] == 0)


def test_graph_option_refused(lib, ctx):
    kh = np.ones((1, 16, 16))
    with pytest.raises(lib.MlmcError):
        solve_batch(lib, ctx, kh, lib.mlmc_solver_opts_default(graph=2))


# ------------------------------------------------------------------ on-chip 64 x 64 solver
@pytest.mark.parametrize("gamma,glev,omega", [(2, 2, 1.9), (1, 2, 1.9), (2, 1, 1.9), (2, 0, 1.9),
                                              (2, 2, 2.0)])
def test_onchip_64_matches_tiled(lib, ctx, gamma, glev, omega):
    """The one-workgroup solve of 64 x 64 samples (variant 0) against the tiled
    kernels (variant 2) with the same hierarchy and cycle: same status, the same
    iteration counts up to one, pressures to 1e-12 and QoIs to 1e-12 relative, and
    QoIs within 1e-10 of the oracle.  omega = 2 exercises the V-cycle restart."""
    model, m = FULL.model, 64
    ids = [31, 601, 672, 0, 1, 2, 3, 4]
    kk = f64(len(ids), m, m)
    sid = torch.tensor(ids, dtype=torch.int32, device=DEV)
    lib.mlmc_sample_field_ids(ctx, model, m, 0, sid, len(ids), kk)
    kh = kk.cpu().numpy()
    kw = dict(gamma=gamma, gamma_levels=glev, omega=omega)
    oc = solve_batch(lib, ctx, kh, lib.mlmc_solver_opts_default(variant=0, **kw))
    ti = solve_batch(lib, ctx, kh, lib.mlmc_solver_opts_default(variant=2, **kw))
    print("on-chip iterations", oc["iters"], "tiled", ti["iters"], flush=True)
    assert np.array_equal(oc["status"], ti["status"]) and np.all(oc["status"] == 0)
    assert np.max(np.abs(oc["iters"] - ti["iters"])) <= 1
    assert np.all(oc["relres"] < 1e-12)
    np.testing.assert_allclose(oc["q_out"], ti["q_out"], rtol=1e-12)
    assert np.max(np.abs(oc["p"] - ti["p"])) <= 1e-12
    for s in (0, 3):
        q = omlmc.solve_qoi(kh[s])[0]
        assert abs(oc["q_out"][s] - q) <= QTOL * q


def test_onchip_64_level_run_full_size(lib, ctx):
    """The 64^2 level of the layered workload (4096 samples) through the on-chip
    solver: no failures, batch-invariant results and oracle parity on samples."""
    m, n = 64, 4096
    sums, qf, _, _ = level_run(lib, ctx, FULL.model, 0, m, 0, n, False)
    assert sums.n_failed == 0
    sums2, qf2, _, _ = level_run(lib, ctx, FULL.model, 0, m, 100, 7, False)
    assert np.array_equal(qf[100:107], qf2)
    for s in (0, 2047, 4095):
        q = omlmc.solve_qoi(ofield.sample_k(FULL.model, 0, s, m))[0]
        assert abs(qf[s] - q) <= QTOL * q


@pytest.mark.parametrize("m,glev", [(128, 2), (128, 0), (256, 2), (512, 3)])
def test_onchip_subcycle_matches_tiled(lib, ctx, m, glev):
    """Larger solves run the cycle of their 64^2 level (and below) in one workgroup
    per sample (variant 0); against the all-tiled cycle (variant 2): the same
    status, iterations up to one and QoIs to 1e-12."""
    rng = np.random.default_rng(700 + m)
    kh = np.exp(1.5 * rng.standard_normal((3, m, m)))
    kw = dict(gamma_levels=glev)
    oc = solve_batch(lib, ctx, kh, lib.mlmc_solver_opts_default(variant=0, **kw))
    ti = solve_batch(lib, ctx, kh, lib.mlmc_solver_opts_default(variant=2, **kw))
    print("m %d sub-cycle iterations %s tiled %s" % (m, oc["iters"], ti["iters"]), flush=True)
    assert np.all(oc["status"] == 0) and np.all(ti["status"] == 0)
    assert np.max(np.abs(oc["iters"] - ti["iters"])) <= 1
    np.testing.assert_allclose(oc["q_out"], ti["q_out"], rtol=1e-12)
