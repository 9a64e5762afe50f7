"""GPU parity of the 3-D path (7-point TPFA, tilted planar interface, 3-D
circulant embedding, 2 x 2 x 2 multigrid) against the CPU oracle, through the
C ABI.  Tolerances as in the 2-D parity tests: exact layer decisions, 1e-14
relative for k of piecewise constant layers and for assembly, 1e-11 absolute
in log k for embedded fields, 1e-10 relative for every QoI.
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
from oracle import mlmc as omlmc  # noqa: E402
from oracle import qoi as oqoi  # noqa: E402
from oracle import solve as osolve  # noqa: E402

QTOL = 1e-10
DEV = "cuda:0"
MODEL = W.TILTED3


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


def solve3(lib, ctx, kh, opts=None):
    batch, m = kh.shape[0], kh.shape[1]
    k = torch.from_numpy(np.ascontiguousarray(kh)).to(DEV)
    T, tb, b, p = f64(batch, 3, m, m, m), f64(batch, 3, m, m), f64(batch, m, m, m), f64(batch, m, m, m)
    st, it, rr, qo, qi = i32(batch), i32(batch), f64(batch), f64(batch), f64(batch)
    opts = opts or lib.mlmc_solver_opts_default()
    lib.mlmc_assemble(ctx, 3, m, batch, k, T, tb, b)
    lib.mlmc_solve(ctx, 3, m, batch, T, tb, b, p, opts, st, it, rr)
    lib.mlmc_qoi_outflow(ctx, 3, m, batch, k, p, qo, qi)
    torch.cuda.synchronize()
    return {"status": st.cpu().numpy(), "iters": it.cpu().numpy(), "relres": rr.cpu().numpy(),
            "q_out": qo.cpu().numpy(), "q_in": qi.cpu().numpy(), "p": p.cpu().numpy(),
            "T": T.cpu().numpy(), "tb": tb.cpu().numpy(), "b": b.cpu().numpy()}


# ------------------------------------------------------------------ fields
@pytest.mark.parametrize("m,level,batch", [(8, 0, 3), (16, 1, 3), (32, 0, 2), (64, 1, 2)])
def test_field_3d_circulant_embedding(lib, ctx, m, level, batch):
    """The served grids' fields too (32^3 and 64^3, embeddings of 75^3 and 225^3)."""
    print("3-D field m=%d level=%d" % (m, level), flush=True)
    k, kc = f64(batch, m, m, m), f64(batch, m // 2, m // 2, m // 2)
    lib.mlmc_sample_field(ctx, MODEL, m, level, 5, batch, k, kc)
    torch.cuda.synchronize()
    k, kc = k.cpu().numpy(), kc.cpu().numpy()
    for s in range(batch):
        kr, kcr = ofield.sample_k(MODEL, level, 5 + s, m, with_coarse=True)
        assert np.max(np.abs(np.log(k[s]) - np.log(kr))) <= 1e-11
        assert np.max(np.abs(np.log(kc[s]) - np.log(kcr))) <= 1e-11


FIELD128 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "tilted3_field_128.json")


def test_field_3d_128_against_stored_oracle_cells(lib, ctx):
    """The 128^3 field (embedding 540^3; a launch of two samples, the first of
    them the stored one): log k at 4096 and the plain coarse companion at 2048
    cells that the oracle sampled, stored with the model's parameters."""
    with open(FIELD128) as f:
        rec = json.load(f)
    assert {int(a): b for a, b in rec["n_ce"].items()} == MODEL.n_ce
    for key in ("norm_r", "lam", "sigma2", "mu", "interface_kind", "seed"):
        v = getattr(MODEL, key)
        assert (list(v) if isinstance(v, tuple) else v) == rec["model"][key], key
    fr = rec["field"]
    m, level, s0 = fr["m"], fr["level"], fr["sample"]
    print("3-D field m=%d level=%d (stored)" % (m, level), flush=True)
    k, kc = f64(2, m, m, m), f64(2, m // 2, m // 2, m // 2)
    lib.mlmc_sample_field(ctx, MODEL, m, level, s0, 2, k, kc)
    torch.cuda.synchronize()
    lk = torch.log(k[0]).flatten().cpu().numpy()[np.array(fr["cells"])]
    lkc = torch.log(kc[0]).flatten().cpu().numpy()[np.array(fr["coarse_cells"])]
    assert np.max(np.abs(lk - np.array(fr["log_k"]))) <= 1e-11
    assert np.max(np.abs(lkc - np.array(fr["log_k_coarse"]))) <= 1e-11


def test_field_3d_piecewise_constant(lib, ctx):
    model = MODEL.with_(field_kind=W.PIECEWISE_CONSTANT)
    m, batch = 12, 4
    k, kc = f64(batch, m, m, m), f64(batch, m // 2, m // 2, m // 2)
    lib.mlmc_sample_field(ctx, model, m, 2, 0, batch, k, kc)
    torch.cuda.synchronize()
    for s in range(batch):
        kr, kcr = ofield.sample_k(model, 2, s, m, with_coarse=True)
        np.testing.assert_allclose(k[s].cpu().numpy(), kr, rtol=1e-14)
        np.testing.assert_allclose(kc[s].cpu().numpy(), kcr, rtol=1e-14)


def test_cgv_extract_3d_exact(lib, ctx):
    rng = np.random.default_rng(2)
    m, batch = 6, 2
    kh = rng.random((batch, m, m, m))
    ks = f64(batch * 8, m // 2, m // 2, m // 2)
    lib.mlmc_cgv_extract(ctx, 3, m, batch, torch.from_numpy(kh).to(DEV), ks)
    torch.cuda.synchronize()
    ks = ks.cpu().numpy()
    for s in range(batch):
        for j, sub in enumerate(ofield.cgv_sublattices(kh[s])):
            np.testing.assert_array_equal(ks[s * 8 + j], sub)


# ------------------------------------------------------------------ assembly, solve, QoI
def test_assemble_3d_matches_oracle(lib, ctx):
    rng = np.random.default_rng(4)
    m, batch = 6, 2
    kh = np.exp(rng.standard_normal((batch, m, m, m)))
    out = solve3(lib, ctx, kh)
    for s in range(batch):
        Tint, Tb = ofv.face_transmissibilities(kh[s])
        T = out["T"][s]
        # oracle axes (x3, x2, x1): T[2] faces along x1, T[1] along x2, T[0] along x3
        np.testing.assert_allclose(T[0][:, :, :-1], Tint[2], rtol=1e-14)
        np.testing.assert_allclose(T[1][:, :-1, :], Tint[1], rtol=1e-14)
        np.testing.assert_allclose(T[2][:-1, :, :], Tint[0], rtol=1e-14)
        np.testing.assert_allclose(T[0][:, :, -1], Tb[:, :, -1], rtol=1e-15)
        assert np.all(T[1][:, -1, :] == 0) and np.all(T[2][-1] == 0)
        np.testing.assert_allclose(out["tb"][s][0], Tb[:, :, 0], rtol=1e-15)
        assert np.all(out["tb"][s][1] == 0) and np.all(out["tb"][s][2] == 0)
        _, bref = ofv.assemble(kh[s])
        np.testing.assert_allclose(out["b"][s].ravel(), bref, rtol=1e-15)


@pytest.mark.parametrize("m", [1, 2, 3, 4, 6, 8, 12, 16, 24])
def test_solve_3d_random_lognormal(lib, ctx, m):
    print("3-D solve m=%d" % m, flush=True)
    rng = np.random.default_rng(900 + m)
    batch = 3
    kh = np.exp(1.5 * rng.standard_normal((batch, m, m, m)))
    out = solve3(lib, ctx, kh)
    assert np.all(out["status"] == 0), out["status"]
    assert np.all(out["relres"] < 1e-12), out["relres"]
    for s in range(batch):
        A, b = ofv.assemble(kh[s])
        pr = osolve.direct_solve(A, b)
        q = oqoi.outflow(kh[s], pr)
        assert abs(out["q_out"][s] - q) <= QTOL * q, (s, out["q_out"][s], q)
        assert abs(out["q_in"][s] - q) <= 1e-9 * q


@pytest.mark.parametrize("m,variant,nu,prec", [(6, 1, 1, 0), (12, 1, 1, 0), (24, 1, 1, 1),
                                               (24, 0, 2, 0), (16, 0, 2, 1), (32, 0, 1, 0),
                                               (8, 0, 1, 0), (16, 0, 1, 1)])
def test_solve_3d_pressure_field_matches_oracle(lib, ctx, m, variant, nu, prec):
    """The whole pressure field against the oracle's direct solve, with the
    levels swept per launch (vectors and faces in colour-split order) reaching
    down to the dense coarsest grid of side 3 or 4 (variant 1, or two sweeps
    per visit), stopping above the in-LDS levels (the defaults), or absent (the
    finest level in LDS: m = 8 in FP64, 16 in FP32).  The solution comes back in
    natural order: its true residual is below 1e-12 and every cell matches."""
    print("3-D pressure field m=%d variant=%d nu=%d precision=%d" % (m, variant, nu, prec),
          flush=True)
    rng = np.random.default_rng(1300 + m + 7 * nu + 3 * variant)
    batch = 2
    kh = np.exp(1.5 * rng.standard_normal((batch, m, m, m)))
    opts = lib.mlmc_solver_opts_default(variant=variant, nu1=nu, nu2=nu, precision=prec)
    out = solve3(lib, ctx, kh, opts)
    assert np.all(out["status"] == 0), out["status"]
    assert np.all(out["relres"] < 1e-12), out["relres"]
    for s in range(batch):
        A, b = ofv.assemble(kh[s])
        pref = osolve.direct_solve(A, b).reshape(m, m, m)
        assert np.max(np.abs(out["p"][s] - pref)) <= 1e-9, np.max(np.abs(out["p"][s] - pref))


@pytest.mark.parametrize("gamma,glev", [(1, 2), (2, 2), (2, 0)])
def test_solve_3d_cycles_same_solution(lib, ctx, gamma, glev):
    rng = np.random.default_rng(31)
    m = 16
    kh = np.exp(rng.standard_normal((2, m, m, m)))
    out = solve3(lib, ctx, kh, lib.mlmc_solver_opts_default(gamma=gamma, gamma_levels=glev))
    assert np.all(out["status"] == 0)
    print("3-D m=16 gamma %d levels %d iterations %s" % (gamma, glev, out["iters"]), flush=True)
    assert np.all(out["iters"] <= 40)
    for s in range(2):
        A, b = ofv.assemble(kh[s])
        q = oqoi.outflow(kh[s], osolve.direct_solve(A, b))
        assert abs(out["q_out"][s] - q) <= QTOL * q


@pytest.mark.parametrize("m,coarse_max,glev,prec", [(6, 4, 2, 0), (8, 1, 0, 0), (8, 2, 0, 1),
                                                    (12, 4, 0, 0), (12, 2, 2, 1), (16, 1, 2, 1),
                                                    (24, 2, 0, 0), (24, 4, 0, 1), (32, 1, 0, 1),
                                                    (32, 4, 2, 1)])
def test_solve_3d_small_level_cycle(lib, ctx, m, coarse_max, glev, prec):
    """The levels of side <= 8 (FP64 hierarchy) or <= 16 (FP32) run as one
    in-LDS cycle: hierarchies of two to five such levels (coarsest 1, 2, 3 or
    4), W on every level or on the two finest, the cycle starting at the finest
    level or below it.  QoIs at the oracle's value, iterations bounded."""
    print("3-D small-level cycle m=%d coarse_max=%d gamma_levels=%d precision=%d"
          % (m, coarse_max, glev, prec), flush=True)
    rng = np.random.default_rng(1100 + m + coarse_max)
    batch = 3
    kh = np.exp(1.5 * rng.standard_normal((batch, m, m, m)))
    opts = lib.mlmc_solver_opts_default(gamma=2, gamma_levels=glev, coarse_max=coarse_max,
                                        precision=prec)
    out = solve3(lib, ctx, kh, opts)
    assert np.all(out["status"] == 0), out["status"]
    assert np.all(out["iters"] <= 40), out["iters"]
    for s in range(batch):
        A, b = ofv.assemble(kh[s])
        q = oqoi.outflow(kh[s], osolve.direct_solve(A, b))
        assert abs(out["q_out"][s] - q) <= QTOL * q, (s, out["q_out"][s], q)


def test_solve_3d_closed_forms(lib, ctx):
    m = 8
    kh = np.full((1, m, m, m), 3.7)
    out = solve3(lib, ctx, kh)
    assert abs(out["q_out"][0] - 3.7) <= 1e-11 * 3.7
    x1 = (np.arange(m) + 0.5) / m
    assert np.max(np.abs(out["p"][0] - (1.0 - x1)[None, None, :])) < 1e-10
    rng = np.random.default_rng(8)
    kj = np.exp(rng.standard_normal(m))
    kh = np.broadcast_to(kj[None, :, None], (m, m, m))[None].copy()   # layers along the flow
    out = solve3(lib, ctx, kh)
    assert abs(out["q_out"][0] - kj.mean()) <= 1e-11 * kj.mean()


@pytest.mark.parametrize("m", [4, 8, 16, 32])
def test_solve_3d_fp32_hierarchy(lib, ctx, m):
    """The multigrid hierarchy in FP32 inside the flexible FP64 CG: every QoI at
    the oracle's value (1e-10), iteration counts within a few of the FP64 ones."""
    print("3-D FP32 hierarchy m=%d" % m, flush=True)
    rng = np.random.default_rng(700 + m)
    batch = 3
    kh = np.exp(1.5 * rng.standard_normal((batch, m, m, m)))
    o32 = solve3(lib, ctx, kh, lib.mlmc_solver_opts_default(precision=lib.MLMC_PREC_FP32))
    o64 = solve3(lib, ctx, kh)
    assert np.all(o32["status"] == 0), o32["status"]
    assert np.all(o32["iters"] <= o64["iters"] + 3), (o32["iters"], o64["iters"])
    for s in range(batch):
        A, b = ofv.assemble(kh[s])
        q = oqoi.outflow(kh[s], osolve.direct_solve(A, b))
        assert abs(o32["q_out"][s] - q) <= QTOL * q, (s, o32["q_out"][s], q)


def test_level_run_3d_fp32_matches_oracle(lib, ctx):
    m, n = 32, 3
    print("3-D level run FP32 hierarchy m=%d" % m, flush=True)
    qf, qc = f64(n), f64(n)
    sums = lib.mlmc_level_run(ctx, MODEL, 1, m, 40, n, False,
                              lib.mlmc_solver_opts_default(precision=lib.MLMC_PREC_FP32),
                              q_f=qf, q_c=qc)
    torch.cuda.synchronize()
    assert sums.n_failed == 0
    qf, qc = qf.cpu().numpy(), qc.cpu().numpy()
    for s in range(n):
        ref = omlmc.level_sample(MODEL, 1, 40 + s, m)
        assert abs(qf[s] - ref["Q_f"]) <= QTOL * ref["Q_f"], (s, qf[s], ref["Q_f"])
        assert abs(qc[s] - ref["Q_c"]) <= QTOL * ref["Q_c"], (s, qc[s], ref["Q_c"])


def test_solve_3d_refusals(lib, ctx):
    kh = np.ones((1, 8, 8, 8))
    with pytest.raises(lib.MlmcError):
        solve3(lib, ctx, kh, lib.mlmc_solver_opts_default(precision=lib.MLMC_PREC_BF16))
    with pytest.raises(lib.MlmcError):
        solve3(lib, ctx, np.ones((1, 10, 10, 10)))          # coarsest 5 > 4


# ------------------------------------------------------------------ level runs
@pytest.mark.parametrize("cgv", [False, True])
def test_level_run_3d_matches_oracle(lib, ctx, cgv):
    m, n = 16, 4
    print("3-D level run m=%d cgv=%d" % (m, cgv), flush=True)
    qf, qc, y = f64(n), f64(n), f64(n)
    sums = lib.mlmc_level_run(ctx, MODEL, 1, m, 11, n, cgv, lib.mlmc_solver_opts_default(),
                              q_f=qf, q_c=qc, y=y)
    torch.cuda.synchronize()
    assert sums.n == n and sums.n_failed == 0
    qf, qc = qf.cpu().numpy(), qc.cpu().numpy()
    for s in range(n):
        ref = omlmc.level_sample(MODEL, 1, 11 + s, m, cgv=cgv)
        assert abs(qf[s] - ref["Q_f"]) <= QTOL * ref["Q_f"], (s, qf[s], ref["Q_f"])
        assert abs(qc[s] - ref["Q_c"]) <= QTOL * ref["Q_c"], (s, qc[s], ref["Q_c"])


GOLDEN3 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                       "tilted3_64_128_plain.json")


def _served_opts(lib, prec):
    return lib.mlmc_solver_opts_default(
        precision=lib.MLMC_PREC_FP32 if prec == "f32" else lib.MLMC_PREC_FP64)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_level_run_3d_served_sizes(lib, ctx, prec):
    """The served 3-D level runs (32^3/64, 64^3/16, 128^3/4 samples) with the
    FP64 hierarchy and with the FP32 hierarchy the served mix uses: every solve
    converges; the 32^3 sample matches the oracle's direct solve; samples 0 and
    1 of the 64^3 and 128^3 levels match the oracle's conjugate gradient solve
    to 1e-14 (stored by tests/golden/make_golden.py), fine and coarse QoI."""
    with open(GOLDEN3) as f:
        gold = {lv["level"]: lv for lv in json.load(f)["levels"]}
    for level, (m, n) in enumerate(zip(W.SERVED_3D.m_levels, W.SERVED_3D.n_samples)):
        print("3-D served level %d m=%d n=%d %s" % (level, m, n, prec), flush=True)
        qf, qc = f64(n), f64(n)
        sums = lib.mlmc_level_run(ctx, MODEL, level, m, 0, n, False, _served_opts(lib, prec),
                                  q_f=qf, q_c=qc)
        torch.cuda.synchronize()
        assert sums.n_failed == 0
        assert sums.iters_fine / n <= 30, sums.iters_fine / n
        qf, qc = qf.cpu().numpy(), qc.cpu().numpy()
        if m == 32:
            ref = omlmc.level_sample(MODEL, level, 0, m)
            assert abs(qf[0] - ref["Q_f"]) <= QTOL * ref["Q_f"]
            assert abs(qc[0] - ref["Q_c"]) <= QTOL * ref["Q_c"]
        else:
            lv = gold[level]
            assert lv["m"] == m
            for row in lv["samples"]:
                s = row["sample"]
                assert abs(qf[s] - row["Q_f"]) <= QTOL * row["Q_f"], (m, s, qf[s], row["Q_f"])
                assert abs(qc[s] - row["Q_c"]) <= QTOL * row["Q_c"], (m, s, qc[s], row["Q_c"])


def test_level_run_3d_served_sizes_fp32_equals_fp64(lib, ctx):
    """Per sample, the FP32-hierarchy served level runs give the FP64
    hierarchy's QoIs to 1e-10 on every sample of 64^3 and 128^3."""
    for level, (m, n) in enumerate(zip(W.SERVED_3D.m_levels, W.SERVED_3D.n_samples)):
        if m < 64:
            continue
        print("3-D served FP32 vs FP64 m=%d" % m, flush=True)
        out = {}
        for prec in ("f64", "f32"):
            qf, qc = f64(n), f64(n)
            sums = lib.mlmc_level_run(ctx, MODEL, level, m, 100, n, False,
                                      _served_opts(lib, prec), q_f=qf, q_c=qc)
            torch.cuda.synchronize()
            assert sums.n_failed == 0
            out[prec] = (qf.cpu().numpy(), qc.cpu().numpy())
        np.testing.assert_allclose(out["f32"][0], out["f64"][0], rtol=QTOL, atol=0)
        np.testing.assert_allclose(out["f32"][1], out["f64"][1], rtol=QTOL, atol=0)


@pytest.mark.parametrize("m", [8, 16, 32])
@pytest.mark.parametrize("gamma,gamma_levels", [(1, 2), (2, 2), (2, 0)])
def test_in_lds_cycle_equals_per_sweep_cycle(lib, ctx, m, gamma, gamma_levels):
    """The in-LDS coarse cycle takes the per-sweep cycle's steps in its order:
    with the FP64 hierarchy both give the same per-sample iteration counts (a
    wrongly ordered visit or restriction would change them) and the same QoIs
    to rounding; variant 1 forces the per-sweep cycle on every level."""
    print("3-D in-LDS vs per-sweep m=%d gamma=%d/%d" % (m, gamma, gamma_levels), flush=True)
    rng = np.random.default_rng(1200 + m)
    kh = np.exp(1.5 * rng.standard_normal((4, m, m, m)))
    lds = solve3(lib, ctx, kh, lib.mlmc_solver_opts_default(gamma=gamma,
                                                            gamma_levels=gamma_levels))
    per = solve3(lib, ctx, kh, lib.mlmc_solver_opts_default(gamma=gamma, gamma_levels=gamma_levels,
                                                            variant=1))
    assert np.all(lds["status"] == 0) and np.all(per["status"] == 0)
    np.testing.assert_array_equal(lds["iters"], per["iters"])
    np.testing.assert_allclose(lds["q_out"], per["q_out"], rtol=1e-12, atol=0)


@pytest.mark.parametrize("m,prec", [(16, "f64"), (32, "f32"), (64, "f32"), (64, "f64"),
                                    (128, "f64"), (128, "f32")])
def test_default_cycle_equals_per_sweep_cycle_large(lib, ctx, m, prec):
    """The default cycle (small levels in the in-LDS kernel) against variant 1
    (one launch per half-sweep on every level) up to 128^3, with both
    hierarchies and W on every level: the same iteration counts and, to
    rounding, the same QoIs and pressures."""
    print("3-D default vs per-sweep m=%d %s" % (m, prec), flush=True)
    rng = np.random.default_rng(1300 + m)
    kh = np.exp(1.5 * rng.standard_normal((3, m, m, m)))
    p = lib.MLMC_PREC_FP32 if prec == "f32" else lib.MLMC_PREC_FP64
    a = solve3(lib, ctx, kh, lib.mlmc_solver_opts_default(precision=p, gamma_levels=0))
    b = solve3(lib, ctx, kh, lib.mlmc_solver_opts_default(precision=p, gamma_levels=0, variant=1))
    assert np.all(a["status"] == 0) and np.all(b["status"] == 0)
    np.testing.assert_array_equal(a["iters"], b["iters"])
    np.testing.assert_allclose(a["q_out"], b["q_out"], rtol=1e-12, atol=0)
    np.testing.assert_allclose(a["p"], b["p"], rtol=0, atol=1e-12)


def test_serve_3d(lib, ctx):
    grids = [16, 32]
    opts = lib.serve_opts_for(MODEL, grids, n_workers=2, max_batch=8)
    srv = lib.mlmc_serve_start(MODEL, opts)
    try:
        reqs = [(0, 16, 40 + i) for i in range(5)] + [(1, 32, 60 + i) for i in range(3)]
        ids = [lib.mlmc_serve_submit(srv, *r) for r in reqs]
        import time
        out, t0 = {}, time.time()
        while len(out) < len(ids):
            res, _ = lib.mlmc_serve_poll(srv)
            for r in res:
                out[r["id"]] = r
            assert time.time() - t0 < 60
            time.sleep(0.002)
    finally:
        lib.mlmc_serve_stop(srv)
    for r, i in zip(reqs, ids):
        assert out[i]["failed"] == 0 and out[i]["status"] == 0
    level, m, sample = reqs[-1]
    ref = omlmc.level_sample(MODEL, level, sample, m)
    got = out[ids[-1]]
    assert abs(got["q_f"] - ref["Q_f"]) <= QTOL * ref["Q_f"]
    assert abs(got["q_c"] - ref["Q_c"]) <= QTOL * ref["Q_c"]
