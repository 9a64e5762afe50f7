"""Serving form: continuous batching of MLMC sample requests (GPU).

* Every request's (Q_f, Q_c, Y) is bitwise the same when served alone and in a
  mixed load (levels and grid sizes interleaved, several workers in flight),
  equal to the library's direct level run, and within 1e-10 of the oracle.
* A device-memory budget smaller than two requests serialises the batches
  (batch size 1, never two running) without failures.
* Malformed requests are refused.
* One server serves several models (2-D with an FP32 multigrid, 3-D in FP64):
  each result equals the direct level run of its own model and options.
"""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import workloads as W  # noqa: E402
from oracle import field as ofield  # noqa: E402
from oracle import mlmc as omlmc  # noqa: E402

MODEL = W.CE2
GRIDS = [32, 64, 128]


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1506_04694_amd as lib
    return lib


def drain(lib, srv, count, timeout=60.0):
    out = {}
    t0 = time.time()
    while len(out) < count:
        res, _ = lib.mlmc_serve_poll(srv)
        for r in res:
            out[r["id"]] = r
        if time.time() - t0 > timeout:
            raise TimeoutError("server did not finish %d requests" % count)
        time.sleep(0.002)
    return out


def mixed_requests():
    reqs = []
    for i in range(12):
        reqs.append((0, 32, 100 + i))
        reqs.append((1, 64, 200 + i))
        if i % 2 == 0:
            reqs.append((2, 128, 300 + i))
    return reqs


def test_serve_same_alone_and_in_mix(lib):
    print("serve mixed", flush=True)
    opts = lib.serve_opts_for(MODEL, GRIDS, n_workers=3, max_batch=16)
    srv = lib.mlmc_serve_start(MODEL, opts)
    try:
        reqs = mixed_requests()
        ids = [lib.mlmc_serve_submit(srv, *r) for r in reqs]
        mixed = drain(lib, srv, len(ids))
        assert all(mixed[i]["failed"] == 0 and mixed[i]["status"] == 0 for i in ids)
        assert max(mixed[i]["batch_size"] for i in ids) > 1
        alone = {}
        for r in reqs[::5]:
            rid = lib.mlmc_serve_submit(srv, *r)
            alone[r] = drain(lib, srv, 1)[rid]
            assert alone[r]["batch_size"] == 1
        by_req = {r: mixed[i] for r, i in zip(reqs, ids)}
        for r, a in alone.items():
            b = by_req[r]
            assert (a["q_f"], a["q_c"], a["y"]) == (b["q_f"], b["q_c"], b["y"]), r
    finally:
        lib.mlmc_serve_stop(srv)
    # the direct batched call gives the same numbers
    ctx = lib.mlmc_ctx_create(0, torch.cuda.current_stream(0))
    try:
        for level, m in ((0, 32), (1, 64)):
            rs = [r for r in reqs if r[0] == level]
            sid = torch.tensor([r[2] for r in rs], dtype=torch.int32, device="cuda:0")
            qf = torch.empty(len(rs), dtype=torch.float64, device="cuda:0")
            qc = torch.empty_like(qf)
            lib.mlmc_level_run_ids(ctx, MODEL, level, m, sid, len(rs), False,
                                   lib.mlmc_solver_opts_default(), q_f=qf, q_c=qc)
            torch.cuda.synchronize()
            for q, r in enumerate(rs):
                assert qf[q].item() == by_req[r]["q_f"] and qc[q].item() == by_req[r]["q_c"]
    finally:
        lib.mlmc_ctx_destroy(ctx)
    # and the oracle agrees to the parity tolerance
    for r in (reqs[0], reqs[1]):
        level, m, sample = r
        k, kc = ofield.sample_k(MODEL, level, sample, m, with_coarse=True)
        qf_ref = omlmc.solve_qoi(k)[0]
        assert abs(by_req[r]["q_f"] - qf_ref) <= 1e-10 * qf_ref
        if level > 0:
            qc_ref = omlmc.solve_qoi(kc)[0]
            assert abs(by_req[r]["q_c"] - qc_ref) <= 1e-10 * qc_ref


def test_serve_tiny_budget_serialises(lib):
    print("serve tiny budget", flush=True)
    opts = lib.serve_opts_for(MODEL, GRIDS, n_workers=3, max_batch=16, hbm_budget_bytes=1)
    srv = lib.mlmc_serve_start(MODEL, opts)
    try:
        ids = [lib.mlmc_serve_submit(srv, 1, 64, 400 + i) for i in range(6)]
        res = drain(lib, srv, len(ids))
        assert all(res[i]["batch_size"] == 1 and res[i]["failed"] == 0 for i in ids)
        spans = sorted((res[i]["t_start"], res[i]["t_done"]) for i in ids)
        for (a0, a1), (b0, b1) in zip(spans[:-1], spans[1:]):
            assert b0 >= a1 - 1e-6, "two batches ran at once under a one-request budget"
    finally:
        lib.mlmc_serve_stop(srv)


def test_serve_rejects_bad_requests(lib):
    opts = lib.serve_opts_for(MODEL, GRIDS)
    srv = lib.mlmc_serve_start(MODEL, opts)
    try:
        with pytest.raises(lib.MlmcError):
            lib.mlmc_serve_submit(srv, 1, 33, 0)      # odd fine grid on level >= 1
        with pytest.raises(lib.MlmcError):
            lib.mlmc_serve_submit(srv, 0, 48, 0)      # grid without an embedding size
    finally:
        lib.mlmc_serve_stop(srv)


def test_serve_two_models_2d_fp32_and_3d(lib):
    """One server for a 2-D model (multigrid in FP32 inside the FP64 CG) and the
    3-D model (FP64): interleaved requests of both come back bitwise equal to
    the direct level runs of their own model and options, and within 1e-10 of
    the oracle."""
    print("serve 2-D + 3-D", flush=True)
    m3 = W.TILTED3
    opts = lib.serve_opts_for_models([(MODEL, [32, 64]), (m3, [16, 32])], n_workers=3,
                                     max_batch=8)
    s2 = lib.mlmc_solver_opts_default(precision=lib.MLMC_PREC_FP32)
    s3 = lib.mlmc_solver_opts_default()
    srv = lib.mlmc_serve_start_models([MODEL, m3], opts, solvers=[s2, s3])
    reqs = []
    for i in range(6):
        reqs += [(0, 32, 500 + i, 0), (1, 64, 600 + i, 0), (0, 16, 700 + i, 1)]
        if i % 2 == 0:
            reqs.append((1, 32, 800 + i, 1))
    try:
        with pytest.raises(lib.MlmcError):
            lib.mlmc_serve_submit(srv, 0, 32, 0, model=2)      # no such model
        with pytest.raises(lib.MlmcError):
            lib.mlmc_serve_submit(srv, 0, 64, 0, model=1)      # 64 is not a 3-D grid here
        ids = [lib.mlmc_serve_submit(srv, *r) for r in reqs]
        got = drain(lib, srv, len(ids))
    finally:
        lib.mlmc_serve_stop(srv)
    by_req = {r: got[i] for r, i in zip(reqs, ids)}
    assert all(v["failed"] == 0 and v["status"] == 0 for v in by_req.values())
    assert all(v["model"] == r[3] for r, v in by_req.items())
    ctx = lib.mlmc_ctx_create(0, torch.cuda.current_stream(0))
    try:
        for model_i, model, sol in ((0, MODEL, s2), (1, m3, s3)):
            for level in (0, 1):
                rs = [r for r in reqs if r[3] == model_i and r[0] == level]
                m = rs[0][1]
                sid = torch.tensor([r[2] for r in rs], dtype=torch.int32, device="cuda:0")
                qf = torch.empty(len(rs), dtype=torch.float64, device="cuda:0")
                qc = torch.empty_like(qf)
                lib.mlmc_level_run_ids(ctx, model, level, m, sid, len(rs), False, sol,
                                       q_f=qf, q_c=qc)
                torch.cuda.synchronize()
                for q, r in enumerate(rs):
                    assert qf[q].item() == by_req[r]["q_f"], r
                    assert qc[q].item() == by_req[r]["q_c"], r
    finally:
        lib.mlmc_ctx_destroy(ctx)
    for r in ((1, 64, 600, 0), (1, 32, 800, 1)):
        level, m, sample, mi = r
        model = (MODEL, m3)[mi]
        k, kc = ofield.sample_k(model, level, sample, m, with_coarse=True)
        qf_ref, qc_ref = omlmc.solve_qoi(k)[0], omlmc.solve_qoi(kc)[0]
        assert abs(by_req[r]["q_f"] - qf_ref) <= 1e-10 * qf_ref, r
        assert abs(by_req[r]["q_c"] - qc_ref) <= 1e-10 * qc_ref, r


def test_serve_start_models_refusals(lib):
    opts = lib.serve_opts_for_models([(MODEL, [32])])
    opts.grid_model[0] = 1                                   # grid of a model not given
    with pytest.raises(lib.MlmcError):
        lib.mlmc_serve_start_models([MODEL], opts)
    with pytest.raises(lib.MlmcError):
        lib.mlmc_serve_start_models([], lib.serve_opts_for_models([(MODEL, [32])]))


def test_serve_model_problems_and_three_layers(lib):
    """One server for the layered model under Model Problem 2 and under Model
    Problem 1, and for the paper's three-layer model (two embedding samples per
    field): each result is bitwise the direct level run of its own model and
    within 1e-10 of the oracle's QoI of its problem."""
    print("serve MP2 + MP1 + three layers", flush=True)
    models = [MODEL, W.MP1_CE2, W.PAPER3_CE]
    opts = lib.serve_opts_for_models([(mdl, [32, 64]) for mdl in models], n_workers=3,
                                     max_batch=8)
    srv = lib.mlmc_serve_start_models(models, opts)
    reqs = []
    for i in range(5):
        for mi in range(3):
            reqs.append((i % 2, 32 if i % 2 == 0 else 64, 900 + 10 * mi + i, mi))
    try:
        ids = [lib.mlmc_serve_submit(srv, *r) for r in reqs]
        got = drain(lib, srv, len(ids))
    finally:
        lib.mlmc_serve_stop(srv)
    by_req = {r: got[i] for r, i in zip(reqs, ids)}
    assert all(v["failed"] == 0 and v["status"] == 0 for v in by_req.values())
    ctx = lib.mlmc_ctx_create(0, torch.cuda.current_stream(0))
    try:
        for r, v in by_req.items():
            level, m, sample, mi = r
            qf = torch.empty(1, dtype=torch.float64, device="cuda:0")
            qc = torch.empty_like(qf)
            lib.mlmc_level_run(ctx, models[mi], level, m, sample, 1, False,
                               lib.mlmc_solver_opts_default(), q_f=qf, q_c=qc)
            torch.cuda.synchronize()
            assert qf.item() == v["q_f"] and qc.item() == v["q_c"], r
    finally:
        lib.mlmc_ctx_destroy(ctx)
    for r in ((1, 64, 911, 1), (0, 32, 920, 2)):
        level, m, sample, mi = r
        ref = omlmc.level_sample(models[mi], level, sample, m)
        assert abs(by_req[r]["q_f"] - ref["Q_f"]) <= 1e-10 * ref["Q_f"], r
        assert abs(by_req[r]["q_c"] - ref["Q_c"]) <= 1e-10 * abs(ref["Q_c"]) + 1e-300, r
