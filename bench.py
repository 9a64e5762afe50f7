#!/usr/bin/env python
"""Throughput of the MLMC hot path on one MI355X.

One step = one pass of the whole path over the layered correlated workload:
for each level l (grids 64^2, 128^2, 256^2, 512^2 with 4096/1024/256/64
samples) sample k by circulant embedding, assemble the finite volume system,
solve it by multigrid-preconditioned CG to relative residual 1e-13, take the
outflow QoI, do the same for the plain coarse companion (levels >= 1), and
reduce Y = Q_f - Q_c into the level sums.  Every step draws fresh samples.
The levels run one after another (each on its own context and stream);
--concurrent-levels runs them at once from four host threads.

Prints one JSON line: value = Y-samples per second over all levels (the
per-level rates are in "per_level"), a roofline entry for the dominant
kernel timed live with HIP events, and the CPU oracle timed on a bounded
sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

METRIC = "MLMC samples solved/s per level at 1e-10 QoI rel-err; HBM GB/s; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
# The dominant kernel of the step: the W second visit on the finest grid of
# every solve, k_mg_mid_p<64, 32, 768, double, true> (its own instantiation, the
# top line of the rocprofv3 summary).  "@0" selects that level's launches.
DOMINANT = "k_mg_mid@0"
DOMINANT_SYMBOL = "mlmc::k_mg_mid_p<64, 32, 768, double, true>"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--kernel", default=DOMINANT, help="kernel label timed for the roofline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-sample", action="store_true",
                    help="skip timing the unbatched one-sample-per-call GPU path")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work")
    ap.add_argument("--serve-rates", default="0.5,0.8,0.95",
                    help="offered request rates as fractions of the batched throughput ('' = skip)")
    ap.add_argument("--serve-seconds", type=float, default=2.0,
                    help="seconds of Poisson arrivals per offered rate")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip timing the all-levels-in-one-call and FP32-multigrid forms")
    ap.add_argument("--concurrent-levels", action="store_true",
                    help="run the levels of a step at once (own streams and host threads)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration) and exit")
    ap.add_argument("--served-3d-only", action="store_true",
                    help="only time the served 3-D model's level runs (served_3d) and print them")
    return ap.parse_args()


def _oracle_levels(wl, budget_s, first_sample=0):
    """The oracle (as it is) on consecutive samples of each level from first_sample,
    one thread, for about budget_s seconds in all: seconds per Y-sample per level."""
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(1)
    except Exception:  # pragma: no cover
        limiter = None
    from oracle import field as ofield
    from oracle import mlmc as omlmc
    per_level = []
    share = budget_s / len(wl.m_levels)
    for level, (m, n) in enumerate(zip(wl.m_levels, wl.n_samples)):
        lam = ofield.ce_eigenvalues(wl.model.n_ce[m], m, wl.model.sigma2[0], wl.model.lam[0],
                                    wl.model.norm_r)
        done, t0 = 0, time.perf_counter()
        while True:
            omlmc.level_sample(wl.model, level, first_sample + done, m, cgv=wl.cgv, lam_eig=lam)
            done += 1
            el = time.perf_counter() - t0
            if el >= share or done >= n:
                break
        per_level.append((done, el))
    if limiter is not None and hasattr(limiter, "unregister"):
        limiter.unregister()
    return per_level


def _oracle_worker(args):
    wl_name, budget_s, first_sample = args
    wl = {w.name: w for w in (W.LAYERED_CE,)}[wl_name]
    return _oracle_levels(wl, budget_s, first_sample)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, budget_s):
    """The oracle (as it is) on the first samples of each level: one thread for
    budget_s seconds (the single-core rate), then C single-threaded processes at
    once on disjoint samples (C = the host cores this process may use, at most 16,
    the machine's CPU share) for budget_s / 2 seconds each (the aggregate host rate).
    Rates are Y-samples/s extrapolated to the full level sizes."""
    one = _oracle_levels(wl, budget_s)
    s_per = [el / done for done, el in one]
    single = sum(wl.n_samples) / sum(sp * n for sp, n in zip(s_per, wl.n_samples))
    cores = min(len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
                else os.cpu_count() or 1, 16)
    agg = None
    if cores > 1:
        import multiprocessing as mp
        t0 = time.perf_counter()
        with mp.get_context("spawn").Pool(cores) as pool:
            res = pool.map(_oracle_worker, [(wl.name, budget_s / 2, 10 ** 6 * (c + 1))
                                            for c in range(cores)])
        wall = time.perf_counter() - t0
        # per level: samples done by all processes over the slowest process's time there
        rate_lv = []
        for lv in range(len(wl.m_levels)):
            done = sum(r[lv][0] for r in res)
            el = max(r[lv][1] for r in res)
            rate_lv.append(done / el)
        agg = {"value": sum(wl.n_samples) / sum(n / r for n, r in zip(wl.n_samples, rate_lv)),
               "cores": cores, "wall_s": wall,
               "samples_per_level": [sum(r[lv][0] for r in res) for lv in range(len(wl.m_levels))]}
    return {"value": agg["value"] if agg else single, "unit": "samples/s",
            "cores": cores if agg else 1, "kind": "oracle", "cpu_model": cpu_model(),
            "sample": "oracle on the first samples of levels %s (of %s): %s samples on one "
                      "thread in %.1f s%s; Y-samples incl. coarse companion, rates extrapolated "
                      "to the full level sizes; the oracle solves directly (sparse LU) where the "
                      "GPU uses multigrid, so the ratio mixes an algorithmic and a hardware gap"
                      % ("/".join("%d^2" % m for m in wl.m_levels),
                         "/".join(str(n) for n in wl.n_samples),
                         "/".join(str(d) for d, _ in one), sum(el for _, el in one),
                         ("" if not agg else "; then %d single-threaded processes at once on "
                          "disjoint samples (%s per level)" % (cores, "/".join(
                              str(x) for x in agg["samples_per_level"])))),
            "single_core": {"value": single, "cores": 1, "per_level_s_per_sample": s_per},
            "aggregate": agg}


SERVE_WORKERS = 4
SERVE_MAX_BATCH = 64


def serve_setup(lib, kinds, models, solvers):
    """Server options for request kinds [(model index, level, m, count)]."""
    grids = [[] for _ in models]
    for mi, _, m, _ in kinds:
        if m not in grids[mi]:
            grids[mi].append(m)
    return lib.serve_opts_for_models(list(zip(models, grids)), n_workers=SERVE_WORKERS,
                                     max_batch=SERVE_MAX_BATCH)


def pass_rate(lib, torch, kinds, models, solvers, reps=2):
    """Requests/s of one batched pass over every kind (count samples each, level
    runs one after another with the kind's model and solver options), after one
    warm-up pass: the saturation estimate the offered loads are scaled to."""
    ctx = lib.mlmc_ctx_create(0, torch.cuda.current_stream(0))
    first = 0
    try:
        for rep in range(reps + 1):
            if rep == 1:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
            for mi, level, m, n in kinds:
                lib.mlmc_level_run(ctx, models[mi], level, m, first, n, False, solvers[mi])
            first += max(k[3] for k in kinds)
        torch.cuda.synchronize()
        per_pass = (time.perf_counter() - t0) / reps
    finally:
        lib.mlmc_ctx_destroy(ctx)
    return sum(k[3] for k in kinds) / per_pass, per_pass


def serving_latency(lib, kinds, models, solvers, rate, seconds, seed=1):
    """Poisson arrivals at `rate` of single-sample requests of the given kinds
    (probability proportional to each kind's count), served by one continuous-
    batching server for all models; latency = completion - submission on the
    server clock."""
    import numpy as np
    rng = np.random.default_rng(seed)
    probs = np.array([k[3] for k in kinds], dtype=float)
    probs /= probs.sum()
    n_req = max(50, int(rate * seconds))
    gaps = rng.exponential(1.0 / rate, size=n_req)
    picks = rng.choice(len(kinds), size=n_req, p=probs)
    srv = lib.mlmc_serve_start_models(models, serve_setup(lib, kinds, models, solvers),
                                      solvers=solvers)
    results = {}
    counters = [10 ** 7] * len(kinds)
    try:
        t = lib.mlmc_serve_now(srv) + 0.05
        for g, kq in zip(gaps, picks):
            t += g
            while lib.mlmc_serve_now(srv) < t:
                pass
            mi, level, m, _ = kinds[kq]
            lib.mlmc_serve_submit(srv, level, m, counters[kq], model=mi)
            counters[kq] += 1
            if len(results) % 64 == 0:
                for r in lib.mlmc_serve_poll(srv)[0]:
                    results[r["id"]] = r
        t_end = time.time() + 60
        while len(results) < n_req and time.time() < t_end:
            for r in lib.mlmc_serve_poll(srv)[0]:
                results[r["id"]] = r
            time.sleep(0.001)
        stats = lib.mlmc_serve_stats(srv)
    finally:
        lib.mlmc_serve_stop(srv)
    rs = list(results.values())
    lat = np.array([r["t_done"] - r["t_submit"] for r in rs])
    span = max(r["t_done"] for r in rs) - min(r["t_submit"] for r in rs)
    per_kind = []
    for mi, level, m, _ in kinds:
        ll = np.array([r["t_done"] - r["t_submit"] for r in rs
                       if r["model"] == mi and r["level"] == level and r["m_fine"] == m])
        if ll.size:
            sel = [r for r in rs if r["model"] == mi and r["level"] == level and r["m_fine"] == m]
            wait = np.array([r["t_start"] - r["t_submit"] for r in sel])
            serv = np.array([r["t_done"] - r["t_start"] for r in sel])
            per_kind.append({"model": mi, "dim": int(models[mi].dim), "level": level, "m": m,
                             "requests": int(ll.size),
                             "p50_ms": 1e3 * float(np.percentile(ll, 50)),
                             "p99_ms": 1e3 * float(np.percentile(ll, 99)),
                             "wait_p50_ms": 1e3 * float(np.percentile(wait, 50)),
                             "wait_p99_ms": 1e3 * float(np.percentile(wait, 99)),
                             "service_p50_ms": 1e3 * float(np.percentile(serv, 50)),
                             "service_p99_ms": 1e3 * float(np.percentile(serv, 99)),
                             "mean_batch": float(np.mean([r["batch_size"] for r in sel]))})
    return {"offered_per_s": rate, "completed": len(rs), "submitted": n_req,
            "achieved_per_s": len(rs) / span, "failed": int(sum(r["failed"] for r in rs)),
            "p50_ms": 1e3 * float(np.percentile(lat, 50)), "p99_ms": 1e3 * float(np.percentile(lat, 99)),
            "mean_batch": float(np.mean([r["batch_size"] for r in rs])), "batches": stats["batches"],
            "per_kind": per_kind}


KERNEL_SOURCES = {"k_mg_mid@0": "mg_fused.hip", "k_mg_mid": "mg_fused.hip", "k_mg_up": "mg_fused.hip",
                  "k_mg_down": "mg_fused.hip", "k_mg_coarse_cycle": "mg_fused.hip",
                  "k_cg_direction_t": "mg_fused.hip", "k_spmv_dot": "mg_pcg.hip",
                  "k_axpy_dot": "mg_pcg.hip", "k_ce_pass_a": "field.hip", "k_ce_pass_b": "field.hip"}


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary
    (profiles/traffic_<kernel>.json, "@<level>" written "_level<level>"), or None when there is none or the kernel's
    source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % kernel.replace("@", "_level"))
    src = KERNEL_SOURCES.get(kernel)
    if not os.path.exists(path) or src is None:
        return None
    with open(path) as f:
        rec = json.load(f)
    with open(os.path.join(ROOT, "paper_1506_04694_amd", "csrc", src), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if rec.get("source_sha256") != sha:
        return None
    return rec["hbm_bytes_per_launch"]


def copy_calibration():
    """A plain device copy of 1 GiB (read 1 GiB, write 1 GiB), three times."""
    import torch
    n = 2 ** 27
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 3
    print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n,
                      "ms": 1e3 * dt, "GB_s_read_plus_write": 16 * n / dt / 1e9}), flush=True)


def path_variants(lib, torch, wl, ctx, opts, args):
    """Other forms of the same step, timed over args.steps steps each after the
    main measurement (not part of `value`):
    * all levels in one call (mlmc_run_levels: each level's pipeline on its own
      stream, concurrently), FP64, with eager launches and with the PCG
      iterations replayed from captured HIP graphs;
    * the per-level step with graph-replayed iterations;
    * the per-level step with the multigrid hierarchy stored in FP32 inside the FP64
      flexible CG, with the largest relative QoI difference to the FP64 solve of
      the same samples."""
    nlev = len(wl.m_levels)
    base = 100  # step numbers (sample ranges) not used by the main measurement

    def timed(f):
        f(base)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            f(base + 1 + k)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps

    def merged(idx):
        lib.mlmc_run_levels(ctx, wl.model, wl.m_levels, [idx * n for n in wl.n_samples],
                            wl.n_samples, wl.cgv, opts)

    o32 = lib.mlmc_solver_opts_default(precision=lib.MLMC_PREC_FP32)

    def per_level(o, idx, q=None):
        for level, (m, n) in enumerate(zip(wl.m_levels, wl.n_samples)):
            kw = {} if q is None else {"q_f": q[level][0], "q_c": q[level][1]}
            lib.mlmc_level_run(ctx, wl.model, level, m, idx * n, n, wl.cgv, o, **kw)

    og = lib.mlmc_solver_opts_default(graph=1)

    def merged_graph(idx):
        lib.mlmc_run_levels(ctx, wl.model, wl.m_levels, [idx * n for n in wl.n_samples],
                            wl.n_samples, wl.cgv, og)

    t_merged = timed(merged)
    t_merged_graph = timed(merged_graph)
    t_graph = timed(lambda idx: per_level(og, idx))
    t_fp32 = timed(lambda idx: per_level(o32, idx))
    qs = []
    for o in (opts, o32):
        q = [(torch.empty(n, dtype=torch.float64, device="cuda"),
              torch.empty(n, dtype=torch.float64, device="cuda")) for n in wl.n_samples]
        per_level(o, base, q)
        qs.append(q)
    torch.cuda.synchronize()
    dev = 0.0
    for level in range(nlev):
        for which in ((0,) if level == 0 else (0, 1)):   # Q_f, and Q_c on levels >= 1
            a, b = qs[0][level][which], qs[1][level][which]
            dev = max(dev, ((a - b).abs() / a.abs()).max().item())
    total = sum(wl.n_samples)
    return {"all_levels_one_call_fp64": {"value": total / t_merged, "ms_per_step": 1e3 * t_merged},
            "all_levels_one_call_fp64_graph": {"value": total / t_merged_graph,
                                               "ms_per_step": 1e3 * t_merged_graph},
            "per_level_fp64_graph": {"value": total / t_graph, "ms_per_step": 1e3 * t_graph},
            "multigrid_fp32_in_fp64_cg": {"value": total / t_fp32, "ms_per_step": 1e3 * t_fp32,
                                          "max_qoi_rel_diff_vs_fp64": dev}}


def cgv_variance(lib, torch, ctx, opts):
    """Section 4.2's experiment: the sample variance of Y_l = Q_l - Q_{l-1} with one
    coarse companion (the plain estimator; the coarse sample is the fine field's
    sub-lattice of even indices) and with Coarse Grid Variates (the mean over the
    2^d sub-lattices, eq. (4.1)), from the same fine samples, on the stationary
    log-normal field with the 1-norm covariance, lambda 0.3, sigma^2 1, Model
    Problem 2, fine grids h_l = 1/8 upwards in 2-D and 3-D."""
    out = {"model": "stationary log-normal, exp. covariance r=1, sigma2=1, lambda=0.3 "
                    "(no layers)", "qoi": "outflow at x1 = 1 (Model Problem 2)"}
    for key, model, levels in (("2d", W.STATIONARY_1NORM, W.CGV_VARIANCE_2D),
                               ("3d", W.STATIONARY_1NORM_3D, W.CGV_VARIANCE_3D)):
        rows = []
        for level, (m, n) in enumerate(levels, start=1):
            row = {"h": 1.0 / m, "m_fine": m, "samples": n}
            for name, cgv in (("plain", False), ("cgv", True)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                s = lib.mlmc_level_run(ctx, model, level, m, 0, n, cgv, opts)
                torch.cuda.synchronize()
                t = time.perf_counter() - t0
                mean = s.sum_y / s.n
                var = (s.sum_y2 - s.n * mean * mean) / (s.n - 1)
                row[name] = {"var_y": var, "mean_y": mean, "ms": 1e3 * t,
                             "samples_per_s": n / t, "failed_solves": int(s.n_failed)}
            row["variance_ratio"] = row["plain"]["var_y"] / row["cgv"]["var_y"]
            rows.append(row)
        out[key] = rows
    return out


def rates_vs_reference(lib, torch, ctx, opts):
    """Section 3.4's convergence observations from reference solutions: for the
    paper's three piecewise constant layers (the sample -- two random lines and
    three log-normal constants -- does not depend on the grid, so each sample is
    solved on every grid and on the reference grid h* = 1/512 in 2-D, 1/128 in
    3-D), the weak error |E[Q_h - Q_h*]| per grid from the paired differences,
    its standard error, the least squares rate alpha_ref, and beside it the rate
    alpha_Y of |E[Q_h - Q_2h]| (the MLMC differences of the same samples), for
    the outflow (Model Problem 2) and the mean pressure (Model Problem 1)."""
    import numpy as np
    out = {}
    for key, model, grids, ref, n in W.RATES_REFERENCE:
        q = {}
        t0 = time.perf_counter()
        for m in grids + [ref]:
            qt = torch.empty(n, dtype=torch.float64, device="cuda")
            lib.mlmc_level_run(ctx, model, 0, m, 0, n, False, opts, q_f=qt)
            q[m] = qt.cpu().numpy()
        rows = []
        for m in grids:
            d = q[m] - q[ref]
            row = {"h": 1.0 / m, "m": m, "weak_error": float(abs(d.mean())),
                   "std_error": float(d.std(ddof=1) / math.sqrt(n))}
            if m // 2 in q:
                y = q[m] - q[m // 2]
                row["mean_y"] = float(y.mean())
                row["var_y"] = float(y.var(ddof=1))
            rows.append(row)
        h = np.array([r["h"] for r in rows])
        e = np.array([r["weak_error"] for r in rows])
        alpha_ref = float(np.polyfit(np.log2(h), np.log2(e), 1)[0])
        hy = np.array([r["h"] for r in rows if "mean_y" in r])
        ey = np.abs(np.array([r["mean_y"] for r in rows if "mean_y" in r]))
        alpha_y = float(np.polyfit(np.log2(hy), np.log2(ey), 1)[0]) if len(hy) >= 2 else None
        vy = np.array([r["var_y"] for r in rows if "var_y" in r])
        beta = float(np.polyfit(np.log2(hy), np.log2(vy), 1)[0]) if len(hy) >= 2 else None
        out[key] = {"dim": int(model.dim), "problem": int(model.problem), "reference_m": ref,
                    "samples": n, "grids": rows, "alpha_ref": alpha_ref, "alpha_y": alpha_y,
                    "beta": beta, "seconds": time.perf_counter() - t0}
    return out


def served_3d(lib, torch, ctx, steps):
    """Level runs of the served 3-D model (tilted plane, two correlated layers,
    2-norm covariance; 32^3, 64^3, 128^3 with 64/16/4 samples, fine solve plus
    plain coarse companion): per level the median over `steps` calls after one
    warm-up, with the FP32 hierarchy (and the level's tuned W depth) and with
    the FP64 one, the mean fine PCG iterations, and the time of the field
    sampler alone (circulant embedding, n_ce^3 points per sample) for the same
    samples."""
    wl = W.SERVED_3D
    out = []
    for level, (m, n) in enumerate(zip(wl.m_levels, wl.n_samples)):
        row = {"level": level, "m": m, "samples": n, "n_ce": wl.model.n_ce[m]}
        for name, prec in (("f32", lib.MLMC_PREC_FP32), ("f64", lib.MLMC_PREC_FP64)):
            o = lib.mlmc_solver_opts_default(precision=prec)
            for key, v in W.SERVED_3D_LEVEL_OPTS[level].items():
                setattr(o, key, v)
            ts, its = [], 0
            for k in range(steps + 1):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                s = lib.mlmc_level_run(ctx, wl.model, level, m, k * n, n, False, o)
                torch.cuda.synchronize()
                if k > 0:
                    ts.append(time.perf_counter() - t0)
                    its += s.iters_fine
            row[name] = {"ms": 1e3 * sorted(ts)[len(ts) // 2],
                         "mean_iters_fine": its / (steps * n),
                         "opts": dict(W.SERVED_3D_LEVEL_OPTS[level])}
        k = torch.empty(n, m, m, m, dtype=torch.float64, device="cuda")
        kc = torch.empty(n, m // 2, m // 2, m // 2, dtype=torch.float64, device="cuda")
        ts = []
        for j in range(steps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lib.mlmc_sample_field(ctx, wl.model, m, level, j * n, n, k, kc)
            torch.cuda.synchronize()
            if j > 0:
                ts.append(time.perf_counter() - t0)
        row["sampler_ms"] = 1e3 * sorted(ts)[len(ts) // 2]
        out.append(row)
    # roofline of the fine grid's red-black half-sweep (the 3-D path's largest
    # kernel by time) in one more 128^3 level run, FP32 hierarchy: algorithmic
    # bytes (every face, r of the swept colour, z of both colours once, scaled
    # by the share of samples still iterating) over its event-timed launches
    level = len(wl.m_levels) - 1
    m, n = wl.m_levels[level], wl.n_samples[level]
    o = lib.mlmc_solver_opts_default(precision=lib.MLMC_PREC_FP32)
    for key, v in W.SERVED_3D_LEVEL_OPTS[level].items():
        setattr(o, key, v)
    lib.mlmc_profile_enable(ctx, "k_rbgs3@0")
    lib.mlmc_level_run(ctx, wl.model, level, m, 0, n, False, o)
    torch.cuda.synchronize()
    pr = lib.mlmc_profile_read(ctx)
    lib.mlmc_profile_enable(ctx, None)
    roof = None
    if pr["launches"] > 0 and pr["total_ms"] > 0:
        ach = pr["algorithmic_bytes"] / (pr["total_ms"] * 1e-3) / 1e9
        roof = {"kernel": "k_rbgs3@0", "grid": "%d^3 x %d, FP32 hierarchy" % (m, n),
                "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "launches": pr["launches"],
                "avg_launch_ms": pr["total_ms"] / pr["launches"],
                "algorithmic_bytes_per_launch": pr["algorithmic_bytes"] / pr["launches"]}
    return {"workload": wl.name, "per_level": out, "roofline": roof}


def other_configs(lib, torch, steps):
    """The other batched workloads, each timed over `steps` passes after one warm-up
    pass (not part of `value`):
    * Coarse Grid Variates on the piecewise constant model, levels 64^2..512^2
      (4096/1024/256/64 samples, 2^d = 4 sub-lattice companions per fine sample),
      all levels in one call (mlmc_run_levels, levels concurrently) and level by
      level; FP64;
    * the high-contrast field on 1024^2 (256 samples) with the multigrid in FP64,
      FP32 and bfloat16 inside the FP64 CG, with the largest relative QoI
      difference of each reduced precision to the FP64 solve of the same samples;
    * Section 4.2's variance experiment (cgv_variance);
    * Model Problem 1 on the bench workload's levels, level by level;
    * Section 3.4's three-layer correlated model (per-layer correlation lengths),
      both model problems, all levels in one call;
    * adaptive MLMC to a root mean square error (Section 3.2), plain and CGV;
    * the served 3-D model's level runs (served_3d);
    * weak-error rates against reference solutions (rates_vs_reference)."""
    ctx = lib.mlmc_ctx_create(0, torch.cuda.current_stream(0))
    opts = lib.mlmc_solver_opts_default()

    def timed(f):
        f(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            f(1 + k)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    out = {}
    try:
        wl = W.CGV_PC
        total = sum(wl.n_samples)

        def merged(idx):
            lib.mlmc_run_levels(ctx, wl.model, wl.m_levels, [idx * n for n in wl.n_samples],
                                wl.n_samples, True, opts)

        def per_level(idx):
            for level, (m, n) in enumerate(zip(wl.m_levels, wl.n_samples)):
                lib.mlmc_level_run(ctx, wl.model, level, m, idx * n, n, True, opts)

        t_merged, t_level = timed(merged), timed(per_level)
        out["cgv"] = {"workload": wl.name, "levels_m": wl.m_levels, "samples": wl.n_samples,
                      "companions_per_sample": 4, "dtype": "f64",
                      "all_levels_one_call": {"value": total / t_merged,
                                              "ms_per_step": 1e3 * t_merged},
                      "level_by_level": {"value": total / t_level, "ms_per_step": 1e3 * t_level}}

        wl = W.HIGH_CONTRAST
        m, n = wl.m_levels[0], wl.n_samples[0]
        runs, qs = {}, {}
        for name, prec in (("f64", lib.MLMC_PREC_FP64), ("f32", lib.MLMC_PREC_FP32),
                           ("bf16", lib.MLMC_PREC_BF16)):
            o = lib.mlmc_solver_opts_default(precision=prec, tol=wl.tol)
            if prec == lib.MLMC_PREC_BF16:
                o.omega = wl.omega_bf16
            sums = []

            def run(idx):
                sums.append(lib.mlmc_level_run(ctx, wl.model, 0, m, idx * n, n, False, o,
                                               allow_noconv=True))

            t = timed(run)
            q = torch.empty(n, dtype=torch.float64, device="cuda")
            lib.mlmc_level_run(ctx, wl.model, 0, m, 0, n, False, o, q_f=q, allow_noconv=True)
            qs[name] = q
            runs[name] = {"value": n / t, "ms_per_step": 1e3 * t,
                          "mean_iters": sums[-1].iters_fine / n,
                          "failed_solves": int(sum(x.n_failed for x in sums))}
        torch.cuda.synchronize()
        for name in ("f32", "bf16"):
            runs[name]["max_qoi_rel_diff_vs_fp64"] = \
                ((qs[name] - qs["f64"]).abs() / qs["f64"].abs()).max().item()
        # per-QoI error against the FP64 oracle (direct sparse solve) on the
        # samples stored by tests/golden/make_golden.py from the oracle alone
        gold = os.path.join(ROOT, "tests", "golden", "ce_hc_1024_fine.json")
        if os.path.exists(gold):
            import numpy as np
            with open(gold) as f:
                rows = json.load(f)["levels"][0]["samples"]
            ids = [r["sample"] for r in rows]
            ref = np.array([r["Q_f"] for r in rows])
            for name in runs:
                got = qs[name].cpu().numpy()[ids]
                err = np.abs(got - ref) / np.abs(ref)
                runs[name]["qoi_rel_err_vs_oracle"] = {
                    "samples": ids, "max": float(err.max()), "median": float(np.median(err))}
        out["high_contrast"] = {"workload": wl.name, "m": m, "samples": n, "tol_relres": wl.tol,
                                "omega_bf16": wl.omega_bf16,
                                "multigrid_precision": runs}
        out["cgv_variance"] = cgv_variance(lib, torch, ctx, opts)

        # Model Problem 1 on the bench model's levels (f = 1, p = 0 on the boundary,
        # mean pressure over the centred box of side 1/8)
        wl = W.MP1_LAYERED
        total = sum(wl.n_samples)
        lv_ms = {}
        iters = {}

        def mp1_levels(idx):
            for level, (m, n) in enumerate(zip(wl.m_levels, wl.n_samples)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                s = lib.mlmc_level_run(ctx, wl.model, level, m, idx * n, n, False, opts)
                torch.cuda.synchronize()
                lv_ms.setdefault(level, []).append(1e3 * (time.perf_counter() - t0))
                iters[level] = s.iters_fine / n

        t = timed(mp1_levels)
        mp1 = {
            "workload": wl.name, "levels_m": wl.m_levels, "samples": wl.n_samples,
            "qoi": "mean pressure over [7/16, 9/16]^2", "dtype": "f64",
            "value": total / t, "ms_per_step": 1e3 * t,
            "per_level": [{"level": l, "m": m, "ms": sorted(lv_ms[l])[len(lv_ms[l]) // 2],
                           "mean_iters_fine": iters[l]}
                          for l, m in enumerate(wl.m_levels)]}
        out["model_problem_1"] = mp1

        # Section 3.4's three layers (lambda 0.3 / 0.1 / 0.3, means 0 / 4 / 0; two
        # embedding samples per field) on the bench levels, both model problems
        wl = W.PAPER3_LAYERED
        total = sum(wl.n_samples)
        runs = {}
        for name, problem in (("model_problem_2", 0), ("model_problem_1", 1)):
            mdl = wl.model.with_(problem=problem)

            def levels(idx):
                lib.mlmc_run_levels(ctx, mdl, wl.m_levels, [idx * n for n in wl.n_samples],
                                    wl.n_samples, False, opts)

            t = timed(levels)
            runs[name] = {"value": total / t, "ms_per_step": 1e3 * t}
        out["paper_three_layers"] = {"workload": wl.name, "levels_m": wl.m_levels,
                                     "samples": wl.n_samples, "dtype": "f64",
                                     "all_levels_one_call": runs}

        # adaptive MLMC (Section 3.2) on the layered bench model, plain and CGV
        ada = {}
        for name, cgv in (("plain", 0), ("cgv", 1)):
            ao = lib.mlmc_adaptive_opts_default(eps=W.ADAPTIVE_EPS, n_initial=64, cgv=cgv)
            r = lib.mlmc_adaptive(ctx, W.CE2, W.ADAPTIVE_LEVELS, ao, opts)
            L1 = r.n_levels
            ada[name] = {"converged": bool(r.converged), "levels": L1,
                         "m": W.ADAPTIVE_LEVELS[:L1], "estimate": r.estimate,
                         "rmse_bound": math.sqrt(r.variance + r.bias ** 2),
                         "seconds": r.seconds, "n": [r.n[l] for l in range(L1)],
                         "var_y": [r.var_y[l] for l in range(L1)],
                         "cost_ms_per_sample": [1e3 * r.cost[l] for l in range(L1)],
                         "alpha": r.alpha, "beta": r.beta, "gamma": r.gamma}
        out["adaptive"] = {"model": "layered CE (bench model)", "eps": W.ADAPTIVE_EPS,
                           "runs": ada}
        out["served_3d"] = served_3d(lib, torch, ctx, steps)
        out["rates_vs_reference"] = rates_vs_reference(lib, torch, ctx, opts)
    finally:
        lib.mlmc_ctx_destroy(ctx)
    return out


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return 0
    if args.served_3d_only:
        import torch

        import paper_1506_04694_amd as lib
        ctx = lib.mlmc_ctx_create(0, torch.cuda.current_stream(0))
        try:
            print(json.dumps({"served_3d": served_3d(lib, torch, ctx, args.steps)}), flush=True)
        finally:
            lib.mlmc_ctx_destroy(ctx)
        return 0
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs the sample-parallel path on a single "
              "MI355X; --gpus %d is not supported" % args.gpus, file=sys.stderr)
        return 2
    # the CPU baseline first: its worker processes start before this process
    # touches the GPU
    cpu = None if args.no_cpu_baseline else cpu_baseline(W.LAYERED_CE, args.cpu_budget)
    import torch

    import paper_1506_04694_amd as lib

    wl = W.LAYERED_CE
    dev = 0
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    ctx = lib.mlmc_ctx_create(dev, stream)
    opts = lib.mlmc_solver_opts_default()
    lopts = [lib.mlmc_solver_opts_default(**o) for o in W.LAYERED_CE_LEVEL_OPTS]
    nlev = len(wl.m_levels)
    level_times = [[] for _ in range(nlev)]
    iters = [[] for _ in range(nlev)]
    # Each level runs on its own context and stream.  With --concurrent-levels
    # the levels (independent of each other) also run from their own host
    # threads, so one level's latency-bound coarse-grid launches overlap
    # another's bandwidth-bound fine-grid launches; kernel durations then
    # include that overlap, so the roofline entry is only meaningful without it.
    lstreams = [torch.cuda.Stream(dev) for _ in range(nlev)]
    lctx = [lib.mlmc_ctx_create(dev, st) for st in lstreams]

    def step(idx, record):
        sums = [None] * nlev
        errors = []

        def run(level):
            m, n = wl.m_levels[level], wl.n_samples[level]
            try:
                t0 = time.perf_counter()
                s = lib.mlmc_level_run(lctx[level], wl.model, level, m, idx * n, n, wl.cgv,
                                       lopts[level])
                lstreams[level].synchronize()
                dt = time.perf_counter() - t0
            except Exception as e:  # noqa: BLE001 - re-raised below on the main thread
                errors.append(e)
                return
            if record:
                level_times[level].append(dt)
                iters[level].append((s.iters_fine / n, s.iters_coarse / max(n, 1)))
            sums[level] = s

        if not args.concurrent_levels:
            for level in range(nlev):
                run(level)
        else:
            threads = [threading.Thread(target=run, args=(level,)) for level in range(nlev)]
            for th in threads:
                th.start()
            for th in threads:
                th.join()
        if errors:
            raise errors[0]
        return sums

    def per_sample_baseline(budget_s=1.5):
        """The same FP64 path with one sample per call (no batching), a few samples
        per level: the plain per-sample GPU solve the batched form is compared to."""
        out = []
        for level, (m, n) in enumerate(zip(wl.m_levels, wl.n_samples)):
            lib.mlmc_level_run(ctx, wl.model, level, m, 10 ** 6, 1, wl.cgv, lopts[level])  # warm
            done, t0 = 0, time.perf_counter()
            while time.perf_counter() - t0 < budget_s / len(wl.m_levels) and done < n:
                lib.mlmc_level_run(ctx, wl.model, level, m, 10 ** 6 + 1 + done, 1, wl.cgv,
                                   lopts[level])
                done += 1
            dt = (time.perf_counter() - t0) / done
            out.append({"level": level, "m": m, "samples_timed": done, "ms_per_sample": 1e3 * dt,
                        "samples_per_s": 1.0 / dt})
        t_step = sum(n * o["ms_per_sample"] * 1e-3 for n, o in zip(wl.n_samples, out))
        return {"value": sum(wl.n_samples) / t_step, "unit": "samples/s", "per_level": out}

    for w in range(args.warmup):
        step(w, False)
    torch.cuda.synchronize()
    for c in lctx:
        lib.mlmc_profile_enable(c, args.kernel)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        sums = step(args.warmup + k, True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = {"launches": 0, "total_ms": 0.0, "algorithmic_bytes": 0.0}
    for c in lctx:
        pr = lib.mlmc_profile_read(c)
        for key in prof:
            prof[key] += pr[key]
        lib.mlmc_profile_enable(c, None)
    # the same kernel function over every level (all instantiations), one more step
    prof_all = None
    base_kernel = args.kernel.split("@")[0]
    if base_kernel != args.kernel:
        for c in lctx:
            lib.mlmc_profile_enable(c, base_kernel)
        step(args.warmup + args.steps, False)
        torch.cuda.synchronize()
        prof_all = {"launches": 0, "total_ms": 0.0, "algorithmic_bytes": 0.0}
        for c in lctx:
            pr = lib.mlmc_profile_read(c)
            for key in prof_all:
                prof_all[key] += pr[key]
            lib.mlmc_profile_enable(c, None)
    # the same kernel split by launch size, one more step each: the level runs'
    # 2^24-cell fine solves (working set per launch larger than the 256 MB
    # Infinity Cache) apart from the 2^22-cell companions
    by_size = None
    if args.kernel == DOMINANT:
        by_size = {}
        for cells in (1 << 24, 1 << 22):
            label = "%s#%d" % (args.kernel, cells)
            for c in lctx:
                lib.mlmc_profile_enable(c, label)
            step(args.warmup + args.steps + 1, False)
            torch.cuda.synchronize()
            pb = {"launches": 0, "total_ms": 0.0, "algorithmic_bytes": 0.0}
            for c in lctx:
                pr = lib.mlmc_profile_read(c)
                for key in pb:
                    pb[key] += pr[key]
                lib.mlmc_profile_enable(c, None)
            if pb["launches"] and pb["total_ms"] > 0:
                ach = pb["algorithmic_bytes"] / (pb["total_ms"] * 1e-3) / 1e9
                by_size[str(cells)] = {
                    "label": label, "achieved": round(ach, 1), "frac": round(ach / HBM_PEAK_GBS, 4),
                    "launches": pb["launches"], "avg_launch_ms": pb["total_ms"] / pb["launches"],
                    "algorithmic_bytes_per_launch": pb["algorithmic_bytes"] / pb["launches"]}
    # the other finest-grid kernels of a PCG iteration (down, up, CG direction,
    # axpy), one more step each, timed and credited like the dominant kernel
    others = None
    if args.kernel == DOMINANT:
        others = {}
        for label in ("k_mg_down@0", "k_mg_up@0", "k_cg_direction_t", "k_axpy_dot"):
            for c in lctx:
                lib.mlmc_profile_enable(c, label)
            step(args.warmup + args.steps + 2, False)
            torch.cuda.synchronize()
            pb = {"launches": 0, "total_ms": 0.0, "algorithmic_bytes": 0.0}
            for c in lctx:
                pr = lib.mlmc_profile_read(c)
                for key in pb:
                    pb[key] += pr[key]
                lib.mlmc_profile_enable(c, None)
            if pb["launches"] and pb["total_ms"] > 0:
                ach = pb["algorithmic_bytes"] / (pb["total_ms"] * 1e-3) / 1e9
                others[label] = {
                    "achieved": round(ach, 1), "frac": round(ach / HBM_PEAK_GBS, 4),
                    "launches": pb["launches"], "avg_launch_ms": pb["total_ms"] / pb["launches"],
                    "algorithmic_bytes_per_launch": pb["algorithmic_bytes"] / pb["launches"]}
    est = lib.mlmc_estimate(sums)
    single = per_sample_baseline() if not args.no_per_sample else None
    variants = None if args.no_variants else path_variants(lib, torch, wl, ctx, opts, args)
    configs = None if args.no_variants else other_configs(lib, torch, args.steps)
    for c in lctx:
        lib.mlmc_ctx_destroy(c)
    lib.mlmc_ctx_destroy(ctx)

    ms_per_step = 1e3 * elapsed / args.steps
    total = sum(wl.n_samples)
    serving = None
    if args.serve_rates and args.serve_rates != "none":
        rates = [float(f) for f in args.serve_rates.split(",") if f]
        # the bench workload's levels, FP64, one model
        kinds = [(0, level, m, n) for level, (m, n) in enumerate(zip(wl.m_levels, wl.n_samples))]
        sat = total / (elapsed / args.steps)
        serving = {"workload": wl.name, "saturation_estimate_per_s": sat,
                   "workers": SERVE_WORKERS, "max_batch": SERVE_MAX_BATCH,
                   "precision": "f64",
                   "runs": [serving_latency(lib, kinds, [wl.model], [opts], f * sat,
                                            args.serve_seconds) for f in rates]}
        # the mixed 2-D / 3-D stream: three models in one server
        models = W.SERVED_MIX_MODELS
        solvers = [lib.mlmc_solver_opts_default(
            precision=lib.MLMC_PREC_FP32 if p == "f32" else lib.MLMC_PREC_FP64, tol=tl)
            for p, tl in zip(W.SERVED_MIX_PRECISION, W.SERVED_MIX_TOL)]
        sat_mix, pass_mix = pass_rate(lib, torch, W.SERVED_MIX_KINDS, models, solvers)
        serving["mixed_2d_3d"] = {
            "kinds": [{"model": mi, "dim": int(models[mi].dim), "level": lv, "m": m, "count": c}
                      for mi, lv, m, c in W.SERVED_MIX_KINDS],
            "precision": W.SERVED_MIX_PRECISION, "tol_relres": W.SERVED_MIX_TOL,
            "batched_pass_ms": 1e3 * pass_mix, "saturation_estimate_per_s": sat_mix,
            "runs": [serving_latency(lib, W.SERVED_MIX_KINDS, models, solvers, f * sat_mix,
                                     args.serve_seconds) for f in rates]}
    per_level = []
    for level, (m, n) in enumerate(zip(wl.m_levels, wl.n_samples)):
        t = sorted(level_times[level])[len(level_times[level]) // 2]
        per_level.append({"level": level, "m": m, "samples": n, "ms": 1e3 * t,
                          "samples_per_s": n / t,
                          "mean_iters_fine": sum(a for a, _ in iters[level]) / len(iters[level]),
                          "mean_iters_coarse": sum(b for _, b in iters[level]) / len(iters[level])})
    roof = None
    if prof["launches"] > 0 and prof["total_ms"] > 0:
        avg_ms = prof["total_ms"] / prof["launches"]
        achieved = prof["algorithmic_bytes"] / (prof["total_ms"] * 1e-3) / 1e9
        roof = {"kernel": args.kernel,
                "symbol": DOMINANT_SYMBOL if args.kernel == DOMINANT else None,
                "bound": "hbm", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(args.kernel), "launches": prof["launches"],
                "avg_launch_ms": avg_ms,
                "algorithmic_bytes_per_launch": prof["algorithmic_bytes"] / prof["launches"]}
        if by_size:
            roof["by_launch_cells"] = by_size
        if others:
            roof["other_kernels"] = others
        if prof_all and prof_all["launches"] > 0:
            ach = prof_all["algorithmic_bytes"] / (prof_all["total_ms"] * 1e-3) / 1e9
            roof["all_levels"] = {
                "kernel": base_kernel, "achieved": round(ach, 1),
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": measured_traffic(base_kernel),
                "launches": prof_all["launches"],
                "avg_launch_ms": prof_all["total_ms"] / prof_all["launches"],
                "algorithmic_bytes_per_launch": prof_all["algorithmic_bytes"] / prof_all["launches"]}
    out = {"metric": METRIC, "value": total / (elapsed / args.steps), "unit": "samples/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": wl.name, "levels_m": wl.m_levels, "samples": wl.n_samples,
                      "estimator": "cgv" if wl.cgv else "plain", "tol_relres": opts.tol,
                      "n_ce": [wl.model.n_ce[m] for m in wl.m_levels],
                      "solver_overrides_per_level": list(W.LAYERED_CE_LEVEL_OPTS),
                      "model": "2 layers, 8-node interface, exp. covariance r=2, sigma2=1, "
                               "lambda=0.3, means 0/2"},
           "levels_concurrent": bool(args.concurrent_levels),
           "per_level": per_level, "estimate": est, "roofline": roof,
           "per_sample_fp64_gpu": single, "variants": variants, "other_configs": configs,
           "serving": serving}
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
