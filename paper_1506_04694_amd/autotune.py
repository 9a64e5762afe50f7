"""Autotuner for the batched multigrid-PCG solve.

For each fine grid size of a workload it times ``mlmc_level_run`` on a
calibration batch drawn from the workload itself, for every combination of
the tunable solver options (multigrid storage precision, coarse-grid
correction scaling omega, V- or W-cycle and the number of W levels, smoothing
sweeps nu = nu1 = nu2, coarsest grid size, host convergence-check interval,
on-chip cycle threshold, tile shapes of the multigrid kernels).  A combination is admissible only if every QoI of the calibration
batch stays within ``qoi_rtol`` (default 1e-10) of the FP64 default
solver's QoI for the same samples; the fastest admissible one is kept.

Results are cached as JSON keyed by device name and grid size.  All work runs
through the C ABI (``mlmc_level_run``); this module only chooses options.
"""
import itertools
import json
import os
import time

import paper_1506_04694_amd as lib

DEFAULT_SPACE = {
    "precision": [lib.MLMC_PREC_FP64, lib.MLMC_PREC_FP32, lib.MLMC_PREC_BF16],
    "omega": [1.8, 1.9, 2.0],
    "gamma": [1, 2],
    "gamma_levels": [2, 3],
    "nu": [1, 2],
    "coarse_max": [2, 4, 8],
    "check_every": [4, 8],
    "cycle_max": [16, 32],
    "tile_shape": [0, 1],
}


def make_opts(**kw):
    """mlmc_solver_opts from a point of the search space; "nu" sets the
    symmetric pair nu1 = nu2 (pre- and post-smoothing sweeps)."""
    kw = dict(kw)
    if "nu" in kw:
        kw["nu1"] = kw["nu2"] = kw.pop("nu")
    return lib.mlmc_solver_opts_default(**kw)


def _time_level(ctx, model, level, m, n, opts, first, reps):
    import torch
    qf = torch.empty(n, dtype=torch.float64, device="cuda")
    qc = torch.empty_like(qf)
    best = float("inf")
    sums = None
    for r in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sums = lib.mlmc_level_run(ctx, model, level, m, first, n, False, opts, q_f=qf, q_c=qc,
                                  allow_noconv=True)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best, qf.cpu().numpy(), qc.cpu().numpy(), sums


def tune_level(ctx, model, level, m, n, space=None, qoi_rtol=1e-10, reps=2, first=10 ** 6):
    """Best solver options for one level (grid m, calibration batch of n samples)."""
    import numpy as np
    space = space or DEFAULT_SPACE
    ref_opts = lib.mlmc_solver_opts_default()
    _, ref_f, ref_c, _ = _time_level(ctx, model, level, m, n, ref_opts, first, 1)
    trials = []
    keys = list(space)
    for combo in itertools.product(*(space[k] for k in keys)):
        kw = dict(zip(keys, combo))
        opts = make_opts(**kw)
        try:
            t, qf, qc, sums = _time_level(ctx, model, level, m, n, opts, first, reps)
        except lib.MlmcError as e:
            trials.append({"opts": kw, "error": str(e)})
            continue
        err = float(np.max(np.abs(qf - ref_f) / np.abs(ref_f)))
        if level > 0:
            err = max(err, float(np.max(np.abs(qc - ref_c) / np.abs(ref_c))))
        ok = sums.n_failed == 0 and err <= qoi_rtol
        trials.append({"opts": kw, "seconds": t, "samples_per_s": n / t, "max_qoi_rel_dev": err,
                       "mean_iters": sums.iters_fine / n, "admissible": ok})
    good = [t for t in trials if t.get("admissible")]
    best = min(good, key=lambda t: t["seconds"]) if good else None
    return {"level": level, "m": m, "calibration_samples": n, "best": best, "trials": trials}


def tune_workload(workload, calib_samples=None, cache_path=None, space=None, reps=2):
    """Tunes every level of a workloads.Workload; returns {m: result}."""
    import torch
    dev_name = torch.cuda.get_device_name(0)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    ctx = lib.mlmc_ctx_create(0, torch.cuda.current_stream(0))
    out = {}
    try:
        for level, (m, n) in enumerate(zip(workload.m_levels, workload.n_samples)):
            key = "%s|%s|%d" % (dev_name, workload.name, m)
            if key in cache:
                out[m] = cache[key]
                continue
            nc = calib_samples.get(m, n) if calib_samples else n
            res = tune_level(ctx, workload.model, level, m, nc, space=space, reps=reps)
            out[m] = cache[key] = res
    finally:
        lib.mlmc_ctx_destroy(ctx)
    if cache_path:
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return out


def best_opts(tuned, m):
    """mlmc_solver_opts for grid m from a tune_workload result (defaults if untuned)."""
    res = tuned.get(m) or tuned.get(str(m))
    if not res or not res.get("best"):
        return lib.mlmc_solver_opts_default()
    return make_opts(**res["best"]["opts"])
