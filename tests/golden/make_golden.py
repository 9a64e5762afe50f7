"""Writes the stored expected values under tests/golden/ from the oracle alone.

Run from the repository root:  python tests/golden/make_golden.py [file ...]
(no argument: every file).  Each file records the workload parameters it was
made from and the oracle solver behind each grid (direct sparse solve, or the
Jacobi-preconditioned conjugate gradient solve to 1e-14 on 3-D grids above
32^3; the 128^3 samples take a few minutes).
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import field, mlmc, solve  # noqa: E402


def level_records(model, m_levels, n_per_level, cgv, levels=None):
    out = []
    for level, m in enumerate(m_levels):
        if levels is not None and level not in levels:
            continue
        rows = []
        for s in range(n_per_level):
            r = mlmc.level_sample(model, level, s, m, cgv=cgv)
            rows.append({"sample": s, "Q_f": r["Q_f"], "Q_c": r["Q_c"], "Y": r["Y"],
                         "companions": r["companions"]})
        out.append({"level": level, "m": m, "samples": rows,
                    "fine_solver": "cg" if solve.uses_cg(model.dim, m) else "direct",
                    "coarse_solver": "cg" if solve.uses_cg(model.dim, m // 2) else "direct"})
        print("  level %d m=%d done" % (level, m), flush=True)
    return out


FILES = {
    "pc2_16_32_plain.json": (W.PC2, [16, 32], 16, False, None),
    "pc2_16_32_cgv.json": (W.PC2, [16, 32], 8, True, None),
    "ce2_16_32_plain.json": (W.CE2, [16, 32], 8, False, None),
    "ce2_16_32_cgv.json": (W.CE2, [16, 32], 8, True, None),
    # the served 3-D model on its two largest grids: samples 0 and 1 of level 1
    # (64^3, companions 32^3) and level 2 (128^3, companions 64^3)
    "tilted3_64_128_plain.json": (W.TILTED3, [32, 64, 128], 2, False, (1, 2)),
    # the high-contrast field on 1024^2 (sigma^2 = 3, lambda = 0.1): samples 0-15,
    # the subset the reduced-precision multigrid errors are stated on
    "ce_hc_1024_fine.json": (W.CE_HC, [1024], 16, False, None),
}


def field_record(model, level, sample, m, n_cells, rng_seed):
    """log k of one oracle sample at n_cells fixed pseudo-random cells of the
    m^3 grid, and log of its plain coarse companion at n_cells / 2 cells."""
    import numpy as np
    k, kc = field.sample_k(model, level, sample, m, with_coarse=True)
    rng = np.random.default_rng(rng_seed)
    idx = rng.integers(0, k.size, size=n_cells)
    idc = rng.integers(0, kc.size, size=n_cells // 2)
    return {"level": level, "sample": sample, "m": m,
            "cells": idx.tolist(), "log_k": np.log(k.ravel()[idx]).tolist(),
            "coarse_cells": idc.tolist(), "log_k_coarse": np.log(kc.ravel()[idc]).tolist()}


FIELDS = {
    # the served 3-D model's 128^3 field (embedding 540^3): too large for the
    # oracle to sample inside a GPU test
    "tilted3_field_128.json": (W.TILTED3, 2, 0, 128, 4096, 7),
}


def main(names):
    for name in names:
        if name in FIELDS:
            model, level, sample, m, cells, seed = FIELDS[name]
            rec = {"source": "oracle/field.py sample_k (FP64)",
                   "model": {k: (list(v) if isinstance(v, tuple) else v)
                             for k, v in model.__dict__.items() if k != "n_ce"},
                   "n_ce": {str(k): v for k, v in model.n_ce.items()},
                   "field": field_record(model, level, sample, m, cells, seed)}
            with open(os.path.join(HERE, name), "w") as f:
                json.dump(rec, f)
            print("wrote", name)
            continue
        model, ms, n, cgv, levels = FILES[name]
        rec = {"source": "oracle/ (FP64; solver per level in fine_solver / coarse_solver)",
               "model": {k: (list(v) if isinstance(v, tuple) else v)
                         for k, v in model.__dict__.items() if k != "n_ce"},
               "n_ce": {str(k): v for k, v in model.n_ce.items()},
               "cgv": cgv, "levels": level_records(model, ms, n, cgv, levels)}
        with open(os.path.join(HERE, name), "w") as f:
            json.dump(rec, f, indent=1)
        print("wrote", name)


if __name__ == "__main__":
    main(sys.argv[1:] or list(FILES) + list(FIELDS))
