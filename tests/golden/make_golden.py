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
from oracle import mlmc, solve  # noqa: E402


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


def main(names):
    for name in names:
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
    main(sys.argv[1:] or list(FILES))
