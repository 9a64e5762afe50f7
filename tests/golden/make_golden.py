"""Writes the stored expected values under tests/golden/ from the oracle alone.

Run from the repository root:  python tests/golden/make_golden.py
Each file records the workload parameters it was made from.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import mlmc  # noqa: E402


def level_records(model, m_levels, n_per_level, cgv):
    out = []
    for level, m in enumerate(m_levels):
        rows = []
        for s in range(n_per_level):
            r = mlmc.level_sample(model, level, s, m, cgv=cgv)
            rows.append({"sample": s, "Q_f": r["Q_f"], "Q_c": r["Q_c"], "Y": r["Y"],
                         "companions": r["companions"]})
        out.append({"level": level, "m": m, "samples": rows})
    return out


def main():
    files = {
        "pc2_16_32_plain.json": (W.PC2, [16, 32], 16, False),
        "pc2_16_32_cgv.json": (W.PC2, [16, 32], 8, True),
        "ce2_16_32_plain.json": (W.CE2, [16, 32], 8, False),
        "ce2_16_32_cgv.json": (W.CE2, [16, 32], 8, True),
    }
    for name, (model, ms, n, cgv) in files.items():
        rec = {"source": "oracle/ (direct sparse solve, FP64)",
               "model": {k: (list(v) if isinstance(v, tuple) else v)
                         for k, v in model.__dict__.items() if k != "n_ce"},
               "n_ce": {str(k): v for k, v in model.n_ce.items()},
               "cgv": cgv, "levels": level_records(model, ms, n, cgv)}
        with open(os.path.join(HERE, name), "w") as f:
            json.dump(rec, f, indent=1)
        print("wrote", name)


if __name__ == "__main__":
    main()
