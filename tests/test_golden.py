"""The stored expected values under tests/golden/ are reproduced by the oracle."""
import json
import os

import pytest

import workloads as W
from oracle import mlmc

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
MODELS = {"pc2": W.PC2, "ce2": W.CE2, "til": W.TILTED3, "ce_": W.CE_HC}


@pytest.mark.parametrize("name", ["pc2_16_32_plain.json", "pc2_16_32_cgv.json",
                                  "ce2_16_32_plain.json", "ce2_16_32_cgv.json",
                                  "tilted3_64_128_plain.json", "ce_hc_1024_fine.json"])
def test_golden_reproduced_by_oracle(name):
    with open(os.path.join(GOLDEN, name)) as f:
        rec = json.load(f)
    model = MODELS[name[:3]]
    for lv in rec["levels"]:
        if name.startswith("tilted3") and lv["m"] > 64:
            continue   # 128^3 conjugate gradient solves take minutes: 64^3 only here
        for row in lv["samples"][:3 if lv["m"] <= 32 else 1]:
            r = mlmc.level_sample(model, lv["level"], row["sample"], lv["m"], cgv=rec["cgv"])
            assert abs(r["Q_f"] - row["Q_f"]) <= 1e-13 * abs(row["Q_f"])
            assert abs(r["Y"] - row["Y"]) <= 1e-13 * abs(row["Q_f"])
