"""The C-ABI library loads, exports every entry point its header declares,
and the binding's struct layouts match the header (checked by compiling a C
probe against include/mlmc_darcy.h).  Host-only entry points (defaults and
the estimator arithmetic of eq. (3.6)/(3.7)) are checked against the oracle;
no device call is made here."""
import ctypes
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mlmc_darcy.h")


@pytest.fixture(scope="module")
def lib():
    import paper_1506_04694_amd as lib
    return lib


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+char\*|mlmc_status|double)\s+(mlmc_\w+)\s*\(", text, re.M)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib._lib, name), name
    assert sorted(lib.EXPORTED) == names
    out = subprocess.check_output(["nm", "-D", "--defined-only", lib.LIB_PATH]).decode()
    for name in names:
        assert re.search(r"\sT\s%s$" % name, out, re.M), name


PROBE = r"""
#include <stdio.h>
#include <stddef.h>
#include "mlmc_darcy.h"
#define P(T, f) printf("%s.%s %zu\n", #T, #f, offsetof(T, f))
int main(void) {
  printf("mlmc_model %zu\nmlmc_solver_opts %zu\nmlmc_level_sums %zu\nmlmc_estimate_t %zu\n",
         sizeof(mlmc_model), sizeof(mlmc_solver_opts), sizeof(mlmc_level_sums),
         sizeof(mlmc_estimate_t));
  P(mlmc_model, y_lo); P(mlmc_model, mu); P(mlmc_model, sigma2); P(mlmc_model, lambda);
  P(mlmc_model, seed); P(mlmc_model, problem); P(mlmc_solver_opts, maxit); P(mlmc_solver_opts, check_every); P(mlmc_solver_opts, gamma); P(mlmc_solver_opts, gamma_levels); P(mlmc_solver_opts, graph);
  P(mlmc_level_sums, sum_y); P(mlmc_level_sums, iters_coarse);
  printf("mlmc_serve_opts %zu\nmlmc_request %zu\nmlmc_result %zu\n", sizeof(mlmc_serve_opts),
         sizeof(mlmc_request), sizeof(mlmc_result));
  P(mlmc_serve_opts, hbm_budget_bytes); P(mlmc_serve_opts, grid_model); P(mlmc_serve_opts, solver);
  P(mlmc_request, model); P(mlmc_result, model); P(mlmc_result, q_f); P(mlmc_result, t_done);
  printf("mlmc_adaptive_opts %zu\nmlmc_adaptive_result %zu\n", sizeof(mlmc_adaptive_opts),
         sizeof(mlmc_adaptive_result));
  P(mlmc_adaptive_opts, max_samples); P(mlmc_adaptive_result, n); P(mlmc_adaptive_result, cost);
  P(mlmc_adaptive_result, sums);
  return 0;
}
"""


def test_struct_layouts_match_header(lib, tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    src = tmp_path / "probe.c"
    src.write_text(PROBE)
    exe = tmp_path / "probe"
    subprocess.check_call([gcc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    vals = dict(line.split() for line in subprocess.check_output([str(exe)]).decode().splitlines())
    assert int(vals["mlmc_model"]) == ctypes.sizeof(lib.mlmc_model)
    assert int(vals["mlmc_solver_opts"]) == ctypes.sizeof(lib.mlmc_solver_opts)
    assert int(vals["mlmc_level_sums"]) == ctypes.sizeof(lib.mlmc_level_sums)
    assert int(vals["mlmc_estimate_t"]) == ctypes.sizeof(lib.mlmc_estimate_t)
    assert int(vals["mlmc_model.lambda"]) == lib.mlmc_model.lambda_.offset
    assert int(vals["mlmc_model.seed"]) == lib.mlmc_model.seed.offset
    assert int(vals["mlmc_model.y_lo"]) == lib.mlmc_model.y_lo.offset
    assert int(vals["mlmc_model.problem"]) == lib.mlmc_model.problem.offset
    assert int(vals["mlmc_solver_opts.check_every"]) == lib.mlmc_solver_opts.check_every.offset
    assert int(vals["mlmc_solver_opts.gamma"]) == lib.mlmc_solver_opts.gamma.offset
    assert int(vals["mlmc_solver_opts.gamma_levels"]) == lib.mlmc_solver_opts.gamma_levels.offset
    assert int(vals["mlmc_solver_opts.graph"]) == lib.mlmc_solver_opts.graph.offset
    assert int(vals["mlmc_level_sums.iters_coarse"]) == lib.mlmc_level_sums.iters_coarse.offset
    for st in ("mlmc_serve_opts", "mlmc_request", "mlmc_result", "mlmc_adaptive_opts",
               "mlmc_adaptive_result"):
        assert int(vals[st]) == ctypes.sizeof(getattr(lib, st)), st
    for st, f in (("mlmc_serve_opts", "hbm_budget_bytes"), ("mlmc_serve_opts", "grid_model"),
                  ("mlmc_serve_opts", "solver"), ("mlmc_request", "model"),
                  ("mlmc_result", "model"), ("mlmc_result", "q_f"), ("mlmc_result", "t_done"),
                  ("mlmc_adaptive_opts", "max_samples"), ("mlmc_adaptive_result", "n"),
                  ("mlmc_adaptive_result", "cost"), ("mlmc_adaptive_result", "sums")):
        assert int(vals["%s.%s" % (st, f)]) == getattr(getattr(lib, st), f).offset, (st, f)


def test_solver_defaults(lib):
    o = lib.mlmc_solver_opts_default()
    assert o.tol == 1e-13 and o.omega == 1.9 and o.nu1 == o.nu2 == 1 and o.maxit == 200
    assert o.gamma == 2 and o.gamma_levels == 2 and o.variant == 0 and o.precision == lib.MLMC_PREC_FP64
    assert o.graph == 0


def test_estimate_matches_oracle(lib):
    from oracle import mlmc as omlmc
    rng = np.random.default_rng(3)
    ys = [rng.standard_normal(n) * s + mu for n, s, mu in ((40, 1.0, 1.6), (25, 0.1, 0.01), (9, 0.02, 0.0))]
    levels = []
    for y in ys:
        s = lib.mlmc_level_sums()
        s.n = len(y)
        s.sum_y = float(np.sum(y))
        s.sum_y2 = float(np.sum(y * y))
        levels.append(s)
    got = lib.mlmc_estimate(levels)
    ref = omlmc.estimate([omlmc.level_sums(y, y, np.zeros_like(y)) for y in ys])
    assert abs(got["estimate"] - ref["estimate"]) < 1e-13
    assert abs(got["variance"] - ref["variance_of_estimate"]) < 1e-13 * ref["variance_of_estimate"]
    bad = lib.mlmc_level_sums()
    bad.n = 1
    with pytest.raises(lib.MlmcError):
        lib.mlmc_estimate([bad])


def test_product_path_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_1506_04694_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in re.sub(r"#.*|//.*", "", text).lower() or f == "__init__.py" and \
                    "import oracle" not in text, f


def test_autotune_space_point_to_opts(lib):
    """The autotuner's "nu" sets the symmetric pair nu1 = nu2; other keys are
    solver option fields (host-only: no device work)."""
    from paper_1506_04694_amd import autotune
    o = autotune.make_opts(nu=2, gamma_levels=3, precision=lib.MLMC_PREC_FP32)
    assert o.nu1 == 2 and o.nu2 == 2 and o.gamma_levels == 3
    assert o.precision == lib.MLMC_PREC_FP32
    assert set(autotune.DEFAULT_SPACE) >= {"nu", "coarse_max", "tile_shape", "gamma_levels"}
