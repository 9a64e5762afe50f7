"""The autotuner on the GPU: over a small option space on small grids (2-D and
3-D) every admissible setting reproduces the FP64 defaults' QoIs within 1e-10,
the chosen one is the fastest admissible trial, and refused combinations are
recorded as errors rather than raised."""
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import workloads as W  # noqa: E402


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1506_04694_amd as lib
    return lib


@pytest.mark.parametrize("model,m", [("ce2", 64), ("ce2", 128), ("tilted3", 16)])
def test_tune_level_small_space(lib, model, m):
    from paper_1506_04694_amd import autotune
    mdl = {"ce2": W.CE2, "tilted3": W.TILTED3}[model]
    print("autotune %s m=%d" % (model, m), flush=True)
    ctx = lib.mlmc_ctx_create(0, torch.cuda.current_stream(0))
    try:
        space = {"precision": [lib.MLMC_PREC_FP64, lib.MLMC_PREC_FP32, lib.MLMC_PREC_BF16],
                 "gamma_levels": [2, 3]}
        if m == 128:   # tile shapes instead of W depth on a tiled grid
            space = {"precision": space["precision"], "tile_shape": [0, 1]}
        res = autotune.tune_level(ctx, mdl, 1, m, 8, space=space, reps=1)
    finally:
        lib.mlmc_ctx_destroy(ctx)
    assert res["m"] == m and len(res["trials"]) == 6
    good = [t for t in res["trials"] if t.get("admissible")]
    assert good, res["trials"]
    assert res["best"] is not None
    assert res["best"]["seconds"] == min(t["seconds"] for t in good)
    for t in good:
        assert t["max_qoi_rel_dev"] <= 1e-10
    if model == "tilted3":
        # bfloat16 hierarchies are 2-D only: recorded as errors
        assert all("error" in t for t in res["trials"]
                   if t["opts"]["precision"] == lib.MLMC_PREC_BF16)


def test_tune_level_smoothing_sweeps(lib):
    """nu = 1 (fused tile kernels) and nu = 2 (per-sweep cycle) both reach the
    FP64 default's QoIs; the tuner keeps the faster admissible one."""
    from paper_1506_04694_amd import autotune
    print("autotune nu m=128", flush=True)
    ctx = lib.mlmc_ctx_create(0, torch.cuda.current_stream(0))
    try:
        res = autotune.tune_level(ctx, W.CE2, 1, 128, 8, space={"nu": [1, 2]}, reps=1)
    finally:
        lib.mlmc_ctx_destroy(ctx)
    assert [t["opts"]["nu"] for t in res["trials"]] == [1, 2]
    assert all(t.get("admissible") for t in res["trials"]), res["trials"]
    assert all(t["max_qoi_rel_dev"] <= 1e-10 for t in res["trials"])
    assert res["best"]["seconds"] == min(t["seconds"] for t in res["trials"])
    o = autotune.best_opts({128: res}, 128)
    assert o.nu1 == o.nu2 == res["best"]["opts"]["nu"]
