"""Kernel timing through the C ABI (mlmc_profile_enable / mlmc_profile_read):
the label forms "<name>", "<name>@<level>" and "<name>@<level>#<cells>"
select the launches the bench's roofline entries are computed from.  On a
256^2 level run (8 samples, plain 128^2 companions) the finest-grid mid
launches split exactly into the fine solve's (8 x 256^2 cells) and the
companions' (8 x 128^2), and each launch is credited at most its
algorithmic bytes (T two words, r, z_pre, the coarse z and residual a
quarter word each, z: 44 bytes per cell in FP64), scaled down only by the
share of samples still iterating."""
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


def _profiled(lib, ctx, label, opts):
    lib.mlmc_profile_enable(ctx, label)
    lib.mlmc_level_run(ctx, W.CE2, 2, 256, 0, 8, False, opts)
    torch.cuda.synchronize()
    pr = lib.mlmc_profile_read(ctx)
    lib.mlmc_profile_enable(ctx, None)
    return pr


def test_profile_labels_split_launches_by_level_and_size(lib):
    print("profile labels on a 256^2 level run", flush=True)
    ctx = lib.mlmc_ctx_create(0, torch.cuda.current_stream(0))
    try:
        opts = lib.mlmc_solver_opts_default()
        lib.mlmc_level_run(ctx, W.CE2, 2, 256, 0, 8, False, opts)      # warm
        every = _profiled(lib, ctx, "k_mg_mid", opts)
        top = _profiled(lib, ctx, "k_mg_mid@0", opts)
        fine = _profiled(lib, ctx, "k_mg_mid@0#%d" % (8 * 256 * 256), opts)
        comp = _profiled(lib, ctx, "k_mg_mid@0#%d" % (8 * 128 * 128), opts)
        none = _profiled(lib, ctx, "k_mg_mid@0#12345", opts)
    finally:
        lib.mlmc_ctx_destroy(ctx)
    assert none["launches"] == 0
    assert fine["launches"] > 0 and comp["launches"] > 0
    assert fine["launches"] + comp["launches"] == top["launches"] <= every["launches"]
    for pr, cells in ((fine, 8 * 256 * 256), (comp, 8 * 128 * 128)):
        assert pr["total_ms"] > 0
        per_launch = pr["algorithmic_bytes"] / pr["launches"]
        assert 0 < per_launch <= 44.0 * cells * (1 + 1e-12), (per_launch, cells)
    assert abs(fine["algorithmic_bytes"] + comp["algorithmic_bytes"] - top["algorithmic_bytes"]) \
        <= 1e-9 * top["algorithmic_bytes"]
