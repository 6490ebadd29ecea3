"""The allocation-free spectral forward (fno_spectral_fwd_noalloc) against the
workspace entry point fno_spectral_fwd: same kernels, so the outputs and the
cache must be bit-identical, on two calls in a row (the second on a smaller
problem, whose intermediates reuse the front of the same static device array),
in both activation dtypes; sizes beyond the static array are rejected on the
host before anything is launched."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2211_12709_amd import inputs  # noqa: E402


@pytest.fixture(scope="module")
def fno():
    from paper_2211_12709_amd import fno as f
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    f.load_library()
    return f


# (B, C_in, C_out, grid, modes): a larger problem first, then a smaller one
CASES = [
    (2, 8, 8, (16, 16, 16, 8), (4, 4, 4, 4)),  # matrix-core path, about 2.6 MB of intermediates
    (1, 3, 5, (12, 10, 9, 7), (3, 2, 4, 4)),    # ragged grid (odd Nt: the scalar kernels)
]


def run_pair(fno, plan, seed):
    x = inputs.normal_field((plan.B, plan.C_in, *plan.grid), seed=seed)
    w, _, _ = inputs.block_params(plan.C_in, plan.C_out, plan.kshape, block=seed % 7)
    tx = torch.from_numpy(x).cuda().to(plan.act_dtype)
    tw = torch.from_numpy(w).cuda()
    assert plan.workspace_bytes(fno.OP_SPECTRAL_FWD) <= fno.NOALLOC_SCRATCH_BYTES
    ref_cache, cache = plan.new_cache(), plan.new_cache()
    y_ref = plan.spectral_fwd(tx, tw, cache=ref_cache)
    y = torch.full_like(y_ref, float("nan"))
    plan.spectral_fwd_noalloc(tx, tw, y, cache=cache)
    y_nc = torch.full_like(y_ref, float("nan"))
    plan.spectral_fwd_noalloc(tx, tw, y_nc)  # without a cache
    torch.cuda.synchronize()
    return y_ref, y, y_nc, ref_cache, cache


@pytest.mark.parametrize("code", [0, 1], ids=["f32", "bf16"])
def test_noalloc_matches_workspace_entry_point(fno, code):
    for i, (B, Ci, Co, grid, modes) in enumerate(CASES):
        print(f"noalloc case {i}: B={B} Ci={Ci} Co={Co} grid={grid} modes={modes} dtype={code}", flush=True)
        plan = fno.Plan(B, Ci, Co, grid, modes, code)
        y_ref, y, y_nc, ref_cache, cache = run_pair(fno, plan, seed=11 + i)
        assert torch.equal(y.view(torch.int16 if code else torch.int32),
                           y_ref.view(torch.int16 if code else torch.int32)), f"case {i}: y differs"
        assert torch.equal(y_nc.view(torch.int16 if code else torch.int32),
                           y_ref.view(torch.int16 if code else torch.int32)), f"case {i}: y (no cache) differs"
        assert torch.equal(cache, ref_cache), f"case {i}: cache differs"
        assert np.isfinite(y.float().cpu().numpy()).all()


def test_noalloc_rejects_sizes_beyond_the_static_array(fno):
    plan = fno.Plan(1, 20, 20, (64, 64, 64, 16), (12, 12, 12, 8), fno.FNO_BF16)
    assert plan.workspace_bytes(fno.OP_SPECTRAL_FWD) > fno.NOALLOC_SCRATCH_BYTES
    x = torch.zeros(plan.act_shape(20), dtype=plan.act_dtype, device="cuda")
    w = torch.zeros((20, 20, *plan.kshape), dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    with pytest.raises(fno.FnoError) as e:
        plan.spectral_fwd_noalloc(x, w, y)
    assert e.value.code == fno.FNO_ERR_WORKSPACE
