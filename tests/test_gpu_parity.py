"""Parity of the HIP path (through the C-ABI) with the FP64 CPU oracle.

Tolerances: relative L2 error (||a - ref|| / ||ref|| over the whole tensor,
complex as (re, im) pairs) of at most 1e-5 for the FP32 path and 1e-2 for the
BF16 path.  Inputs are seeded (paper_2211_12709_amd.inputs); the oracle
consumes the exact float32 values handed to the GPU, so BF16 errors include
the quantisation of activations to bfloat16.
"""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2211_12709_amd import inputs  # noqa: E402

F32_TOL = 1e-5
BF16_TOL = 1e-2

SHAPES = {
    # name: (B, Ci, Co, grid, modes)
    "single_layer_16^3x8": (1, 8, 8, (16, 16, 16, 8), (4, 4, 4, 4)),
    "odd_ragged": (2, 3, 5, (12, 10, 9, 7), (3, 2, 4, 4)),
    "full_retention_nyquist": (1, 4, 6, (8, 6, 10, 16), (4, 3, 5, 9)),
    "long_t_plane": (1, 2, 3, (4, 6, 40, 32), (2, 3, 16, 8)),
    "ns_shape_small": (1, 20, 20, (24, 20, 16, 16), (6, 5, 4, 8)),
    # the z,t kernel variants of the CO2-shaped block (width 20, Nt 32, Kt 8: three source K
    # chunks per tile, two t tiles) and of the batched CO2 block (width 32, Kt 10: two
    # (re/im, kt) tiles), and the batched block's z modes (2 mz = 40)
    "co2_tiles_w20_t32": (1, 20, 20, (4, 4, 32, 32), (2, 2, 8, 8)),
    "batched_tiles_w32_kt10": (2, 32, 32, (4, 4, 32, 32), (2, 2, 8, 10)),
    "batched_modes_kz40": (1, 32, 32, (4, 3, 48, 32), (2, 1, 20, 10)),
    # the batched CO2 block's y and z modes together (2 my = 2 mz = 40, 10 t bins): the general
    # forward t,z,y kernel (three kz blocks, six y-step row tiles)
    "batched_modes_ky40_kz40": (1, 32, 32, (4, 40, 48, 32), (2, 20, 20, 10)),
    # reduced copies of the paper's own grids (Sec. V): Navier-Stokes 130^3 x 64 (Nz 130, Nt 64,
    # two t slices) and CO2 262 x 118 x 64 x 86 (Nt 86: rows not 4-aligned), about 20% of the
    # frequencies kept per axis, at small and at full width
    "ns_true_z130_t64": (1, 3, 4, (4, 3, 130, 64), (2, 1, 13, 7)),
    "ns_true_w20": (1, 20, 20, (3, 3, 40, 64), (1, 1, 8, 7)),
    "co2_true_t86": (1, 4, 4, (10, 6, 64, 86), (5, 3, 6, 9)),
    "co2_true_w20": (1, 20, 20, (4, 4, 64, 86), (2, 2, 6, 9)),
    # odd Nt beyond one t slice (element-wise rows), and more t bins than the matrix-core
    # kernels take (the scalar kernels)
    "odd_t45": (1, 3, 5, (4, 5, 20, 45), (2, 2, 5, 12)),
    "scalar_kt21": (1, 2, 3, (4, 4, 6, 40), (2, 2, 3, 21)),
    # batch 4 at width 32 (the batched CO2 block's): the mix holds the batch in registers and
    # its backward takes 32-mode tiles (64 would not fit in LDS)
    "batch4_w32": (4, 32, 32, (4, 4, 16, 8), (2, 2, 4, 4)),
    # three chunks of 32 y planes, the last one ragged: the bfloat16 k_tzy_fwd's y basis
    # double-buffered a chunk ahead and its plane slots over several chunks
    "tall_y_chunks": (1, 4, 4, (2, 80, 16, 8), (1, 10, 4, 4)),
}

# the kernels each shape must run on: forward t,z,y (k_tzy_fwd "tzy_fwd", the general
# "tzy_gen", or the scalar "fwd_tz") and z,t epilogue (matrix-core "zt_*", t-sliced "zt_*_tsl",
# or the scalar "inv_zt_*"); a pair (float, bfloat16) where the dtypes differ: float plans take
# the general forward kernel wherever the bfloat16 ones take k_tzy_fwd, and at width 32 with
# 2 mz = 40 the float epilogue's U tile alone needs more LDS than a workgroup has
PAIR = ("tzy_gen", "tzy_fwd")
PATHS = {
    "single_layer_16^3x8": (PAIR, "zt_block"),
    "odd_ragged": ("tzy_gen", "zt_block_tsl"),
    "full_retention_nyquist": (PAIR, "zt_block"),
    "long_t_plane": (PAIR, "zt_block"),
    "ns_shape_small": (PAIR, "zt_block"),
    "co2_tiles_w20_t32": (PAIR, "zt_block"),
    "batched_tiles_w32_kt10": (PAIR, "zt_block"),
    "batched_modes_kz40": ("tzy_gen", ("inv_zt_block", "zt_block")),
    "batched_modes_ky40_kz40": ("tzy_gen", ("inv_zt_block", "zt_block")),
    "ns_true_z130_t64": ("tzy_gen", "zt_block_tsl"),
    "ns_true_w20": ("tzy_gen", "zt_block_tsl"),
    "co2_true_t86": ("tzy_gen", "zt_block_tsl"),
    "co2_true_w20": ("tzy_gen", "zt_block_tsl"),
    "odd_t45": ("tzy_gen", "zt_block_tsl"),
    "scalar_kt21": ("fwd_tz", "inv_zt_block"),
    "batch4_w32": (PAIR, "zt_block"),
    "tall_y_chunks": (PAIR, "zt_block"),
}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fno():
    from paper_2211_12709_amd import fno as f
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    f.load_library()
    return f


@pytest.fixture(scope="module")
def o():
    from oracle import oracle as orc
    orc.lib()
    return orc


def rel(a, ref):
    a = np.asarray(a)
    ref = np.asarray(ref)
    return float(np.linalg.norm((a - ref).ravel()) / max(np.linalg.norm(ref.ravel()), 1e-300))


def to_np(t):
    t = t.detach().cpu()
    if t.is_complex():
        return t.numpy().astype(np.complex128)
    return t.float().numpy().astype(np.float64)


def dev_act(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda().to(dtype).contiguous()


def case(name, dtype_code, seed=0):
    B, Ci, Co, grid, modes = SHAPES[name]
    ksh = (2 * modes[0], 2 * modes[1], 2 * modes[2], modes[3])
    x = inputs.normal_field((B, Ci, *grid), seed=seed)
    w, wpw, bpw = inputs.block_params(Ci, Co, ksh, block=seed)
    gy = inputs.normal_field((B, Co, *grid), seed=seed + 1000)
    return (B, Ci, Co, grid, modes), x, w, wpw, bpw, gy


def tol(dtype_code):
    return F32_TOL if dtype_code == 0 else BF16_TOL


@pytest.mark.parametrize("name", sorted(SHAPES))
@pytest.mark.parametrize("dt", [0, 1], ids=["f32", "bf16"])
def test_spectral_fwd_and_cache(fno, o, name, dt):
    (B, Ci, Co, grid, modes), x, w, _, _, _ = case(name, dt)
    say(f"spectral_fwd {name} dtype={dt}")
    d = o.Dims(B, Ci, Co, grid, modes)
    plan = fno.Plan(B, Ci, Co, grid, modes, dt)
    xq = dev_act(x, plan.act_dtype)
    cache = plan.new_cache()
    y = plan.spectral_fwd(xq, torch.from_numpy(w).cuda(), cache=cache)
    torch.cuda.synchronize()
    y_ref, xh_ref, _ = o.spectral_fwd(d, x, w, return_spectra=True)
    e = rel(to_np(y), y_ref)
    nxh = B * Ci * d.nmode
    xh = cache[: nxh * 8].view(torch.complex64).reshape(B, Ci, *d.kshape)
    exh = rel(to_np(xh), xh_ref)
    say(f"  rel y={e:.2e} xhat={exh:.2e}")
    assert e < tol(dt)
    assert exh < tol(dt)


@pytest.mark.parametrize("name", sorted(SHAPES))
@pytest.mark.parametrize("dt", [0, 1], ids=["f32", "bf16"])
def test_spectral_bwd(fno, o, name, dt):
    (B, Ci, Co, grid, modes), x, w, _, _, gy = case(name, dt)
    say(f"spectral_bwd {name} dtype={dt}")
    d = o.Dims(B, Ci, Co, grid, modes)
    plan = fno.Plan(B, Ci, Co, grid, modes, dt)
    xq, gyq = dev_act(x, plan.act_dtype), dev_act(gy, plan.act_dtype)
    tw = torch.from_numpy(w).cuda()
    cache = plan.new_cache()
    plan.spectral_fwd(xq, tw, cache=cache)
    gx, gw = plan.spectral_bwd(gyq, tw, x=xq, cache=cache)
    gx2, gw2 = plan.spectral_bwd(gyq, tw, x=xq, cache=None)       # recompute X^ from x
    torch.cuda.synchronize()
    gx_ref, gw_ref = o.spectral_bwd(d, x, w, gy)
    e1, e2 = rel(to_np(gx), gx_ref), rel(to_np(gw), gw_ref)
    say(f"  rel gx={e1:.2e} gw={e2:.2e}")
    assert e1 < tol(dt) and e2 < tol(dt)
    assert torch.equal(gx, gx2) and torch.equal(gw, gw2)


@pytest.mark.parametrize("name", sorted(SHAPES))
@pytest.mark.parametrize("dt", [0, 1], ids=["f32", "bf16"])
def test_block_fwd_bwd(fno, o, name, dt):
    (B, Ci, Co, grid, modes), x, w, wpw, bpw, gy = case(name, dt, seed=3)
    if Ci != Co:
        wpw, bpw = inputs.linear_weights(Co, Ci, seed=inputs.SEED_POINTWISE + 3)
    say(f"block {name} dtype={dt}")
    d = o.Dims(B, Ci, Co, grid, modes)
    plan = fno.Plan(B, Ci, Co, grid, modes, dt)
    xq, gyq = dev_act(x, plan.act_dtype), dev_act(gy, plan.act_dtype)
    tw, twp, tb = (torch.from_numpy(a).cuda() for a in (w, wpw, bpw))
    cache = plan.new_cache()
    y = plan.block_fwd(xq, tw, twp, tb, cache=cache)
    gx, gw, gwpw, gb = plan.block_bwd(xq, cache, tw, twp, tb, gyq)
    torch.cuda.synchronize()
    y_ref = o.block_fwd(d, x, w, wpw, bpw)
    gx_ref, gw_ref, gwpw_ref, gb_ref = o.block_bwd(d, x, w, wpw, bpw, gy)
    errs = dict(y=rel(to_np(y), y_ref), gx=rel(to_np(gx), gx_ref), gw=rel(to_np(gw), gw_ref),
                gw_pw=rel(to_np(gwpw), gwpw_ref), gb=rel(to_np(gb), gb_ref))
    say("  rel " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v < tol(dt), (k, v)


@pytest.mark.parametrize("name", sorted(SHAPES))
def test_kernel_paths(fno, name):
    """Each shape runs on the kernels it is meant to exercise (names from the per-kernel timing)."""
    B, Ci, Co, grid, modes = SHAPES[name]
    want_fwd, want_epi = PATHS[name]
    for dt in (0, 1):
        plan = fno.Plan(B, Ci, Co, grid, modes, dt)
        x = torch.zeros((B, Ci, *grid), dtype=plan.act_dtype, device="cuda")
        w = torch.zeros((Ci, Co, *plan.kshape), dtype=torch.complex64, device="cuda")
        wpw = torch.zeros((Co, Ci), device="cuda")
        plan.timing(True)
        plan.block_fwd(x, w, wpw)
        names = set(plan.timing_read())
        plan.timing(False)
        say(f"{name} dtype={dt}: {sorted(names)}")
        fwd = {n.split("<")[0] for n in names} & {"tzy_fwd", "tzy_gen", "fwd_tz"}
        assert fwd == {want_fwd if isinstance(want_fwd, str) else want_fwd[dt]}, (name, dt, names)
        epi = want_epi if isinstance(want_epi, str) else want_epi[dt]
        assert epi in names, (name, dt, names)


def test_block_without_bias_and_accumulate(fno, o):
    (B, Ci, Co, grid, modes), x, w, wpw, _, gy = case("odd_ragged", 0, seed=5)
    wpw, _ = inputs.linear_weights(Co, Ci, seed=77)
    say("block no-bias + accumulate")
    d = o.Dims(B, Ci, Co, grid, modes)
    plan = fno.Plan(B, Ci, Co, grid, modes, 0)
    xq, gyq = dev_act(x, torch.float32), dev_act(gy, torch.float32)
    tw, twp = torch.from_numpy(w).cuda(), torch.from_numpy(wpw).cuda()
    cache = plan.new_cache()
    y = plan.block_fwd(xq, tw, twp, None, cache=cache)
    gx0 = torch.full_like(xq, 0.25)
    gw0 = torch.full((Ci, Co, *d.kshape), 0.5 + 0.5j, dtype=torch.complex64, device="cuda")
    gwpw0 = torch.full((Co, Ci), -1.0, device="cuda")
    gx, gw, gwpw, gb = plan.block_bwd(xq, cache, tw, twp, None, gyq, gx=gx0.clone(), gw=gw0.clone(),
                                      gw_pw=gwpw0.clone(), need_gb=False, accumulate=True)
    torch.cuda.synchronize()
    y_ref = o.block_fwd(d, x, w, wpw, None)
    gx_ref, gw_ref, gwpw_ref, _ = o.block_bwd(d, x, w, wpw, None, gy)
    assert rel(to_np(y), y_ref) < F32_TOL
    assert rel(to_np(gx), gx_ref + 0.25) < F32_TOL
    assert rel(to_np(gw), gw_ref + (0.5 + 0.5j)) < F32_TOL
    assert rel(to_np(gwpw), gwpw_ref - 1.0) < F32_TOL


@pytest.mark.parametrize("name", ["ns_shape_small", "long_t_plane"])
@pytest.mark.parametrize("dt", [0, 1], ids=["f32", "bf16"])
def test_accumulate_on_matrix_core_path(fno, o, name, dt):
    """accumulate=True adds every gradient into the given buffers on the matrix-core z,t path
    (Nt a multiple of 4), for the block and for the spectral layer alone."""
    (B, Ci, Co, grid, modes), x, w, wpw, bpw, gy = case(name, dt, seed=9)
    say(f"accumulate {name} dtype={dt}")
    d = o.Dims(B, Ci, Co, grid, modes)
    plan = fno.Plan(B, Ci, Co, grid, modes, dt)
    xq, gyq = dev_act(x, plan.act_dtype), dev_act(gy, plan.act_dtype)
    tw, twp, tb = (torch.from_numpy(a).cuda() for a in (w, wpw, bpw))
    cache = plan.new_cache()
    plan.block_fwd(xq, tw, twp, tb, cache=cache)
    gx0 = torch.full_like(xq, 0.25)
    gw0 = torch.full((Ci, Co, *d.kshape), 0.5 + 0.5j, dtype=torch.complex64, device="cuda")
    gwpw0 = torch.full((Co, Ci), -1.0, device="cuda")
    gb0 = torch.full((Co,), 2.0, device="cuda")
    gx, gw, gwpw, gb = plan.block_bwd(xq, cache, tw, twp, tb, gyq, gx=gx0.clone(), gw=gw0.clone(),
                                      gw_pw=gwpw0.clone(), gb_pw=gb0.clone(), accumulate=True)
    gxs, gws = plan.spectral_bwd(gyq, tw, x=xq, gx=gx0.clone(), gw=gw0.clone(), accumulate=True)
    torch.cuda.synchronize()
    gx_ref, gw_ref, gwpw_ref, gb_ref = o.block_bwd(d, x, w, wpw, bpw, gy)
    gxs_ref, gws_ref = o.spectral_bwd(d, x, w, gy)
    errs = dict(gx=rel(to_np(gx), gx_ref + 0.25), gw=rel(to_np(gw), gw_ref + (0.5 + 0.5j)),
                gw_pw=rel(to_np(gwpw), gwpw_ref - 1.0), gb=rel(to_np(gb), gb_ref + 2.0),
                spectral_gx=rel(to_np(gxs), gxs_ref + 0.25), spectral_gw=rel(to_np(gws), gws_ref + (0.5 + 0.5j)))
    say("  rel " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v < tol(dt), (k, v)


def test_adjoint_dot_product_on_gpu(fno):
    """<S u, v> = <u, S* v> for the spectral layer, with both sides from the GPU."""
    B, Ci, Co, grid, modes = SHAPES["odd_ragged"]
    plan = fno.Plan(B, Ci, Co, grid, modes, 0)
    ksh = plan.kshape
    u = dev_act(inputs.normal_field((B, Ci, *grid), seed=11), torch.float32)
    v = dev_act(inputs.normal_field((B, Co, *grid), seed=12), torch.float32)
    w = torch.from_numpy(inputs.spectral_weights(Ci, Co, ksh, seed=13)).cuda()
    y = plan.spectral_fwd(u, w)
    gx, _ = plan.spectral_bwd(v, w, need_gw=False)
    lhs = float((y.double() * v.double()).sum())
    rhs = float((u.double() * gx.double()).sum())
    assert abs(lhs - rhs) <= 1e-5 * (abs(lhs) + abs(rhs))


def test_deterministic_reruns(fno):
    B, Ci, Co, grid, modes = SHAPES["ns_shape_small"]
    plan = fno.Plan(B, Ci, Co, grid, modes, 1)
    (B, Ci, Co, grid, modes), x, w, wpw, bpw, gy = case("ns_shape_small", 1)
    xq, gyq = dev_act(x, plan.act_dtype), dev_act(gy, plan.act_dtype)
    tw, twp, tb = (torch.from_numpy(a).cuda() for a in (w, wpw, bpw))
    outs = []
    for _ in range(2):
        cache = plan.new_cache()
        y = plan.block_fwd(xq, tw, twp, tb, cache=cache)
        outs.append((y, *plan.block_bwd(xq, cache, tw, twp, tb, gyq)))
    torch.cuda.synchronize()
    for a, b in zip(*outs):
        assert torch.equal(a, b)


def test_error_codes_on_gpu(fno):
    import ctypes
    B, Ci, Co, grid, modes = SHAPES["single_layer_16^3x8"]
    plan = fno.Plan(B, Ci, Co, grid, modes, 0)
    lib = fno.load_library()
    x = torch.zeros((B, Ci, *grid), device="cuda")
    y = torch.zeros((B, Co, *grid), device="cuda")
    w = torch.zeros((Ci, Co, *plan.kshape), dtype=torch.complex64, device="cuda")
    need = plan.workspace_bytes(fno.OP_SPECTRAL_FWD)
    ws = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    P = lambda t, off=0: ctypes.c_void_p(t.data_ptr() + off)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.fno_spectral_fwd(plan._h, P(x), P(w), P(y), None, P(ws), need - 1, st) == fno.FNO_ERR_WORKSPACE
    assert lib.fno_spectral_fwd(plan._h, P(x, 4), P(w), P(y), None, P(ws), need, st) == fno.FNO_ERR_ALIGNMENT
    assert lib.fno_spectral_fwd(plan._h, None, P(w), P(y), None, P(ws), need, st) == fno.FNO_ERR_INVALID_ARG
    assert lib.fno_block_bwd(plan._h, P(x), None, P(w), P(w), None, P(y), P(x), None, None, None, 0, P(ws), need,
                             st) == fno.FNO_ERR_INVALID_ARG   # block backward needs the forward cache
    assert lib.fno_spectral_fwd(plan._h, P(x), P(w), P(y), None, P(ws), need, st) == fno.FNO_OK
    torch.cuda.synchronize()


def test_autograd_functions(fno, o):
    (B, Ci, Co, grid, modes), x, w, wpw, bpw, gy = case("odd_ragged", 0, seed=9)
    wpw, bpw = inputs.linear_weights(Co, Ci, seed=99)
    d = o.Dims(B, Ci, Co, grid, modes)
    plan = fno.Plan(B, Ci, Co, grid, modes, 0)
    tx = dev_act(x, torch.float32).requires_grad_(True)
    tw = torch.from_numpy(w).cuda().requires_grad_(True)
    twp = torch.from_numpy(wpw).cuda().requires_grad_(True)
    tb = torch.from_numpy(bpw).cuda().requires_grad_(True)
    y = fno.FNOBlockFn.apply(tx, tw, twp, tb, plan)
    (y * dev_act(gy, torch.float32)).sum().backward()
    gx_ref, gw_ref, gwpw_ref, gb_ref = o.block_bwd(d, x, w, wpw, bpw, gy)
    assert rel(to_np(tx.grad), gx_ref) < F32_TOL
    assert rel(to_np(tw.grad), gw_ref) < F32_TOL
    assert rel(to_np(twp.grad), gwpw_ref) < F32_TOL
    assert rel(to_np(tb.grad), gb_ref) < F32_TOL
    tx.grad = None
    tw.grad = None
    ys = fno.SpectralConv4dFn.apply(tx, tw, plan)
    (ys * dev_act(gy, torch.float32)[:, :Co]).sum().backward()
    gx_ref, gw_ref = o.spectral_bwd(d, x, w, gy)
    assert rel(to_np(tx.grad), gx_ref) < F32_TOL
    assert rel(to_np(tw.grad), gw_ref) < F32_TOL
