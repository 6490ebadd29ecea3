"""Packed FP8 (OCP E4M3) spectral weights: fno_pack_weights against the E4M3 reference written
from the format's definition (bit-exact codes, power-of-two scale per channel pair), the block
fwd + bwd of an FNO_W_FP8 plan against the FP64 oracle evaluated with the dequantized weights
(the plan's usual tolerance: only the weights' storage differs), and the error the 8-bit weights
add against the oracle with the original weights (reported; bounded loosely)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import e4m3_ref  # noqa: E402
from paper_2211_12709_amd import inputs  # noqa: E402

TOL = {0: 1e-5, 1: 1e-2}
SHAPES = {
    "ns_shape_small": (1, 20, 20, (24, 20, 16, 16), (6, 5, 4, 8)),
    "batch4_w32": (4, 32, 32, (4, 4, 16, 8), (2, 2, 4, 4)),
}


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
    return float(np.linalg.norm((np.asarray(a) - ref).ravel()) / np.linalg.norm(np.ravel(ref)))


def np64(t):
    t = t.detach().cpu()
    return t.numpy().astype(np.complex128) if t.is_complex() else t.float().numpy().astype(np.float64)


def unpack(plan, packed, Ci, Co):
    """(codes [Ci][Co][modes][2] uint8, scales [Ci][Co]) of a packed buffer."""
    raw = packed.cpu().numpy()
    n = Ci * Co * int(np.prod(plan.kshape))
    codes = raw[: 2 * n].reshape(Ci, Co, *plan.kshape, 2)
    off = (2 * n + 255) // 256 * 256
    scales = raw[off: off + 4 * Ci * Co].view(np.float32).reshape(Ci, Co)
    return codes, scales


@pytest.mark.parametrize("name", sorted(SHAPES))
def test_pack_weights_matches_reference(fno, name):
    B, Ci, Co, grid, modes = SHAPES[name]
    plan = fno.Plan(B, Ci, Co, grid, modes, fno.FNO_BF16, fno.FNO_W_FP8)
    w = inputs.spectral_weights(Ci, Co, plan.kshape, seed=inputs.SEED_SPECTRAL_W)
    packed = plan.pack_weights(torch.from_numpy(w).cuda())
    torch.cuda.synchronize()
    codes, scales = unpack(plan, packed, Ci, Co)
    wr = np.stack([w.real, w.imag], axis=-1).astype(np.float64)  # the float32 values, widened
    for i in range(Ci):
        for k in range(Co):
            rms = np.sqrt(np.mean(wr[i, k] ** 2))
            e = np.log2(rms)
            s = scales[i, k]
            # power of two, 2^round(log2 RMS) (a float32 sum decides exact ties of the rounding)
            assert s == 2.0 ** np.round(np.log2(s))
            if abs(e - np.floor(e) - 0.5) > 1e-5:
                assert s == 2.0 ** np.round(e), (i, k, s, rms)
            ref = e4m3_ref.encode_array(wr[i, k] / s)
            assert np.array_equal(codes[i, k], ref), (i, k)


@pytest.mark.parametrize("name", sorted(SHAPES))
@pytest.mark.parametrize("code", [0, 1], ids=["f32", "bf16"])
def test_block_with_fp8_weights(fno, o, name, code):
    B, Ci, Co, grid, modes = SHAPES[name]
    plan = fno.Plan(B, Ci, Co, grid, modes, code, fno.FNO_W_FP8)
    d = o.Dims(B, Ci, Co, grid, modes)
    x = inputs.normal_field((B, Ci, *grid), seed=3)
    gy = inputs.normal_field((B, Co, *grid), seed=1003)
    w, wpw, bpw = inputs.block_params(Ci, Co, plan.kshape, block=3)
    tw = torch.from_numpy(w).cuda()
    packed = plan.pack_weights(tw)
    codes, scales = unpack(plan, packed, Ci, Co)
    # the weights the packed form represents (exact in float64)
    deq = e4m3_ref.decode_array(codes) * scales.astype(np.float64)[:, :, None, None, None, None, None]
    wq = (deq[..., 0] + 1j * deq[..., 1]).astype(np.complex128)
    xq = torch.from_numpy(x).cuda().to(plan.act_dtype)
    gyq = torch.from_numpy(gy).cuda().to(plan.act_dtype)
    twp, tb = torch.from_numpy(wpw).cuda(), torch.from_numpy(bpw).cuda()
    cache = plan.new_cache()
    y = plan.block_fwd(xq, packed, twp, tb, cache=cache)
    gx, gw, gwpw, gb = plan.block_bwd(xq, cache, packed, twp, tb, gyq)
    torch.cuda.synchronize()
    got = dict(y=np64(y), gx=np64(gx), gw=np64(gw), gw_pw=np64(gwpw), gb=np64(gb))
    # parity: the oracle with the dequantized weights
    yq = o.block_fwd(d, x, wq, wpw, bpw)
    gq = o.block_bwd(d, x, wq, wpw, bpw, gy)
    refq = dict(y=yq, gx=gq[0], gw=gq[1], gw_pw=gq[2], gb=gq[3])
    errs = {k: rel(got[k], refq[k]) for k in got}
    # error budget: the oracle with the original weights
    y0 = o.block_fwd(d, x, w, wpw, bpw)
    g0 = o.block_bwd(d, x, w, wpw, bpw, gy)
    ref0 = dict(y=y0, gx=g0[0], gw=g0[1], gw_pw=g0[2], gb=g0[3])
    budget = {k: rel(got[k], ref0[k]) for k in got}
    print(f"{name} dtype={code} parity (dequantized W) " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()),
          flush=True)
    print(f"{name} dtype={code} vs original W " + " ".join(f"{k}={v:.2e}" for k, v in budget.items()), flush=True)
    for k, v in errs.items():
        assert v < TOL[code], (k, v)
    for k, v in budget.items():
        assert v < 0.1, (k, v)
