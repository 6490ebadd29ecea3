"""Network glue of Alg. 1 on the GPU (encoder, decoder, loss) and the whole
FNO (encoder -> 4 blocks -> decoder -> MSE) against the FP64 oracle, plus
central finite differences of the FP64 oracle loss against the GPU gradient
on the 16^3 x 8 copy of the Navier-Stokes-shaped network."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2211_12709_amd import inputs  # noqa: E402

F32_TOL, BF16_TOL = 1e-5, 1e-2


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
    return float(np.linalg.norm((np.asarray(a) - ref).ravel()) / max(np.linalg.norm(np.ravel(ref)), 1e-300))


def np64(t):
    t = t.detach().cpu()
    return t.numpy().astype(np.complex128) if t.is_complex() else t.float().numpy().astype(np.float64)


def dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda().to(dtype).contiguous()


# (grid, input channels): N = 7680 (vector path), N = 525 (odd length: element path and a
# ragged last work item), and the CO2 encoder's 3 channels
LIFT_CASES = {"n7680_c4": ((12, 10, 8, 8), 4), "n525_c4": ((5, 3, 7, 5), 4), "n4608_c3": ((8, 8, 9, 8), 3)}


@pytest.mark.parametrize("dt", [torch.float32, torch.bfloat16], ids=["f32", "bf16"])
@pytest.mark.parametrize("case", sorted(LIFT_CASES))
def test_lift(fno, o, dt, case):
    grid, ci = LIFT_CASES[case]
    x = inputs.normal_field((2, ci, *grid), seed=3)
    we, be = inputs.linear_weights(20, ci, seed=inputs.SEED_LIFT)
    gy = inputs.normal_field((2, 20, *grid), seed=7)
    y = fno.lift_fwd(dev(x, dt), dev(we), dev(be))
    gw, gb = fno.lift_bwd(dev(x, dt), dev(we), dev(be), dev(gy, dt))
    torch.cuda.synchronize()
    tol = F32_TOL if dt == torch.float32 else BF16_TOL
    assert rel(np64(y), o.lift_fwd(x, we, be)) < tol
    _, gw_ref, gb_ref = o.lift_bwd(x, we, be, gy)
    assert rel(np64(gw), gw_ref) < tol
    assert rel(np64(gb), gb_ref) < tol
    # accumulate: a second call adds the same gradients again
    fno.lift_bwd(dev(x, dt), dev(we), dev(be), dev(gy, dt), out=(gw, gb))
    torch.cuda.synchronize()
    assert rel(np64(gw), 2 * gw_ref) < tol
    assert rel(np64(gb), 2 * gb_ref) < tol


# (grid, input channels, hidden channels): the first layer's K chunks (inputs plus the bias row)
# are 2 for 20 channels, 1 for 8 and 3 for 32; N = 4320 is a whole number of 16-point tiles,
# N = 525 an odd length (element path, ragged last tile); H = 100 leaves hidden rows unused.
PROJ_CASES = {"n4320_c20_h128": ((10, 6, 9, 8), 20, 128), "n525_c20_h128": ((5, 3, 7, 5), 20, 128),
              "n4320_c8_h100": ((10, 6, 9, 8), 8, 100), "n525_c32_h128": ((5, 3, 7, 5), 32, 128)}


@pytest.mark.parametrize("dt", [torch.float32, torch.bfloat16], ids=["f32", "bf16"])
@pytest.mark.parametrize("case", sorted(PROJ_CASES))
def test_projection(fno, o, dt, case):
    grid, ci, hid = PROJ_CASES[case]
    x = inputs.normal_field((2, ci, *grid), seed=5)
    w1, b1 = inputs.linear_weights(hid, ci, seed=inputs.SEED_PROJ1)
    w2, b2 = inputs.linear_weights(1, hid, seed=inputs.SEED_PROJ2)
    gy = inputs.normal_field((2, 1, *grid), seed=9)
    y = fno.proj_fwd(dev(x, dt), dev(w1), dev(b1), dev(w2), dev(b2))
    outs = fno.proj_bwd(dev(x, dt), dev(w1), dev(b1), dev(w2), dev(b2), dev(gy, dt))
    torch.cuda.synchronize()
    tol = F32_TOL if dt == torch.float32 else BF16_TOL
    assert rel(np64(y), o.proj_fwd(x, w1, b1, w2, b2)) < tol
    refs = o.proj_bwd(x, w1, b1, w2, b2, gy)
    for name, a, r in zip(("gx", "gw1", "gb1", "gw2", "gb2"), outs, refs):
        assert rel(np64(a), r) < tol, name
    # accumulate: a second call adds the same gradients again
    fno.proj_bwd(dev(x, dt), dev(w1), dev(b1), dev(w2), dev(b2), dev(gy, dt), out=outs)
    torch.cuda.synchronize()
    for name, a, r in zip(("gx", "gw1", "gb1", "gw2", "gb2"), outs, refs):
        assert rel(np64(a), 2 * r) < tol, name + " (accumulated)"


def test_mse(fno, o):
    y = inputs.normal_field((3, 1, 7, 5, 4, 4), seed=1)
    t = inputs.normal_field((3, 1, 7, 5, 4, 4), seed=2)
    loss, gy = fno.mse(dev(y), dev(t))
    torch.cuda.synchronize()
    L, g = o.mse(y, t)
    assert abs(float(loss.item()) - L) <= 1e-6 * abs(L)
    assert rel(np64(gy), g) < F32_TOL


def ns_params(width, kshape, nblocks=4, hidden=128, cin=4):
    we, be = inputs.linear_weights(width, cin, seed=inputs.SEED_LIFT)
    blocks = [inputs.block_params(width, width, kshape, block=i) for i in range(nblocks)]
    w1, b1 = inputs.linear_weights(hidden, width, seed=inputs.SEED_PROJ1)
    w2, b2 = inputs.linear_weights(1, hidden, seed=inputs.SEED_PROJ2)
    return {"lift": (we, be), "blocks": blocks, "proj": (w1, b1, w2, b2)}


def run_net(fno, params, x, target, grid, modes, dt, width):
    net = fno.FNO4d(4, width, grid, modes, nblocks=len(params["blocks"]), dtype=dt, params=params)
    y = net(dev(x, dt))
    loss = fno.MseFn.apply(y, dev(target, dt))
    loss.backward()
    torch.cuda.synchronize()
    grads = {"lift": [p.grad for p in net.lift], "blocks": [[p.grad for p in b] for b in net.blocks],
             "proj": [p.grad for p in net.proj]}
    return y, float(loss.item()), grads


@pytest.mark.parametrize("dt", [torch.float32, torch.bfloat16], ids=["f32", "bf16"])
def test_network_step_vs_oracle(fno, o, dt):
    """The 16^3 x 8 copy of the NS-shaped network (width 20, modes 4,4,4,4, 4 blocks, 20 -> 128 -> 1)."""
    grid, modes, width = (16, 16, 16, 8), (4, 4, 4, 4), 20
    d = o.Dims(1, width, width, grid, modes)
    params = ns_params(width, d.kshape)
    x = inputs.ns_like_input(1, grid)
    target = inputs.normal_field((1, 1, *grid), seed=inputs.SEED_TARGET)
    y, loss, grads = run_net(fno, params, x, target, grid, modes, dt, width)
    y_ref, acts = o.fno_fwd(d, x, params)
    L_ref, gy_ref = o.mse(y_ref, target)
    g_ref = o.fno_bwd(d, x, params, acts, gy_ref)
    tol = F32_TOL if dt == torch.float32 else BF16_TOL
    errs = {"y": rel(np64(y), y_ref), "loss": abs(loss - L_ref) / abs(L_ref)}
    for k, (a, r) in enumerate(zip(grads["lift"], g_ref["lift"])):
        errs[f"lift{k}"] = rel(np64(a), r)
    for bi, (gb, rb) in enumerate(zip(grads["blocks"], g_ref["blocks"])):
        for k, (a, r) in enumerate(zip(gb, rb)):
            errs[f"block{bi}.{k}"] = rel(np64(a), r)
    for k, (a, r) in enumerate(zip(grads["proj"], g_ref["proj"])):
        errs[f"proj{k}"] = rel(np64(a), r)
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    bad = {k: v for k, v in errs.items() if not v < tol}
    assert not bad, bad


def test_network_finite_differences(fno, o):
    """Central differences (eps 1e-3) of the FP64 oracle loss on 32 sampled
    weights against the GPU's FP32 analytic gradient (16^3 x 8 copy)."""
    grid, modes, width = (16, 16, 16, 8), (4, 4, 4, 4), 20
    d = o.Dims(1, width, width, grid, modes)
    params = ns_params(width, d.kshape)
    x = inputs.ns_like_input(1, grid)
    target = inputs.normal_field((1, 1, *grid), seed=inputs.SEED_TARGET)
    _, _, grads = run_net(fno, params, x, target, grid, modes, torch.float32, width)
    # work on float64 copies of the float32 parameters
    p64 = {"lift": [np.array(a, dtype=np.float64) for a in params["lift"]],
           "blocks": [[np.array(a, dtype=np.complex128 if np.iscomplexobj(a) else np.float64) for a in b]
                      for b in params["blocks"]],
           "proj": [np.array(a, dtype=np.float64) for a in params["proj"]]}

    def loss64():
        y, _ = o.fno_fwd(d, x, p64)
        return o.mse(y, target)[0]

    rng = np.random.default_rng(inputs.SEED_FD)
    sites = [("lift", 0), ("lift", 1), ("blocks", (0, 0)), ("blocks", (3, 0)), ("blocks", (1, 1)),
             ("blocks", (2, 2)), ("proj", 0), ("proj", 1), ("proj", 2), ("proj", 3)]
    eps, checks = 1e-3, []
    for k in range(32):
        grp, sub = sites[k % len(sites)]
        if grp == "blocks":
            arr, g = p64["blocks"][sub[0]][sub[1]], np64(grads["blocks"][sub[0]][sub[1]])
        else:
            arr, g = p64[grp][sub], np64(grads[grp][sub])
        idx = tuple(int(rng.integers(0, s)) for s in arr.shape)
        unit, part = (1j, "im") if (np.iscomplexobj(arr) and k % 2) else (1.0, "re")
        orig = arr[idx]
        arr[idx] = orig + eps * unit
        lp = loss64()
        arr[idx] = orig - eps * unit
        lm = loss64()
        arr[idx] = orig
        fd = (lp - lm) / (2 * eps)
        an = g[idx].real if part == "re" else g[idx].imag
        checks.append((grp, sub, idx, part, fd, an))
    scale = max(abs(c[-1]) for c in checks)
    for c in checks:
        fd, an = c[-2], c[-1]
        assert abs(fd - an) <= 2e-3 * abs(fd) + 1e-4 * scale, c


# ---------------------------------------------------------------- Navier-Stokes-shaped network at full size
NS_GRID, NS_MODES, NS_WIDTH = (64, 64, 64, 16), (12, 12, 12, 8), 20


@pytest.fixture(scope="module")
def ns_full(o):
    """The full Navier-Stokes-shaped FNO (4-channel input on 64^3 x 16, lifting to width 20,
    4 blocks with modes 12,12,12,8, projection 20 -> 128 -> 1) and an MSE loss against a
    seeded target: FP64 oracle forward (every block's output kept) and gradients, once."""
    d = o.Dims(1, NS_WIDTH, NS_WIDTH, NS_GRID, NS_MODES)
    params = ns_params(NS_WIDTH, d.kshape)
    x = inputs.ns_like_input(1, NS_GRID)
    target = inputs.normal_field((1, 1, *NS_GRID), seed=inputs.SEED_TARGET)
    print("ns network 64^3x16: FP64 oracle forward + backward", flush=True)
    y_ref, acts = o.fno_fwd(d, x, params)
    L_ref, gy_ref = o.mse(y_ref, target)
    g_ref = o.fno_bwd(d, x, params, acts, gy_ref)
    return dict(d=d, params=params, x=x, target=target, y=y_ref, acts=acts, L=L_ref, grads=g_ref)


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("dt", [torch.float32, torch.bfloat16], ids=["f32", "bf16"])
def test_ns_network_full_size(fno, o, ns_full, dt):
    """Forward of the whole network (every block's output and the network output) and the
    gradient of every parameter of the training step, against the FP64 oracle at full size."""
    print(f"ns network 64^3x16 dtype={dt}", flush=True)
    tol = F32_TOL if dt == torch.float32 else BF16_TOL
    params = ns_full["params"]
    net = fno.FNO4d(4, NS_WIDTH, NS_GRID, NS_MODES, nblocks=4, dtype=dt, params=params)
    errs = {}
    # per-block forward outputs (Alg. 1: lifting, then each block)
    with torch.no_grad():
        h = fno.LiftFn.apply(dev(ns_full["x"], dt), *net.lift)
        errs["lift_out"] = rel(np64(h), ns_full["acts"][0])
        for bi, (w, wpw, bpw) in enumerate(net.blocks):
            h = fno.FNOBlockFn.apply(h, w, wpw, bpw, net.plan)
            errs[f"block{bi}_out"] = rel(np64(h), ns_full["acts"][bi + 1])
        del h
    y, loss, grads = run_net(fno, params, ns_full["x"], ns_full["target"], NS_GRID, NS_MODES, dt, NS_WIDTH)
    g_ref = ns_full["grads"]
    errs["y"] = rel(np64(y), ns_full["y"])
    errs["loss"] = abs(loss - ns_full["L"]) / abs(ns_full["L"])
    for k, (a, r) in enumerate(zip(grads["lift"], g_ref["lift"])):
        errs[f"lift{k}"] = rel(np64(a), r)
    for bi, (gb, rb) in enumerate(zip(grads["blocks"], g_ref["blocks"])):
        for k, (a, r) in enumerate(zip(gb, rb)):
            errs[f"block{bi}.{k}"] = rel(np64(a), r)
    for k, (a, r) in enumerate(zip(grads["proj"], g_ref["proj"])):
        errs[f"proj{k}"] = rel(np64(a), r)
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    bad = {k: v for k, v in errs.items() if not v < tol}
    assert not bad, bad
