"""Pins of the oracle's network glue (Alg. 1: encoder, FNO blocks, decoder)
and the MSE loss: torch float64 autograd as an independent gradient, and
central finite differences on sampled weights of every parameter group."""
import numpy as np
import pytest

from paper_2211_12709_amd import inputs

D_SPEC = (1, 5, 5, (6, 5, 4, 6), (2, 2, 1, 3))


def make_params(rng, cin, width, hidden, cout, kshape, nblocks):
    def lin(o, i):
        return rng.standard_normal((o, i)) / np.sqrt(i), rng.standard_normal(o) * 0.1
    we, be = lin(width, cin)
    blocks = []
    for _ in range(nblocks):
        w = (rng.standard_normal((width, width, *kshape)) + 1j * rng.standard_normal((width, width, *kshape))) * 0.2
        wpw, bpw = lin(width, width)
        blocks.append((w, wpw, bpw))
    w1, b1 = lin(hidden, width)
    w2, b2 = lin(cout, hidden)
    return {"lift": (we, be), "blocks": blocks, "proj": (w1, b1, w2, b2)}


def net_loss(o, d, x, params, target):
    y, _ = o.fno_fwd(d, x, params)
    return o.mse(y, target)[0]


def test_network_gradient_vs_torch_autograd(oracle):
    torch = pytest.importorskip("torch")
    o = oracle
    B, W, _, grid, modes = D_SPEC
    d = o.Dims(B, W, W, grid, modes)
    rng = np.random.default_rng(31)
    x = rng.standard_normal((B, 3, *grid))
    target = rng.standard_normal((B, 1, *grid))
    params = make_params(rng, 3, W, 7, 1, d.kshape, 2)
    y, acts = o.fno_fwd(d, x, params)
    L, gy = o.mse(y, target)
    grads = o.fno_bwd(d, x, params, acts, gy)

    T = lambda a: torch.tensor(a, requires_grad=True)
    tp = {"lift": [T(a) for a in params["lift"]], "blocks": [[T(a) for a in b] for b in params["blocks"]],
          "proj": [T(a) for a in params["proj"]]}
    (nx, ny, nz, nt), (mx, my, mz, mt) = grid, modes
    kset = lambda n, m: list(range(m)) + list(range(n - m, n))
    ix, iy, iz = (torch.tensor(kset(n, m)) for n, m in ((nx, mx), (ny, my), (nz, mz)))
    gelu = torch.nn.functional.gelu

    def pw(wm, bv, h):
        return torch.einsum("oi,bixyzt->boxyzt", wm, h) + bv[None, :, None, None, None, None]

    h = gelu(pw(tp["lift"][0], tp["lift"][1], torch.tensor(x)))
    for (w, wpw, bpw) in tp["blocks"]:
        X = torch.fft.rfftn(h, dim=(2, 3, 4, 5))
        Xk = X.index_select(2, ix).index_select(3, iy).index_select(4, iz)[..., :mt]
        Yk = torch.einsum("bikxyz,iokxyz->bokxyz", Xk, w)
        full = torch.zeros((B, W, nx, ny, nz, nt // 2 + 1), dtype=torch.complex128)
        full[:, :, ix[:, None, None], iy[None, :, None], iz[None, None, :], :mt] = Yk
        h = gelu(torch.fft.irfftn(full, s=grid, dim=(2, 3, 4, 5)) + pw(wpw, bpw, h))
    w1, b1, w2, b2 = tp["proj"]
    yt = pw(w2, b2, gelu(pw(w1, b1, h)))
    Lt = ((yt - torch.tensor(target)) ** 2).mean()
    Lt.backward()
    assert abs(float(Lt) - L) < 1e-12 * abs(L)
    rel = lambda a, b: np.linalg.norm(a - b) / np.linalg.norm(b)
    for a, t in zip(grads["lift"], tp["lift"]):
        assert rel(a, t.grad.numpy()) < 1e-11
    for gb, tb in zip(grads["blocks"], tp["blocks"]):
        for a, t in zip(gb, tb):
            assert rel(a, t.grad.numpy()) < 1e-11
    for a, t in zip(grads["proj"], tp["proj"]):
        assert rel(a, t.grad.numpy()) < 1e-11


def test_network_finite_differences(oracle):
    o = oracle
    B, W, _, grid, modes = D_SPEC
    d = o.Dims(B, W, W, grid, modes)
    rng = np.random.default_rng(inputs.SEED_FD)
    x = rng.standard_normal((B, 3, *grid))
    target = rng.standard_normal((B, 1, *grid))
    params = make_params(rng, 3, W, 7, 1, d.kshape, 2)
    y, acts = o.fno_fwd(d, x, params)
    _, gy = o.mse(y, target)
    grads = o.fno_bwd(d, x, params, acts, gy)
    eps = 1e-3
    groups = [("lift", 0), ("lift", 1), ("blocks", (0, 0)), ("blocks", (1, 0)), ("blocks", (0, 1)),
              ("blocks", (1, 2)), ("proj", 0), ("proj", 1), ("proj", 2), ("proj", 3)]
    checks = []
    for k in range(32):
        grp, sub = groups[k % len(groups)]
        if grp == "blocks":
            bi, pi = sub
            arr = params["blocks"][bi][pi]
            g = grads["blocks"][bi][pi]
        else:
            arr = params[grp][sub]
            g = grads[grp][sub]
        idx = tuple(int(rng.integers(0, s)) for s in arr.shape)
        for unit, part in ((1.0, "re"), (1j, "im")) if np.iscomplexobj(arr) else ((1.0, "re"),):
            orig = arr[idx]
            arr[idx] = orig + eps * unit
            lp = net_loss(o, d, x, params, target)
            arr[idx] = orig - eps * unit
            lm = net_loss(o, d, x, params, target)
            arr[idx] = orig
            fd = (lp - lm) / (2 * eps)
            an = g[idx].real if part == "re" else g[idx].imag
            checks.append((grp, sub, idx, part, fd, an))
    assert len(checks) >= 32
    scale = max(abs(c[-1]) for c in checks)
    for c in checks:
        fd, an = c[-2], c[-1]
        # central differences: O(eps^2) truncation error
        assert abs(fd - an) <= 1e-4 * abs(an) + 1e-6 * scale, c


def test_mse_closed_form(oracle):
    y = np.array([1.0, -2.0, 0.5, 3.0])
    t = np.array([0.0, -1.0, 0.5, 1.0])
    L, g = oracle.mse(y, t)
    assert L == pytest.approx((1 + 1 + 0 + 4) / 4, abs=1e-15)
    assert np.allclose(g, [0.5, -0.5, 0.0, 1.0], atol=1e-15)
