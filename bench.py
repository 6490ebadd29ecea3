"""Benchmark: FNO block forward + backward on one MI355X.

A step is one pass of the whole hot path over one batch: fno_block_fwd
(truncated forward DFT over t, z, y, x; per-mode channel mix; inverse DFT;
fused pointwise 1x1 + bias + GELU) followed by fno_block_bwd (recomputation
of the pre-activation, GELU gradient, pointwise gradients, spectral adjoint
and complex weight gradient).

Workload (default): the CO2-flow-shaped block of arXiv 2211.12709 Sec. V-B
at grid 128^3 x 32, batch 1, width 20, modes 16,16,16,8.  The block input and
the upstream gradient are smooth seeded synthetic fields
(paper_2211_12709_amd.inputs.smooth_spacetime_field); weights are seeded.

The BF16 path (bfloat16 activations, FP32 accumulation) is the reported value;
the FP32 path runs the same kernels in float32 for the ratio.  Relative L2
errors of y, gx, gw, gw_pw and gb against the FP64 CPU oracle are measured at
the full size in the same run; that oracle run is also the cpu_baseline.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

WORKLOADS = {
    # name: (B, C, grid, modes)
    "co2_block_128^3x32": (1, 20, (128, 128, 128, 32), (16, 16, 16, 8)),
    "ns_block_64^3x16": (1, 20, (64, 64, 64, 16), (12, 12, 12, 8)),
    "co2_batched_block_128^3x32": (4, 32, (128, 128, 128, 32), (20, 20, 20, 10)),
    "single_layer_16^3x8": (1, 8, (16, 16, 16, 8), (4, 4, 4, 4)),
    # the paper's own grids (Sec. V-A: Navier-Stokes 130^3 x 64; Sec. V-B: CO2 262 x 118 x 64 x 86)
    # at width 20, keeping about 20% of the frequencies per axis (2 m ~ N / 5, 2 mt - 1 ~ Nt / 5)
    "ns_true_130^3x64": (1, 20, (130, 130, 130, 64), (13, 13, 13, 7)),
    "co2_true_262x118x64x86": (1, 20, (262, 118, 64, 86), (26, 12, 6, 9)),
}
# timed beside the headline in a default run (BF16 only, device-generated inputs, no oracle: their
# parity is tested at reduced grids that run the same kernel variants)
EXTRA_WORKLOADS = ("ns_true_130^3x64", "co2_true_262x118x64x86", "co2_batched_block_128^3x32",
                   "co2_block_128^3x32+w_fp8", "co2_batched_block_128^3x32+w_fp8")
# "+w_fp8": the plan takes the spectral weights packed as OCP E4M3 with per-channel-pair scales
# (FNO_W_FP8); the step packs them (fno_pack_weights) before the block fwd+bwd, as a training
# step whose weights change every step must.

HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "f32": 157.3}
METRIC = "FNO block fwd+bwd ms/step & TFLOP/s, BF16 vs FP32 at stated rel err"
REL_L2_TARGET = {"bf16": 1e-2, "f32": 1e-5}  # relative L2 error against the FP64 oracle, every output


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# ------------------------------------------------------------------ work model
def flop_model(B, Ci, Co, grid, modes):
    """Model flops of the block (truncated separable DFT, counted per stage)."""
    nx, ny, nz, nt = grid
    mx, my, mz, mt = modes
    N = nx * ny * nz * nt
    M = (2 * mx) * (2 * my) * (2 * mz) * mt

    def dft(C):
        t = 4 * B * C * N * mt
        z = 8 * B * C * nx * ny * mt * nz * 2 * mz
        y = 8 * B * C * nx * 2 * mz * mt * ny * 2 * my
        x = 8 * B * C * 2 * my * 2 * mz * mt * nx * 2 * mx
        return t + z + y + x, (t, z, y, x)

    dft_in, _ = dft(Ci)
    dft_out, stages = dft(Co)
    mix = 8 * B * Ci * Co * M
    pw = 2 * B * Ci * Co * N
    fwd = dft_in + mix + dft_out + pw
    bwd = dft_out + 2 * mix + dft_in + 2 * pw
    recompute = (stages[2] + stages[3]) + (stages[0] + stages[1]) + pw
    return dict(fwd=fwd, bwd=bwd, recompute=recompute, stages_t_z_y_x=stages, mix=mix, pointwise=pw)


def kernel_model(name, B, Ci, Co, grid, modes, act_bytes):
    """Algorithmic HBM bytes and model flops of ONE launch of a library kernel
    in the block step: what the kernel must read and write across its own
    boundary (activations, spectra, weights), and the flops of the truncated
    separable transform stages it performs."""
    nx, ny, nz, nt = grid
    mx, my, mz, mt = modes
    N = nx * ny * nz * nt
    C = Co  # the benchmark block has Ci == Co
    A = B * C * N * act_bytes                                # one activation tensor
    kx, ky, kz = 2 * mx, 2 * my, 2 * mz
    t1 = B * C * nx * ny * kz * mt * 8                       # t,z spectrum, complex64
    u1 = B * C * nx * ny * kz * mt * 2 * act_bytes           # its y-inverse as the z,t kernels read it
    t2 = B * C * nx * ky * kz * mt * 8                       # t,z,y spectrum
    sp = B * C * kx * ky * kz * mt * 8                       # retained spectrum
    W = Ci * Co * kx * ky * kz * mt * 8
    t_fl = 4 * B * C * N * mt
    z_fl = 8 * B * C * nx * ny * mt * nz * kz
    y_fl = 8 * B * C * nx * kz * mt * ny * ky
    x_fl = 8 * B * C * ky * kz * mt * nx * kx
    pw = 2 * B * Ci * Co * N
    models = {
        "tzy_fwd<bf16>": (B * C * N * 2 + t2, t_fl + z_fl + y_fl),
        "tzy_fwd<f32>": (B * C * N * 4 + t2, t_fl + z_fl + y_fl),
        "tzy_gen<bf16>": (B * C * N * 2 + t2, t_fl + z_fl + y_fl),
        "tzy_gen<f32>": (B * C * N * 4 + t2, t_fl + z_fl + y_fl),
        "zt_plain": (u1 + A, t_fl + z_fl),
        "zt_block": (u1 + 2 * A, t_fl + z_fl + pw),
        "zt_bwd": (u1 + 3 * A, t_fl + z_fl + 2 * pw),
        "zt_adj": (u1 + 2 * A, t_fl + z_fl + pw),
        "axis_fwd_x": (t2 + sp, x_fl),
        "axis_inv_x": (sp + t2, x_fl),
        "axis_inv_y": (t2 + u1, y_fl),
        "axis_fwd_y": (t1 + t2, y_fl),
        "mix_fwd": (2 * sp + W, 8 * B * Ci * Co * kx * ky * kz * mt),
        "mix_bwd": (3 * sp + 2 * W, 16 * B * Ci * Co * kx * ky * kz * mt),
    }
    name = name[:-4] if name.endswith("_tsl") else name  # t-sliced variants do the same work
    if name not in models:
        return None
    by, fl = models[name]
    return dict(bytes=by, flops=fl)


# ------------------------------------------------------------------ measured HBM traffic
HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "paper_2211_12709_amd", "csrc")
# sources whose text decides a kernel's memory traffic (a counter figure is stale once they change)
KERNEL_SOURCES = {
    "zt": ["zt_epi.h", "zt_epi.hip", "zt_epi_block.hip", "zt_epi_bwd.hip", "zt_epi_adj.hip", "zt_epi_plain.hip",
           "tables.hip", "mfma_common.h", "fno_internal.h"],
    "tzy": ["fwd_tzy.hip", "fwd_tzy_gen.hip", "tables.hip", "mfma_common.h", "fno_internal.h"],
}


def _code_only(text):
    """Source text without comments and with whitespace collapsed: what the compiler sees."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def source_hash(label):
    """Hash of the code (comments and layout excluded) of the sources kernel `label` is built from."""
    key = "zt" if label.startswith("zt_") else "tzy" if label.startswith("tzy") else None
    if key is None:
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[key]:
        with open(os.path.join(CSRC, f), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def profiled_traffic(label, dtype, workload):
    """HBM bytes per launch of kernel `label` from the committed rocprofv3 counter summaries
    (FETCH_SIZE and WRITE_SIZE scaled by a plain-copy calibration), or None when there is no
    figure for this kernel, dtype and workload or its sources changed since it was taken."""
    want = source_hash(label)
    if want is None:
        return None
    for path in sorted(glob.glob(os.path.join(HERE, "profiles", "*hbm_counters*.txt"))):
        with open(path) as fh:
            for line in fh:
                f = line.split()
                if len(f) == 6 and f[0] == "traffic" and f[1] == label and f[2] == dtype and f[3] == workload:
                    kv = dict(x.split("=", 1) for x in f[4:])
                    if kv.get("src") == want:
                        return int(kv["bytes"])
    return None


# ------------------------------------------------------------------ helpers
def median_ci(xs, level=0.95):
    """Median of the per-step times and a distribution-free confidence interval for it: the
    order statistics (x_(j), x_(n+1-j)) with the largest j whose binomial coverage is >= level."""
    from math import comb
    v = sorted(xs)
    n = len(v)
    med = float(np.median(v))
    lo, hi = v[0], v[-1]
    for j in range(1, n // 2 + 1):
        cover = sum(comb(n, i) for i in range(j, n - j + 1)) / 2.0 ** n
        if cover >= level:
            lo, hi = v[j - 1], v[n - j]
        else:
            break
    return med, float(lo), float(hi)


def rel(a, ref):
    return float(np.linalg.norm((a - ref).ravel()) / max(np.linalg.norm(ref.ravel()), 1e-300))


def roofline_of(kern, wl, workload):
    """Roofline object of the dominant (longest) kernel of a BF16 step from its per-kernel timings
    {name: (launches, total_ms)}: algorithmic bytes (or flops) of one launch over its average time."""
    B, C, grid, modes = wl
    name, (launches, tot_ms) = max(kern.items(), key=lambda kv: kv[1][1])
    avg_ms = tot_ms / launches
    km = kernel_model(name, B, C, C, grid, modes, 2)
    if km is None:
        return None
    t_hbm = km["bytes"] / (HBM_PEAK_GBS * 1e9)
    t_mfma = km["flops"] / (MFMA_PEAK_TFLOPS["bf16"] * 1e12)
    if t_hbm >= t_mfma:
        ach = km["bytes"] / (avg_ms * 1e-3) / 1e9
        return dict(bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS,
                    traffic=profiled_traffic(name, "bf16", workload), kernel=name, avg_ms=avg_ms,
                    bytes_per_launch=km["bytes"])
    ach = km["flops"] / (avg_ms * 1e-3) / 1e12
    return dict(bound="mfma", achieved=ach, peak=MFMA_PEAK_TFLOPS["bf16"], unit="TFLOP/s",
                frac=ach / MFMA_PEAK_TFLOPS["bf16"], traffic=None, kernel=name, avg_ms=avg_ms)


def time_steps(step, steps, warmup, kernel_steps, plan):
    """Times `steps` back-to-back calls of step() with one event between consecutive steps, then
    a separate pass of kernel_steps steps with every kernel launch bracketed by events."""
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record(stream)
    for k in range(steps):
        step()
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_step = [evs[k].elapsed_time(evs[k + 1]) for k in range(steps)]
    ms = evs[0].elapsed_time(evs[-1]) / steps
    plan.timing(True)
    plan.timing_read()
    for _ in range(kernel_steps):
        step()
    torch.cuda.synchronize()
    plan.timing(False)
    kern = plan.timing_read()
    med, lo, hi = median_ci(per_step)
    return dict(ms=ms, wall_ms=wall * 1000 / steps, kernels=kern, median_ms=med, ci95_ms=[lo, hi],
                kernel_steps=kernel_steps)


def run_extra(name, steps, warmup):
    """BF16 block fwd+bwd timing of another workload: inputs and weights drawn on the device (seeded
    normal values; the kernels' work does not depend on them), no oracle."""
    import torch

    from paper_2211_12709_amd import fno, inputs

    base, _, variant = name.partition("+")
    fp8 = variant == "w_fp8"
    B, C, grid, modes = WORKLOADS[base]
    dev = torch.device("cuda", 0)
    ksh = (2 * modes[0], 2 * modes[1], 2 * modes[2], modes[3])
    log(f"[bench] {name}: B={B} C={C} grid={grid} modes={modes}")
    g = torch.Generator(device=dev)
    g.manual_seed(inputs.SEED_INPUT)
    plan = fno.Plan(B, C, C, grid, modes, fno.FNO_BF16, fno.FNO_W_FP8 if fp8 else 0)
    packed = torch.empty(plan.packed_weight_bytes(), dtype=torch.uint8, device=dev) if fp8 else None
    xa = torch.randn((B, C, *grid), generator=g, device=dev, dtype=torch.bfloat16)
    gya = torch.randn((B, C, *grid), generator=g, device=dev, dtype=torch.bfloat16)
    tw = torch.randn((C, C, *ksh), generator=g, device=dev, dtype=torch.complex64) / C
    twp = torch.randn((C, C), generator=g, device=dev) / C ** 0.5
    tb = torch.zeros((C,), device=dev)
    cache = plan.new_cache()
    y, gx = torch.empty_like(xa), torch.empty_like(xa)
    gw = torch.empty_like(tw)
    gwpw = torch.empty_like(twp)
    gb = torch.empty_like(tb)

    def step():
        wv = plan.pack_weights(tw, packed) if fp8 else tw
        plan.block_fwd(xa, wv, twp, tb, y=y, cache=cache)
        plan.block_bwd(xa, cache, wv, twp, tb, gya, gx=gx, gw=gw, gw_pw=gwpw, gb_pw=gb)

    r = time_steps(step, steps, warmup, 1, plan)
    fm = flop_model(B, C, C, grid, modes)
    wl = WORKLOADS[base]
    out = dict(config={"batch": B, "width": C, "grid": list(grid), "modes": list(modes)}, dtype="bf16",
               ms_per_step=r["ms"], median_ms_per_step=r["median_ms"], ci95_ms_per_step=r["ci95_ms"],
               tflops=(fm["fwd"] + fm["bwd"]) / (r["ms"] * 1e-3) / 1e12,
               kernels_ms_per_step={k: v[1] for k, v in r["kernels"].items()},
               roofline=roofline_of(r["kernels"], wl, base), data="synthetic (device normal draws)")
    log(f"[bench] {name}: {r['ms']:.3f} ms/step")
    del plan, xa, gya, cache, y, gx, tw, gw
    torch.cuda.empty_cache()
    return out


def run_network_leg(steps, warmup):
    """BF16 training step of the CO2-shaped 4-block FNO (Alg. 1) at 128^3 x 32: the 3-channel
    CO2-like input (ln k, porosity, injection-well column; paper_2211_12709_amd.inputs), lifting
    to width 20, four blocks with modes 16,16,16,8 (per-block recomputation in the backward),
    projection 20 -> 128 -> 1, MSE against a seeded target; seeded weights.  No oracle (the
    network's parity is tested at full size on the Navier-Stokes-shaped grid)."""
    import torch

    from paper_2211_12709_amd import fno, inputs

    B, C, grid, modes = WORKLOADS["co2_block_128^3x32"]
    dev = torch.device("cuda", 0)
    ksh = (2 * modes[0], 2 * modes[1], 2 * modes[2], modes[3])
    log(f"[bench] co2_network_128^3x32: 4 blocks, width {C}, grid {grid}, modes {modes}")
    we, be = inputs.linear_weights(C, 3, seed=inputs.SEED_LIFT)
    blocks = [inputs.block_params(C, C, ksh, block=i) for i in range(4)]
    w1, b1 = inputs.linear_weights(128, C, seed=inputs.SEED_PROJ1)
    w2, b2 = inputs.linear_weights(1, 128, seed=inputs.SEED_PROJ2)
    params = {"lift": (we, be), "blocks": blocks, "proj": (w1, b1, w2, b2)}
    net = fno.FNO4d(3, C, grid, modes, nblocks=4, dtype=torch.bfloat16, params=params)
    x = torch.from_numpy(inputs.co2_like_input(1, grid)).to(dev).to(torch.bfloat16)
    g = torch.Generator(device=dev)
    g.manual_seed(inputs.SEED_TARGET)
    target = torch.randn((1, 1, *grid), generator=g, device=dev).to(torch.bfloat16)

    def step():
        for p_ in net.parameters():
            p_.grad = None
        loss = fno.MseFn.apply(net(x), target)
        loss.backward()

    r = time_steps(step, steps, warmup, 1, net.plan)
    fm = flop_model(B, C, C, grid, modes)
    out = dict(config={"batch": B, "width": C, "grid": list(grid), "modes": list(modes), "blocks": 4,
                       "lift": [3, C], "projection": [C, 128, 1]}, dtype="bf16",
               ms_per_step=r["ms"], median_ms_per_step=r["median_ms"], ci95_ms_per_step=r["ci95_ms"],
               block_tflops=4 * (fm["fwd"] + fm["bwd"]) / (r["ms"] * 1e-3) / 1e12,
               kernels_ms_per_step={k: v[1] for k, v in r["kernels"].items()},
               data="synthetic (CO2-like input fields, device normal target)")
    log(f"[bench] co2_network_128^3x32: {r['ms']:.3f} ms/step")
    del net, x, target
    torch.cuda.empty_cache()
    return out


def run_gpu(args, wl):
    import torch

    from paper_2211_12709_amd import fno, inputs

    B, C, grid, modes = wl
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    ksh = (2 * modes[0], 2 * modes[1], 2 * modes[2], modes[3])
    log(f"[bench] generating inputs B={B} C={C} grid={grid} modes={modes}")
    x = inputs.smooth_spacetime_field(B, C, grid, seed=inputs.SEED_INPUT)
    gy = inputs.smooth_spacetime_field(B, C, grid, seed=inputs.SEED_TARGET)
    w, wpw, bpw = inputs.block_params(C, C, ksh, block=0)
    tw, twp, tb = (torch.from_numpy(a).to(dev) for a in (w, wpw, bpw))
    x32 = torch.from_numpy(x).to(dev)
    gy32 = torch.from_numpy(gy).to(dev)
    results = {}
    outputs = {}
    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)   # 1 GiB
        a.fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("[bench] copy calibration: 1 GiB read + 1 GiB written by one copy kernel")
        del a, b
        torch.cuda.empty_cache()
    for dt_name, code in (("bf16", fno.FNO_BF16), ("f32", fno.FNO_F32)):
        if dt_name == "f32" and args.no_fp32:
            continue
        plan = fno.Plan(B, C, C, grid, modes, code)
        xa = x32.to(plan.act_dtype).contiguous()
        gya = gy32.to(plan.act_dtype).contiguous()
        cache = plan.new_cache()
        y = torch.empty_like(xa)
        gx = torch.empty_like(xa)
        gw = torch.empty((C, C, *ksh), dtype=torch.complex64, device=dev)
        gwpw = torch.empty((C, C), dtype=torch.float32, device=dev)
        gb = torch.empty((C,), dtype=torch.float32, device=dev)

        def step():
            plan.block_fwd(xa, tw, twp, tb, y=y, cache=cache)
            plan.block_bwd(xa, cache, tw, twp, tb, gya, gx=gx, gw=gw, gw_pw=gwpw, gb_pw=gb)

        log(f"[bench] {dt_name}: warmup {args.warmup}, timing {args.steps} steps")
        results[dt_name] = time_steps(step, args.steps, args.warmup, args.kernel_steps, plan)
        ms = results[dt_name]["ms"]
        log(f"[bench] {dt_name}: {ms:.3f} ms/step")
        if not args.no_oracle:
            # activations stay in their own dtype on the host (compared a channel at a time)
            outputs[dt_name] = dict(y=y.cpu(), gx=gx.cpu(), gw=gw.cpu().numpy(), gw_pw=gwpw.cpu().numpy(),
                                    gb=gb.cpu().numpy())
        del plan, xa, gya, cache, y, gx
        torch.cuda.empty_cache()
    return results, outputs, (x, gy, w, wpw, bpw)


class ErrAcc:
    """Relative L2 error accumulated over slices: sqrt(sum |a - ref|^2 / sum |ref|^2)."""

    def __init__(self):
        self.num = self.den = 0.0

    def add(self, a, ref):
        a = np.asarray(a, dtype=np.complex128 if np.iscomplexobj(ref) else np.float64)
        self.num += float(np.sum(np.abs(a - ref) ** 2))
        self.den += float(np.sum(np.abs(ref) ** 2))

    def value(self):
        return float(np.sqrt(self.num / max(self.den, 1e-300)))


def compare_acts(acc, dev_cpu, ref, b0=0):
    """Adds to `acc` the error of a host copy of a device activation [B][C][...] (any dtype) against
    an FP64 oracle array covering batch elements b0.. of it, one (b, c) slice at a time."""
    for b in range(ref.shape[0]):
        for c in range(ref.shape[1]):
            acc.add(dev_cpu[b0 + b, c].float().numpy(), ref[b, c])


def run_oracle(wl, data, outputs):
    """FP64 oracle block fwd + bwd on the benchmark inputs and the relative L2 errors of every
    output of `outputs` ({dtype: {name: host array}}).  Batch elements are run one at a time
    (memory stays at one element's FP64 activations): output and input-gradient errors are
    accumulated over them, and the weight gradients, sums over the batch, are summed first."""
    from oracle import oracle as o
    B, C, grid, modes = wl
    x, gy, w, wpw, bpw = data
    d1 = o.Dims(1, C, C, grid, modes)
    log("[bench] oracle (FP64 CPU) block fwd+bwd" + (f", streamed over {B} batch elements" if B > 1 else ""))
    acc = {dt: dict(y=ErrAcc(), gx=ErrAcc()) for dt in outputs}
    sums = None
    sec = 0.0
    for b in range(B):
        t0 = time.perf_counter()
        y = o.block_fwd(d1, x[b:b + 1], w, wpw, bpw)
        sec += time.perf_counter() - t0
        for dt, out in outputs.items():
            compare_acts(acc[dt]["y"], out["y"], y, b0=b)
        del y
        t0 = time.perf_counter()
        gx, gw, gwpw, gb = o.block_bwd(d1, x[b:b + 1], w, wpw, bpw, gy[b:b + 1])
        sec += time.perf_counter() - t0
        for dt, out in outputs.items():
            compare_acts(acc[dt]["gx"], out["gx"], gx, b0=b)
        del gx
        sums = [gw, gwpw, gb] if sums is None else [sums[0] + gw, sums[1] + gwpw, sums[2] + gb]
        log(f"[bench] oracle: batch element {b} done ({sec:.1f} s)")
    errs = {}
    for dt, out in outputs.items():
        e = {k: acc[dt][k].value() for k in ("y", "gx")}
        for k, ref in zip(("gw", "gw_pw", "gb"), sums):
            ea = ErrAcc()
            ea.add(out[k], ref)
            e[k] = ea.value()
        errs[dt] = e
    log(f"[bench] oracle: {sec:.1f} s")
    return errs, sec


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--kernel-steps", type=int, default=4,
                    help="steps of the separate pass whose kernels are timed one by one")
    ap.add_argument("--workload", default="co2_block_128^3x32", choices=sorted(WORKLOADS))
    ap.add_argument("--no-oracle", action="store_true", help="skip the FP64 oracle (errors and cpu_baseline)")
    ap.add_argument("--no-fp32", action="store_true", help="time the BF16 path only")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the BF16 timings of the paper's own grids and the batched block")
    ap.add_argument("--extra-steps", type=int, default=5, help="timed steps of each extra workload")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one plain 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--network-only", action="store_true",
                    help="time only the four-block network step (for profiling it) and print its JSON object")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs as a single process on one GPU.", file=sys.stderr)
        sys.exit(2)

    if args.network_only:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps(run_network_leg(args.extra_steps, 2)), flush=True)
        return

    wl = WORKLOADS[args.workload]
    B, C, grid, modes = wl
    fm = flop_model(B, C, C, grid, modes)
    model_flops = fm["fwd"] + fm["bwd"]
    results, outputs, data = run_gpu(args, wl)

    errs, cpu = {}, None
    if not args.no_oracle:
        errs, sec = run_oracle(wl, data, outputs)
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
        cpu = dict(value=model_flops / sec / 1e12, unit="TFLOP/s", cores=threads, kind="oracle",
                   sample=f"one full block fwd+bwd of the benchmark workload ({args.workload}), FP64, "
                          f"{sec:.1f} s wall")

    bf = results["bf16"]
    ms = bf["ms"]
    value = model_flops / (ms * 1e-3) / 1e12
    roof = roofline_of(bf["kernels"], wl, args.workload)
    others = {}
    if args.workload == "co2_block_128^3x32" and not args.no_extra:
        for name in EXTRA_WORKLOADS:
            others[name] = run_extra(name, args.extra_steps, 2)
        others["co2_network_128^3x32"] = run_network_leg(args.extra_steps, 2)
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": args.workload, "batch": B, "width": C, "grid": list(grid), "modes": list(modes)},
        "fp32_ms_per_step": results.get("f32", {}).get("ms"),
        "bf16_speedup_vs_fp32": (results["f32"]["ms"] / ms) if "f32" in results else None,
        "model_gflop_per_step": model_flops / 1e9,
        "rel_l2_vs_fp64_oracle": errs or None,
        "rel_l2_targets": REL_L2_TARGET,
        "rel_l2_within_targets": (all(v <= REL_L2_TARGET[dt] for dt, e in errs.items() for v in e.values())
                                  if errs else None),
        "median_ms_per_step": {dt: r["median_ms"] for dt, r in results.items()},
        "ci95_ms_per_step": {dt: r["ci95_ms"] for dt, r in results.items()},
        "kernels_ms_per_step": {dt: {k: v[1] / r["kernel_steps"] for k, v in r["kernels"].items()}
                                for dt, r in results.items()},
        "roofline": roof,
        "cpu_baseline": cpu,
        "other_workloads": others or None,
    }
    print(json.dumps(line), flush=True)
    if errs and not line["rel_l2_within_targets"]:
        log(f"[bench] relative L2 error above target: {errs}")
        sys.exit(3)


if __name__ == "__main__":
    main()
