"""ctypes front end of the FP64 CPU oracle (oracle/fno_oracle.c).

TEST INFRASTRUCTURE ONLY.  The product path (paper_2211_12709_amd) never
imports this module.  Arrays are numpy float64, C-contiguous; complex tensors
are numpy complex128 (same memory as interleaved re/im doubles).

Shapes follow Sec. IV-C of arXiv 2211.12709:
  x   [B, C_in, Nx, Ny, Nz, Nt]              real
  xh  [B, C_in, 2mx, 2my, 2mz, mt]           complex (retained modes only)
  w   [C_in, C_out, 2mx, 2my, 2mz, mt]       complex
  wpw [C_out, C_in], bpw [C_out]             real
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fno_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libfno_oracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_lp = ctypes.POINTER(ctypes.c_long)


def build_oracle(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def load(path: str):
    """Load an oracle shared object and declare its C signatures."""
    L = ctypes.CDLL(path)
    L.oracle_check_dims.argtypes = [_ip]
    L.oracle_check_dims.restype = ctypes.c_int
    L.oracle_ct.argtypes = [ctypes.c_long, ctypes.c_long]
    L.oracle_ct.restype = ctypes.c_double
    L.oracle_gelu.argtypes = [ctypes.c_double]
    L.oracle_gelu.restype = ctypes.c_double
    L.oracle_gelu_grad.argtypes = [ctypes.c_double]
    L.oracle_gelu_grad.restype = ctypes.c_double
    L.oracle_dft_fwd.argtypes = [_ip, ctypes.c_int, _dp, _dp, _dp]
    L.oracle_synth.argtypes = [_ip, ctypes.c_int, _dp, _dp, _dp]
    L.oracle_dft_fwd_direct.argtypes = [_ip, ctypes.c_int, _dp, _dp]
    L.oracle_dft_fwd_modes.argtypes = [_ip, ctypes.c_int, _dp, ctypes.c_long, _ip, _dp]
    L.oracle_synth_points.argtypes = [_ip, ctypes.c_int, _dp, _dp, ctypes.c_long, _lp, _dp]
    L.oracle_mix.argtypes = [_ip, _dp, _dp, _dp]
    L.oracle_mix_bwd.argtypes = [_ip, _dp, _dp, _dp, _dp, _dp]
    L.oracle_spectral_fwd.argtypes = [_ip, _dp, _dp, _dp, _dp, _dp]
    L.oracle_spectral_bwd.argtypes = [_ip, _dp, _dp, _dp, _dp, _dp]
    L.oracle_block_fwd.argtypes = [_ip, _dp, _dp, _dp, _dp, _dp]
    L.oracle_block_bwd.argtypes = [_ip, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    L.oracle_lift_fwd.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_long, _dp, _dp, _dp, _dp]
    L.oracle_lift_bwd.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_long, _dp, _dp, _dp, _dp, _dp,
                                  _dp, _dp]
    L.oracle_proj_fwd.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_long, _dp, _dp,
                                  _dp, _dp, _dp, _dp]
    L.oracle_proj_bwd.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_long, _dp, _dp,
                                  _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    L.oracle_mse.argtypes = [ctypes.c_long, _dp, _dp, _dp]
    L.oracle_mse.restype = ctypes.c_double
    for f in ("oracle_lift_fwd", "oracle_lift_bwd", "oracle_proj_fwd", "oracle_proj_bwd"):
        getattr(L, f).restype = None
    for f in ("oracle_dft_fwd", "oracle_synth", "oracle_dft_fwd_direct", "oracle_dft_fwd_modes",
              "oracle_synth_points", "oracle_mix", "oracle_mix_bwd", "oracle_spectral_fwd",
              "oracle_spectral_bwd", "oracle_block_fwd", "oracle_block_bwd"):
        getattr(L, f).restype = None
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_oracle(force=True)
        _lib = load(_LIB_PATH)
    return _lib


@dataclass(frozen=True)
class Dims:
    """Problem description: batch, channels, grid (x, y, z, t), modes (x, y, z, t)."""
    B: int
    Ci: int
    Co: int
    grid: tuple
    modes: tuple

    @property
    def kshape(self):
        mx, my, mz, mt = self.modes
        return (2 * mx, 2 * my, 2 * mz, mt)

    @property
    def ncell(self):
        return int(np.prod(self.grid))

    @property
    def nmode(self):
        return int(np.prod(self.kshape))

    def vec(self):
        v = [self.B, self.Ci, self.Co, *self.grid, *self.modes]
        return (ctypes.c_int * 11)(*v)


def _p(a):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be C-contiguous"
    if a.dtype == np.complex128:
        return a.ctypes.data_as(_dp)
    assert a.dtype == np.float64, a.dtype
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def check_dims(d: Dims) -> bool:
    return lib().oracle_check_dims(d.vec()) == 0


def ct(kt: int, nt: int) -> float:
    return lib().oracle_ct(kt, nt)


def gelu(u: float) -> float:
    return lib().oracle_gelu(float(u))


def gelu_grad(u: float) -> float:
    return lib().oracle_gelu_grad(float(u))


def inverse_weights(d: Dims) -> np.ndarray:
    """c(kt)/N for the real inverse transform."""
    return np.array([ct(k, d.grid[3]) / d.ncell for k in range(d.modes[3])], dtype=np.float64)


def dft_fwd(d: Dims, x, wt=None, direct=False):
    """Truncated forward DFT of a real field x [B, C, grid] -> [B, C, kshape] complex."""
    x = _f64(x)
    C = x.shape[1]
    out = np.zeros((d.B, C, *d.kshape), dtype=np.complex128)
    if direct:
        assert wt is None
        lib().oracle_dft_fwd_direct(d.vec(), C, _p(x), _p(out))
    else:
        lib().oracle_dft_fwd(d.vec(), C, _p(x), _p(_f64(wt) if wt is not None else None), _p(out))
    return out


def synth(d: Dims, F, wt=None):
    """sum_k wt[kt] Re(F[k] e^{+i theta(k,n)}) -> real [B, C, grid]."""
    F = _c128(F)
    C = F.shape[1]
    out = np.zeros((d.B, C, *d.grid), dtype=np.float64)
    lib().oracle_synth(d.vec(), C, _p(F), _p(_f64(wt) if wt is not None else None), _p(out))
    return out


def synth_points(d: Dims, F, pts, wt=None):
    """synth() evaluated directly (4-D sum) at flat grid points pts -> [B, C, len(pts)]."""
    F = _c128(F)
    C = F.shape[1]
    pts = np.ascontiguousarray(pts, dtype=np.int64)
    out = np.zeros((d.B, C, len(pts)), dtype=np.float64)
    lib().oracle_synth_points(d.vec(), C, _p(F), _p(_f64(wt) if wt is not None else None),
                              len(pts), pts.ctypes.data_as(_lp), _p(out))
    return out


def dft_modes(d: Dims, x, kidx):
    """Forward DFT at the listed compact mode indices kidx [n, 4] -> [B, C, n] complex."""
    x = _f64(x)
    C = x.shape[1]
    kidx = np.ascontiguousarray(kidx, dtype=np.int32)
    out = np.zeros((d.B, C, kidx.shape[0]), dtype=np.complex128)
    lib().oracle_dft_fwd_modes(d.vec(), C, _p(x), kidx.shape[0], kidx.ctypes.data_as(_ip), _p(out))
    return out


def mix(d: Dims, xh, w):
    out = np.zeros((d.B, d.Co, *d.kshape), dtype=np.complex128)
    lib().oracle_mix(d.vec(), _p(_c128(xh)), _p(_c128(w)), _p(out))
    return out


def mix_bwd(d: Dims, xh, w, gyh):
    gxh = np.zeros((d.B, d.Ci, *d.kshape), dtype=np.complex128)
    gw = np.zeros((d.Ci, d.Co, *d.kshape), dtype=np.complex128)
    lib().oracle_mix_bwd(d.vec(), _p(_c128(xh)), _p(_c128(w)), _p(_c128(gyh)), _p(gxh), _p(gw))
    return gxh, gw


def spectral_fwd(d: Dims, x, w, return_spectra=False):
    y = np.zeros((d.B, d.Co, *d.grid), dtype=np.float64)
    xh = np.zeros((d.B, d.Ci, *d.kshape), dtype=np.complex128)
    yh = np.zeros((d.B, d.Co, *d.kshape), dtype=np.complex128)
    lib().oracle_spectral_fwd(d.vec(), _p(_f64(x)), _p(_c128(w)), _p(y), _p(xh), _p(yh))
    return (y, xh, yh) if return_spectra else y


def spectral_bwd(d: Dims, x, w, gy):
    gx = np.zeros((d.B, d.Ci, *d.grid), dtype=np.float64)
    gw = np.zeros((d.Ci, d.Co, *d.kshape), dtype=np.complex128)
    lib().oracle_spectral_bwd(d.vec(), _p(_f64(x)), _p(_c128(w)), _p(_f64(gy)), _p(gx), _p(gw))
    return gx, gw


def block_fwd(d: Dims, x, w, wpw, bpw):
    y = np.zeros((d.B, d.Co, *d.grid), dtype=np.float64)
    lib().oracle_block_fwd(d.vec(), _p(_f64(x)), _p(_c128(w)), _p(_f64(wpw)),
                           _p(_f64(bpw) if bpw is not None else None), _p(y))
    return y


def block_bwd(d: Dims, x, w, wpw, bpw, gy):
    gx = np.zeros((d.B, d.Ci, *d.grid), dtype=np.float64)
    gw = np.zeros((d.Ci, d.Co, *d.kshape), dtype=np.complex128)
    gwpw = np.zeros((d.Co, d.Ci), dtype=np.float64)
    gb = np.zeros((d.Co,), dtype=np.float64)
    lib().oracle_block_bwd(d.vec(), _p(_f64(x)), _p(_c128(w)), _p(_f64(wpw)),
                           _p(_f64(bpw) if bpw is not None else None), _p(_f64(gy)),
                           _p(gx), _p(gw), _p(gwpw), _p(gb))
    return gx, gw, gwpw, gb


# ------------------------------------------------------------------ network glue (Alg. 1)
def lift_fwd(x, we, be):
    """Encoder: GELU(we x + be) pointwise; x [B, Ci, *grid] -> [B, Co, *grid]."""
    x = _f64(x)
    B, Ci = x.shape[:2]
    Co = we.shape[0]
    N = int(np.prod(x.shape[2:]))
    y = np.zeros((B, Co, *x.shape[2:]))
    lib().oracle_lift_fwd(B, Ci, Co, N, _p(x), _p(_f64(we)), _p(_f64(be) if be is not None else None), _p(y))
    return y


def lift_bwd(x, we, be, gy, need_gx=False):
    x = _f64(x)
    B, Ci = x.shape[:2]
    Co = we.shape[0]
    N = int(np.prod(x.shape[2:]))
    gx = np.zeros_like(x) if need_gx else None
    gwe = np.zeros((Co, Ci))
    gbe = np.zeros(Co)
    lib().oracle_lift_bwd(B, Ci, Co, N, _p(x), _p(_f64(we)), _p(_f64(be) if be is not None else None),
                          _p(_f64(gy)), _p(gx), _p(gwe), _p(gbe))
    return gx, gwe, gbe


def proj_fwd(x, w1, b1, w2, b2):
    """Decoder: w2 GELU(w1 x + b1) + b2 pointwise."""
    x = _f64(x)
    B, Ci = x.shape[:2]
    H, Co = w1.shape[0], w2.shape[0]
    N = int(np.prod(x.shape[2:]))
    y = np.zeros((B, Co, *x.shape[2:]))
    lib().oracle_proj_fwd(B, Ci, H, Co, N, _p(x), _p(_f64(w1)), _p(_f64(b1)), _p(_f64(w2)), _p(_f64(b2)), _p(y))
    return y


def proj_bwd(x, w1, b1, w2, b2, gy):
    x = _f64(x)
    B, Ci = x.shape[:2]
    H, Co = w1.shape[0], w2.shape[0]
    N = int(np.prod(x.shape[2:]))
    gx = np.zeros_like(x)
    gw1, gb1 = np.zeros((H, Ci)), np.zeros(H)
    gw2, gb2 = np.zeros((Co, H)), np.zeros(Co)
    lib().oracle_proj_bwd(B, Ci, H, Co, N, _p(x), _p(_f64(w1)), _p(_f64(b1)), _p(_f64(w2)), _p(_f64(b2)),
                          _p(_f64(gy)), _p(gx), _p(gw1), _p(gb1), _p(gw2), _p(gb2))
    return gx, gw1, gb1, gw2, gb2


def mse(y, t):
    """(loss, gradient) of the mean-squared error."""
    y = _f64(y)
    g = np.zeros_like(y)
    L = lib().oracle_mse(y.size, _p(y), _p(_f64(t)), _p(g))
    return L, g


def fno_fwd(d: Dims, x, params):
    """Alg. 1 on one device: lift -> blocks -> projection.  params holds
    'lift': (we, be), 'blocks': [(w, wpw, bpw), ...], 'proj': (w1, b1, w2, b2).
    Returns the output and the list of block inputs (for the backward)."""
    h = lift_fwd(x, *params["lift"])
    acts = [h]
    for (w, wpw, bpw) in params["blocks"]:
        h = block_fwd(d, h, w, wpw, bpw)
        acts.append(h)
    y = proj_fwd(h, *params["proj"])
    return y, acts


def fno_bwd(d: Dims, x, params, acts, gy):
    """Gradients of every parameter for the upstream gradient gy (same structure as params)."""
    g, gw1, gb1, gw2, gb2 = proj_bwd(acts[-1], *params["proj"], gy)
    grads_blocks = []
    for bi in range(len(params["blocks"]) - 1, -1, -1):
        w, wpw, bpw = params["blocks"][bi]
        g, gw, gwpw, gb = block_bwd(d, acts[bi], w, wpw, bpw, g)
        grads_blocks.append((gw, gwpw, gb))
    grads_blocks.reverse()
    _, gwe, gbe = lift_bwd(x, *params["lift"], g)
    return {"lift": (gwe, gbe), "blocks": grads_blocks, "proj": (gw1, gb1, gw2, gb2)}


__all__ = ["lift_fwd", "lift_bwd", "proj_fwd", "proj_bwd", "mse", "fno_fwd", "fno_bwd",
           "Dims", "build_oracle", "check_dims", "ct", "gelu", "gelu_grad", "inverse_weights",
           "dft_fwd", "synth", "synth_points", "dft_modes", "mix", "mix_bwd", "spectral_fwd",
           "spectral_bwd", "block_fwd", "block_bwd"]
