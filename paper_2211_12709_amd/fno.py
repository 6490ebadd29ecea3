"""Python binding of libfno_mi355x.so (C-ABI in include/fno_mi355x.h).

Argument marshalling only: every arithmetic step of the spectral block runs
in the HIP library.  PyTorch provides device memory and the current stream.
Importing this module loads the library and raises if it is not built.

Names follow the C entry points:
    Plan(...).spectral_fwd / spectral_bwd / block_fwd / block_bwd
and torch.autograd.Function wrappers SpectralConv4dFn and FNOBlockFn
(the FNO block of arXiv 2211.12709, Alg. 1 and Alg. 2).
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfno_mi355x.so")

FNO_OK, FNO_ERR_INVALID_ARG, FNO_ERR_UNSUPPORTED, FNO_ERR_ALIGNMENT, FNO_ERR_WORKSPACE, FNO_ERR_HIP, FNO_ERR_OOM = range(7)
FNO_F32, FNO_BF16 = 0, 1
FNO_W_FP8 = 1
OP_SPECTRAL_FWD, OP_SPECTRAL_BWD, OP_BLOCK_FWD, OP_BLOCK_BWD = range(4)

EXPORTS = ("fno_desc_validate", "fno_plan_create", "fno_plan_destroy", "fno_workspace_bytes", "fno_cache_bytes",
           "fno_spectral_fwd", "fno_spectral_fwd_noalloc", "fno_spectral_bwd", "fno_block_fwd", "fno_block_bwd",
           "fno_lift_fwd", "fno_lift_bwd", "fno_proj_fwd", "fno_proj_bwd", "fno_mse", "fno_glue_workspace_bytes",
           "fno_timing_enable", "fno_timing_read", "fno_packed_weight_bytes", "fno_pack_weights", "fno_status_str")
NOALLOC_SCRATCH_BYTES = 32 << 20  # FNO_NOALLOC_SCRATCH_BYTES


class Desc(ctypes.Structure):
    _fields_ = [("B", ctypes.c_int32), ("C_in", ctypes.c_int32), ("C_out", ctypes.c_int32),
                ("grid", ctypes.c_int32 * 4), ("modes", ctypes.c_int32 * 4),
                ("dtype", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class FnoError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {status_str(code)} ({code})")
        self.code = code


_lib = None
_vp = ctypes.c_void_p
_sz = ctypes.c_size_t


def load_library(path: str = LIB_PATH):
    """Load the HIP library (no GPU needed to load it)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run __graft_entry__.build() (hipcc, gfx950) first")
    L = ctypes.CDLL(path)
    L.fno_desc_validate.argtypes = [ctypes.POINTER(Desc)]
    L.fno_plan_create.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(Desc)]
    L.fno_plan_destroy.argtypes = [_vp]
    L.fno_workspace_bytes.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(_sz)]
    L.fno_cache_bytes.argtypes = [_vp, ctypes.POINTER(_sz)]
    L.fno_spectral_fwd.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]
    L.fno_spectral_fwd_noalloc.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
    L.fno_spectral_bwd.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_int, _vp, _sz, _vp]
    L.fno_block_fwd.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]
    L.fno_block_bwd.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_int, _vp, _sz, _vp]
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    L.fno_lift_fwd.argtypes = [i32, i32, i32, i32, i64, _vp, _vp, _vp, _vp, _vp]
    L.fno_lift_bwd.argtypes = [i32, i32, i32, i32, i64, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_int, _vp, _sz, _vp]
    L.fno_proj_fwd.argtypes = [i32, i32, i32, i32, i32, i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    L.fno_proj_bwd.argtypes = [i32, i32, i32, i32, i32, i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                               ctypes.c_int, _vp, _sz, _vp]
    L.fno_mse.argtypes = [i32, i64, _vp, _vp, _vp, _vp, _vp, _sz, _vp]
    L.fno_glue_workspace_bytes.argtypes = [i32, i32, i32, ctypes.POINTER(_sz)]
    L.fno_timing_enable.argtypes = [_vp, ctypes.c_int]
    L.fno_timing_read.argtypes = [_vp, ctypes.c_char_p, _sz]
    L.fno_packed_weight_bytes.argtypes = [_vp, ctypes.POINTER(_sz)]
    L.fno_pack_weights.argtypes = [_vp, _vp, _vp, _sz, _vp]
    L.fno_status_str.argtypes = [ctypes.c_int]
    L.fno_status_str.restype = ctypes.c_char_p
    for f in EXPORTS[:-1]:
        getattr(L, f).restype = ctypes.c_int
    _lib = L
    return L


def status_str(code: int) -> str:
    return load_library().fno_status_str(int(code)).decode()


def _check(code, what):
    if code != FNO_OK:
        raise FnoError(code, what)


def make_desc(B, C_in, C_out, grid, modes, dtype=FNO_F32, flags=0) -> Desc:
    d = Desc()
    d.B, d.C_in, d.C_out = B, C_in, C_out
    d.grid[:] = list(grid)
    d.modes[:] = list(modes)
    d.dtype = dtype
    d.flags = flags
    return d


def validate(desc: Desc) -> int:
    return load_library().fno_desc_validate(ctypes.byref(desc))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


_TORCH_DTYPE = {FNO_F32: torch.float32, FNO_BF16: torch.bfloat16}


class Plan:
    """A plan for one block shape: basis tables on the current device."""

    def __init__(self, B, C_in, C_out, grid, modes, dtype=FNO_F32, flags=0):
        L = load_library()
        self.desc = make_desc(B, C_in, C_out, grid, modes, dtype, flags)
        self.flags = flags
        self.B, self.C_in, self.C_out = B, C_in, C_out
        self.grid, self.modes, self.dtype = tuple(grid), tuple(modes), dtype
        self.kshape = (2 * modes[0], 2 * modes[1], 2 * modes[2], modes[3])
        self.act_dtype = _TORCH_DTYPE[dtype]
        self.device = torch.device("cuda", torch.cuda.current_device())
        h = _vp()
        _check(L.fno_plan_create(ctypes.byref(h), ctypes.byref(self.desc)), "fno_plan_create")
        self._h = h
        self._ws = {}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.fno_plan_destroy(h)
            self._h = None

    # ---------------------------------------------------------------- sizes
    def workspace_bytes(self, op):
        n = _sz()
        _check(_lib.fno_workspace_bytes(self._h, op, ctypes.byref(n)), "fno_workspace_bytes")
        return n.value

    def cache_bytes(self):
        n = _sz()
        _check(_lib.fno_cache_bytes(self._h, ctypes.byref(n)), "fno_cache_bytes")
        return n.value

    def workspace(self, op):
        """A reusable workspace for `op` on the current stream: one per (op, stream), so calls that
        share this plan on different streams never share a workspace, while the calls of one stream
        (which run in order) reuse theirs."""
        n = self.workspace_bytes(op)
        key = (op, torch.cuda.current_stream().cuda_stream)
        ws = self._ws.get(key)
        if ws is None or ws.numel() < n:
            ws = torch.empty(max(n, 256), dtype=torch.uint8, device=self.device)
            self._ws[key] = ws
        return ws

    def packed_weight_bytes(self):
        n = _sz()
        _check(_lib.fno_packed_weight_bytes(self._h, ctypes.byref(n)), "fno_packed_weight_bytes")
        return n.value

    def pack_weights(self, w, out=None):
        """fno_pack_weights: complex64 weights -> the packed E4M3 form (uint8 tensor) that plans
        created with FNO_W_FP8 take in place of w."""
        if out is None:
            out = torch.empty(self.packed_weight_bytes(), dtype=torch.uint8, device=self.device)
        _check(_lib.fno_pack_weights(self._h, _ptr(w), _ptr(out), out.numel(), _stream()), "fno_pack_weights")
        return out

    def new_cache(self):
        return torch.empty(self.cache_bytes(), dtype=torch.uint8, device=self.device)

    def act_shape(self, C):
        return (self.B, C, *self.grid)

    # ---------------------------------------------------------------- timing
    def timing(self, enable: bool):
        _check(_lib.fno_timing_enable(self._h, int(enable)), "fno_timing_enable")

    def timing_read(self):
        """{kernel: (launches, total_ms)} of the launches recorded since the last read."""
        import json
        buf = ctypes.create_string_buffer(1 << 16)
        _check(_lib.fno_timing_read(self._h, buf, len(buf)), "fno_timing_read")
        return {k: (int(v[0]), float(v[1])) for k, v in json.loads(buf.value.decode()).items()}

    # ---------------------------------------------------------------- calls
    def spectral_fwd(self, x, w, y=None, cache=None):
        if y is None:
            y = torch.empty(self.act_shape(self.C_out), dtype=self.act_dtype, device=self.device)
        ws = self.workspace(OP_SPECTRAL_FWD)
        _check(_lib.fno_spectral_fwd(self._h, _ptr(x), _ptr(w), _ptr(y), _ptr(cache), _ptr(ws), ws.numel(),
                                     _stream()), "fno_spectral_fwd")
        return y

    def spectral_fwd_noalloc(self, x, w, y, cache=None):
        """fno_spectral_fwd_noalloc: the forward without a workspace (the library's static device
        array holds the intermediates); y (and cache) are caller-allocated."""
        _check(_lib.fno_spectral_fwd_noalloc(self._h, _ptr(x), _ptr(w), _ptr(y), _ptr(cache), _stream()),
               "fno_spectral_fwd_noalloc")
        return y

    def spectral_bwd(self, gy, w, x=None, cache=None, gx=None, gw=None, need_gx=True, need_gw=True, accumulate=False):
        if need_gx and gx is None:
            gx = torch.empty(self.act_shape(self.C_in), dtype=self.act_dtype, device=self.device)
        if need_gw and gw is None:
            gw = torch.empty((self.C_in, self.C_out, *self.kshape), dtype=torch.complex64, device=self.device)
        ws = self.workspace(OP_SPECTRAL_BWD)
        _check(_lib.fno_spectral_bwd(self._h, _ptr(x), _ptr(cache), _ptr(w), _ptr(gy), _ptr(gx if need_gx else None),
                                     _ptr(gw if need_gw else None), int(accumulate), _ptr(ws), ws.numel(), _stream()),
               "fno_spectral_bwd")
        return gx, gw

    def block_fwd(self, x, w, w_pw, b_pw=None, y=None, cache=None):
        if y is None:
            y = torch.empty(self.act_shape(self.C_out), dtype=self.act_dtype, device=self.device)
        ws = self.workspace(OP_BLOCK_FWD)
        _check(_lib.fno_block_fwd(self._h, _ptr(x), _ptr(w), _ptr(w_pw), _ptr(b_pw), _ptr(y), _ptr(cache), _ptr(ws),
                                  ws.numel(), _stream()), "fno_block_fwd")
        return y

    def block_bwd(self, x, cache, w, w_pw, b_pw, gy, gx=None, gw=None, gw_pw=None, gb_pw=None, need_gw=True,
                  need_gw_pw=True, need_gb=True, accumulate=False):
        if gx is None:
            gx = torch.empty(self.act_shape(self.C_in), dtype=self.act_dtype, device=self.device)
        if need_gw and gw is None:
            gw = torch.empty((self.C_in, self.C_out, *self.kshape), dtype=torch.complex64, device=self.device)
        if need_gw_pw and gw_pw is None:
            gw_pw = torch.empty((self.C_out, self.C_in), dtype=torch.float32, device=self.device)
        if need_gb and gb_pw is None:
            gb_pw = torch.empty((self.C_out,), dtype=torch.float32, device=self.device)
        ws = self.workspace(OP_BLOCK_BWD)
        _check(_lib.fno_block_bwd(self._h, _ptr(x), _ptr(cache), _ptr(w), _ptr(w_pw), _ptr(b_pw), _ptr(gy), _ptr(gx),
                                  _ptr(gw if need_gw else None), _ptr(gw_pw if need_gw_pw else None),
                                  _ptr(gb_pw if need_gb else None), int(accumulate), _ptr(ws), ws.numel(), _stream()),
               "fno_block_bwd")
        return gx, gw, gw_pw, gb_pw


def _c(t):
    return t if t.is_contiguous() else t.contiguous()


class SpectralConv4dFn(torch.autograd.Function):
    """y = spectral convolution of x with complex weights w (Alg. 2)."""

    @staticmethod
    def forward(ctx, x, w, plan: Plan):
        x, w = _c(x), _c(w)
        cache = plan.new_cache()
        y = plan.spectral_fwd(x, w, cache=cache)
        ctx.plan = plan
        ctx.save_for_backward(x, w, cache)
        return y

    @staticmethod
    def backward(ctx, gy):
        x, w, cache = ctx.saved_tensors
        plan = ctx.plan
        gx, gw = plan.spectral_bwd(_c(gy.to(plan.act_dtype)), w, x=x, cache=cache,
                                   need_gx=ctx.needs_input_grad[0], need_gw=ctx.needs_input_grad[1])
        return gx, gw, None


class FNOBlockFn(torch.autograd.Function):
    """y = GELU(spectral(x, w) + w_pw x + b_pw) with per-block recomputation:
    only x and the small forward cache are kept for the backward."""

    @staticmethod
    def forward(ctx, x, w, w_pw, b_pw, plan: Plan):
        x, w, w_pw = _c(x), _c(w), _c(w_pw)
        b_pw = _c(b_pw) if b_pw is not None else None
        cache = plan.new_cache()
        y = plan.block_fwd(x, w, w_pw, b_pw, cache=cache)
        ctx.plan = plan
        ctx.has_bias = b_pw is not None
        ctx.save_for_backward(x, w, w_pw, b_pw if b_pw is not None else torch.empty(0, device=x.device), cache)
        return y

    @staticmethod
    def backward(ctx, gy):
        x, w, w_pw, b_pw, cache = ctx.saved_tensors
        plan = ctx.plan
        gx, gw, gwpw, gb = plan.block_bwd(x, cache, w, w_pw, b_pw if ctx.has_bias else None,
                                          _c(gy.to(plan.act_dtype)), need_gw=ctx.needs_input_grad[1],
                                          need_gw_pw=ctx.needs_input_grad[2],
                                          need_gb=ctx.has_bias and ctx.needs_input_grad[3])
        return gx, gw, gwpw, (gb if ctx.has_bias else None), None


# ---------------------------------------------------------------------------
# Network glue of Alg. 1: encoder (lifting), decoder (projection), MSE loss.
_DTYPE_CODE = {torch.float32: FNO_F32, torch.bfloat16: FNO_BF16}
_glue_ws = {}


def _glue_workspace(device, ci, h, co):
    n = _sz()
    _check(load_library().fno_glue_workspace_bytes(ci, h, co, ctypes.byref(n)), "fno_glue_workspace_bytes")
    # one workspace per (device, stream): calls on one stream run in order and may share it
    key = (str(device), torch.cuda.current_stream(device).cuda_stream)
    ws = _glue_ws.get(key)
    if ws is None or ws.numel() < n.value:
        ws = torch.empty(max(n.value, 256), dtype=torch.uint8, device=device)
        _glue_ws[key] = ws
    return ws


def _npts(t):
    n = 1
    for s in t.shape[2:]:
        n *= s
    return n


def lift_fwd(x, w, b):
    B, ci = x.shape[:2]
    co = w.shape[0]
    y = torch.empty((B, co, *x.shape[2:]), dtype=x.dtype, device=x.device)
    _check(load_library().fno_lift_fwd(_DTYPE_CODE[x.dtype], B, ci, co, _npts(x), _ptr(x), _ptr(w), _ptr(b), _ptr(y),
                                       _stream()), "fno_lift_fwd")
    return y


def lift_bwd(x, w, b, gy, need_gw=True, need_gb=True, out=None):
    """(gw, gb) of the encoder; with out = (gw, gb) the gradients are added into those tensors."""
    B, ci = x.shape[:2]
    co = w.shape[0]
    if out is not None:
        gw, gb = out
    else:
        gw = torch.empty_like(w) if need_gw else None
        gb = torch.empty((co,), dtype=torch.float32, device=x.device) if need_gb else None
    ws = _glue_workspace(x.device, ci, 1, co)
    _check(load_library().fno_lift_bwd(_DTYPE_CODE[x.dtype], B, ci, co, _npts(x), _ptr(x), _ptr(w), _ptr(b),
                                       _ptr(gy), _ptr(gw), _ptr(gb), int(out is not None), _ptr(ws), ws.numel(),
                                       _stream()), "fno_lift_bwd")
    return gw, gb


def proj_fwd(x, w1, b1, w2, b2):
    B, ci = x.shape[:2]
    h, co = w1.shape[0], w2.shape[0]
    y = torch.empty((B, co, *x.shape[2:]), dtype=x.dtype, device=x.device)
    _check(load_library().fno_proj_fwd(_DTYPE_CODE[x.dtype], B, ci, h, co, _npts(x), _ptr(x), _ptr(w1), _ptr(b1),
                                       _ptr(w2), _ptr(b2), _ptr(y), _stream()), "fno_proj_fwd")
    return y


def proj_bwd(x, w1, b1, w2, b2, gy, out=None):
    """(gx, gw1, gb1, gw2, gb2) of the decoder; with out = those five tensors the gradients are
    added into them."""
    B, ci = x.shape[:2]
    h, co = w1.shape[0], w2.shape[0]
    if out is not None:
        gx, gw1, gb1, gw2, gb2 = out
    else:
        gx = torch.empty_like(x)
        gw1, gw2 = torch.empty_like(w1), torch.empty_like(w2)
        gb1 = torch.empty((h,), dtype=torch.float32, device=x.device)
        gb2 = torch.empty((co,), dtype=torch.float32, device=x.device)
    ws = _glue_workspace(x.device, ci, h, co)
    _check(load_library().fno_proj_bwd(_DTYPE_CODE[x.dtype], B, ci, h, co, _npts(x), _ptr(x), _ptr(w1), _ptr(b1),
                                       _ptr(w2), _ptr(b2), _ptr(gy), _ptr(gx), _ptr(gw1), _ptr(gb1), _ptr(gw2),
                                       _ptr(gb2), int(out is not None), _ptr(ws), ws.numel(), _stream()),
           "fno_proj_bwd")
    return gx, gw1, gb1, gw2, gb2


def mse(y, target, need_grad=True):
    loss = torch.empty((1,), dtype=torch.float32, device=y.device)
    gy = torch.empty_like(y) if need_grad else None
    ws = _glue_workspace(y.device, 1, 1, 1)
    _check(load_library().fno_mse(_DTYPE_CODE[y.dtype], y.numel(), _ptr(y), _ptr(target), _ptr(loss), _ptr(gy),
                                  _ptr(ws), ws.numel(), _stream()), "fno_mse")
    return loss, gy


class LiftFn(torch.autograd.Function):
    """Encoder of Alg. 1: GELU(w x + b) pointwise; no gradient to the (data) input."""

    @staticmethod
    def forward(ctx, x, w, b):
        x, w, b = _c(x), _c(w), _c(b)
        ctx.save_for_backward(x, w, b)
        return lift_fwd(x, w, b)

    @staticmethod
    def backward(ctx, gy):
        x, w, b = ctx.saved_tensors
        gw, gb = lift_bwd(x, w, b, _c(gy.to(x.dtype)))
        return None, gw, gb


class ProjFn(torch.autograd.Function):
    """Decoder of Alg. 1: w2 GELU(w1 x + b1) + b2 pointwise (hidden layer never stored)."""

    @staticmethod
    def forward(ctx, x, w1, b1, w2, b2):
        x, w1, b1, w2, b2 = (_c(t) for t in (x, w1, b1, w2, b2))
        ctx.save_for_backward(x, w1, b1, w2, b2)
        return proj_fwd(x, w1, b1, w2, b2)

    @staticmethod
    def backward(ctx, gy):
        x, w1, b1, w2, b2 = ctx.saved_tensors
        gx, gw1, gb1, gw2, gb2 = proj_bwd(x, w1, b1, w2, b2, _c(gy.to(x.dtype)))
        return gx, gw1, gb1, gw2, gb2


class MseFn(torch.autograd.Function):
    """Mean-squared error; returns a float32 scalar tensor."""

    @staticmethod
    def forward(ctx, y, target):
        y, target = _c(y), _c(target.to(y.dtype))
        loss, gy = mse(y, target, need_grad=True)
        ctx.save_for_backward(gy)
        return loss.reshape(())

    @staticmethod
    def backward(ctx, gl):
        (gy,) = ctx.saved_tensors
        return gy * gl.to(gy.dtype), None


class FNO4d:
    """The model-parallel FNO of Alg. 1 on one GPU: encoder (lifting 1x1 + GELU),
    `nblocks` FNO blocks (spectral convolution + 1x1 + GELU, with per-block
    recomputation in the backward), decoder (1x1 -> GELU -> 1x1).

    Parameters are float32 tensors with requires_grad; activations use `dtype`
    (torch.float32 or torch.bfloat16)."""

    def __init__(self, in_ch, width, grid, modes, nblocks=4, hidden=128, out_ch=1, batch=1,
                 dtype=torch.float32, params=None, device=None):
        self.device = device or torch.device("cuda", torch.cuda.current_device())
        self.dtype = dtype
        self.plan = Plan(batch, width, width, grid, modes, FNO_BF16 if dtype == torch.bfloat16 else FNO_F32)
        t = lambda a: torch.as_tensor(a).to(self.device).contiguous().requires_grad_(True)
        if params is None:
            raise ValueError("pass params = {'lift': (we, be), 'blocks': [(w, wpw, bpw), ...], 'proj': (w1, b1, w2, b2)}")
        self.lift = [t(a) for a in params["lift"]]
        self.blocks = [[t(a) for a in blk] for blk in params["blocks"]]
        self.proj = [t(a) for a in params["proj"]]

    def parameters(self):
        out = list(self.lift)
        for blk in self.blocks:
            out += blk
        return out + list(self.proj)

    def __call__(self, x):
        h = LiftFn.apply(x.to(self.dtype), *self.lift)
        for (w, wpw, bpw) in self.blocks:
            h = FNOBlockFn.apply(h, w, wpw, bpw, self.plan)
        return ProjFn.apply(h, *self.proj)
