"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds input synthesis only (random fields, weights, targets); it
contains none of the spectral-convolution arithmetic and is shared by the
HIP path's tests and benchmark and by the oracle's tests.

All draws use numpy's PCG64 (``numpy.random.default_rng(seed)``) in float64
and are rounded once to float32: the float32 values are what the GPU gets and
what the oracle consumes (widened back to float64).

Workloads (arXiv 2211.12709, Sec. V):
  * Navier-Stokes-like (Sec. V-A): 4 channels -- a smooth Gaussian random
    field with power spectrum ~ |k|^-3 and its x, y, z coordinate channels --
    on a 3-D grid repeated along t (the paper's inputs are 3-D maps repeated
    along time).
  * CO2-flow-like (Sec. V-B): 3 channels -- log-permeability ln k ~ N(0, 1)
    with Gaussian covariance of correlation length 16 cells, porosity
    0.1 + 0.05 tanh(ln k), and a one-hot injection-well column at a random
    (x, y) -- repeated along t.
The paper's datasets (WaterLily vorticity, Sleipner/OPM saturation) are not
available; these fields stand in for them at the same tensor shapes.
"""
from __future__ import annotations

import numpy as np

# Seed plan: input 0; spectral weights of block i: 100 + i; pointwise weights
# of block i: 200 + i; lifting 300; projection 301 / 302; target 400;
# finite-difference sample indices 500; GRF 600; permeability 700; well 701.
SEED_INPUT = 0
SEED_SPECTRAL_W = 100
SEED_POINTWISE = 200
SEED_LIFT = 300
SEED_PROJ1 = 301
SEED_PROJ2 = 302
SEED_TARGET = 400
SEED_FD = 500
SEED_GRF = 600
SEED_PERM = 700
SEED_WELL = 701


def f32(a) -> np.ndarray:
    """Round float64 draws to the float32 values handed to both sides."""
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def normal_field(shape, seed=SEED_INPUT, std=1.0) -> np.ndarray:
    """i.i.d. N(0, std^2) field, float32."""
    rng = np.random.default_rng(seed)
    return f32(rng.standard_normal(size=shape) * std)


def spectral_weights(ci, co, kshape, seed=SEED_SPECTRAL_W) -> np.ndarray:
    """Complex weights [ci, co, *kshape], real and imaginary parts i.i.d.
    N(0, 1/(ci*co)) (variance), rounded to complex64."""
    rng = np.random.default_rng(seed)
    std = 1.0 / np.sqrt(ci * co)
    re = rng.standard_normal(size=(ci, co, *kshape)) * std
    im = rng.standard_normal(size=(ci, co, *kshape)) * std
    return np.ascontiguousarray((re + 1j * im).astype(np.complex64))


def linear_weights(fan_out, fan_in, seed, bias=True):
    """W [fan_out, fan_in] and b [fan_out] ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)), float32."""
    rng = np.random.default_rng(seed)
    bound = 1.0 / np.sqrt(fan_in)
    w = f32(rng.uniform(-bound, bound, size=(fan_out, fan_in)))
    b = f32(rng.uniform(-bound, bound, size=(fan_out,))) if bias else None
    return w, b


def _kgrid(shape3):
    """Integer wavenumbers (cycles per domain) of a 3-D FFT grid."""
    ks = [np.fft.fftfreq(n) * n for n in shape3]
    return np.meshgrid(*ks, indexing="ij")


def _standardize(f):
    f = f - f.mean()
    s = f.std()
    return f / s if s > 0 else f


def grf_power_law(shape3, seed=SEED_GRF, exponent=3.0) -> np.ndarray:
    """3-D Gaussian random field with power spectrum ~ |k|^-exponent
    (DC removed), standardised to zero mean and unit variance, float64."""
    rng = np.random.default_rng(seed)
    white = rng.standard_normal(size=shape3)
    kx, ky, kz = _kgrid(shape3)
    kk = np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)
    amp = np.zeros_like(kk)
    nz = kk > 0
    amp[nz] = kk[nz] ** (-exponent / 2.0)
    f = np.fft.ifftn(np.fft.fftn(white) * amp).real
    return _standardize(f)


def grf_gaussian_cov(shape3, corr_len=16.0, seed=SEED_PERM) -> np.ndarray:
    """3-D Gaussian random field with Gaussian covariance of correlation
    length corr_len cells (spectral amplitude exp(-kappa^2 l^2 / 4),
    kappa in rad/cell), standardised to N(0, 1), float64."""
    rng = np.random.default_rng(seed)
    white = rng.standard_normal(size=shape3)
    kx, ky, kz = _kgrid(shape3)
    kappa2 = sum((2 * np.pi * k / n) ** 2 for k, n in zip((kx, ky, kz), shape3))
    amp = np.exp(-kappa2 * corr_len ** 2 / 4.0)
    f = np.fft.ifftn(np.fft.fftn(white) * amp).real
    return _standardize(f)


def ns_like_input(batch, grid, seed=SEED_GRF) -> np.ndarray:
    """[batch, 4, Nx, Ny, Nz, Nt]: power-law GRF + x, y, z coordinates in
    [0, 1] (inclusive linspace), every channel constant along t."""
    nx, ny, nz, nt = grid
    out = np.empty((batch, 4, nx, ny, nz, nt), dtype=np.float32)
    cx, cy, cz = np.meshgrid(np.linspace(0, 1, nx), np.linspace(0, 1, ny), np.linspace(0, 1, nz),
                             indexing="ij")
    for b in range(batch):
        g = grf_power_law((nx, ny, nz), seed=seed + b)
        for c, f in enumerate((g, cx, cy, cz)):
            out[b, c] = f32(f)[..., None]
    return out


def co2_like_input(batch, grid, corr_len=16.0, seed=SEED_PERM, well_seed=SEED_WELL) -> np.ndarray:
    """[batch, 3, Nx, Ny, Nz, Nt]: ln k, porosity 0.1 + 0.05 tanh(ln k), and a
    one-hot well column at a random (x0, y0) over all z; constant along t."""
    nx, ny, nz, nt = grid
    out = np.empty((batch, 3, nx, ny, nz, nt), dtype=np.float32)
    for b in range(batch):
        lnk = grf_gaussian_cov((nx, ny, nz), corr_len=corr_len, seed=seed + b)
        por = 0.1 + 0.05 * np.tanh(lnk)
        rng = np.random.default_rng(well_seed + b)
        x0, y0 = int(rng.integers(0, nx)), int(rng.integers(0, ny))
        well = np.zeros((nx, ny, nz))
        well[x0, y0, :] = 1.0
        for c, f in enumerate((lnk, por, well)):
            out[b, c] = f32(f)[..., None]
    return out


def block_params(ci, co, kshape, block=0):
    """Seeded parameters of FNO block `block`: spectral W (complex64), W_pw, b_pw (float32)."""
    w = spectral_weights(ci, co, kshape, seed=SEED_SPECTRAL_W + block)
    wpw, bpw = linear_weights(co, ci, seed=SEED_POINTWISE + block)
    return w, wpw, bpw


def smooth_spacetime_field(batch, channels, grid, seed, corr_len=16.0) -> np.ndarray:
    """[batch, channels, Nx, Ny, Nz, Nt] float32 stand-in for a hidden FNO
    activation on a CO2- or NS-shaped grid: per (b, c) two independent 3-D
    Gaussian-covariance fields g1, g2 (correlation length corr_len cells) and
    x = (g1 + g2 sin(2 pi f t / Nt + phi)) / sqrt(1.5), with f in {1, 2, 3} and
    phi uniform, drawn from the seed.  Smooth in space, periodic in time, with
    unit variance on average."""
    nx, ny, nz, nt = grid
    rng = np.random.default_rng(seed)
    out = np.empty((batch, channels, nx, ny, nz, nt), dtype=np.float32)
    t = np.arange(nt)
    for b in range(batch):
        for c in range(channels):
            s1, s2 = (int(v) for v in rng.integers(0, 2 ** 31, size=2))
            f = int(rng.integers(1, 4))
            phi = float(rng.uniform(0, 2 * np.pi))
            cl = min(corr_len, max(nx, ny, nz) / 8.0)
            g1 = grf_gaussian_cov((nx, ny, nz), corr_len=cl, seed=s1).astype(np.float32)
            g2 = grf_gaussian_cov((nx, ny, nz), corr_len=cl, seed=s2).astype(np.float32)
            prof = np.sin(2 * np.pi * f * t / nt + phi).astype(np.float32)
            out[b, c] = (g1[..., None] + g2[..., None] * prof) / np.float32(np.sqrt(1.5))
    return out
