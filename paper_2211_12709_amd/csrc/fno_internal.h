// fno_internal.h -- shared definitions of the HIP library (plan layout,
// kernel launcher prototypes, small device helpers).  Not part of the C-ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "fno_mi355x.h"

namespace fno {

// ---------------------------------------------------------------- plan
// Basis tables live in device memory owned by the plan.  Every table is
// generated in FP64 with the phase k*n reduced modulo N in 64-bit integers,
// then rounded once to float.
struct Tables {
    // Per axis d = x, y, z, t: (cos, sin) of theta = 2*pi*((k_j n) mod N_d)/N_d,
    // laid out [K_d][N_d] (retained index j major, grid point n minor).
    float2 *cs[4];
    // c(kt)/N per kt (weights of the real inverse transform) and ones.
    float *wt_inv;
    float *wt_one;
    // Fragment-ordered tables of the MFMA kernels (tables.hip): float copy and
    // bfloat16 hi/lo split of each.  y tables exist for the float kernels'
    // y chunk (16 planes) and the bfloat16 kernels' (32 planes).
    struct Frag {
        float *f;
        short *hi, *lo;
    };
    Frag t_fwd, t_bwd, z_fwd, y_fwd_f32, y_fwd_bf16;
    Frag z_syn, t_syn_inv, t_syn_adj;  // z and t synthesis (inverse / adjoint weights)
    Frag ax_fwd[2], ax_inv[2];           // one-axis contractions along x (0) and y (1)
};

struct Dims {
    int B, Ci, Co;
    int N[4];  // Nx, Ny, Nz, Nt
    int m[4];  // mx, my, mz, mt
    int K[4];  // 2mx, 2my, 2mz, mt
    long long ncell;      // Nx Ny Nz Nt
    long long nmode;      // Kx Ky Kz Kt
    long long plane;      // Nz Nt  (one (b, c, x, y) plane of an activation)
    long long kplane;     // Kz Kt  (its truncated t, z spectrum)
    long long P;          // Ky Kz Kt
};

// Geometry of the forward t, z, y kernels (fwd_tzy.hip, fwd_tzy_gen.hip): y, z, t sizes and retained
// counts; t chunks of 16, z blocks of 16, kz blocks of 16 and z-step row tiles (cos, sin), y-step
// row tiles (re, im), y planes per staged chunk, its K chunks, and the chunk count.
struct TzyArgs {
    int Ny, Nz, Nt, Ky, Kz, Kt;
    int NQ, NZB, KB, MZ, MY, Yc, QY, NYC;
};
// Basis tables of the forward t, z, y kernels (fragment order; lo: the bfloat16 hi + lo split).
struct TzyTabs {
    const void *t, *t_lo, *z, *z_lo, *y, *y_lo;
};

}  // namespace fno

namespace fno {
// Opt-in per-kernel event timing of a plan's launches.
struct TimingRec {
    const char *name;
    hipEvent_t start, stop;
};
struct Timing {
    bool on = false;
    std::vector<TimingRec> recs;
    std::vector<hipEvent_t> pool;
};
}  // namespace fno

struct fno_plan {
    fno_desc_t desc;
    fno::Dims d;
    int device;
    fno::Tables tab;
    void *table_mem;
    mutable fno::Timing timing;
};

namespace fno {

// Workspace carve-up shared by the host code of every entry point.
struct Workspace {
    float2 *t1;    // [B*C][Nx][Ny][Kz*Kt]  t,z spectrum (also its inverse-side twin)
    float2 *t2;    // [B*C][Nx][Ky*Kz*Kt]   t,z,y spectrum
    float2 *sp;    // [B*C][Kx*Ky*Kz*Kt]    retained spectrum (mix input or output)
    float2 *sp2;   // [B*C][Kx*Ky*Kz*Kt]
    float *gz;     // [B*Co][N]             gradient of the pre-activation (block bwd)
    float *part;   // partial sums for the pointwise weight gradients
    size_t bytes;
};

// ---------------------------------------------------------------- device helpers
__device__ __forceinline__ float to_f32(float v) { return v; }
__device__ __forceinline__ float to_f32(__bf16 v) { return (float)v; }
template <typename T> __device__ __forceinline__ T from_f32(float v);
template <> __device__ __forceinline__ float from_f32<float>(float v) { return v; }
template <> __device__ __forceinline__ __bf16 from_f32<__bf16>(float v) { return (__bf16)v; }

__device__ __forceinline__ float gelu_f(float u) { return 0.5f * u * (1.0f + erff(u * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float u)
{
    return 0.5f * (1.0f + erff(u * 0.70710678118654752f)) + u * 0.39894228040143268f * expf(-0.5f * u * u);
}

// GELU and its derivative from one evaluation of erf by Abramowitz & Stegun,
// Handbook of Mathematical Functions, formula 7.1.26:
//   1 - erf(w) = (a1 s + a2 s^2 + a3 s^3 + a4 s^4 + a5 s^5) exp(-w^2),  s = 1/(1 + p w),  w >= 0,
// with absolute error at most 1.5e-7.  At w = |u|/sqrt(2), q = (1 - erf(w)) / 2 is the Gaussian
// tail beyond |u|, so Phi(u) = 1 - q for u >= 0 and q for u < 0, and
//   GELU(u)  = u Phi(u) = max(u, 0) - |u| q,
//   GELU'(u) = Phi(u) + u phi(u),  phi(u) = exp(-u^2/2) / sqrt(2 pi) (the same exponential).
// q is formed directly (no 1 - erf cancellation for u < 0); one exponential and one
// reciprocal per value.  Coefficients below: a_k / 2 and p / sqrt(2).
__device__ __forceinline__ void gelu_tail(float u, float &q, float &e)
{
    const float s = __builtin_amdgcn_rcpf(fmaf(0.23164189f, fabsf(u), 1.0f));
    const float hp = fmaf(s, fmaf(s, fmaf(s, fmaf(s, 0.5307027145f, -0.7265760135f), 0.7107068705f), -0.142248368f),
                          0.127414796f);
    e = __builtin_amdgcn_exp2f(u * (u * -0.72134752044448170f));  // exp(-u^2 / 2)
    q = s * hp * e;
}
__device__ __forceinline__ void gelu_as(float u, float &g, float &dg)
{
    float q, e;
    gelu_tail(u, q, e);
    g = fmaf(-fabsf(u), q, fmaxf(u, 0.0f));
    dg = fmaf(u * 0.39894228040143268f, e, u >= 0.0f ? 1.0f - q : q);
}
__device__ __forceinline__ float gelu_fast(float u)
{
    float q, e;
    gelu_tail(u, q, e);
    return fmaf(-fabsf(u), q, fmaxf(u, 0.0f));
}
__device__ __forceinline__ float gelu_grad_fast(float u)
{
    float q, e;
    gelu_tail(u, q, e);
    return fmaf(u * 0.39894228040143268f, e, u >= 0.0f ? 1.0f - q : q);
}

// Cheaper forms for the bfloat16 epilogues, whose results are rounded to bfloat16 (relative step
// 2^-8): Phi by the logistic approximation of Bowling, Khasawneh, Kaewkuekool and Cho (2009), "A
// logistic approximation to the cumulative normal distribution",
//   Phi(u) ~ 1 / (1 + exp(-(1.5976 u + 0.07056 u^3))),  |error| <= 1.4e-4,
// so GELU(u) = u Phi(u) is within 1.1e-4 (|u| + 1) and GELU'(u) = Phi(u) + u phi(u) (phi exact)
// within 1.4e-4; 7 and 10 instructions per value against 14 and 18 above.  The constants below
// carry the factor log2(e) of the base-2 exponential.
__device__ __forceinline__ float phi_logistic(float u, float u2)
{
    const float a = u * fmaf(u2, -0.10179656f, -2.30484960f);  // -(1.5976 u + 0.07056 u^3) log2(e)
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(a));
}
__device__ __forceinline__ float gelu_lg(float u) { return u * phi_logistic(u, u * u); }
__device__ __forceinline__ float gelu_grad_lg(float u)
{
    const float u2 = u * u;
    const float e = __builtin_amdgcn_exp2f(u2 * -0.72134752044448170f);  // exp(-u^2 / 2)
    return fmaf(u * 0.39894228040143268f, e, phi_logistic(u, u2));
}
// The derivative of u P(u) with P the logistic approximation itself, P' = P (1 - P) g'(u),
// g(u) = 1.5976 u + 0.07056 u^3: within 7.9e-4 of the exact GELU', one exponential fewer.
__device__ __forceinline__ float gelu_grad_lgd(float u)
{
    const float u2 = u * u;
    const float P = phi_logistic(u, u2);
    const float gp = fmaf(u2, 0.21168f, 1.5976f);
    return fmaf(u * fmaf(-P, P, P), gp, P);
}

// OCP 8-bit floating point E4M3 (sign, 4 exponent bits with bias 7, 3 mantissa bits; no
// infinities, S.1111.111 is NaN, largest finite 448, subnormals m 2^-9).
__device__ __forceinline__ float e4m3_to_f32(unsigned b)
{
    const unsigned sgn = (b & 0x80u) << 24, e = (b >> 3) & 15u, m = b & 7u;
    const float nrm = __uint_as_float(sgn | ((e + 120u) << 23) | (m << 20));   // 2^(e-7) (1 + m/8)
    const float sub = __uint_as_float(sgn | __float_as_uint((float)m * 0.001953125f));  // m 2^-9
    return e ? nrm : sub;
}
// Nearest E4M3 value, ties to even, magnitudes beyond 448 saturating to 448 (finite inputs).
__device__ __forceinline__ unsigned f32_to_e4m3(float v)
{
    const unsigned sgn = (__float_as_uint(v) >> 24) & 0x80u;
    const float a = fabsf(v);
    if (a >= 448.0f) return sgn | 0x7eu;
    if (a < 0.015625f) return sgn | (unsigned)rintf(a * 512.0f);  // subnormal grid; 8 -> 2^-6, code 0x08
    unsigned u = __float_as_uint(a);
    u += 0x7ffffu + ((u >> 20) & 1u);  // round the 23-bit mantissa to 3 bits, ties to even
    const unsigned r = (((u >> 23) - 120u) << 3) | ((u >> 20) & 7u);
    return sgn | (r > 0x7eu ? 0x7eu : r);
}

}  // namespace fno
