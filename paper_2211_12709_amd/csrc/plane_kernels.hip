// plane_kernels.hip -- kernels that touch full-size activations, one
// (b, x, y) plane of Nz x Nt points per workgroup:
//   * k_fwd_tz: truncated real DFT over t, then complex DFT over z of one
//     channel plane (the t and z part of F_yzt, S_yzt in Alg. 2 line 1);
//   * k_inv_zt: z and real-output t synthesis from the truncated spectrum
//     (the t and z part of F_yzt^T S_yzt^T in Alg. 2 line 3) with one of three
//     epilogues: plain output, the FNO block epilogue sigma(S + W_pw x + b)
//     (Alg. 1), or the accumulation of an adjoint into an input gradient;
//   * k_bwd_gz: recomputation of the block pre-activation and the gradient
//     through GELU.
#include "fno_internal.h"

namespace fno {

// in: [planes][Nz][Nt] activations; out: [planes][Kz][Kt] complex.
// A[z][kt] = wt[kt] sum_t v[z][t] exp(-i 2 pi kt t / Nt);  out[kz][kt] = sum_z exp(-i th) A[z][kt]
template <typename T>
__global__ void __launch_bounds__(256) k_fwd_tz(const T *__restrict__ in, float2 *__restrict__ out,
                                                const float2 *__restrict__ cs_t, const float2 *__restrict__ cs_z,
                                                const float *__restrict__ wt, int Nz, int Nt, int Kz, int Kt)
{
    extern __shared__ float smem[];
    float *xs = smem;                                             // Nz*Nt
    float2 *A = reinterpret_cast<float2 *>(smem + ((Nz * Nt + 1) & ~1));  // Nz*Kt
    const long long p = blockIdx.x;
    const T *src = in + p * (long long)Nz * Nt;
    for (int e = threadIdx.x; e < Nz * Nt; e += blockDim.x) xs[e] = to_f32(src[e]);
    __syncthreads();
    for (int e = threadIdx.x; e < Nz * Kt; e += blockDim.x) {
        const int z = e / Kt, kt = e % Kt;
        float re = 0.f, im = 0.f;
        for (int t = 0; t < Nt; t++) {
            const float2 c = cs_t[kt * Nt + t];
            const float v = xs[z * Nt + t];
            re += v * c.x;
            im -= v * c.y;
        }
        A[e] = make_float2(re * wt[kt], im * wt[kt]);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < Kz * Kt; e += blockDim.x) {
        const int kz = e / Kt, kt = e % Kt;
        float re = 0.f, im = 0.f;
        for (int z = 0; z < Nz; z++) {
            const float2 c = cs_z[kz * Nz + z];
            const float2 a = A[z * Kt + kt];
            re += c.x * a.x + c.y * a.y;
            im += c.x * a.y - c.y * a.x;
        }
        out[p * Kz * Kt + e] = make_float2(re, im);
    }
}

enum { EPI_PLAIN = 0, EPI_BLOCK = 1, EPI_ADJ = 2 };

// One workgroup per (b, x, y) plane; loops over the C channels of the
// spectrum u [B*C][Nx][Ny][Kz][Kt].  For channel c:
//   V[z][kt] = sum_kz exp(+i th) u[kz][kt];  s[z][t] = sum_kt wt[kt] Re(V[z][kt] exp(+i 2 pi kt t/Nt))
// then, at every point of the plane:
//   EPI_PLAIN: out[c] = s
//   EPI_BLOCK: out[c] = GELU(s + sum_i wpw[c][i] x[i] + b[c])          (C = Co, x has Ci channels)
//   EPI_ADJ:   out[c] = (acc ? out[c] : 0) + s + sum_o wpw[o][c] gz[o] (C = Ci; gz, wpw nullable)
template <typename T, int EPI>
__global__ void __launch_bounds__(256) k_inv_zt(const float2 *__restrict__ u, T *__restrict__ out,
                                                const float2 *__restrict__ cs_t, const float2 *__restrict__ cs_z,
                                                const float *__restrict__ wt, const T *__restrict__ x,
                                                const float *__restrict__ wpw, const float *__restrict__ bpw,
                                                const float *__restrict__ gz, int C, int Cx, int Nx, int Ny, int Nz,
                                                int Nt, int Kz, int Kt, int accumulate)
{
    extern __shared__ float smem[];
    float2 *U = reinterpret_cast<float2 *>(smem);  // Kz*Kt
    float2 *V = U + Kz * Kt;                       // Nz*Kt
    const long long pl = blockIdx.x;               // (b, x, y)
    const long long xy = pl % ((long long)Nx * Ny);
    const int b = (int)(pl / ((long long)Nx * Ny));
    const long long plane = (long long)Nz * Nt;
    const long long ncell = (long long)Nx * Ny * plane;
    for (int c = 0; c < C; c++) {
        const float2 *uc = u + (((long long)b * C + c) * Nx * Ny + xy) * Kz * Kt;
        __syncthreads();
        for (int e = threadIdx.x; e < Kz * Kt; e += blockDim.x) U[e] = uc[e];
        __syncthreads();
        for (int e = threadIdx.x; e < Nz * Kt; e += blockDim.x) {
            const int z = e / Kt, kt = e % Kt;
            float re = 0.f, im = 0.f;
            for (int kz = 0; kz < Kz; kz++) {
                const float2 cz = cs_z[kz * Nz + z];
                const float2 a = U[kz * Kt + kt];
                re += cz.x * a.x - cz.y * a.y;
                im += cz.x * a.y + cz.y * a.x;
            }
            V[e] = make_float2(re, im);
        }
        __syncthreads();
        T *oc = out + ((long long)b * C + c) * ncell + xy * plane;
        for (int e = threadIdx.x; e < plane; e += blockDim.x) {
            const int z = e / Nt, t = e % Nt;
            float s = 0.f;
            for (int kt = 0; kt < Kt; kt++) {
                const float2 ct = cs_t[kt * Nt + t];
                const float2 v = V[z * Kt + kt];
                s += wt[kt] * (v.x * ct.x - v.y * ct.y);
            }
            if (EPI == EPI_BLOCK) {
                float a = bpw ? bpw[c] : 0.f;
                for (int i = 0; i < Cx; i++)
                    a += wpw[c * Cx + i] * to_f32(x[((long long)b * Cx + i) * ncell + xy * plane + e]);
                oc[e] = from_f32<T>(gelu_f(s + a));
            } else if (EPI == EPI_ADJ) {
                float a = accumulate ? to_f32(oc[e]) : 0.f;
                if (gz)
                    for (int o = 0; o < Cx; o++)
                        a += wpw[o * C + c] * gz[((long long)b * Cx + o) * ncell + xy * plane + e];
                oc[e] = from_f32<T>(a + s);
            } else {
                oc[e] = from_f32<T>(s);
            }
        }
    }
}

// Block backward, first pass: with s from the spectrum u (as in k_inv_zt),
// z = s + sum_i wpw[o][i] x[i] + b[o] and gz[o] = gy[o] * GELU'(z).
template <typename T>
__global__ void __launch_bounds__(256) k_bwd_gz(const float2 *__restrict__ u, const T *__restrict__ x,
                                                const T *__restrict__ gy, float *__restrict__ gz,
                                                const float2 *__restrict__ cs_t, const float2 *__restrict__ cs_z,
                                                const float *__restrict__ wt, const float *__restrict__ wpw,
                                                const float *__restrict__ bpw, int Ci, int Co, int Nx, int Ny, int Nz,
                                                int Nt, int Kz, int Kt)
{
    extern __shared__ float smem[];
    float2 *U = reinterpret_cast<float2 *>(smem);
    float2 *V = U + Kz * Kt;
    const long long pl = blockIdx.x;
    const long long xy = pl % ((long long)Nx * Ny);
    const int b = (int)(pl / ((long long)Nx * Ny));
    const long long plane = (long long)Nz * Nt;
    const long long ncell = (long long)Nx * Ny * plane;
    for (int o = 0; o < Co; o++) {
        const float2 *uc = u + (((long long)b * Co + o) * Nx * Ny + xy) * Kz * Kt;
        __syncthreads();
        for (int e = threadIdx.x; e < Kz * Kt; e += blockDim.x) U[e] = uc[e];
        __syncthreads();
        for (int e = threadIdx.x; e < Nz * Kt; e += blockDim.x) {
            const int z = e / Kt, kt = e % Kt;
            float re = 0.f, im = 0.f;
            for (int kz = 0; kz < Kz; kz++) {
                const float2 cz = cs_z[kz * Nz + z];
                const float2 a = U[kz * Kt + kt];
                re += cz.x * a.x - cz.y * a.y;
                im += cz.x * a.y + cz.y * a.x;
            }
            V[e] = make_float2(re, im);
        }
        __syncthreads();
        const long long base = ((long long)b * Co + o) * ncell + xy * plane;
        for (int e = threadIdx.x; e < plane; e += blockDim.x) {
            const int z = e / Nt, t = e % Nt;
            float s = 0.f;
            for (int kt = 0; kt < Kt; kt++) {
                const float2 ct = cs_t[kt * Nt + t];
                const float2 v = V[z * Kt + kt];
                s += wt[kt] * (v.x * ct.x - v.y * ct.y);
            }
            float a = bpw ? bpw[o] : 0.f;
            for (int i = 0; i < Ci; i++) a += wpw[o * Ci + i] * to_f32(x[((long long)b * Ci + i) * ncell + xy * plane + e]);
            gz[base + e] = to_f32(gy[base + e]) * gelu_grad_f(s + a);
        }
    }
}

// ---------------------------------------------------------------- launchers
template <typename T>
void launch_fwd_tz(const T *in, float2 *out, long long planes, const Dims &d, const Tables &tab, const float *wt,
                   hipStream_t st)
{
    const int Nz = d.N[2], Nt = d.N[3], Kz = d.K[2], Kt = d.K[3];
    const size_t lds = sizeof(float) * ((Nz * Nt + 1) & ~1) + sizeof(float2) * Nz * Kt;
    hipLaunchKernelGGL(k_fwd_tz<T>, dim3((unsigned)planes), dim3(256), lds, st, in, out, tab.cs[3], tab.cs[2], wt, Nz,
                       Nt, Kz, Kt);
}

size_t fwd_tz_lds(const Dims &d) { return sizeof(float) * ((d.N[2] * d.N[3] + 1) & ~1) + sizeof(float2) * d.N[2] * d.K[3]; }
size_t inv_zt_lds(const Dims &d) { return sizeof(float2) * (d.K[2] * d.K[3] + d.N[2] * d.K[3]); }

template <typename T>
void launch_inv_zt(int epi, const float2 *u, T *out, int C, const Dims &d, const Tables &tab, const float *wt,
                   const T *x, const float *wpw, const float *bpw, const float *gz, int Cx, int accumulate,
                   hipStream_t st)
{
    const size_t lds = inv_zt_lds(d);
    const dim3 grid((unsigned)((long long)d.B * d.N[0] * d.N[1]));
#define FNO_INV_ARGS u, out, tab.cs[3], tab.cs[2], wt, x, wpw, bpw, gz, C, Cx, d.N[0], d.N[1], d.N[2], d.N[3], d.K[2], d.K[3], accumulate
    if (epi == EPI_BLOCK)
        hipLaunchKernelGGL((k_inv_zt<T, EPI_BLOCK>), grid, dim3(256), lds, st, FNO_INV_ARGS);
    else if (epi == EPI_ADJ)
        hipLaunchKernelGGL((k_inv_zt<T, EPI_ADJ>), grid, dim3(256), lds, st, FNO_INV_ARGS);
    else
        hipLaunchKernelGGL((k_inv_zt<T, EPI_PLAIN>), grid, dim3(256), lds, st, FNO_INV_ARGS);
#undef FNO_INV_ARGS
}

template <typename T>
void launch_bwd_gz(const float2 *u, const T *x, const T *gy, float *gz, const Dims &d, const Tables &tab,
                   const float *wpw, const float *bpw, hipStream_t st)
{
    const size_t lds = inv_zt_lds(d);
    hipLaunchKernelGGL(k_bwd_gz<T>, dim3((unsigned)((long long)d.B * d.N[0] * d.N[1])), dim3(256), lds, st, u, x, gy,
                       gz, tab.cs[3], tab.cs[2], tab.wt_inv, wpw, bpw, d.Ci, d.Co, d.N[0], d.N[1], d.N[2], d.N[3],
                       d.K[2], d.K[3]);
}

#define FNO_INST(T)                                                                                                   \
    template void launch_fwd_tz<T>(const T *, float2 *, long long, const Dims &, const Tables &, const float *,       \
                                   hipStream_t);                                                                      \
    template void launch_inv_zt<T>(int, const float2 *, T *, int, const Dims &, const Tables &, const float *,       \
                                   const T *, const float *, const float *, const float *, int, int, hipStream_t);   \
    template void launch_bwd_gz<T>(const float2 *, const T *, const T *, float *, const Dims &, const Tables &,       \
                                   const float *, const float *, hipStream_t);
FNO_INST(float)
FNO_INST(__bf16)
#undef FNO_INST

}  // namespace fno
