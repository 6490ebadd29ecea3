// mode_kernels.hip -- kernels that act on truncated spectra: one-axis complex
// basis contractions (the x and y stages of the forward DFT, Alg. 2 line 1,
// and of its inverse/adjoint, Alg. 2 line 3), the per-mode channel mix
// (Alg. 2 line 2) and its gradients, and the deterministic reduction of the
// pointwise-weight gradient partial sums.
#include "fno_internal.h"

namespace fno {

// out[o][j][i] = sum_n E(j, n) in[o][n][i] along one axis of grid size N.
//   forward (inverse == 0): j runs over retained frequencies (Nout = K), n over
//     grid points (Nin = N), E = cos - i sin of tab[j][n]  (exp(-i theta));
//   inverse (inverse != 0): j runs over grid points (Nout = N), n over retained
//     frequencies (Nin = K), E = cos + i sin of tab[n][j]  (exp(+i theta)).
// Thread per output element; inner (contiguous) index fastest across threads.
__global__ void k_axis(const float2 *__restrict__ in, float2 *__restrict__ out, const float2 *__restrict__ tab,
                       long long outer, int Nin, int Nout, long long inner, int N, int inverse)
{
    const long long total = outer * Nout * inner;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long i = e % inner;
        const long long r = e / inner;
        const int j = (int)(r % Nout);
        const long long o = r / Nout;
        const float2 *src = in + o * Nin * inner + i;
        float re = 0.f, im = 0.f;
        for (int n = 0; n < Nin; n++) {
            const float2 c = inverse ? tab[(long long)n * N + j] : tab[(long long)j * N + n];
            const float s = inverse ? c.y : -c.y;
            const float2 v = src[(long long)n * inner];
            re += c.x * v.x - s * v.y;
            im += c.x * v.y + s * v.x;
        }
        out[e] = make_float2(re, im);
    }
}

// Y^[b][o][k] = sum_i X^[b][i][k] W[i][o][k]
__global__ void k_mix_fwd(const float2 *__restrict__ xh, const float2 *__restrict__ w, float2 *__restrict__ yh,
                          int B, int Ci, int Co, long long M)
{
    const long long total = (long long)B * Co * M;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long k = e % M;
        const long long r = e / M;
        const int o = (int)(r % Co), b = (int)(r / Co);
        float re = 0.f, im = 0.f;
        for (int i = 0; i < Ci; i++) {
            const float2 a = xh[((long long)b * Ci + i) * M + k];
            const float2 q = w[((long long)i * Co + o) * M + k];
            re += a.x * q.x - a.y * q.y;
            im += a.x * q.y + a.y * q.x;
        }
        yh[e] = make_float2(re, im);
    }
}

// gX^[b][i][k] = sum_o gY^[b][o][k] conj(W[i][o][k])
__global__ void k_mix_bwd_x(const float2 *__restrict__ gyh, const float2 *__restrict__ w, float2 *__restrict__ gxh,
                            int B, int Ci, int Co, long long M)
{
    const long long total = (long long)B * Ci * M;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long k = e % M;
        const long long r = e / M;
        const int i = (int)(r % Ci), b = (int)(r / Ci);
        float re = 0.f, im = 0.f;
        for (int o = 0; o < Co; o++) {
            const float2 g = gyh[((long long)b * Co + o) * M + k];
            const float2 q = w[((long long)i * Co + o) * M + k];
            re += g.x * q.x + g.y * q.y;
            im += g.y * q.x - g.x * q.y;
        }
        gxh[e] = make_float2(re, im);
    }
}

// gW[i][o][k] (+)= sum_b conj(X^[b][i][k]) gY^[b][o][k]
__global__ void k_mix_bwd_w(const float2 *__restrict__ xh, const float2 *__restrict__ gyh, float2 *__restrict__ gw,
                            int B, int Ci, int Co, long long M, int accumulate)
{
    const long long total = (long long)Ci * Co * M;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long k = e % M;
        const long long r = e / M;
        const int o = (int)(r % Co), i = (int)(r / Co);
        float re = 0.f, im = 0.f;
        for (int b = 0; b < B; b++) {
            const float2 a = xh[((long long)b * Ci + i) * M + k];
            const float2 g = gyh[((long long)b * Co + o) * M + k];
            re += a.x * g.x + a.y * g.y;
            im += a.x * g.y - a.y * g.x;
        }
        if (accumulate) {
            const float2 p = gw[e];
            re += p.x;
            im += p.y;
        }
        gw[e] = make_float2(re, im);
    }
}

// Weight access of the mix kernels: complex64 W, or W packed as two OCP e4m3 bytes per complex
// value with one power-of-two scale per (i, o) channel pair (fno_pack_weights, fp8.hip).
struct WComplex {
    const float2 *w;
    __device__ __forceinline__ float2 get(long long idx, int) const { return w[idx]; }
};
struct WFp8 {
    const unsigned short *q;
    const float *scale;
    __device__ __forceinline__ float2 get(long long idx, int io) const
    {
        const unsigned v = q[idx];
        const float sc = scale[io];
        return make_float2(e4m3_to_f32(v & 0xffu) * sc, e4m3_to_f32(v >> 8) * sc);
    }
};

// Tiled mix: a workgroup owns KM (64 or 32) consecutive retained modes; the batch's X^ (or gY^)
// of all channels at those modes is staged in LDS once, and the 256 / KM groups of KM lanes split
// the output channels.  The batch is held in registers (BM >= B), so every W element is read
// once (and, in the backward, gW written once) in coalesced rows of KM complex values while X^ /
// gY^ are read once.

// Y^[b][o][k] = sum_i X^[b][i][k] W[i][o][k]
template <int KM, int BM, typename WL>
__global__ void __launch_bounds__(256) k_mix_fwd_t(const float2 *__restrict__ xh, const WL w,
                                                   float2 *__restrict__ yh, int B, int Ci, int Co, long long M)
{
    constexpr int NG = 256 / KM;
    extern __shared__ float2 xs[];  // [b][i][KM]
    const int tk = threadIdx.x % KM, to = threadIdx.x / KM;
    const long long k0 = (long long)blockIdx.x * KM, k = k0 + tk;
    for (int e = threadIdx.x; e < B * Ci * KM; e += 256) {
        const int bi = e / KM, kk = e % KM;
        xs[e] = k0 + kk < M ? xh[(long long)bi * M + k0 + kk] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    if (k >= M) return;
    for (int o = to; o < Co; o += NG) {
        float re[BM], im[BM];
#pragma unroll
        for (int b = 0; b < BM; b++) re[b] = im[b] = 0.f;
        for (int i = 0; i < Ci; i++) {
            const float2 q = w.get(((long long)i * Co + o) * M + k, i * Co + o);
#pragma unroll
            for (int b = 0; b < BM; b++)
                if (b < B) {
                    const float2 a = xs[(b * Ci + i) * KM + tk];
                    re[b] += a.x * q.x - a.y * q.y;
                    im[b] += a.x * q.y + a.y * q.x;
                }
        }
#pragma unroll
        for (int b = 0; b < BM; b++)
            if (b < B) yh[((long long)b * Co + o) * M + k] = make_float2(re[b], im[b]);
    }
}

// gX^[b][i][k] = sum_o gY^[b][o][k] conj(W[i][o][k]) and gW[i][o][k] (+)= sum_b conj(X^[b][i][k]) gY^[b][o][k],
// one pass over W and gW (either output may be null; with gw null, xh may be null).
template <int KM, int BM, typename WL>
__global__ void __launch_bounds__(256) k_mix_bwd_t(const float2 *__restrict__ xh, const WL w,
                                                   const float2 *__restrict__ gyh, float2 *__restrict__ gxh,
                                                   float2 *__restrict__ gw, int B, int Ci, int Co, long long M,
                                                   int accumulate)
{
    constexpr int NG = 256 / KM;
    extern __shared__ float2 sh[];  // gs [b][o][KM], then xs [b][i][KM]
    float2 *gs = sh, *xs = sh + (size_t)B * Co * KM;
    const int tk = threadIdx.x % KM, ti = threadIdx.x / KM;
    const long long k0 = (long long)blockIdx.x * KM, k = k0 + tk;
    for (int e = threadIdx.x; e < B * Co * KM; e += 256) {
        const int bo = e / KM, kk = e % KM;
        gs[e] = k0 + kk < M ? gyh[(long long)bo * M + k0 + kk] : make_float2(0.f, 0.f);
    }
    if (gw)
        for (int e = threadIdx.x; e < B * Ci * KM; e += 256) {
            const int bi = e / KM, kk = e % KM;
            xs[e] = k0 + kk < M ? xh[(long long)bi * M + k0 + kk] : make_float2(0.f, 0.f);
        }
    __syncthreads();
    if (k >= M) return;
    for (int i = ti; i < Ci; i += NG) {
        float gre[BM], gim[BM];
#pragma unroll
        for (int b = 0; b < BM; b++) gre[b] = gim[b] = 0.f;
        for (int o = 0; o < Co; o++) {
            const long long wi = ((long long)i * Co + o) * M + k;
            if (gxh) {
                const float2 q = w.get(wi, i * Co + o);
#pragma unroll
                for (int b = 0; b < BM; b++)
                    if (b < B) {
                        const float2 g = gs[(b * Co + o) * KM + tk];
                        gre[b] += g.x * q.x + g.y * q.y;
                        gim[b] += g.y * q.x - g.x * q.y;
                    }
            }
            if (gw) {
                float re = 0.f, im = 0.f;
#pragma unroll
                for (int b = 0; b < BM; b++)
                    if (b < B) {
                        const float2 a = xs[(b * Ci + i) * KM + tk], g = gs[(b * Co + o) * KM + tk];
                        re += a.x * g.x + a.y * g.y;
                        im += a.x * g.y - a.y * g.x;
                    }
                if (accumulate) {
                    const float2 p0 = gw[wi];
                    re += p0.x;
                    im += p0.y;
                }
                gw[wi] = make_float2(re, im);
            }
        }
        if (gxh) {
#pragma unroll
            for (int b = 0; b < BM; b++)
                if (b < B) gxh[((long long)b * Ci + i) * M + k] = make_float2(gre[b], gim[b]);
        }
    }
}

// Pointwise-weight gradient partials: for chunk c of the flat (b, n) range and
// channel o, part[c][o][i] = sum gz[b][o][n] x[b][i][n] (i < Ci) and
// part[c][o][Ci] = sum gz[b][o][n].  One workgroup per (chunk, o).
template <typename T>
__global__ void __launch_bounds__(256) k_pw_wgrad_partial(const float *__restrict__ gz, const T *__restrict__ x,
                                                          float *__restrict__ part, int B, int Ci, int Co,
                                                          long long ncell, long long chunk)
{
    constexpr int MAXC = 64;
    const int o = blockIdx.y;
    const long long c = blockIdx.x;
    const long long total = (long long)B * ncell;
    const long long beg = c * chunk;
    const long long end = beg + chunk < total ? beg + chunk : total;
    float acc[MAXC + 1];
#pragma unroll
    for (int i = 0; i <= MAXC; i++) acc[i] = 0.f;
    for (long long e = beg + threadIdx.x; e < end; e += blockDim.x) {
        const long long b = e / ncell, n = e % ncell;
        const float g = gz[(b * Co + o) * ncell + n];
        acc[MAXC] += g;
#pragma unroll
        for (int i = 0; i < MAXC; i++)
            if (i < Ci) acc[i] += g * to_f32(x[(b * Ci + i) * ncell + n]);
    }
    __shared__ float red[256];
#pragma unroll
    for (int i = 0; i <= MAXC; i++) {
        if (i <= Ci) {  // Ci is uniform across the workgroup
            red[threadIdx.x] = (i == Ci) ? acc[MAXC] : acc[i];
            __syncthreads();
            for (int s = 128; s > 0; s >>= 1) {
                if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
                __syncthreads();
            }
            if (threadIdx.x == 0) part[(c * Co + o) * (Ci + 1) + i] = red[0];
            __syncthreads();
        }
    }
}

// gw_pw[o][i] (+)= sum_c part[c][o][i]; gb[o] (+)= sum_c part[c][o][Ci].
// One workgroup per (o, i) entry; a fixed-order tree over the chunks keeps the
// result deterministic.
__global__ void __launch_bounds__(256) k_pw_wgrad_reduce(const float *__restrict__ part, float *__restrict__ gwpw,
                                                         float *__restrict__ gb, int Ci, int Co, int nchunk,
                                                         int accumulate)
{
    const int e = blockIdx.x;
    const int o = e / (Ci + 1), i = e % (Ci + 1);
    const long long stride = (long long)Co * (Ci + 1);
    float s = 0.f;
    for (int c = threadIdx.x; c < nchunk; c += 256) s += part[c * stride + e];
    __shared__ float red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        s = red[0];
        if (i < Ci) {
            if (gwpw) gwpw[o * Ci + i] = (accumulate ? gwpw[o * Ci + i] : 0.f) + s;
        } else {
            if (gb) gb[o] = (accumulate ? gb[o] : 0.f) + s;
        }
    }
}

// ---------------------------------------------------------------- launchers
static inline int grid_for(long long total, int block)
{
    long long g = (total + block - 1) / block;
    if (g > 1048576) g = 1048576;
    return (int)(g < 1 ? 1 : g);
}

void launch_axis(const float2 *in, float2 *out, const float2 *tab, long long outer, int Nin, int Nout,
                 long long inner, int N, int inverse, hipStream_t st)
{
    hipLaunchKernelGGL(k_axis, dim3(grid_for(outer * Nout * inner, 256)), dim3(256), 0, st, in, out, tab, outer, Nin,
                       Nout, inner, N, inverse);
}

// Tiled mix launch: the mode tile (64, else 32) whose LDS stage fits 64 KB, for B <= 8; 0 if none.
static int mix_tile(int B, int C)
{
    if (B > 8) return 0;
    if (sizeof(float2) * (size_t)B * C * 64 <= 64 * 1024) return 64;
    if (sizeof(float2) * (size_t)B * C * 32 <= 64 * 1024) return 32;
    return 0;
}

// Whether both mix directions run on the tiled kernels (the only ones that read packed weights).
bool mix_tiled(int B, int Ci, int Co) { return mix_tile(B, Ci) != 0 && mix_tile(B, Co + Ci) != 0; }

template <int KM, typename WL>
static void launch_mix_fwd_km(const float2 *xh, const WL w, float2 *yh, int B, int Ci, int Co, long long M,
                              hipStream_t st)
{
    const size_t lds = sizeof(float2) * (size_t)B * Ci * KM;
    const dim3 grid((unsigned)((M + KM - 1) / KM));
    if (B <= 1) hipLaunchKernelGGL((k_mix_fwd_t<KM, 1, WL>), grid, dim3(256), lds, st, xh, w, yh, B, Ci, Co, M);
    else if (B <= 2) hipLaunchKernelGGL((k_mix_fwd_t<KM, 2, WL>), grid, dim3(256), lds, st, xh, w, yh, B, Ci, Co, M);
    else if (B <= 4) hipLaunchKernelGGL((k_mix_fwd_t<KM, 4, WL>), grid, dim3(256), lds, st, xh, w, yh, B, Ci, Co, M);
    else hipLaunchKernelGGL((k_mix_fwd_t<KM, 8, WL>), grid, dim3(256), lds, st, xh, w, yh, B, Ci, Co, M);
}

template <int KM, typename WL>
static void launch_mix_bwd_km(const float2 *xh, const WL w, const float2 *gyh, float2 *gxh, float2 *gw, int B,
                              int Ci, int Co, long long M, int accumulate, hipStream_t st)
{
    const size_t lds = sizeof(float2) * (size_t)B * (Co + (gw ? Ci : 0)) * KM;
    const dim3 grid((unsigned)((M + KM - 1) / KM));
#define FNO_MIX_BWD(BM_)                                                                                         \
    hipLaunchKernelGGL((k_mix_bwd_t<KM, BM_, WL>), grid, dim3(256), lds, st, xh, w, gyh, gxh, gw, B, Ci, Co, M, \
                       accumulate)
    if (B <= 1) FNO_MIX_BWD(1);
    else if (B <= 2) FNO_MIX_BWD(2);
    else if (B <= 4) FNO_MIX_BWD(4);
    else FNO_MIX_BWD(8);
#undef FNO_MIX_BWD
}

// w: complex64 weights, or (wq != null) packed e4m3 weights wq with per-channel-pair scales wscale.
void launch_mix_fwd(const float2 *xh, const float2 *w, const unsigned short *wq, const float *wscale, float2 *yh,
                    int B, int Ci, int Co, long long M, hipStream_t st)
{
    const int km = mix_tile(B, Ci);
    if (wq) {
        const WFp8 wl{wq, wscale};
        if (km == 64) return launch_mix_fwd_km<64>(xh, wl, yh, B, Ci, Co, M, st);
        return launch_mix_fwd_km<32>(xh, wl, yh, B, Ci, Co, M, st);  // the plan checked mix_tiled
    }
    const WComplex wl{w};
    if (km == 64) return launch_mix_fwd_km<64>(xh, wl, yh, B, Ci, Co, M, st);
    if (km == 32) return launch_mix_fwd_km<32>(xh, wl, yh, B, Ci, Co, M, st);
    hipLaunchKernelGGL(k_mix_fwd, dim3(grid_for((long long)B * Co * M, 256)), dim3(256), 0, st, xh, w, yh, B, Ci, Co, M);
}

void launch_mix_bwd(const float2 *xh, const float2 *w, const unsigned short *wq, const float *wscale,
                    const float2 *gyh, float2 *gxh, float2 *gw, int B, int Ci, int Co, long long M, int accumulate,
                    hipStream_t st)
{
    const int km = mix_tile(B, Co + (gw ? Ci : 0));
    if (wq) {
        const WFp8 wl{wq, wscale};
        if (km == 64) return launch_mix_bwd_km<64>(xh, wl, gyh, gxh, gw, B, Ci, Co, M, accumulate, st);
        return launch_mix_bwd_km<32>(xh, wl, gyh, gxh, gw, B, Ci, Co, M, accumulate, st);
    }
    const WComplex wl{w};
    if (km == 64) return launch_mix_bwd_km<64>(xh, wl, gyh, gxh, gw, B, Ci, Co, M, accumulate, st);
    if (km == 32) return launch_mix_bwd_km<32>(xh, wl, gyh, gxh, gw, B, Ci, Co, M, accumulate, st);
    if (gxh)
        hipLaunchKernelGGL(k_mix_bwd_x, dim3(grid_for((long long)B * Ci * M, 256)), dim3(256), 0, st, gyh, w, gxh, B,
                           Ci, Co, M);
    if (gw)
        hipLaunchKernelGGL(k_mix_bwd_w, dim3(grid_for((long long)Ci * Co * M, 256)), dim3(256), 0, st, xh, gyh, gw, B,
                           Ci, Co, M, accumulate);
}

int pw_wgrad_chunks(long long total) { return (int)((total + 65535) / 65536); }

template <typename T>
void launch_pw_wgrad(const float *gz, const T *x, float *part, float *gwpw, float *gb, int B, int Ci, int Co,
                     long long ncell, int accumulate, hipStream_t st)
{
    const long long total = (long long)B * ncell;
    const long long chunk = 65536;
    const int nchunk = pw_wgrad_chunks(total);
    hipLaunchKernelGGL(k_pw_wgrad_partial<T>, dim3(nchunk, Co), dim3(256), 0, st, gz, x, part, B, Ci, Co, ncell, chunk);
    hipLaunchKernelGGL(k_pw_wgrad_reduce, dim3(Co * (Ci + 1)), dim3(256), 0, st, part, gwpw, gb, Ci, Co, nchunk,
                       accumulate);
}

void launch_pw_reduce(const float *part, float *gwpw, float *gb, int Ci, int Co, int nchunk, int accumulate,
                      hipStream_t st)
{
    hipLaunchKernelGGL(k_pw_wgrad_reduce, dim3(Co * (Ci + 1)), dim3(256), 0, st, part, gwpw, gb, Ci, Co, nchunk,
                       accumulate);
}

template void launch_pw_wgrad<float>(const float *, const float *, float *, float *, float *, int, int, int, long long,
                                     int, hipStream_t);
template void launch_pw_wgrad<__bf16>(const float *, const __bf16 *, float *, float *, float *, int, int, int,
                                      long long, int, hipStream_t);

}  // namespace fno
