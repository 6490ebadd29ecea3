// glue.hip -- the network around the FNO blocks (Alg. 1): the encoder (lifting
// 1x1 + GELU), the two-layer decoder (projection 1x1 -> GELU -> 1x1) and the
// mean-squared-error loss, forward and backward.  Everything is pointwise in
// space, so every kernel streams points; the decoder's hidden layer (H = 128
// channels per point) is never written to memory.
//
// Decoder on the matrix cores, per tile of 16 points p and one wave (details at the kernels):
//   Z1[h][p]  = sum_ci W1[h][ci] x[ci][p] + b1[h]          (A = W1 fragments, B = x)
//   Hd[h][p]  = GELU(Z1)                                    (accumulator rows h = K rows of the next product)
//   y[o][p]   = sum_h W2[o][h] Hd[h][p] + b2[o]
// backward, per tile:
//   gH[h][p]  = (sum_o W2[o][h] gy[o][p]) GELU'(Z1[h][p])
//   gx[ci][p] = sum_h W1[h][ci] gH[h][p]
//   gW1[h][ci] += sum_p gH[h][p] x[ci][p], gW2[o][h] += sum_p gy[o][p] Hd[h][p]
// Tiles change between "point across lanes" and "channel across lanes" by a product with the
// identity fragment on the matrix cores, not through memory.
#include <algorithm>
#include <atomic>

#include "fno_internal.h"
#include "mfma_common.h"

namespace fno {

// ---------------------------------------------------------------- shared helpers
// GELU of the encoder and decoder: the logistic form for bfloat16 activations (their values are
// rounded to bfloat16, relative step 2^-8), the Abramowitz-Stegun erf for float.
template <typename T> __device__ __forceinline__ float glue_gelu(float u)
{
    return sizeof(T) == 2 ? gelu_lg(u) : gelu_fast(u);
}
template <typename T> __device__ __forceinline__ float glue_gelu_grad(float u)
{
    return sizeof(T) == 2 ? gelu_grad_lg(u) : gelu_grad_fast(u);
}
// GELU(u) and GELU'(u) from one evaluation.
template <typename T> __device__ __forceinline__ void glue_gelu2(float u, float &g, float &dg)
{
    if (sizeof(T) == 2) {
        const float u2 = u * u;
        const float P = phi_logistic(u, u2);
        g = u * P;
        dg = fmaf(u * 0.39894228040143268f, __builtin_amdgcn_exp2f(u2 * -0.72134752044448170f), P);
    } else {
        gelu_as(u, g, dg);
    }
}

// Four consecutive points p .. p + 3 of one channel row as floats; zeros past n (the row's
// length).  VEC: the row start and p are multiples of 4 elements, so one aligned vector access.
template <bool VEC, typename T> __device__ __forceinline__ void ld4(const T *row, long long p, long long n, float (&v)[4])
{
    if (VEC && p + 4 <= n) {
        load4(row + p, v);
    } else {
#pragma unroll
        for (int j = 0; j < 4; j++) v[j] = p + j < n ? to_f32(row[p + j]) : 0.f;
    }
}
template <bool VEC, typename T> __device__ __forceinline__ void st4(T *row, long long p, long long n, const float (&v)[4])
{
    if (VEC && p + 4 <= n) {
        store4(row + p, v);
    } else {
#pragma unroll
        for (int j = 0; j < 4; j++)
            if (p + j < n) row[p + j] = from_f32<T>(v[j]);
    }
}

// ---------------------------------------------------------------- lifting
// y[b][o][n] = GELU(sum_i w[o][i] x[b][i][n] + bias[o]).  A thread takes 4 consecutive points of
// one batch element for all channels; work items of 1024 points, grid-strided.  CI: the input
// channel count (the encoder's few data channels, at most 8).

template <typename T, int CI, bool VEC>
__global__ void __launch_bounds__(256) k_lift_fwd(const T *__restrict__ x, T *__restrict__ y,
                                                  const float *__restrict__ w, const float *__restrict__ bias, int B,
                                                  int Co, long long N)
{
    const long long nchunk = (N + 1023) / 1024, items = (long long)B * nchunk;
    for (long long it = blockIdx.x; it < items; it += gridDim.x) {
        const long long b = it / nchunk, p = (it - b * nchunk) * 1024 + 4 * threadIdx.x;
        if (p >= N) continue;
        float xv[CI][4];
#pragma unroll
        for (int i = 0; i < CI; i++) ld4<VEC>(x + (b * CI + i) * N, p, N, xv[i]);
        for (int o = 0; o < Co; o++) {
            const float b0 = bias ? bias[o] : 0.f;
            float z[4] = {b0, b0, b0, b0};
#pragma unroll
            for (int i = 0; i < CI; i++) {
                const float wv = w[o * CI + i];
#pragma unroll
                for (int j = 0; j < 4; j++) z[j] = fmaf(wv, xv[i][j], z[j]);
            }
#pragma unroll
            for (int j = 0; j < 4; j++) z[j] = glue_gelu<T>(z[j]);
            st4<VEC>(y + (b * Co + o) * N, p, N, z);
        }
    }
}

// The derivative used by the encoder's backward: for bfloat16 that of the logistic form itself
// (as in the decoder), for float the A&S form.
template <typename T> __device__ __forceinline__ float lift_gelu_grad(float u)
{
    return sizeof(T) == 2 ? gelu_grad_lgd(u) : gelu_grad_fast(u);
}

// Partial sums of gw[o][i] = sum gz[o] x[i] and gb[o] = sum gz[o], gz = gy GELU'(w x + b), per
// block: part[block][o * Ci + i] and part[block][Co * Ci + o].  Output channels are taken in
// groups of OG (x is read once per group, gy once in all); each thread sums over its points, then
// the block in a fixed order (wave shuffles, then the four waves).
template <typename T, int CI, bool VEC>
__global__ void __launch_bounds__(256) k_lift_bwd(const T *__restrict__ x, const T *__restrict__ gy,
                                                  const float *__restrict__ w, const float *__restrict__ bias,
                                                  float *__restrict__ part, int B, int Co, long long N)
{
    constexpr int OG = 8;
    const long long nchunk = (N + 1023) / 1024, items = (long long)B * nchunk;
    const size_t row = (size_t)Co * (CI + 1);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __shared__ float red[4][OG * (CI + 1)];
    for (int o0 = 0; o0 < Co; o0 += OG) {
        float acc[OG][CI + 1];
#pragma unroll
        for (int k = 0; k < OG; k++)
#pragma unroll
            for (int i = 0; i <= CI; i++) acc[k][i] = 0.f;
        for (long long it = blockIdx.x; it < items; it += gridDim.x) {
            const long long b = it / nchunk, p = (it - b * nchunk) * 1024 + 4 * threadIdx.x;
            if (p >= N) continue;
            float xv[CI][4];
#pragma unroll
            for (int i = 0; i < CI; i++) ld4<VEC>(x + (b * CI + i) * N, p, N, xv[i]);
#pragma unroll
            for (int k = 0; k < OG; k++) {
                const int o = o0 + k;
                if (o < Co) {
                    const float b0 = bias ? bias[o] : 0.f;
                    float z[4] = {b0, b0, b0, b0}, g[4];
#pragma unroll
                    for (int i = 0; i < CI; i++) {
                        const float wo = w[o * CI + i];
#pragma unroll
                        for (int j = 0; j < 4; j++) z[j] = fmaf(wo, xv[i][j], z[j]);
                    }
                    ld4<VEC>(gy + (b * Co + o) * N, p, N, g);  // zero past N
#pragma unroll
                    for (int j = 0; j < 4; j++) {
                        const float gz = g[j] * lift_gelu_grad<T>(z[j]);
#pragma unroll
                        for (int i = 0; i < CI; i++) acc[k][i] = fmaf(gz, xv[i][j], acc[k][i]);
                        acc[k][CI] += gz;
                    }
                }
            }
        }
        // block sum: butterfly over the wave's 64 lanes, then the 4 waves in order
#pragma unroll
        for (int k = 0; k < OG; k++)
#pragma unroll
            for (int i = 0; i <= CI; i++) {
                float v = acc[k][i];
#pragma unroll
                for (int sh = 1; sh < 64; sh <<= 1) v += __shfl_xor(v, sh);
                if (lane == 0) red[wv][k * (CI + 1) + i] = v;
            }
        __syncthreads();
        for (int e = threadIdx.x; e < OG * (CI + 1); e += 256) {
            const int k = e / (CI + 1), i = e - k * (CI + 1), o = o0 + k;
            if (o < Co) {
                const float v = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
                part[(size_t)blockIdx.x * row + (i == CI ? (size_t)Co * CI + o : (size_t)o * CI + i)] = v;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- projection
struct ProjArgs {
    int B, Ci, H, Co;
    long long N;
    int accumulate;
};

// Identity B fragment: lane (c, g), element j is 1 where 4 g + j == c.  mma16(a, I, 0) returns,
// in accumulator layout, the matrix whose A fragment a is: element r of lane (c, g) becomes row
// 4 g + r, column c of that matrix, i.e. what lane (4 g + r, c / 4) held in element c % 4.  So
// a tile held with one index across lanes and the other across elements comes back with the two
// roles swapped, exactly (one nonzero product per sum).
template <typename T> __device__ __forceinline__ typename OpOf<T>::type op_identity(int c, int g)
{
    return op_from4<T>(4 * g == c ? 1.f : 0.f, 4 * g + 1 == c ? 1.f : 0.f, 4 * g + 2 == c ? 1.f : 0.f,
                       4 * g + 3 == c ? 1.f : 0.f);
}

// The decoder's first-layer weights as A fragments, the bias folded in as input channel Ci (the
// input tile carries a row of ones there): A[h = 16 m + c][k = 16 q + 4 g + j].
template <typename T, int MCI, int MH>
__device__ __forceinline__ void proj_w1_frags(const float *w1, const float *b1, int H, int Ci, int c, int g,
                                              typename OpOf<T>::type (&aw1)[MH][MCI])
{
#pragma unroll
    for (int m = 0; m < MH; m++)
#pragma unroll
        for (int q = 0; q < MCI; q++) {
            float v[4];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int h = 16 * m + c, ci = 16 * q + 4 * g + j;
                v[j] = h >= H ? 0.f : ci < Ci ? w1[h * Ci + ci] : (ci == Ci && b1) ? b1[h] : 0.f;
            }
            aw1[m][q] = op_from4<T>(v[0], v[1], v[2], v[3]);
        }
}

// Input tile of 16 points p0 .. p0 + 15 in A layout: lane (c, g) holds channel 16 q + c at points
// p0 + 4 g + j, with channel Ci a row of ones (the bias input) and zeros past Ci or N.  `rows[q]`
// is the lane's channel row (clamped to a real row: every address is inside the tensor) and
// `sel[q]` its kind: 0 data, 1 ones, 2 zeros.  FULL: the whole tile is inside the row and the
// row starts on 4 elements, so the 4 points are one vector load whose bits are the operand.
template <typename T, int MCI, bool FULL>
__device__ __forceinline__ void proj_load_x(const T *const (&rows)[MCI], const int (&sel)[MCI], int p0, int N, int g,
                                            typename OpOf<T>::type (&xa)[MCI])
{
    typedef typename OpOf<T>::type Op;
    const int p = p0 + 4 * g;
#pragma unroll
    for (int q = 0; q < MCI; q++) {
        Op v;
        if (FULL) {
            v = *reinterpret_cast<const Op *>(rows[q] + p);
        } else {
            float f[4];
#pragma unroll
            for (int j = 0; j < 4; j++) f[j] = p + j < N ? to_f32(rows[q][p + j]) : 0.f;
            v = op_from4<T>(f[0], f[1], f[2], f[3]);
        }
        const Op one = op_from4<T>(1.f, 1.f, 1.f, 1.f);
        xa[q] = sel[q] == 0 ? v : sel[q] == 1 ? one : op_zero<T>();
    }
}

// Per-lane channel rows of batch element b for proj_load_x (lane channel 16 q + c).
template <typename T, int MCI>
__device__ __forceinline__ void proj_rows(const T *x, int b, int Ci, int N, int c, const T *(&rows)[MCI],
                                          int (&sel)[MCI])
{
#pragma unroll
    for (int q = 0; q < MCI; q++) {
        const int ci = 16 * q + c;
        rows[q] = x + ((long long)b * Ci + min(ci, Ci - 1)) * N;
        sel[q] = ci < Ci ? 0 : ci == Ci ? 1 : 2;
    }
}

// Z1 chunk m: sum over the K chunks q of aw1[m][q] bx[q], two chunks per product.  One accumulation
// chain never mixes the 16- and 32-deep instructions (an odd count above one takes a zero chunk):
// the compiler's wait states between a 32-deep product and a 16-deep one reading its result as
// the accumulator were measured to give wrong sums.
template <typename Op, int MCI>
__device__ __forceinline__ f4v proj_z(const Op (&aw)[MCI], const Op (&bx)[MCI])
{
    if (MCI == 1) return mma16(aw[0], bx[0], f4_zero());
    f4v z = f4_zero();
#pragma unroll
    for (int q = 0; q + 1 < MCI; q += 2) z = mma32(aw[q], aw[q + 1], bx[q], bx[q + 1], z);
    if (MCI % 2) z = mma32(aw[MCI - 1], op_zero_of(aw[0]), bx[MCI - 1], op_zero_of(bx[0]), z);
    return z;
}

// Forward of the decoder (Co == 1); one wave per 16-point tile, tiles of one batch element strided
// over the waves of the grid:
//   X   [ci][p]  tile loaded with ci across lanes (vector loads along p), turned into the B
//                fragment (p across lanes, ci along K) by one identity product per K chunk;
//   Z1  [h][p]   = W1' X   (W1' = [W1 | b1]; per 16-row chunk m of h)
//   y   [o][p]  += W2[o][h chunk] GELU(Z1 chunk)     (the accumulator is the next B fragment)
// VEC: N is a multiple of 4 (rows start on 4 elements); the last tile of a row may be partial.
template <typename T, int MCI, bool VEC>
__global__ void __launch_bounds__(256) k_proj_fwd(const T *__restrict__ x, T *__restrict__ y,
                                                  const float *__restrict__ w1, const float *__restrict__ b1,
                                                  const float *__restrict__ w2, const float *__restrict__ b2,
                                                  ProjArgs a)
{
    typedef typename OpOf<T>::type Op;
    constexpr int MH = 8;
    const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
    const int N = (int)a.N, ntile = (N + 15) / 16;
    const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int nwaves = (int)((gridDim.x * blockDim.x) >> 6);
    Op aw1[MH][MCI], aw2[MH];
    proj_w1_frags<T, MCI, MH>(w1, b1, a.H, a.Ci, c, g, aw1);
#pragma unroll
    for (int m = 0; m < MH; m++) {
        float v[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int h = 16 * m + 4 * g + j;
            v[j] = (c < a.Co && h < a.H) ? w2[c * a.H + h] : 0.f;  // A[o = c][h]
        }
        aw2[m] = op_from4<T>(v[0], v[1], v[2], v[3]);
    }
    const Op eye = op_identity<T>(c, g);
    const float bias2 = b2 ? b2[0] : 0.f;
    for (int b = 0; b < a.B; b++) {
        const T *rows[MCI];
        int sel[MCI];
        proj_rows<T, MCI>(x, b, a.Ci, N, c, rows, sel);
        T *yrow = y + (long long)b * N;
        Op xa[MCI];
        if (wave < ntile) {
            if (VEC && 16 * wave + 16 <= N) proj_load_x<T, MCI, true>(rows, sel, 16 * wave, N, g, xa);
            else proj_load_x<T, MCI, false>(rows, sel, 16 * wave, N, g, xa);
        }
        for (int t = wave; t < ntile; t += nwaves) {
            const int p0 = 16 * t;
            Op bx[MCI];
#pragma unroll
            for (int q = 0; q < MCI; q++) bx[q] = to_op<T>(mma16(xa[q], eye, f4_zero()));
            const int tn = t + nwaves;  // next tile's input, loaded while this one computes
            if (tn < ntile) {
                if (VEC && 16 * tn + 16 <= N) proj_load_x<T, MCI, true>(rows, sel, 16 * tn, N, g, xa);
                else proj_load_x<T, MCI, false>(rows, sel, 16 * tn, N, g, xa);
            }
            f4v yo = f4_zero();
#pragma unroll
            for (int m = 0; m < MH; m += 2) {
                f4v hd0, hd1;
                const f4v z0 = proj_z<Op, MCI>(aw1[m], bx), z1 = proj_z<Op, MCI>(aw1[m + 1], bx);
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    hd0[r] = glue_gelu<T>(z0[r]);
                    hd1[r] = glue_gelu<T>(z1[r]);
                }
                yo = mma32(aw2[m], aw2[m + 1], to_op<T>(hd0), to_op<T>(hd1), yo);
            }
            // yo[r] = y[o = 4 g + r][p0 + c]: output channel 0 is g == 0, r == 0
            if (g == 0 && p0 + c < N) yrow[p0 + c] = from_f32<T>(yo[0] + bias2);
        }
    }
}

// GELU(u) and a derivative for the decoder's backward: bfloat16 takes the derivative of the
// logistic form itself, d/du [u P(u)] = P + u P (1 - P) (1.5976 + 0.21168 u^2) (within 7.9e-4 of
// the exact GELU', one exponential and one reciprocal per value); float the A&S pair.
template <typename T> __device__ __forceinline__ void proj_gelu2(float u, float &g, float &dg)
{
    if (sizeof(T) == 2) {
        const float u2 = u * u;
        const float P = phi_logistic(u, u2);
        g = u * P;
        dg = fmaf(u * fmaf(-P, P, P), fmaf(u2, 0.21168f, 1.5976f), P);
    } else {
        gelu_as(u, g, dg);
    }
}

// Backward of the decoder (Co == 1), per 16-point tile, with gH' = gy GELU'(Z1) (the factor
// W2[0][h] is carried by the weights instead, see below):
//   gx^T [p][ci] += gH'^T[p][h chunk] (W2 W1)[h chunk][ci]  (gH' accumulator as A: p across lanes)
//   gW1' [h][ci] += gH'[h][p] X^T[p][ci]                   (gH' turned by an identity product;
//                                                           column ci = Ci, the ones row, is gb1')
//   gW2  [h]     += sum_p gy[p] GELU(Z1[h][p])             (per lane, summed over lanes at the end)
// so gx^T lands with ci across lanes and 4 consecutive points per lane (vector stores), and the
// input tile is read once per wave.  A pair of waves shares each tile, wave hh of the pair taking
// hidden rows 64 hh .. 64 hh + 63 (half the weight fragments and accumulators each, so three
// waves fit a SIMD); the odd wave hands its part of gx^T to the even one through LDS (double
// buffered, one barrier per tile, so every wave of the block runs the same number of tiles).
// Per pair partials, multiplied by W2[0][h] at the end: gW1 [H][Ci], gb1 [H], gW2 [H], gb2 [1] at
// part[(block * 2 + pair) * proj_part_len], the pair's waves writing disjoint rows h.
template <typename T, int MCI, bool VEC>
__global__ void __launch_bounds__(256) k_proj_bwd(const T *__restrict__ x, const T *__restrict__ gy,
                                                  T *__restrict__ gx, const float *__restrict__ w1,
                                                  const float *__restrict__ b1, const float *__restrict__ w2,
                                                  float *__restrict__ part, ProjArgs a)
{
    typedef typename OpOf<T>::type Op;
    constexpr int MH = 4;  // 16-row chunks of h per wave
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), g = lane >> 4,
              c = lane & 15;
    const int pair = w >> 1, hh = w & 1, h0 = 64 * hh;
    const int N = (int)a.N, ntile = (N + 15) / 16;
    const int H = a.H, Ci = a.Ci;
    __shared__ f4v xch[2][2][MCI][64];  // [buffer][pair][q][lane]
    Op aw1[MH][MCI], bw1[MH][MCI];
#pragma unroll
    for (int m = 0; m < MH; m++)
#pragma unroll
        for (int q = 0; q < MCI; q++) {
            float v[4], u[4];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                // A[h = h0 + 16 m + c][k = 16 q + 4 g + j] = [W1 | b1]
                const int h = h0 + 16 * m + c, ci = 16 * q + 4 * g + j;
                v[j] = h >= H ? 0.f : ci < Ci ? w1[h * Ci + ci] : (ci == Ci && b1) ? b1[h] : 0.f;
                // B[h = h0 + 16 m + 4 g + j][ci = 16 q + c] = W2[0][h] W1[h][ci]
                const int h2 = h0 + 16 * m + 4 * g + j, ci2 = 16 * q + c;
                u[j] = (h2 < H && ci2 < Ci) ? w2[h2] * w1[h2 * Ci + ci2] : 0.f;
            }
            aw1[m][q] = op_from4<T>(v[0], v[1], v[2], v[3]);
            bw1[m][q] = op_from4<T>(u[0], u[1], u[2], u[3]);
        }
    const Op eye = op_identity<T>(c, g);
    f4v gw1[MH][MCI];
    float gw2[MH][4], gb2 = 0.f;
#pragma unroll
    for (int m = 0; m < MH; m++) {
#pragma unroll
        for (int q = 0; q < MCI; q++) gw1[m][q] = f4_zero();
#pragma unroll
        for (int r = 0; r < 4; r++) gw2[m][r] = 0.f;
    }
    int buf = 0;
    for (int b = 0; b < a.B; b++) {
        const T *rows[MCI];
        int sel[MCI];
        proj_rows<T, MCI>(x, b, Ci, N, c, rows, sel);
        const T *gyrow = gy + (long long)b * N;
        T *gxrow[MCI];
#pragma unroll
        for (int q = 0; q < MCI; q++) gxrow[q] = gx + ((long long)b * Ci + min(16 * q + c, Ci - 1)) * N;
        for (int t0 = 2 * (int)blockIdx.x; t0 < ntile; t0 += 2 * (int)gridDim.x) {
            const int t = t0 + pair, p0 = 16 * t;
            const bool valid = t < ntile;  // wave-uniform
            const bool full = VEC && p0 + 16 <= N;
            f4v gxt[MCI];
#pragma unroll
            for (int q = 0; q < MCI; q++) gxt[q] = f4_zero();
            if (valid) {
                Op xcur[MCI];
                if (full) proj_load_x<T, MCI, true>(rows, sel, p0, N, g, xcur);
                else proj_load_x<T, MCI, false>(rows, sel, p0, N, g, xcur);
                const float gyp = p0 + c < N ? to_f32(gyrow[p0 + c]) : 0.f;  // gy[p0 + c], zero past N
                Op bx[MCI];
#pragma unroll
                for (int q = 0; q < MCI; q++) bx[q] = to_op<T>(mma16(xcur[q], eye, f4_zero()));
                if (hh == 0) gb2 += gyp;
#pragma unroll
                for (int m = 0; m < MH; m += 2) {
                    Op ghop[2];
#pragma unroll
                    for (int u = 0; u < 2; u++) {
                        const f4v z = proj_z<Op, MCI>(aw1[m + u], bx);
                        f4v gh;
#pragma unroll
                        for (int r = 0; r < 4; r++) {
                            float hd, dg;
                            proj_gelu2<T>(z[r], hd, dg);
                            gh[r] = gyp * dg;
                            gw2[m + u][r] = fmaf(gyp, hd, gw2[m + u][r]);
                        }
                        ghop[u] = to_op<T>(gh);  // gH'[h = h0 + 16 (m + u) + 4 g + r][p0 + c]
                        // gH'[h0 + 16 (m + u) + c][p0 + 4 g + j]
                        const Op ght = to_op<T>(mma16(ghop[u], eye, f4_zero()));
#pragma unroll
                        for (int q = 0; q < MCI; q++) gw1[m + u][q] = mma16(ght, xcur[q], gw1[m + u][q]);
                    }
#pragma unroll
                    for (int q = 0; q < MCI; q++) gxt[q] = mma32(ghop[0], ghop[1], bw1[m][q], bw1[m + 1][q], gxt[q]);
                }
                if (hh == 1) {
#pragma unroll
                    for (int q = 0; q < MCI; q++) xch[buf][pair][q][lane] = gxt[q];
                }
            }
            __syncthreads();
            if (valid && hh == 0) {
                // gx[ci = 16 q + c][p0 + 4 g + r] = both halves of the sum over h
                const int p = p0 + 4 * g;
#pragma unroll
                for (int q = 0; q < MCI; q++) {
                    if (sel[q] != 0) continue;
                    const f4v o = xch[buf][pair][q][lane];
                    float v[4];
                    if (a.accumulate) {
                        if (full) load4(gxrow[q] + p, v);
                        else {
#pragma unroll
                            for (int r = 0; r < 4; r++) v[r] = p + r < N ? to_f32(gxrow[q][p + r]) : 0.f;
                        }
#pragma unroll
                        for (int r = 0; r < 4; r++) v[r] += gxt[q][r] + o[r];
                    } else {
#pragma unroll
                        for (int r = 0; r < 4; r++) v[r] = gxt[q][r] + o[r];
                    }
                    if (full) store4(gxrow[q] + p, v);
                    else {
#pragma unroll
                        for (int r = 0; r < 4; r++)
                            if (p + r < N) gxrow[q][p + r] = from_f32<T>(v[r]);
                    }
                }
            }
            buf ^= 1;
        }
    }
    float *pw = part + ((size_t)blockIdx.x * 2 + pair) * ((size_t)H * Ci + 2 * H + 1);
    // gw1[m][q][r] = gW1'[h = h0 + 16 m + 4 g + r][ci = 16 q + c]; column Ci holds gb1'
#pragma unroll
    for (int m = 0; m < MH; m++)
#pragma unroll
        for (int q = 0; q < MCI; q++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int h = h0 + 16 * m + 4 * g + r, ci = 16 * q + c;
                if (h < H) {
                    if (ci < Ci) pw[h * Ci + ci] = w2[h] * gw1[m][q][r];
                    else if (ci == Ci) pw[(size_t)H * Ci + h] = w2[h] * gw1[m][q][r];
                }
            }
    // gw2[m][r]: h = h0 + 16 m + 4 g + r, summed over this lane's points; add the 16 point lanes c
#pragma unroll
    for (int m = 0; m < MH; m++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
            float s = gw2[m][r];
            s += __shfl_xor(s, 1);
            s += __shfl_xor(s, 2);
            s += __shfl_xor(s, 4);
            s += __shfl_xor(s, 8);
            const int h = h0 + 16 * m + 4 * g + r;
            if (c == 0 && h < H) pw[(size_t)H * Ci + H + h] = s;
        }
    float s = gb2;  // every point lane c carries its gy once per g group: take g == 0
    s += __shfl_xor(s, 1);
    s += __shfl_xor(s, 2);
    s += __shfl_xor(s, 4);
    s += __shfl_xor(s, 8);
    if (hh == 0 && lane == 0) pw[(size_t)H * Ci + 2 * H] = s;
}

// out[e] (+)= sum over k < nchunk of part[k * stride + e], e < len; fixed order.
__global__ void __launch_bounds__(256) k_sum_rows(const float *__restrict__ part, float *__restrict__ out, int len,
                                                  size_t stride, int nchunk, int accumulate)
{
    const int e = blockIdx.x;
    if (e >= len) return;
    float s = 0.f;
    for (int k = threadIdx.x; k < nchunk; k += 256) s += part[(size_t)k * stride + e];
    __shared__ float red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[e] = (accumulate ? out[e] : 0.f) + red[0];
}

// ---------------------------------------------------------------- loss
// part[block] = sum (y - t)^2 over the block's elements; gy = 2 (y - t) / n.
template <typename T>
__global__ void __launch_bounds__(256) k_mse(const T *__restrict__ y, const T *__restrict__ t, T *__restrict__ gy,
                                             float *__restrict__ part, long long n)
{
    float s = 0.f;
    const float scale = 2.0f / (float)n;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const float d = to_f32(y[e]) - to_f32(t[e]);
        s = fmaf(d, d, s);
        if (gy) gy[e] = from_f32<T>(scale * d);
    }
    __shared__ float red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// loss = (sum of the per-block partials) / n, the partials added in a fixed order: 8 consecutive
// ones per thread in double, then a tree over the 256 threads.
__global__ void __launch_bounds__(256) k_mse_final(const float *__restrict__ part, int nb, float *__restrict__ loss,
                                                   long long n)
{
    double s = 0.0;
    const int per = (nb + 255) / 256;
    for (int k = 0; k < per; k++) {
        const int i = threadIdx.x * per + k;
        if (i < nb) s += part[i];
    }
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = (float)(red[0] / (double)n);
}

// ---------------------------------------------------------------- launchers
static const int kGlueBlocks = 2048;

int glue_blocks() { return kGlueBlocks; }

size_t proj_part_len(int Ci, int H) { return (size_t)H * Ci + 2 * (size_t)H + 1; }

// Largest number of partial sums the decoder's backward writes: one per pair of waves.
int proj_part_chunks() { return kGlueBlocks * 2; }

// Blocks of a streaming launch: as many as are resident at once on the device (all have the same
// work, so one round fills the chip without a partial last round), at most kGlueBlocks (the
// partial-sum buffers are sized for that).  Computed once per kernel.
template <typename K> static int resident_blocks(K kernel, int lds_bytes, std::atomic<int> &cache)
{
    int v = cache.load(std::memory_order_relaxed);
    if (v > 0) return v;
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, 256, lds_bytes) != hipSuccess || cus < 1 || per < 1)
        v = kGlueBlocks;
    else
        v = std::min(kGlueBlocks, cus * per);
    cache.store(v, std::memory_order_relaxed);
    return v;
}

template <typename T, int CI, bool VEC>
static void launch_lift_fwd_t(const T *x, T *y, const float *w, const float *b, int B, int Co, long long N,
                              hipStream_t st)
{
    static std::atomic<int> nblk{0};
    const int g = resident_blocks(k_lift_fwd<T, CI, VEC>, 0, nblk);
    hipLaunchKernelGGL((k_lift_fwd<T, CI, VEC>), dim3(g), dim3(256), 0, st, x, y, w, b, B, Co, N);
}

template <typename T, int CI>
static void launch_lift_fwd_c(const T *x, T *y, const float *w, const float *b, int B, int Co, long long N,
                              hipStream_t st)
{
    if (N % 4 == 0) launch_lift_fwd_t<T, CI, true>(x, y, w, b, B, Co, N, st);
    else launch_lift_fwd_t<T, CI, false>(x, y, w, b, B, Co, N, st);
}

template <typename T>
hipError_t launch_lift_fwd(const T *x, T *y, const float *w, const float *b, int B, int Ci, int Co, long long N,
                           hipStream_t st)
{
    switch (Ci) {
    case 1: launch_lift_fwd_c<T, 1>(x, y, w, b, B, Co, N, st); break;
    case 2: launch_lift_fwd_c<T, 2>(x, y, w, b, B, Co, N, st); break;
    case 3: launch_lift_fwd_c<T, 3>(x, y, w, b, B, Co, N, st); break;
    case 4: launch_lift_fwd_c<T, 4>(x, y, w, b, B, Co, N, st); break;
    case 5: launch_lift_fwd_c<T, 5>(x, y, w, b, B, Co, N, st); break;
    case 6: launch_lift_fwd_c<T, 6>(x, y, w, b, B, Co, N, st); break;
    case 7: launch_lift_fwd_c<T, 7>(x, y, w, b, B, Co, N, st); break;
    case 8: launch_lift_fwd_c<T, 8>(x, y, w, b, B, Co, N, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

void launch_sum_rows(const float *part, float *out, int len, size_t stride, int nchunk, int accumulate, hipStream_t st)
{
    if (out && len > 0)
        hipLaunchKernelGGL(k_sum_rows, dim3(len), dim3(256), 0, st, part, out, len, stride, nchunk, accumulate);
}

// Returns the number of blocks launched (partial sums written).
template <typename T, int CI, bool VEC>
static int launch_lift_bwd_t(const T *x, const T *gy, const float *w, const float *b, float *part, int B, int Co,
                             long long N, hipStream_t st)
{
    static std::atomic<int> nblk{0};
    const int g = resident_blocks(k_lift_bwd<T, CI, VEC>, 0, nblk);
    hipLaunchKernelGGL((k_lift_bwd<T, CI, VEC>), dim3(g), dim3(256), 0, st, x, gy, w, b, part, B, Co, N);
    return g;
}

template <typename T, int CI>
static int launch_lift_bwd_c(const T *x, const T *gy, const float *w, const float *b, float *part, int B, int Co,
                             long long N, hipStream_t st)
{
    if (N % 4 == 0) return launch_lift_bwd_t<T, CI, true>(x, gy, w, b, part, B, Co, N, st);
    return launch_lift_bwd_t<T, CI, false>(x, gy, w, b, part, B, Co, N, st);
}

template <typename T>
hipError_t launch_lift_bwd(const T *x, const T *gy, const float *w, const float *b, float *part, float *gw, float *gb,
                           int B, int Ci, int Co, long long N, int accumulate, hipStream_t st)
{
    int nb = 0;
    switch (Ci) {
    case 1: nb = launch_lift_bwd_c<T, 1>(x, gy, w, b, part, B, Co, N, st); break;
    case 2: nb = launch_lift_bwd_c<T, 2>(x, gy, w, b, part, B, Co, N, st); break;
    case 3: nb = launch_lift_bwd_c<T, 3>(x, gy, w, b, part, B, Co, N, st); break;
    case 4: nb = launch_lift_bwd_c<T, 4>(x, gy, w, b, part, B, Co, N, st); break;
    case 5: nb = launch_lift_bwd_c<T, 5>(x, gy, w, b, part, B, Co, N, st); break;
    case 6: nb = launch_lift_bwd_c<T, 6>(x, gy, w, b, part, B, Co, N, st); break;
    case 7: nb = launch_lift_bwd_c<T, 7>(x, gy, w, b, part, B, Co, N, st); break;
    case 8: nb = launch_lift_bwd_c<T, 8>(x, gy, w, b, part, B, Co, N, st); break;
    default: return hipErrorInvalidValue;
    }
    const size_t row = (size_t)Co * (Ci + 1);
    launch_sum_rows(part, gw, Co * Ci, row, nb, accumulate, st);
    launch_sum_rows(part + (size_t)Co * Ci, gb, Co, row, nb, accumulate, st);
    return hipGetLastError();
}

// Returns the number of blocks launched.
template <typename T, int MCI, bool VEC>
static int launch_proj_t(const ProjArgs &a, bool bwd, const T *x, const T *gy, T *y_or_gx, const float *w1,
                         const float *b1, const float *w2, const float *b2, float *part, hipStream_t st)
{
    static std::atomic<int> nfwd{0}, nbwd{0};
    if (!bwd) {
        const int g = resident_blocks(k_proj_fwd<T, MCI, VEC>, 0, nfwd);
        hipLaunchKernelGGL((k_proj_fwd<T, MCI, VEC>), dim3(g), dim3(256), 0, st, x, y_or_gx, w1, b1, w2, b2, a);
        return g;
    }
    const int g = resident_blocks(k_proj_bwd<T, MCI, VEC>, 0, nbwd);
    hipLaunchKernelGGL((k_proj_bwd<T, MCI, VEC>), dim3(g), dim3(256), 0, st, x, gy, y_or_gx, w1, b1, w2, part, a);
    return g;
}

template <typename T, int MCI>
static int launch_proj_m(const ProjArgs &a, bool bwd, const T *x, const T *gy, T *y_or_gx, const float *w1,
                         const float *b1, const float *w2, const float *b2, float *part, hipStream_t st)
{
    if (a.N % 4 == 0) return launch_proj_t<T, MCI, true>(a, bwd, x, gy, y_or_gx, w1, b1, w2, b2, part, st);
    return launch_proj_t<T, MCI, false>(a, bwd, x, gy, y_or_gx, w1, b1, w2, b2, part, st);
}

// The backward's partial sums: *nchunk (one per pair of waves) rows of proj_part_len floats.
template <typename T>
hipError_t launch_proj(bool bwd, int B, int Ci, int H, int Co, long long N, const T *x, const T *gy, T *y_or_gx,
                       const float *w1, const float *b1, const float *w2, const float *b2, float *part, int accumulate,
                       hipStream_t st, int *nchunk)
{
    ProjArgs a{B, Ci, H, Co, N, accumulate};
    // K chunks of the first layer: Ci inputs plus the ones row of the bias
    const int mci = (Ci + 1 + 15) / 16;
    if (H > 128 || Co != 1) return hipErrorInvalidValue;
    int g = 0;
    if (mci == 1) g = launch_proj_m<T, 1>(a, bwd, x, gy, y_or_gx, w1, b1, w2, b2, part, st);
    else if (mci == 2) g = launch_proj_m<T, 2>(a, bwd, x, gy, y_or_gx, w1, b1, w2, b2, part, st);
    else if (mci == 3) g = launch_proj_m<T, 3>(a, bwd, x, gy, y_or_gx, w1, b1, w2, b2, part, st);
    else return hipErrorInvalidValue;
    if (nchunk) *nchunk = 2 * g;
    return hipGetLastError();
}

template <typename T>
hipError_t launch_mse(const T *y, const T *t, T *gy, float *part, float *loss, long long n, hipStream_t st)
{
    hipLaunchKernelGGL(k_mse<T>, dim3(kGlueBlocks), dim3(256), 0, st, y, t, gy, part, n);
    hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(256), 0, st, part, kGlueBlocks, loss, n);
    return hipGetLastError();
}

#define FNO_GLUE_INST(T)                                                                                              \
    template hipError_t launch_lift_fwd<T>(const T *, T *, const float *, const float *, int, int, int, long long,   \
                                           hipStream_t);                                                              \
    template hipError_t launch_lift_bwd<T>(const T *, const T *, const float *, const float *, float *, float *,      \
                                           float *, int, int, int, long long, int, hipStream_t);                      \
    template hipError_t launch_proj<T>(bool, int, int, int, int, long long, const T *, const T *, T *, const float *, \
                                       const float *, const float *, const float *, float *, int, hipStream_t, int *); \
    template hipError_t launch_mse<T>(const T *, const T *, T *, float *, float *, long long, hipStream_t);
FNO_GLUE_INST(float)
FNO_GLUE_INST(__bf16)
#undef FNO_GLUE_INST

}  // namespace fno
