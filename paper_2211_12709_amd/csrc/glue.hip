// glue.hip -- the network around the FNO blocks (Alg. 1): the encoder (lifting
// 1x1 + GELU), the two-layer decoder (projection 1x1 -> GELU -> 1x1) and the
// mean-squared-error loss, forward and backward.  Everything is pointwise in
// space, so every kernel streams points; the decoder's hidden layer (H = 128
// channels per point) is never written to memory.
//
// Decoder on the matrix cores, per tile of 16 points p and one wave:
//   Z1[h][p]  = sum_ci W1[h][ci] x[ci][p] + b1[h]          (A = W1 fragments, B = x)
//   Hd[h][p]  = GELU(Z1)                                    (accumulator rows h = K rows of the next product)
//   y[o][p]   = sum_h W2[o][h] Hd[h][p] + b2[o]
// backward, per tile:
//   gH[h][p]  = (sum_o W2[o][h] gy[o][p]) GELU'(Z1[h][p])
//   gx[ci][p] = sum_h W1[h][ci] gH[h][p]                    (gH tiles are the K chunks)
//   gW1^T[ci][h] += sum_p x[ci][p] gH^T[p][h], gW2[o][h] += sum_p gy[o][p] Hd^T[p][h]
//   (gH and Hd are transposed through LDS for the last two products)
#include "fno_internal.h"
#include "mfma_common.h"

namespace fno {

// ---------------------------------------------------------------- lifting
// y[b][o][n] = GELU(sum_i w[o][i] x[b][i][n] + bias[o]); thread per point, all channels.
template <typename T>
__global__ void __launch_bounds__(256) k_lift_fwd(const T *__restrict__ x, T *__restrict__ y,
                                                  const float *__restrict__ w, const float *__restrict__ bias, int B,
                                                  int Ci, int Co, long long N)
{
    const long long tot = (long long)B * N;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
         e += (long long)gridDim.x * blockDim.x) {
        const long long b = e / N, n = e % N;
        float xv[8];
        for (int i = 0; i < Ci; i++) xv[i] = to_f32(x[(b * Ci + i) * N + n]);
        for (int o = 0; o < Co; o++) {
            float z = bias ? bias[o] : 0.f;
            for (int i = 0; i < Ci; i++) z = fmaf(w[o * Ci + i], xv[i], z);
            y[(b * Co + o) * N + n] = from_f32<T>(gelu_fast(z));
        }
    }
}

// Partial sums of gw[o][i] = sum gz[o] x[i] and gb[o] = sum gz[o] with
// gz = gy GELU'(w x + b), per block: part[block][o * Ci + i] and part[block][Co * Ci + o].
// Output channels are taken in groups of OG to bound the accumulators.
template <typename T>
__global__ void __launch_bounds__(256) k_lift_bwd(const T *__restrict__ x, const T *__restrict__ gy,
                                                  const float *__restrict__ w, const float *__restrict__ bias,
                                                  float *__restrict__ part, int B, int Ci, int Co, long long N)
{
    constexpr int OG = 8, MAXI = 8;
    const long long tot = (long long)B * N;
    const size_t row = (size_t)Co * (Ci + 1);
    __shared__ float red[256];
    for (int o0 = 0; o0 < Co; o0 += OG) {
        float acc[OG][MAXI + 1];
#pragma unroll
        for (int k = 0; k < OG; k++)
#pragma unroll
            for (int i = 0; i <= MAXI; i++) acc[k][i] = 0.f;
        for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
             e += (long long)gridDim.x * blockDim.x) {
            const long long b = e / N, n = e % N;
            float xv[MAXI];
#pragma unroll
            for (int i = 0; i < MAXI; i++) xv[i] = i < Ci ? to_f32(x[(b * Ci + i) * N + n]) : 0.f;
#pragma unroll
            for (int k = 0; k < OG; k++) {
                const int o = o0 + k;
                if (o < Co) {
                    float z = bias ? bias[o] : 0.f;
#pragma unroll
                    for (int i = 0; i < MAXI; i++)
                        if (i < Ci) z = fmaf(w[o * Ci + i], xv[i], z);
                    const float gz = to_f32(gy[(b * Co + o) * N + n]) * gelu_grad_fast(z);
#pragma unroll
                    for (int i = 0; i < MAXI; i++) acc[k][i] = fmaf(gz, xv[i], acc[k][i]);
                    acc[k][MAXI] += gz;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < OG; k++) {
            const int o = o0 + k;
            if (o < Co) {  // uniform across the block
#pragma unroll
                for (int i = 0; i <= MAXI; i++) {
                    if (i < Ci || i == MAXI) {
                        red[threadIdx.x] = acc[k][i];
                        __syncthreads();
                        for (int h = 128; h > 0; h >>= 1) {
                            if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
                            __syncthreads();
                        }
                        if (threadIdx.x == 0)
                            part[(size_t)blockIdx.x * row + (i == MAXI ? (size_t)Co * Ci + o : (size_t)o * Ci + i)] =
                                red[0];
                        __syncthreads();
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------- projection
struct ProjArgs {
    int B, Ci, H, Co;
    long long N;
    int accumulate;
};

// Forward of the decoder; one wave per 16-point tile, tiles strided over the grid.
// CT: compute type of the MFMA operands (float or bf16); T: activation type.
template <typename T, int MCI, int MH>
__global__ void __launch_bounds__(256) k_proj_fwd(const T *__restrict__ x, T *__restrict__ y,
                                                  const float *__restrict__ w1, const float *__restrict__ b1,
                                                  const float *__restrict__ w2, const float *__restrict__ b2,
                                                  ProjArgs a)
{
    typedef typename OpOf<T>::type Op;
    const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
    const long long ntile = (a.N + 15) / 16, tiles = (long long)a.B * ntile;
    const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
    // W1 fragments A[h = 16 m + c][ci = 16 q + 4 g + j]; W2 fragments A[o = c][h = 16 m + 4 g + j]
    Op aw1[MH][MCI], aw2[MH];
    float bias1[MH][4];
#pragma unroll
    for (int m = 0; m < MH; m++) {
#pragma unroll
        for (int q = 0; q < MCI; q++) {
            float v[4];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int h = 16 * m + c, ci = 16 * q + 4 * g + j;
                v[j] = (h < a.H && ci < a.Ci) ? w1[h * a.Ci + ci] : 0.f;
            }
            aw1[m][q] = op_from4<T>(v[0], v[1], v[2], v[3]);
        }
        float v[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int h = 16 * m + 4 * g + j;
            v[j] = (c < a.Co && h < a.H) ? w2[c * a.H + h] : 0.f;
        }
        aw2[m] = op_from4<T>(v[0], v[1], v[2], v[3]);
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int h = 16 * m + 4 * g + r;
            bias1[m][r] = (b1 && h < a.H) ? b1[h] : 0.f;
        }
    }
    for (long long tile = wave; tile < tiles; tile += nwaves) {
        const long long b = tile / ntile, p0 = (tile % ntile) * 16;
        const long long p = p0 + c;
        // B = x[ci = 16 q + 4 g + j][p]
        Op bx[MCI];
#pragma unroll
        for (int q = 0; q < MCI; q++) {
            float v[4];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int ci = 16 * q + 4 * g + j;
                v[j] = (ci < a.Ci && p < a.N) ? to_f32(x[((long long)b * a.Ci + ci) * a.N + p]) : 0.f;
            }
            bx[q] = op_from4<T>(v[0], v[1], v[2], v[3]);
        }
        f4v yo = f4_zero();
#pragma unroll
        for (int m = 0; m < MH; m++) {
            f4v z = f4_zero();
#pragma unroll
            for (int q = 0; q < MCI; q++) z = mma16(aw1[m][q], bx[q], z);
            f4v hd;
#pragma unroll
            for (int r = 0; r < 4; r++) hd[r] = gelu_fast(z[r] + bias1[m][r]);
            yo = mma16(aw2[m], to_op<T>(hd), yo);
        }
        // yo[r] = y[o = 4 g + r][p]
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int o = 4 * g + r;
            if (o < a.Co && p < a.N) y[((long long)b * a.Co + o) * a.N + p] = from_f32<T>(yo[r] + (b2 ? b2[o] : 0.f));
        }
    }
}

// Backward of the decoder.  Per wave partial sums of gW1 [H][Ci], gb1 [H],
// gW2 [Co][H], gb2 [Co] go to part[(block * 4 + wave)][...] (layout in proj_part_len).
template <typename T, int MCI, int MH>
__global__ void __launch_bounds__(256) k_proj_bwd(const T *__restrict__ x, const T *__restrict__ gy,
                                                  T *__restrict__ gx, const float *__restrict__ w1,
                                                  const float *__restrict__ b1, const float *__restrict__ w2,
                                                  float *__restrict__ part, ProjArgs a)
{
    typedef typename OpOf<T>::type Op;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), g = lane >> 4, c = lane & 15;
    const int ldh = 16 * MH + 4;
    T *ghl = reinterpret_cast<T *>(smem) + (size_t)w * 2 * 16 * ldh;  // this wave: gH^T [16 p][ldh], Hd^T [16 p][ldh]
    T *hdl = ghl + 16 * ldh;
    const long long ntile = (a.N + 15) / 16, tiles = (long long)a.B * ntile;
    const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
    Op aw1[MH][MCI], aw1t[MCI][MH];
    float bias1[MH][4], w2v[MH][4];
#pragma unroll
    for (int m = 0; m < MH; m++) {
#pragma unroll
        for (int q = 0; q < MCI; q++) {
            float v[4], vt[4];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int h = 16 * m + c, ci = 16 * q + 4 * g + j;
                v[j] = (h < a.H && ci < a.Ci) ? w1[h * a.Ci + ci] : 0.f;
                // W1^T fragments: A[ci = 16 q + c][h = 16 m + 4 g + j]
                const int ci2 = 16 * q + c, h2 = 16 * m + 4 * g + j;
                vt[j] = (h2 < a.H && ci2 < a.Ci) ? w1[h2 * a.Ci + ci2] : 0.f;
            }
            aw1[m][q] = op_from4<T>(v[0], v[1], v[2], v[3]);
            aw1t[q][m] = op_from4<T>(vt[0], vt[1], vt[2], vt[3]);
        }
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int h = 16 * m + 4 * g + r;
            bias1[m][r] = (b1 && h < a.H) ? b1[h] : 0.f;
            w2v[m][r] = h < a.H ? w2[h] : 0.f;  // decoder output channel 0 (Co == 1)
        }
    }
    // weight-gradient accumulators: gW1^T[ci][h] tiles [q][m]; gW2 row o = 0 via tile (o rows, h cols)
    f4v gw1[MCI][MH], gw2[MH];
#pragma unroll
    for (int q = 0; q < MCI; q++)
#pragma unroll
        for (int m = 0; m < MH; m++) gw1[q][m] = f4_zero();
#pragma unroll
    for (int m = 0; m < MH; m++) gw2[m] = f4_zero();
    float gb1[MH][4], gb2 = 0.f;
#pragma unroll
    for (int m = 0; m < MH; m++)
#pragma unroll
        for (int r = 0; r < 4; r++) gb1[m][r] = 0.f;

    for (long long tile = wave; tile < tiles; tile += nwaves) {
        const long long b = tile / ntile, p0 = (tile % ntile) * 16;
        const long long p = p0 + c;
        Op bx[MCI];
#pragma unroll
        for (int q = 0; q < MCI; q++) {
            float v[4];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int ci = 16 * q + 4 * g + j;
                v[j] = (ci < a.Ci && p < a.N) ? to_f32(x[((long long)b * a.Ci + ci) * a.N + p]) : 0.f;
            }
            bx[q] = op_from4<T>(v[0], v[1], v[2], v[3]);
        }
        const float gyp = p < a.N ? to_f32(gy[(long long)b * a.N + p]) : 0.f;  // Co == 1
        f4v gxa[MCI];
#pragma unroll
        for (int q = 0; q < MCI; q++) gxa[q] = f4_zero();
#pragma unroll
        for (int m = 0; m < MH; m++) {
            f4v z = f4_zero();
#pragma unroll
            for (int q = 0; q < MCI; q++) z = mma16(aw1[m][q], bx[q], z);
            f4v gh, hd;
#pragma unroll
            for (int r = 0; r < 4; r++) {
                float gv, dg;
                gelu_as(z[r] + bias1[m][r], gv, dg);
                hd[r] = gv;
                gh[r] = w2v[m][r] * gyp * dg;
                gb1[m][r] += gh[r];
            }
            const Op ghop = to_op<T>(gh);
#pragma unroll
            for (int q = 0; q < MCI; q++) gxa[q] = mma16(aw1t[q][m], ghop, gxa[q]);
            // transpose gH and Hd through LDS: [p = c][h = 16 m + 4 g + r]
#pragma unroll
            for (int r = 0; r < 4; r++) {
                ghl[c * ldh + 16 * m + 4 * g + r] = from_f32<T>(gh[r]);
                hdl[c * ldh + 16 * m + 4 * g + r] = from_f32<T>(hd[r]);
            }
        }
        gb2 += gyp;
        // gx[ci = 16 q + 4 g + r][p]
#pragma unroll
        for (int q = 0; q < MCI; q++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int ci = 16 * q + 4 * g + r;
                if (ci < a.Ci && p < a.N) {
                    const long long idx = ((long long)b * a.Ci + ci) * a.N + p;
                    gx[idx] = from_f32<T>(gxa[q][r] + (a.accumulate ? to_f32(gx[idx]) : 0.f));
                }
            }
        __builtin_amdgcn_wave_barrier();  // the wave's own LDS writes precede its reads (in order per wave)
        // gW1^T[ci][h] += sum_p x[ci][p] gH^T[p][h]: A[ci = 16 q + c][p = 4 g + j], B[p = 4 g + j][h = 16 m + c]
        Op axt[MCI];
#pragma unroll
        for (int q = 0; q < MCI; q++) {
            float v[4];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int ci = 16 * q + c;
                const long long pj = p0 + 4 * g + j;
                v[j] = (ci < a.Ci && pj < a.N) ? to_f32(x[((long long)b * a.Ci + ci) * a.N + pj]) : 0.f;
            }
            axt[q] = op_from4<T>(v[0], v[1], v[2], v[3]);
        }
        // gy as A[o = c][p = 4 g + j] (only o = 0 is a real row)
        float gv4[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const long long pj = p0 + 4 * g + j;
            gv4[j] = (c == 0 && pj < a.N) ? to_f32(gy[(long long)b * a.N + pj]) : 0.f;
        }
        const Op agy = op_from4<T>(gv4[0], gv4[1], gv4[2], gv4[3]);
#pragma unroll
        for (int m = 0; m < MH; m++) {
            const T *gr = ghl + (4 * g) * ldh + 16 * m + c;
            const T *hr = hdl + (4 * g) * ldh + 16 * m + c;
            const Op bgh = op_from4<T>(to_f32(gr[0]), to_f32(gr[ldh]), to_f32(gr[2 * ldh]), to_f32(gr[3 * ldh]));
            const Op bhd = op_from4<T>(to_f32(hr[0]), to_f32(hr[ldh]), to_f32(hr[2 * ldh]), to_f32(hr[3 * ldh]));
#pragma unroll
            for (int q = 0; q < MCI; q++) gw1[q][m] = mma16(axt[q], bgh, gw1[q][m]);
            gw2[m] = mma16(agy, bhd, gw2[m]);
        }
        __builtin_amdgcn_wave_barrier();
    }
    // partial layout per wave: gW1 [H][Ci], gb1 [H], gW2 [H] (Co == 1), gb2 [1]
    const int H = a.H, Ci = a.Ci;
    float *pw = part + ((size_t)blockIdx.x * 4 + w) * ((size_t)H * Ci + 2 * H + 1);
#pragma unroll
    for (int q = 0; q < MCI; q++)
#pragma unroll
        for (int m = 0; m < MH; m++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int ci = 16 * q + 4 * g + r, h = 16 * m + c;
                if (ci < Ci && h < H) pw[h * Ci + ci] = gw1[q][m][r];
            }
#pragma unroll
    for (int m = 0; m < MH; m++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
            float s = gb1[m][r];
            // lanes with the same g hold the same h rows: sum over the 16 point columns c
            s += __shfl_xor(s, 1);
            s += __shfl_xor(s, 2);
            s += __shfl_xor(s, 4);
            s += __shfl_xor(s, 8);
            const int h = 16 * m + 4 * g + r;
            if (c == 0 && h < H) pw[(size_t)H * Ci + h] = s;
        }
#pragma unroll
    for (int m = 0; m < MH; m++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
            // gw2 tile rows o = 4 g + r, cols h = 16 m + c: row o = 0 is g == 0, r == 0
            if (g == 0 && r == 0 && 16 * m + c < H) pw[(size_t)H * Ci + H + 16 * m + c] = gw2[m][0];
        }
    float s = gb2;
    s += __shfl_xor(s, 1);
    s += __shfl_xor(s, 2);
    s += __shfl_xor(s, 4);
    s += __shfl_xor(s, 8);  // every point column was added once per g group: take g == 0
    if (lane == 0) pw[(size_t)H * Ci + 2 * H] = s;
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

__global__ void k_mse_final(const float *__restrict__ part, int nb, float *__restrict__ loss, long long n)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;  // fixed-order final sum of the per-block partials
    for (int i = 0; i < nb; i++) s += part[i];
    loss[0] = (float)(s / (double)n);
}

// ---------------------------------------------------------------- launchers
static const int kGlueBlocks = 2048;

int glue_blocks() { return kGlueBlocks; }

size_t proj_part_len(int Ci, int H) { return (size_t)H * Ci + 2 * (size_t)H + 1; }

template <typename T>
hipError_t launch_lift_fwd(const T *x, T *y, const float *w, const float *b, int B, int Ci, int Co, long long N,
                           hipStream_t st)
{
    hipLaunchKernelGGL(k_lift_fwd<T>, dim3(kGlueBlocks), dim3(256), 0, st, x, y, w, b, B, Ci, Co, N);
    return hipGetLastError();
}

void launch_sum_rows(const float *part, float *out, int len, size_t stride, int nchunk, int accumulate, hipStream_t st)
{
    if (out && len > 0)
        hipLaunchKernelGGL(k_sum_rows, dim3(len), dim3(256), 0, st, part, out, len, stride, nchunk, accumulate);
}

template <typename T>
hipError_t launch_lift_bwd(const T *x, const T *gy, const float *w, const float *b, float *part, float *gw, float *gb,
                           int B, int Ci, int Co, long long N, int accumulate, hipStream_t st)
{
    hipLaunchKernelGGL(k_lift_bwd<T>, dim3(kGlueBlocks), dim3(256), 0, st, x, gy, w, b, part, B, Ci, Co, N);
    const size_t row = (size_t)Co * (Ci + 1);
    launch_sum_rows(part, gw, Co * Ci, row, kGlueBlocks, accumulate, st);
    launch_sum_rows(part + (size_t)Co * Ci, gb, Co, row, kGlueBlocks, accumulate, st);
    return hipGetLastError();
}

template <typename T, int MCI, int MH>
static hipError_t launch_proj_t(const ProjArgs &a, bool bwd, const T *x, const T *gy, T *y_or_gx, const float *w1,
                                const float *b1, const float *w2, const float *b2, float *part, hipStream_t st)
{
    if (!bwd) {
        hipLaunchKernelGGL((k_proj_fwd<T, MCI, MH>), dim3(kGlueBlocks), dim3(256), 0, st, x, y_or_gx, w1, b1, w2, b2,
                           a);
    } else {
        const size_t lds = (size_t)4 * 2 * 16 * (16 * MH + 4) * sizeof(T);
        hipLaunchKernelGGL((k_proj_bwd<T, MCI, MH>), dim3(kGlueBlocks), dim3(256), lds, st, x, gy, y_or_gx, w1, b1,
                           w2, part, a);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_proj(bool bwd, int B, int Ci, int H, int Co, long long N, const T *x, const T *gy, T *y_or_gx,
                       const float *w1, const float *b1, const float *w2, const float *b2, float *part, int accumulate,
                       hipStream_t st)
{
    ProjArgs a{B, Ci, H, Co, N, accumulate};
    const int mci = (Ci + 15) / 16, mh = (H + 15) / 16;
    if (mci <= 2 && mh <= 8) return launch_proj_t<T, 2, 8>(a, bwd, x, gy, y_or_gx, w1, b1, w2, b2, part, st);
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_mse(const T *y, const T *t, T *gy, float *part, float *loss, long long n, hipStream_t st)
{
    hipLaunchKernelGGL(k_mse<T>, dim3(kGlueBlocks), dim3(256), 0, st, y, t, gy, part, n);
    hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(64), 0, st, part, kGlueBlocks, loss, n);
    return hipGetLastError();
}

#define FNO_GLUE_INST(T)                                                                                              \
    template hipError_t launch_lift_fwd<T>(const T *, T *, const float *, const float *, int, int, int, long long,   \
                                           hipStream_t);                                                              \
    template hipError_t launch_lift_bwd<T>(const T *, const T *, const float *, const float *, float *, float *,      \
                                           float *, int, int, int, long long, int, hipStream_t);                      \
    template hipError_t launch_proj<T>(bool, int, int, int, int, long long, const T *, const T *, T *, const float *, \
                                       const float *, const float *, const float *, float *, int, hipStream_t);       \
    template hipError_t launch_mse<T>(const T *, const T *, T *, float *, float *, long long, hipStream_t);
FNO_GLUE_INST(float)
FNO_GLUE_INST(__bf16)
#undef FNO_GLUE_INST

}  // namespace fno
