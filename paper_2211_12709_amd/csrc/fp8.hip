// fp8.hip -- packing of the spectral weights into OCP 8-bit floating point (E4M3) with one
// power-of-two scale per (input, output) channel pair, for plans created with FNO_W_FP8.
//
// The mode mix (Alg. 2, line 2) at batch 1 is a matrix-vector product per retained mode: every
// weight is used once, so the mix is bound by reading W.  Packed, W takes 2 bytes per complex
// value instead of 8.  E4M3 has a 4-bit exponent (normal range 2^-6 .. 448), so each channel
// pair's weights are stored divided by s = 2^round(log2 RMS) of that pair (RMS over the real
// and imaginary parts of all its retained modes): the values then sit around 1, inside the
// normal range, and dividing by a power of two is exact.  Layout of the packed buffer:
//   [Ci][Co][Kx][Ky][Kz][Kt] 16-bit words (low byte re, high byte im), then at the next 256-byte
//   boundary [Ci][Co] float scales, then the packing's per-chunk sums of squares (scratch).
#include "fno_internal.h"

namespace fno {

// Chunks of modes per (i, o) pair: one workgroup each, in both passes.
constexpr long long kPackChunk = 8192;

static long long pack_chunks(long long M) { return (M + kPackChunk - 1) / kPackChunk; }

// Pass 1: sum of squares of the real and imaginary parts of one chunk of a pair's weights, in a
// fixed order (per thread, then a fixed tree).
__global__ void __launch_bounds__(256) k_pack_sumsq(const float2 *__restrict__ w, float *__restrict__ part,
                                                    long long M, int nch)
{
    const long long io = blockIdx.x / nch, ch = blockIdx.x % nch;
    const float2 *wp = w + io * M;
    const long long k1 = min(M, (ch + 1) * kPackChunk);
    float acc = 0.f;
    for (long long k = ch * kPackChunk + threadIdx.x; k < k1; k += 256) {
        const float2 v = wp[k];
        acc = fmaf(v.x, v.x, fmaf(v.y, v.y, acc));
    }
    __shared__ float red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Pass 2: the pair's scale s = 2^round(log2 RMS) from its chunk sums (every workgroup of the pair
// adds them in the same order, so all agree), then E4M3 codes of this chunk's values / s.
__global__ void __launch_bounds__(256) k_pack_encode(const float2 *__restrict__ w, const float *__restrict__ part,
                                                     unsigned short *__restrict__ q, float *__restrict__ scale,
                                                     long long M, int nch)
{
    const long long io = blockIdx.x / nch, ch = blockIdx.x % nch;
    __shared__ float s_inv;
    if (threadIdx.x == 0) {
        float tot = 0.f;
        for (int c = 0; c < nch; c++) tot += part[io * nch + c];
        const double rms = sqrt((double)tot / (2.0 * (double)M));
        const double s = rms > 0.0 ? ldexp(1.0, (int)rint(log2(rms))) : 1.0;
        if (ch == 0) scale[io] = (float)s;
        s_inv = (float)(1.0 / s);  // exact: a power of two
    }
    __syncthreads();
    const float inv = s_inv;
    const float2 *wp = w + io * M;
    const long long k1 = min(M, (ch + 1) * kPackChunk);
    for (long long k = ch * kPackChunk + threadIdx.x; k < k1; k += 256) {
        const float2 v = wp[k];
        q[io * M + k] = (unsigned short)(f32_to_e4m3(v.x * inv) | (f32_to_e4m3(v.y * inv) << 8));
    }
}

static size_t al256(size_t v) { return (v + 255) & ~size_t(255); }

size_t packed_scale_offset(int Ci, int Co, long long M) { return al256((size_t)2 * Ci * Co * M); }

// codes, scales, then the chunk sums of the packing (scratch of fno_pack_weights)
size_t packed_weight_bytes(int Ci, int Co, long long M)
{
    return packed_scale_offset(Ci, Co, M) + al256((size_t)4 * Ci * Co) +
           al256((size_t)4 * Ci * Co * pack_chunks(M));
}

hipError_t launch_pack_w_fp8(const float2 *w, void *wq, int Ci, int Co, long long M, hipStream_t st)
{
    unsigned short *q = (unsigned short *)wq;
    float *sc = (float *)((char *)wq + packed_scale_offset(Ci, Co, M));
    float *part = (float *)((char *)wq + packed_scale_offset(Ci, Co, M) + al256((size_t)4 * Ci * Co));
    const int nch = (int)pack_chunks(M);
    const unsigned grid = (unsigned)((long long)Ci * Co * nch);
    hipLaunchKernelGGL(k_pack_sumsq, dim3(grid), dim3(256), 0, st, w, part, M, nch);
    hipLaunchKernelGGL(k_pack_encode, dim3(grid), dim3(256), 0, st, w, part, q, sc, M, nch);
    return hipGetLastError();
}

}  // namespace fno
