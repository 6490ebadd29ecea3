// axis_mfma.hip -- one-axis complex DFT contraction of truncated spectra on the
// matrix cores: the x and y stages of the forward transform (Alg. 2 line 1:
// F_x after the y,z,t stages) and of the zero-padded inverse (Alg. 2 line 3).
//
//   out[o][j][col] = sum_n E(j, n) in[o][n][col]      (complex, col contiguous)
//
// Real form: rows (re/im, j), K = (re/im', n):
//   forward  E = exp(-i theta): [[cos, sin], [-sin, cos]]
//   inverse  E = exp(+i theta): [[cos, -sin], [sin, cos]]
// The basis lives in a fragment-ordered table (tables.hip).  OUT16 stores the
// result as bfloat16 (re, im) pairs for a consumer that works in bfloat16.  One workgroup
// owns an (o, 64-column) block: it stages in[o][*][cols] in LDS transposed to
// [col][(re/im', n)] so that every lane's 4 K values are one vector read, and
// each wave computes one 16-column tile for all row tiles.
#include "fno_internal.h"
#include "mfma_common.h"

namespace fno {

struct AxisArgs {
    long long outer;  // independent matrices
    int Nin, Nout;    // contracted / produced length
    int Ninp, Noutp;  // padded to multiples of 16
    long long cols;   // columns (complex) per row
    int MT;           // row tiles: 2 Noutp / 16
    int QK;           // K chunks: 2 Ninp / 16
};

template <typename TC, bool OUT16>
__global__ void __launch_bounds__(256) k_axis_mfma(const float2 *__restrict__ in, void *__restrict__ out_,
                                                   const typename OpOf<TC>::type *__restrict__ tab,
                                                   const typename OpOf<TC>::type *__restrict__ tab_lo, AxisArgs a)
{
    typedef typename OpOf<TC>::type Op;
    constexpr bool SPLIT = sizeof(TC) == 2;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, c = lane & 15;
    const long long nchunk = (a.cols + 63) / 64;
    const long long o = blockIdx.x / nchunk;
    const long long col0 = (blockIdx.x % nchunk) * 64;
    const int ldk = 2 * a.Ninp + 4;
    TC *sl = reinterpret_cast<TC *>(smem);  // [64 cols][(re/im, n)]
    const float2 *src = in + o * a.Nin * a.cols;
    // stage: consecutive threads read consecutive columns of one row n
    for (int e = threadIdx.x; e < a.Ninp * 64; e += 256) {
        const int n = e / 64, cl = e % 64;
        float2 v = make_float2(0.f, 0.f);
        if (n < a.Nin && col0 + cl < a.cols) v = src[(long long)n * a.cols + col0 + cl];
        sl[cl * ldk + n] = from_f32<TC>(v.x);
        sl[cl * ldk + a.Ninp + n] = from_f32<TC>(v.y);
    }
    __syncthreads();
    const int cl = 16 * w + c;  // this wave's column tile, lane column
    const long long col = col0 + cl;
    float2 *dst = reinterpret_cast<float2 *>(out_) + o * a.Nout * a.cols;
    s2v *dst16 = reinterpret_cast<s2v *>(out_) + o * a.Nout * a.cols;
    const int half = a.MT / 2;
    for (int mp = 0; mp < half; mp++) {
        // row tiles mp (re rows) and mp + half (im rows)
        f4v accr = f4_zero(), acci = f4_zero();
        for (int q = 0; q < a.QK; q++) {
            const Op bv = *reinterpret_cast<const Op *>(sl + cl * ldk + 16 * q + 4 * g);
            const int ir = (mp * a.QK + q) * 64 + lane, ii = ((mp + half) * a.QK + q) * 64 + lane;
            accr = mma16(tab[ir], bv, accr);
            acci = mma16(tab[ii], bv, acci);
            if (SPLIT) {
                accr = mma16(tab_lo[ir], bv, accr);
                acci = mma16(tab_lo[ii], bv, acci);
            }
        }
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int j = 16 * mp + 4 * g + r;
            if (j < a.Nout && col < a.cols) {
                if (OUT16)
                    dst16[(long long)j * a.cols + col] = s2v{bf16_bits(accr[r]), bf16_bits(acci[r])};
                else
                    dst[(long long)j * a.cols + col] = make_float2(accr[r], acci[r]);
            }
        }
    }
}

size_t axis_lds_bytes(int Ninp, int elem) { return (size_t)64 * (2 * Ninp + 4) * elem; }

template <typename TC>
hipError_t launch_axis_mfma(const float2 *in, void *out, const void *tab, const void *tab_lo, long long outer,
                            int Nin, int Nout, long long cols, hipStream_t st, bool out16)
{
    typedef typename OpOf<TC>::type Op;
    AxisArgs a;
    a.outer = outer;
    a.Nin = Nin;
    a.Nout = Nout;
    a.Ninp = (Nin + 15) / 16 * 16;
    a.Noutp = (Nout + 15) / 16 * 16;
    a.cols = cols;
    a.MT = 2 * a.Noutp / 16;
    a.QK = 2 * a.Ninp / 16;
    const size_t lds = axis_lds_bytes(a.Ninp, sizeof(TC));
    auto kern = out16 ? k_axis_mfma<TC, true> : k_axis_mfma<TC, false>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const long long blocks = outer * ((cols + 63) / 64);
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), lds, st, in, out, (const Op *)tab, (const Op *)tab_lo,
                       a);
    return hipGetLastError();
}

template hipError_t launch_axis_mfma<float>(const float2 *, void *, const void *, const void *, long long, int, int,
                                            long long, hipStream_t, bool);
template hipError_t launch_axis_mfma<__bf16>(const float2 *, void *, const void *, const void *, long long, int, int,
                                             long long, hipStream_t, bool);

}  // namespace fno
