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

// bfloat16 operands are used for the inverse stages of the bfloat16 path, whose results are
// rounded to bfloat16 next (stored as bfloat16 pairs, or staged so by the following stage): the
// basis is then used once (hi only) unless this is set.
#ifndef FNO_AXIS_BF16_SPLIT
#define FNO_AXIS_BF16_SPLIT 0
#endif

#ifndef FNO_AXIS_X32
#define FNO_AXIS_X32 1  // bfloat16 synthesis: two K chunks per 16x16x32 product
#endif

namespace fno {

struct AxisArgs {
    long long outer;  // independent matrices
    int Nin, Nout;    // contracted / produced length
    int Ninp, Noutp;  // padded to multiples of 16
    long long cols;   // columns (complex) per row
    int MT;           // row tiles: 2 Noutp / 16
    int QK;           // K chunks: 2 Ninp / 16
    int CB;           // columns per workgroup (k_axis_syn)
};

// Stage in[n][col0 + cl] (n < Nin, cl < CB = 2^lcb) into LDS as sl[cl][(re/im, n)], zero padded.
// Consecutive threads read consecutive columns of one row; every thread issues UB loads before
// its LDS writes, so a workgroup waits for one round of loads per UB rows, not one per row.
template <typename TC>
__device__ __forceinline__ void axis_stage(const float2 *__restrict__ src, long long cols, long long col0, int Nin,
                                           int Ninp, int lcb, int ldk, TC *sl)
{
    constexpr int UB = 8;
    const int total = Ninp << lcb, cmask = (1 << lcb) - 1;
    for (int e0 = threadIdx.x; e0 < total; e0 += UB * 256) {
        float2 v[UB];
#pragma unroll
        for (int k = 0; k < UB; k++) {
            const int e = e0 + k * 256, n = e >> lcb, cl = e & cmask;
            v[k] = (e < total && n < Nin && col0 + cl < cols) ? src[(long long)n * cols + col0 + cl]
                                                               : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int k = 0; k < UB; k++) {
            const int e = e0 + k * 256, n = e >> lcb, cl = e & cmask;
            if (e < total) {
                sl[cl * ldk + n] = from_f32<TC>(v[k].x);
                sl[cl * ldk + Ninp + n] = from_f32<TC>(v[k].y);
            }
        }
    }
}

template <typename TC, bool OUT16>
__global__ void __launch_bounds__(256) k_axis_mfma(const float2 *__restrict__ in, void *__restrict__ out_,
                                                   const typename OpOf<TC>::type *__restrict__ tab,
                                                   const typename OpOf<TC>::type *__restrict__ tab_lo, AxisArgs a)
{
    typedef typename OpOf<TC>::type Op;
    constexpr bool SPLIT = sizeof(TC) == 2 && FNO_AXIS_BF16_SPLIT;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), g = lane >> 4, c = lane & 15;
    const long long nchunk = (a.cols + 63) / 64;
    const long long o = blockIdx.x / nchunk;
    const long long col0 = (blockIdx.x % nchunk) * 64;
    const int ldk = 2 * a.Ninp + 4;
    TC *sl = reinterpret_cast<TC *>(smem);  // [64 cols][(re/im, n)]
    const float2 *src = in + o * a.Nin * a.cols;
    axis_stage<TC>(src, a.cols, col0, a.Nin, a.Ninp, 6, ldk, sl);
    __syncthreads();
    const int cl = 16 * w + c;  // this wave's column tile, lane column
    const long long col = col0 + cl;
    float2 *dst = reinterpret_cast<float2 *>(out_) + o * a.Nout * a.cols;
    s2v *dst16 = reinterpret_cast<s2v *>(out_) + o * a.Nout * a.cols;
    const int half = a.MT / 2;
    for (int mp = 0; mp < half; mp++) {
        // row tiles mp (re rows) and mp + half (im rows)
        f4v accr = f4_zero(), acci = f4_zero();
        // QB K chunks at a time: all of their table loads are issued before the first product,
        // so the wave waits for one round of loads per QB chunks instead of one per chunk
        constexpr int QB = 4;
        for (int q0 = 0; q0 < a.QK; q0 += QB) {
            Op tr[QB], ti[QB], trl[QB], til[QB], bv[QB];
#pragma unroll
            for (int k = 0; k < QB; k++)
                if (q0 + k < a.QK) {
                    const int q = q0 + k;
                    const int ir = (mp * a.QK + q) * 64 + lane, ii = ((mp + half) * a.QK + q) * 64 + lane;
                    tr[k] = tab[ir];
                    ti[k] = tab[ii];
                    if (SPLIT) {
                        trl[k] = tab_lo[ir];
                        til[k] = tab_lo[ii];
                    }
                    bv[k] = *reinterpret_cast<const Op *>(sl + cl * ldk + 16 * q + 4 * g);
                }
#pragma unroll
            for (int k = 0; k < QB; k++)
                if (q0 + k < a.QK) {
                    accr = mma16(tr[k], bv[k], accr);
                    acci = mma16(ti[k], bv[k], acci);
                    if (SPLIT) {
                        accr = mma16(trl[k], bv[k], accr);
                        acci = mma16(til[k], bv[k], acci);
                    }
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

// Synthesis-shaped contractions (short K = 2 Nin <= 16 QKM, long output): each wave keeps
// the basis fragments of up to MPW row pairs (re rows mp, im rows mp + MT/2) in registers and
// runs them over every 16-column tile of the workgroup's column block, so the table is read
// once per wave instead of once per tile.  One workgroup owns (o, CB <= 256 columns).
template <typename TC, bool OUT16, int QKM, int MPW>
__global__ void __launch_bounds__(256) k_axis_syn(const float2 *__restrict__ in, void *__restrict__ out_,
                                                  const typename OpOf<TC>::type *__restrict__ tab,
                                                  const typename OpOf<TC>::type *__restrict__ tab_lo, AxisArgs a)
{
    typedef typename OpOf<TC>::type Op;
    constexpr bool SPLIT = sizeof(TC) == 2 && FNO_AXIS_BF16_SPLIT;
    constexpr bool X32 = sizeof(TC) == 2 && !SPLIT && FNO_AXIS_X32 && QKM % 2 == 0;
    const int CB = a.CB;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), g = lane >> 4, c = lane & 15;
    const long long nchunk = (a.cols + CB - 1) / CB;
    const long long o = blockIdx.x / nchunk;
    const long long col0 = (blockIdx.x % nchunk) * CB;
    const int ldk = 2 * a.Ninp + 4;
    TC *sl = reinterpret_cast<TC *>(smem);  // [CB cols][(re/im, n)]
    const float2 *src = in + o * a.Nin * a.cols;
    axis_stage<TC>(src, a.cols, col0, a.Nin, a.Ninp, __builtin_ctz(CB), ldk, sl);
    __syncthreads();
    float2 *dst = reinterpret_cast<float2 *>(out_) + o * a.Nout * a.cols;
    s2v *dst16 = reinterpret_cast<s2v *>(out_) + o * a.Nout * a.cols;
    const int half = a.MT / 2;
    const int ntile = (int)((std::min<long long>(CB, a.cols - col0) + 15) / 16);
    for (int mp0 = w * MPW; mp0 < half; mp0 += 4 * MPW) {
        Op ar[MPW][QKM], ai[MPW][QKM], arl[MPW][QKM], ail[MPW][QKM];
#pragma unroll
        for (int u = 0; u < MPW; u++)
#pragma unroll
            for (int q = 0; q < QKM; q++) {
                const int mp = mp0 + u;
                const bool ok = mp < half && q < a.QK;
                const int ir = (mp * a.QK + q) * 64 + lane, ii = ((mp + half) * a.QK + q) * 64 + lane;
                ar[u][q] = ok ? tab[ir] : op_zero<TC>();
                ai[u][q] = ok ? tab[ii] : op_zero<TC>();
                if (SPLIT) {
                    arl[u][q] = ok ? tab_lo[ir] : op_zero<TC>();
                    ail[u][q] = ok ? tab_lo[ii] : op_zero<TC>();
                }
            }
        for (int ct = 0; ct < ntile; ct++) {
            const int cl = 16 * ct + c;
            const long long col = col0 + cl;
            Op bv[QKM];
#pragma unroll
            for (int q = 0; q < QKM; q++)
                bv[q] = q < a.QK ? *reinterpret_cast<const Op *>(sl + cl * ldk + 16 * q + 4 * g) : op_zero<TC>();
#pragma unroll
            for (int u = 0; u < MPW; u++) {
                const int mp = mp0 + u;
                if (mp < half) {
                    f4v accr = f4_zero(), acci = f4_zero();
                    if constexpr (X32) {
                        // two K chunks per 16x16x32 product (QKM is even; chunks past QK are zero)
#pragma unroll
                        for (int q = 0; q < QKM; q += 2) {
                            accr = mma32(ar[u][q], ar[u][q + 1], bv[q], bv[q + 1], accr);
                            acci = mma32(ai[u][q], ai[u][q + 1], bv[q], bv[q + 1], acci);
                        }
                    } else {
#pragma unroll
                        for (int q = 0; q < QKM; q++) {
                            accr = mma16(ar[u][q], bv[q], accr);
                            acci = mma16(ai[u][q], bv[q], acci);
                            if (SPLIT) {
                                accr = mma16(arl[u][q], bv[q], accr);
                                acci = mma16(ail[u][q], bv[q], acci);
                            }
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
        }
    }
}

// LDS of the launch for a contraction of Ninp (padded) input rows (the larger of the two kernels).
size_t axis_lds_bytes(int Ninp, int elem) { return (size_t)(2 * Ninp / 16 <= 8 ? 256 : 64) * (2 * Ninp + 4) * elem; }

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
    if (a.QK <= 8) {
        // widest column block that still gives at least 1024 workgroups (4 per CU)
        a.CB = 256;
        while (a.CB > 64 && outer * ((cols + a.CB - 1) / a.CB) < 1024) a.CB /= 2;
        const size_t lds = (size_t)a.CB * (2 * a.Ninp + 4) * sizeof(TC);
        auto kern = a.QK <= 4 ? (out16 ? k_axis_syn<TC, true, 4, 2> : k_axis_syn<TC, false, 4, 2>)
                              : (out16 ? k_axis_syn<TC, true, 8, 1> : k_axis_syn<TC, false, 8, 1>);
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        const long long blocks = outer * ((cols + a.CB - 1) / a.CB);
        hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), lds, st, in, out, (const Op *)tab,
                           (const Op *)tab_lo, a);
        return hipGetLastError();
    }
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
