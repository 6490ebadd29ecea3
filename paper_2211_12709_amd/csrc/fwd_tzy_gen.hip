// fwd_tzy_gen.hip -- forward truncated DFT over t, z and y of one (b, c, x)
// slab per workgroup on the matrix cores, for the shapes the plane-pair
// kernel of fwd_tzy.hip does not cover: any Nz, Nt up to 96 (odd or not a
// multiple of 4), up to 48 retained z or y modes (the batched CO2-shaped
// block keeps 40) and 16 retained t bins.  Same operation and fragment
// conventions as fwd_tzy.hip (the F_yzt / S_yzt part of Alg. 2's first line,
// Sec. IV-C, each axis truncated as soon as it is transformed, the t,z
// intermediate never leaving the workgroup):
//   t step:  C1[z][n]  = sum_t x[z][t] Ft[t][n]          n = (re/im, kt)
//   z step:  P[m][n]   = sum_z Ezs[m][z] C1[z][n]        m = (cos/sin, kz)
//   combine: T1[kz][kt] = (Pc_re + Ps_im) + i (Pc_im - Ps_re)
//   y step:  T2[(re/im, ky)][(kz, kt)] += Ay[..][(re/im', y)] T1[(re/im', y)][(kz, kt)]
// Differences from the plane-pair kernel: a wave transforms one y plane at a
// time and streams it one 16-row z block at a time (the next block's loads in
// flight while the current one is multiplied), so the registers a plane needs
// do not grow with Nz or Nt; the t basis sits in LDS beside the z basis; rows
// whose t run is not 4-aligned in memory are read element by element.
#include "fno_internal.h"
#include "mfma_common.h"

#ifndef FNO_TZYG_NW
#define FNO_TZYG_NW 8  // waves per workgroup (the y-step tiles are split over them)
#endif

#ifndef FNO_TZYG_PD_SHORT
#define FNO_TZYG_PD_SHORT 2  // z blocks in flight per wave when a row has at most 2 t chunks
#endif
#ifndef FNO_TZYG_PD_LONG
#define FNO_TZYG_PD_LONG 2  // the same for longer rows
#endif
#ifndef FNO_TZYG_VEC1
#define FNO_TZYG_VEC1 1  // bfloat16, even Nt not a multiple of 4: a run of 4 t as one dword-aligned access (else two)
#endif

#ifndef FNO_TZY_T_X32
#define FNO_TZY_T_X32 1  // bfloat16 t step: t chunks in pairs as 16x16x32 products
#endif
#ifndef FNO_TZY_Y_X32
#define FNO_TZY_Y_X32 1  // bfloat16 y step: hi and lo basis products as one 16x16x32 product
#endif
#ifndef FNO_TZY_TZ_SPLIT
#define FNO_TZY_TZ_SPLIT 0  // bfloat16: hi + lo basis in the t and z steps (0: hi only; their result is staged in bfloat16)
#endif

namespace fno {

TzyArgs tzy_args(const Dims &d, int dtype);

constexpr int kTzgMaxKB = 3;   // kz blocks of 16 (2 mz <= 48)
constexpr int kTzgNBW = 4;     // y-step column tiles per wave (Kz Kt <= 16 * 4 * waves)

// Two consecutive values of storage type T as floats (one 4- or 8-byte access, 2-element aligned).
__device__ __forceinline__ float2 ld_pair_t(const float *p) { return *reinterpret_cast<const float2 *>(p); }
__device__ __forceinline__ float2 ld_pair_t(const __bf16 *p)
{
    const unsigned u = *reinterpret_cast<const unsigned *>(p);
    return make_float2(__uint_as_float(u << 16), __uint_as_float(u & 0xffff0000u));
}

// 4 consecutive t of row z starting at t0 (t0 a multiple of 4) as an operand fragment; values at
// t >= Nt are zero.  ALN 2: the row start is 4-element aligned (Nt % 4 == 0), one vector load;
// ALN 1: Nt even, two pair loads; ALN 0: element by element.
template <typename T, int ALN>
__device__ __forceinline__ typename OpOf<T>::type load_t4(const T *row, int t0, int Nt)
{
    typedef typename OpOf<T>::type Op;
    if (ALN == 2) {
        if (t0 < Nt) return *reinterpret_cast<const Op *>(row + t0);
        return op_zero<T>();
    }
    float v[4];
    if (ALN == 1) {
        // Nt even: the run starts on 4 bytes; a whole run is one dword-aligned access
        if (FNO_TZYG_VEC1 && sizeof(T) == 2 && t0 + 4 <= Nt) return ld_dword_aligned<Op>(row + t0);
#pragma unroll
        for (int j = 0; j < 4; j += 2) {
            const float2 f = t0 + j < Nt ? ld_pair_t(row + t0 + j) : make_float2(0.f, 0.f);
            v[j] = f.x;
            v[j + 1] = f.y;
        }
    } else {
#pragma unroll
        for (int j = 0; j < 4; j++) v[j] = t0 + j < Nt ? to_f32(row[t0 + j]) : 0.f;
    }
    return op_from4<T>(v[0], v[1], v[2], v[3]);
}

// NTT: n tiles of the t/z steps (1: Kt <= 8; 2: Kt <= 16).  MY: row tiles of the y step.
// NQM: t chunks of 16 a z block holds (NQ <= NQM).  ALN: row alignment class (load_t4).
template <typename T, int NTT, bool SPLIT, int MY, int NQM, int ALN>
__global__ void __launch_bounds__(64 * FNO_TZYG_NW) __attribute__((amdgpu_waves_per_eu(2)))
k_tzy_gen(const T *__restrict__ x, float2 *__restrict__ t2, const typename OpOf<T>::type *__restrict__ tabT,
          const typename OpOf<T>::type *__restrict__ tabT_lo, const typename OpOf<T>::type *__restrict__ tabZ,
          const typename OpOf<T>::type *__restrict__ tabZ_lo, const typename OpOf<T>::type *__restrict__ tabY,
          const typename OpOf<T>::type *__restrict__ tabY_lo, TzyArgs a)
{
    typedef typename OpOf<T>::type Op;
    constexpr int NW = FNO_TZYG_NW;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), g = lane >> 4, c = lane & 15;
    const long long slab = blockIdx.x;
    const int Ny = a.Ny, Nz = a.Nz, Nt = a.Nt, Kz = a.Kz, Kt = a.Kt, NQ = a.NQ, NZB = a.NZB, KB = a.KB;
    const T *xs = x + slab * (long long)Ny * Nz * Nt;

    // LDS: z-basis fragments [zb][mb] (hi, then lo), t-basis fragments [q][nt] (hi, then lo),
    // then the T1 chunk [col][k] with row stride ldk
    // (the lo halves only where the t and z steps use them)
    constexpr bool TS = SPLIT && FNO_TZY_TZ_SPLIT;
    const int nzf = NZB * a.MZ * 64, ntf = NQ * NTT * 64;
    Op *zl = reinterpret_cast<Op *>(smem);
    Op *tlb = zl + nzf * (TS ? 2 : 1);
    T *tl = reinterpret_cast<T *>(tlb + ntf * (TS ? 2 : 1));
    const int ldk = 2 * a.Yc + 4;
    const int ncol = Kz * Kt;
    for (int i = threadIdx.x; i < nzf; i += 64 * NW) {
        zl[i] = tabZ[i];
        if (TS) zl[nzf + i] = tabZ_lo[i];
    }
    for (int i = threadIdx.x; i < ntf; i += 64 * NW) {
        tlb[i] = tabT[i];
        if (TS) tlb[ntf + i] = tabT_lo[i];
    }

    f4v acc[kTzgNBW][MY];  // y-step tiles: column block w + NW nbi, row block mb
#pragma unroll
    for (int nbi = 0; nbi < kTzgNBW; nbi++)
#pragma unroll
        for (int mb = 0; mb < MY; mb++) acc[nbi][mb] = f4_zero();
    const int NT2 = (ncol + 15) / 16;
    const int per_wave = a.Yc / NW;
    const int nplanes = a.NYC * per_wave;  // plane slots of this wave (the same for every wave)
    auto plane_y = [&](int s) { return (s / per_wave) * a.Yc + (s % per_wave) * NW + w; };

    // the t-chunk fragments of z block zb of plane y: dst[q] = x[y][16 zb + c][16 q + 4 g .. + 3]
    auto load_zb = [&](int y, int zb, Op (&dst)[NQM]) {
        const int z = 16 * zb + c;
        const bool ok = y < Ny && z < Nz;
        const T *row = xs + ((long long)(ok ? y : 0) * Nz + (ok ? z : 0)) * Nt;
#pragma unroll
        for (int q = 0; q < NQM; q++)
            dst[q] = (ok && q < NQ) ? load_t4<T, ALN>(row, 16 * q + 4 * g, Nt) : op_zero<T>();
    };
    __syncthreads();

    // end of a chunk of Yc planes: the y step on the staged T1
    auto chunk_end = [&](int s) {
        if ((s + 1) % per_wave != 0) return;
        const int ych = s / per_wave;
        __syncthreads();
        for (int q = 0; q < a.QY; q++) {
            Op ay[MY], ayl[MY];
#pragma unroll
            for (int mb = 0; mb < MY; mb++) {
                const int ti = ((ych * a.QY + q) * MY + mb) * 64 + lane;
                ay[mb] = tabY[ti];
                if (SPLIT) ayl[mb] = tabY_lo[ti];
            }
#pragma unroll
            for (int nbi = 0; nbi < kTzgNBW; nbi++) {
                const int nb = w + NW * nbi;
                if (nb < NT2) {
                    const int col = nb * 16 + c;
                    const Op bt = col < ncol ? *reinterpret_cast<const Op *>(tl + col * ldk + 16 * q + 4 * g)
                                             : op_zero<T>();
#pragma unroll
                    for (int mb = 0; mb < MY; mb++) {
                        // bfloat16: the hi and lo basis products in one 16x16x32 product (all of this
                        // accumulator's products are)
                        if (SPLIT && FNO_TZY_Y_X32) {
                            acc[nbi][mb] = mma32(ay[mb], ayl[mb], bt, bt, acc[nbi][mb]);
                        } else {
                            acc[nbi][mb] = mma16(ay[mb], bt, acc[nbi][mb]);
                            if (SPLIT) acc[nbi][mb] = mma16(ayl[mb], bt, acc[nbi][mb]);
                        }
                    }
                }
            }
        }
        __syncthreads();
    };

    // z blocks in flight per wave: PD (a ring shifted by one block per step, so that every index is
    // static); few t chunks per row leave room for more
    constexpr int PD = NQM <= 2 ? FNO_TZYG_PD_SHORT : FNO_TZYG_PD_LONG;
    const int nblk = nplanes * NZB;
    auto load_blk = [&](int L, Op (&dst)[NQM]) {
        if (L < nblk) {
            const int sp = L / NZB;
            load_zb(plane_y(sp), L - sp * NZB, dst);
        }
    };
    Op ring[PD][NQM], cur[NQM];
#pragma unroll
    for (int k = 0; k < PD; k++) load_blk(k, ring[k]);
    for (int s = 0; s < nplanes; s++) {
        const int y = plane_y(s);
        f4v Pc[kTzgMaxKB][NTT], Ps[kTzgMaxKB][NTT];
#pragma unroll
        for (int kb = 0; kb < kTzgMaxKB; kb++)
#pragma unroll
            for (int nt = 0; nt < NTT; nt++) Pc[kb][nt] = Ps[kb][nt] = f4_zero();
        for (int zb = 0; zb < NZB; zb++) {
            // this block leaves the ring; the block PD steps ahead (across planes) enters it
#pragma unroll
            for (int q = 0; q < NQM; q++) cur[q] = ring[0][q];
#pragma unroll
            for (int k = 0; k + 1 < PD; k++)
#pragma unroll
                for (int q = 0; q < NQM; q++) ring[k][q] = ring[k + 1][q];
            load_blk(s * NZB + zb + PD, ring[PD - 1]);
            // t step: C1 tile of this z block, as the z step's B operand
            Op bz[NTT];
#pragma unroll
            for (int nt = 0; nt < NTT; nt++) {
                f4v c1 = f4_zero();
                if constexpr (SPLIT && !TS && FNO_TZY_T_X32) {
                    // t chunks in pairs, one 16x16x32 product each (chunks past Nt are zero: the
                    // fragments by their loads, the basis here)
#pragma unroll
                    for (int q = 0; q < NQM; q += 2)
                        if (q < NQ) {
                            const Op t0 = tlb[(q * NTT + nt) * 64 + lane];
                            const Op t1 = q + 1 < NQ ? tlb[((q + 1) * NTT + nt) * 64 + lane] : op_zero<T>();
                            c1 = mma32(cur[q], q + 1 < NQM ? cur[q + 1] : op_zero<T>(), t0, t1, c1);
                        }
                } else {
#pragma unroll
                    for (int q = 0; q < NQM; q++)
                        if (q < NQ) {
                            const int ti = (q * NTT + nt) * 64 + lane;
                            c1 = mma16(cur[q], tlb[ti], c1);
                            if (TS) c1 = mma16(cur[q], tlb[ntf + ti], c1);
                        }
                }
                bz[nt] = to_op<T>(c1);
            }
            // z step
#pragma unroll
            for (int kb = 0; kb < kTzgMaxKB; kb++)
                if (kb < KB) {
                    const int ic = (zb * a.MZ + kb) * 64 + lane, is = (zb * a.MZ + KB + kb) * 64 + lane;
                    const Op zc = zl[ic], zs = zl[is];
#pragma unroll
                    for (int nt = 0; nt < NTT; nt++) {
                        Pc[kb][nt] = mma16(zc, bz[nt], Pc[kb][nt]);
                        Ps[kb][nt] = mma16(zs, bz[nt], Ps[kb][nt]);
                    }
                    if (TS) {
                        const Op zcl = zl[nzf + ic], zsl = zl[nzf + is];
#pragma unroll
                        for (int nt = 0; nt < NTT; nt++) {
                            Pc[kb][nt] = mma16(zcl, bz[nt], Pc[kb][nt]);
                            Ps[kb][nt] = mma16(zsl, bz[nt], Ps[kb][nt]);
                        }
                    }
                }
        }
        // combine the cos/sin halves into the complex spectrum and stage it in LDS
        const int yl = (s % per_wave) * NW + w;
#pragma unroll
        for (int kb = 0; kb < kTzgMaxKB; kb++) {
            if (kb < KB) {
#pragma unroll
                for (int nt = 0; nt < NTT; nt++) {
                    f4v v;
                    if (NTT == 1) {
#pragma unroll
                        for (int r = 0; r < 4; r++) {
                            const float ps = row_ror8(Ps[kb][0][r]);
                            v[r] = c < 8 ? Pc[kb][0][r] + ps : Pc[kb][0][r] - ps;
                        }
                    } else {
#pragma unroll
                        for (int r = 0; r < 4; r++)
                            v[r] = nt == 0 ? Pc[kb][0][r] + Ps[kb][NTT - 1][r] : Pc[kb][NTT - 1][r] - Ps[kb][0][r];
                    }
                    const int ri = NTT == 1 ? (c >> 3) : nt;
                    const int kt = NTT == 1 ? (c & 7) : c;
#pragma unroll
                    for (int r = 0; r < 4; r++) {
                        const int kz = kb * 16 + 4 * g + r;
                        if (kz < Kz && kt < Kt) tl[(kz * Kt + kt) * ldk + ri * a.Yc + yl] = from_f32<T>(v[r]);
                    }
                }
            }
        }
        (void)y;
        chunk_end(s);
    }

    // T2[slab][ky][(kz, kt)] as (re, im): row block mb holds re rows, mb + MY/2 the matching im rows
#pragma unroll
    for (int nbi = 0; nbi < kTzgNBW; nbi++) {
        const int nb = w + NW * nbi;
        if (nb < NT2) {
            const int col = nb * 16 + c;
#pragma unroll
            for (int mb = 0; mb < MY / 2; mb++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int ky = mb * 16 + 4 * g + r;
                    if (ky < a.Ky && col < ncol)
                        t2[(slab * a.Ky + ky) * (long long)ncol + col] =
                            make_float2(acc[nbi][mb][r], acc[nbi][mb + MY / 2][r]);
                }
        }
    }
}

// ---------------------------------------------------------------- launcher

static size_t tzy_gen_lds(const TzyArgs &a, int elem, bool split)
{
    // bytes of one fragment entry (hi, and lo where the t and z steps use it)
    const size_t op = 4 * (size_t)elem * ((split && FNO_TZY_TZ_SPLIT) ? 2 : 1);
    return (size_t)a.NZB * a.MZ * 64 * op + (size_t)a.NQ * (a.Kt <= 8 ? 1 : 2) * 64 * op +
           (size_t)a.Kz * a.Kt * (2 * a.Yc + 4) * elem;
}

bool tzy_gen_supported(const Dims &d, int dtype)
{
    const TzyArgs a = tzy_args(d, dtype);
    if (a.Kt > 16 || a.KB > kTzgMaxKB || a.MY > 6 || a.NQ > 6) return false;
    if ((a.Kz * a.Kt + 15) / 16 > kTzgNBW * FNO_TZYG_NW) return false;
    if (a.Yc % FNO_TZYG_NW != 0) return false;
    const int elem = dtype == FNO_BF16 ? 2 : 4;
    return tzy_gen_lds(a, elem, dtype == FNO_BF16) <= 160 * 1024;
}

template <typename T, int NTT, int MY, int NQM, int ALN>
static hipError_t launch_tzy_gen_t(const T *x, float2 *t2, long long slabs, const TzyTabs &tb, const TzyArgs &a,
                                   hipStream_t st)
{
    typedef typename OpOf<T>::type Op;
    constexpr bool SPLIT = sizeof(T) == 2;
    const size_t lds = tzy_gen_lds(a, sizeof(T), SPLIT);
    auto kern = k_tzy_gen<T, NTT, SPLIT, MY, NQM, ALN>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)slabs), dim3(64 * FNO_TZYG_NW), lds, st, x, t2, (const Op *)tb.t,
                       (const Op *)tb.t_lo, (const Op *)tb.z, (const Op *)tb.z_lo, (const Op *)tb.y,
                       (const Op *)tb.y_lo, a);
    return hipGetLastError();
}

template <typename T, int NTT, int MY>
static hipError_t launch_tzy_gen_q(const T *x, float2 *t2, long long slabs, const TzyTabs &tb, const TzyArgs &a,
                                   hipStream_t st)
{
    const int aln = a.Nt % 4 == 0 ? 2 : a.Nt % 2 == 0 ? 1 : 0;
#define FNO_TZYG_Q(NQM_)                                                                                          \
    return aln == 2   ? launch_tzy_gen_t<T, NTT, MY, NQM_, 2>(x, t2, slabs, tb, a, st)                             \
           : aln == 1 ? launch_tzy_gen_t<T, NTT, MY, NQM_, 1>(x, t2, slabs, tb, a, st)                             \
                      : launch_tzy_gen_t<T, NTT, MY, NQM_, 0>(x, t2, slabs, tb, a, st)
    if (a.NQ <= 2) FNO_TZYG_Q(2);
    if (a.NQ <= 4) FNO_TZYG_Q(4);
    FNO_TZYG_Q(6);
#undef FNO_TZYG_Q
}

template <typename T, int NTT>
static hipError_t launch_tzy_gen_m(const T *x, float2 *t2, long long slabs, const TzyTabs &tb, const TzyArgs &a,
                                   hipStream_t st)
{
    if (a.MY <= 2) return launch_tzy_gen_q<T, NTT, 2>(x, t2, slabs, tb, a, st);
    if (a.MY <= 4) return launch_tzy_gen_q<T, NTT, 4>(x, t2, slabs, tb, a, st);
    return launch_tzy_gen_q<T, NTT, 6>(x, t2, slabs, tb, a, st);
}

template <typename T>
hipError_t launch_tzy_gen(const T *x, float2 *t2, long long slabs, const TzyTabs &tb, const Dims &d, hipStream_t st)
{
    const TzyArgs a = tzy_args(d, sizeof(T) == 2 ? FNO_BF16 : FNO_F32);
    if (!tzy_gen_supported(d, sizeof(T) == 2 ? FNO_BF16 : FNO_F32)) return hipErrorInvalidValue;
    if (a.Kt <= 8) return launch_tzy_gen_m<T, 1>(x, t2, slabs, tb, a, st);
    return launch_tzy_gen_m<T, 2>(x, t2, slabs, tb, a, st);
}

template hipError_t launch_tzy_gen<float>(const float *, float2 *, long long, const TzyTabs &, const Dims &,
                                          hipStream_t);
template hipError_t launch_tzy_gen<__bf16>(const __bf16 *, float2 *, long long, const TzyTabs &, const Dims &,
                                           hipStream_t);

}  // namespace fno
