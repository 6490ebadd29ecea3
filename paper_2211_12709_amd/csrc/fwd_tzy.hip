// fwd_tzy.hip -- forward truncated DFT over t, z and y of one (b, c, x) slab
// per workgroup, on the matrix cores: the F_yzt / S_yzt part of Alg. 2's first
// line (Sec. IV-C), applied to the non-partitioned axes before anything
// leaves the slab.  Truncating each axis as soon as it is transformed keeps
// every intermediate small (the paper's truncate-before-repartition idea used
// on one GPU): the slab is read from HBM once and only the [Ky][Kz][Kt]
// spectrum is written.
//
// Per y plane [Nz][Nt] (one wave per plane):
//   t step:  C1[z][n]  = sum_t x[z][t] Ft[t][n]          n = (re/im, kt)
//   z step:  P[m][n]   = sum_z Ezs[m][z] C1[z][n]        m = (cos/sin, kz)
//   combine: T1[kz][kt] = (Pc_re + Ps_im) + i (Pc_im - Ps_re)   (exp(-i theta) product)
// T1 of Yc planes is staged in LDS, then
//   y step:  T2[(re/im, ky)][(kz, kt)] += sum_(re/im', y) Ay[..][..] T1[(re/im', y)][(kz, kt)]
// with Ay = [[cos, sin], [-sin, cos]] of exp(-i theta_y), accumulated in
// registers over all chunks of y.
#include "fno_internal.h"
#include "mfma_common.h"

namespace fno {

struct TzyArgs {
    int Ny, Nz, Nt, Ky, Kz, Kt;
    int NQ, NZB, KB, MZ, MY, Yc, QY, NYC;
};

// Accumulator tile i of a wave: column block w + 4 (i / MY); within it, tile
// pairs (2p, 2p + 1) are the re and im row blocks p and p + MY/2.
__device__ __forceinline__ int tile_mb(int i, int MY)
{
    const int rem = i % MY;
    return (rem & 1) * (MY >> 1) + (rem >> 1);
}

// NTT: N tiles of the t/z steps (1: Kt <= 8, re|im in one tile; 2: Kt <= 16).
// MAXT: accumulator tiles per wave in the y step.  NZBM: max z blocks (Nz <= 16*NZBM).
template <typename T, int NTT, bool SPLIT, int MAXT, int NZBM, int MAXKB>
__global__ void __launch_bounds__(256) k_tzy_fwd(const T *__restrict__ x, float2 *__restrict__ t2,
                                                 const typename OpOf<T>::type *__restrict__ tabT,
                                                 const typename OpOf<T>::type *__restrict__ tabT_lo,
                                                 const typename OpOf<T>::type *__restrict__ tabZ,
                                                 const typename OpOf<T>::type *__restrict__ tabZ_lo,
                                                 const typename OpOf<T>::type *__restrict__ tabY,
                                                 const typename OpOf<T>::type *__restrict__ tabY_lo, TzyArgs a)
{
    typedef typename OpOf<T>::type Op;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, c = lane & 15;
    const long long slab = blockIdx.x;
    const int Ny = a.Ny, Nz = a.Nz, Nt = a.Nt, Kz = a.Kz, Kt = a.Kt;
    const T *xs = x + slab * (long long)Ny * Nz * Nt;

    // LDS: z-basis fragments (hi [+ lo]) then the T1 chunk [col][k] with row stride ldk.
    const int nzf = a.NZB * a.MZ * 64;
    Op *zl = reinterpret_cast<Op *>(smem);
    T *tl = reinterpret_cast<T *>(smem + sizeof(Op) * nzf * (SPLIT ? 2 : 1));
    const int ldk = 2 * a.Yc + 4;
    const int ncol = Kz * Kt;
    for (int i = threadIdx.x; i < nzf; i += 256) {
        zl[i] = tabZ[i];
        if (SPLIT) zl[nzf + i] = tabZ_lo[i];
    }
    Op tb[2][NTT], tbl[2][NTT];
#pragma unroll
    for (int q = 0; q < 2; q++)
#pragma unroll
        for (int nt = 0; nt < NTT; nt++) {
            tb[q][nt] = q < a.NQ ? tabT[(q * NTT + nt) * 64 + lane] : op_zero<T>();
            if (SPLIT) tbl[q][nt] = q < a.NQ ? tabT_lo[(q * NTT + nt) * 64 + lane] : op_zero<T>();
        }

    f4v acc[MAXT];
#pragma unroll
    for (int i = 0; i < MAXT; i++) acc[i] = f4_zero();
    const int NT2 = (ncol + 15) / 16;
    const int per_wave = a.Yc / 4;  // planes per wave per chunk

    // fragments of one plane: dst[zb][q] = x[y][zb*16 + c][16 q + 4 g .. + 3]
    auto load_plane = [&](int y, Op (&dst)[NZBM][2]) {
#pragma unroll
        for (int zb = 0; zb < NZBM; zb++)
#pragma unroll
            for (int q = 0; q < 2; q++) {
                const int z = zb * 16 + c, t0 = 16 * q + 4 * g;
                if (y < Ny && zb < a.NZB && q < a.NQ && z < Nz && t0 < Nt)
                    dst[zb][q] = *reinterpret_cast<const Op *>(xs + ((long long)y * Nz + z) * Nt + t0);
                else
                    dst[zb][q] = op_zero<T>();
            }
    };
    __syncthreads();

    const int nplanes = a.NYC * per_wave;  // plane slots of this wave
    auto plane_y = [&](int s) { return (s / per_wave) * a.Yc + (s % per_wave) * 4 + w; };
    // one plane's t and z steps, staged into LDS (or zeros for a padding plane)
    auto do_plane = [&](int s, const Op (&xa)[NZBM][2]) {
        const int yl = (s % per_wave) * 4 + w;
        const int y = plane_y(s);
        // keep the LDS basis reads inside the plane loop (no hoisting into registers)
        asm volatile("" ::: "memory");
        if (y < Ny) {
            // Pc: cos rows (kz block kb), Ps: sin rows, both [kb][nt]
            f4v Pc[MAXKB][NTT], Ps[MAXKB][NTT];
#pragma unroll
            for (int kb = 0; kb < MAXKB; kb++)
#pragma unroll
                for (int nt = 0; nt < NTT; nt++) Pc[kb][nt] = Ps[kb][nt] = f4_zero();
#pragma unroll
            for (int zb = 0; zb < NZBM; zb++) {
                if (zb < a.NZB) {
                    f4v c1[NTT];
#pragma unroll
                    for (int nt = 0; nt < NTT; nt++) {
                        c1[nt] = f4_zero();
#pragma unroll
                        for (int q = 0; q < 2; q++)
                            if (q < a.NQ) {
                                c1[nt] = mma16(xa[zb][q], tb[q][nt], c1[nt]);
                                if (SPLIT) c1[nt] = mma16(xa[zb][q], tbl[q][nt], c1[nt]);
                            }
                    }
#pragma unroll
                    for (int nt = 0; nt < NTT; nt++) {
                        const Op bz = to_op<T>(c1[nt]);
#pragma unroll
                        for (int kb = 0; kb < MAXKB; kb++)
                            if (kb < a.KB) {
                                const int ic = (zb * a.MZ + kb) * 64 + lane, is = (zb * a.MZ + a.KB + kb) * 64 + lane;
                                Pc[kb][nt] = mma16(zl[ic], bz, Pc[kb][nt]);
                                Ps[kb][nt] = mma16(zl[is], bz, Ps[kb][nt]);
                                if (SPLIT) {
                                    Pc[kb][nt] = mma16(zl[nzf + ic], bz, Pc[kb][nt]);
                                    Ps[kb][nt] = mma16(zl[nzf + is], bz, Ps[kb][nt]);
                                }
                            }
                    }
                }
            }
            // combine cos/sin halves into the complex spectrum and stage it in LDS
#pragma unroll
            for (int kb = 0; kb < MAXKB; kb++) {
                if (kb < a.KB) {
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
        } else {
            for (int col = lane; col < ncol; col += 64) {
                tl[col * ldk + yl] = from_f32<T>(0.f);
                tl[col * ldk + a.Yc + yl] = from_f32<T>(0.f);
            }
        }
    };
    // end of a chunk of Yc planes: the y step on the staged T1
    auto chunk_end = [&](int s) {
        if ((s + 1) % per_wave == 0) {
            // chunk complete: y step over its 2*Yc K values
            const int ych = s / per_wave;
            __syncthreads();
#pragma unroll
            for (int i = 0; i < MAXT; i++) {
                const int mb = tile_mb(i, a.MY), nb = w + 4 * (i / a.MY);
                if (nb < NT2) {
                    const int col = nb * 16 + c;
                    for (int q = 0; q < a.QY; q++) {
                        const Op ay = tabY[((ych * a.QY + q) * a.MY + mb) * 64 + lane];
                        const Op bt = col < ncol ? *reinterpret_cast<const Op *>(tl + col * ldk + 16 * q + 4 * g)
                                                 : op_zero<T>();
                        acc[i] = mma16(ay, bt, acc[i]);
                        if (SPLIT) acc[i] = mma16(tabY_lo[((ych * a.QY + q) * a.MY + mb) * 64 + lane], bt, acc[i]);
                    }
                }
            }
            __syncthreads();
        }
    };

    Op xa[NZBM][2], xb[NZBM][2];
    load_plane(plane_y(0), xa);
    for (int s = 0; s < nplanes; s += 2) {  // nplanes is even: ping-pong without register copies
        load_plane(plane_y(s + 1), xb);
        do_plane(s, xa);
        chunk_end(s);
        if (s + 2 < nplanes) load_plane(plane_y(s + 2), xa);
        do_plane(s + 1, xb);
        chunk_end(s + 1);
    }

    // write T2[slab][ky][(kz, kt)] as (re, im): tile i (even) holds re rows, tile i + 1 the matching im rows
#pragma unroll
    for (int i = 0; i < MAXT; i += 2) {
        const int mb = tile_mb(i, a.MY), nb = w + 4 * (i / a.MY);
        if (nb < NT2) {
            const int col = nb * 16 + c;
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int ky = mb * 16 + 4 * g + r;
                if (ky < a.Ky && col < ncol)
                    t2[(slab * a.Ky + ky) * (long long)ncol + col] = make_float2(acc[i][r], acc[i + 1][r]);
            }
        }
    }
}

// ---------------------------------------------------------------- launcher
struct TzyTabs {
    const void *t, *t_lo, *z, *z_lo, *y, *y_lo;
};

size_t tzy_lds_bytes(const TzyArgs &a, int elem, bool split)
{
    const size_t zf = (size_t)a.NZB * a.MZ * 64 * 4 * elem * (split ? 2 : 1);
    const size_t tl = (size_t)a.Kz * a.Kt * (2 * a.Yc + 4) * elem;
    return zf + tl;
}

template <typename T, int NTT, bool SPLIT, int MAXT>
static hipError_t launch_tzy_t(const T *x, float2 *t2, long long slabs, const TzyTabs &tb, const TzyArgs &a,
                               hipStream_t st)
{
    typedef typename OpOf<T>::type Op;
    const size_t lds = tzy_lds_bytes(a, sizeof(T), SPLIT);
    auto kern = k_tzy_fwd<T, NTT, SPLIT, MAXT, 8, 4>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)slabs), dim3(256), lds, st, x, t2, (const Op *)tb.t, (const Op *)tb.t_lo,
                       (const Op *)tb.z, (const Op *)tb.z_lo, (const Op *)tb.y, (const Op *)tb.y_lo, a);
    return hipGetLastError();
}

// Whether the MFMA path covers these dimensions.
bool tzy_supported(const Dims &d, int dtype)
{
    const int Nt = d.N[3], Nz = d.N[2];
    if (Nt % 4 != 0 || Nt > 32 || Nz > 128 || d.K[3] > 16 || d.K[2] > 64) return false;
    const int Kzp = (d.K[2] + 15) / 16 * 16, Kyp = (d.K[1] + 15) / 16 * 16;
    const int MY = 2 * Kyp / 16, NT2 = (d.K[2] * d.K[3] + 15) / 16;
    if (MY * ((NT2 + 3) / 4) > 32) return false;
    TzyArgs a{};
    a.NZB = (Nz + 15) / 16;
    a.MZ = 2 * Kzp / 16;
    a.Kz = d.K[2];
    a.Kt = d.K[3];
    a.Yc = dtype == FNO_BF16 ? 32 : 16;
    return tzy_lds_bytes(a, dtype == FNO_BF16 ? 2 : 4, dtype == FNO_BF16) <= 160 * 1024;
}

TzyArgs tzy_args(const Dims &d, int dtype)
{
    TzyArgs a{};
    a.Ny = d.N[1];
    a.Nz = d.N[2];
    a.Nt = d.N[3];
    a.Ky = d.K[1];
    a.Kz = d.K[2];
    a.Kt = d.K[3];
    a.NQ = (a.Nt + 15) / 16;
    a.NZB = (a.Nz + 15) / 16;
    a.KB = (a.Kz + 15) / 16;
    a.MZ = 2 * a.KB;
    a.MY = 2 * ((a.Ky + 15) / 16);
    a.Yc = dtype == FNO_BF16 ? 32 : 16;
    a.QY = 2 * a.Yc / 16;
    a.NYC = (a.Ny + a.Yc - 1) / a.Yc;
    return a;
}

template <typename T>
hipError_t launch_tzy(const T *x, float2 *t2, long long slabs, const TzyTabs &tb, const Dims &d, hipStream_t st)
{
    const int dtype = sizeof(T) == 2 ? FNO_BF16 : FNO_F32;
    const TzyArgs a = tzy_args(d, dtype);
    const int NT2 = (a.Kz * a.Kt + 15) / 16;
    const int tiles = a.MY * ((NT2 + 3) / 4);
    constexpr bool split = sizeof(T) == 2;  // bfloat16 kernels use the hi/lo basis
    if (d.K[3] <= 8) {
        if (tiles <= 16) return launch_tzy_t<T, 1, split, 16>(x, t2, slabs, tb, a, st);
        return launch_tzy_t<T, 1, split, 32>(x, t2, slabs, tb, a, st);
    }
    if (tiles <= 16) return launch_tzy_t<T, 2, split, 16>(x, t2, slabs, tb, a, st);
    return launch_tzy_t<T, 2, split, 32>(x, t2, slabs, tb, a, st);
}

template hipError_t launch_tzy<float>(const float *, float2 *, long long, const TzyTabs &, const Dims &, hipStream_t);
template hipError_t launch_tzy<__bf16>(const __bf16 *, float2 *, long long, const TzyTabs &, const Dims &,
                                       hipStream_t);

}  // namespace fno
