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
// registers over all chunks of y.  A wave transforms two planes at a time;
// the bfloat16 variants with room keep the first plane of the current pair in
// a per-wave LDS slot (workgroups are one per CU by registers, so LDS is free)
// and have the next pair's loads in flight during the whole pair transform.
#include "fno_internal.h"
#include "mfma_common.h"

#ifndef FNO_TZY_DEPTH
#define FNO_TZY_DEPTH 2  // y planes whose loads are in flight per wave (even)
#endif
#ifndef FNO_TZY_WAVES_BF16
#define FNO_TZY_WAVES_BF16 2  // waves per SIMD the bfloat16 kernel is compiled for
#endif
#ifndef FNO_TZY_NW_BF16
#define FNO_TZY_NW_BF16 8  // waves per workgroup of the bfloat16 kernel (the y-step tiles are split over them)
#endif
#ifndef FNO_TZY_NW_F32
#define FNO_TZY_NW_F32 4  // the same for the float kernel
#endif
template <typename T> constexpr int tzy_nw() { return sizeof(T) == 2 ? FNO_TZY_NW_BF16 : FNO_TZY_NW_F32; }
#ifndef FNO_TZY_LDS_RING
#define FNO_TZY_LDS_RING 1  // bfloat16: one plane of each wave's current pair in LDS, the next pair's loads in flight
#endif
#ifndef FNO_TZY_Y_X32
#define FNO_TZY_Y_X32 1  // bfloat16 y step: hi and lo basis products as one 16x16x32 product
#endif
#ifndef FNO_TZY_T_X32
#define FNO_TZY_T_X32 1  // bfloat16 t step: the two t chunks as one 16x16x32 product
#endif
#ifndef FNO_TZY_YPAIR
#define FNO_TZY_YPAIR 1  // a wave's plane pair adjacent in y: its T1 values staged as pairs
#endif
#ifndef FNO_TZY_USE
#define FNO_TZY_USE 1  // dtypes that take this kernel where it applies (bit 0 bfloat16, bit 1 float; else the general one)
#endif
#ifndef FNO_TZY_TZ_SPLIT
#define FNO_TZY_TZ_SPLIT 0  // bfloat16: hi + lo basis in the t and z steps (0: hi only; their result is staged in bfloat16)
#endif
#ifndef FNO_TZY_WAVES_F32
#define FNO_TZY_WAVES_F32 1  // waves per SIMD the float kernel is compiled for
#endif

namespace fno {


// Two values as one 4-byte (bfloat16) or 8-byte (float) store at p (2-element aligned).
__device__ __forceinline__ void st_pair_t(float *p, float a, float b) { *reinterpret_cast<float2 *>(p) = make_float2(a, b); }
__device__ __forceinline__ void st_pair_t(__bf16 *p, float a, float b) { *reinterpret_cast<unsigned *>(p) = bf16_pack2(a, b); }

// Byte offset of the plane slots in LDS: after the z-basis fragments and the T1 chunk (16-aligned).
__host__ __device__ constexpr int tzy_ring_offset(int zbytes, int tbytes) { return (zbytes + tbytes + 15) / 16 * 16; }
// Whether a kernel variant keeps plane slots in LDS: bfloat16 with one t/z tile and at most 8 y-step
// accumulator tiles per wave (the others have no registers for the second plane's copy).
__host__ __device__ constexpr bool tzy_ring(int elem, int ntt, int my, int nbw)
{
    return elem == 2 && FNO_TZY_LDS_RING && ntt == 1 && my * nbw <= 8;
}

// NTT: N tiles of the t/z steps (1: Kt <= 8, re|im in one tile; 2: Kt <= 16).
// MY: row tiles of the y step (2 ceil(Ky/16)); NBW: its column tiles per wave.
// NZBM: max z blocks (Nz <= 16*NZBM); MAXKB: max kz blocks.
template <typename T, int NTT, bool SPLIT, int MY, int NBW, int NZBM, int MAXKB>
__global__ void __launch_bounds__(64 * tzy_nw<T>()) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 2 ? FNO_TZY_WAVES_BF16 : FNO_TZY_WAVES_F32))) k_tzy_fwd(const T *__restrict__ x, float2 *__restrict__ t2,
                                                 const typename OpOf<T>::type *__restrict__ tabT,
                                                 const typename OpOf<T>::type *__restrict__ tabT_lo,
                                                 const typename OpOf<T>::type *__restrict__ tabZ,
                                                 const typename OpOf<T>::type *__restrict__ tabZ_lo,
                                                 const typename OpOf<T>::type *__restrict__ tabY,
                                                 const typename OpOf<T>::type *__restrict__ tabY_lo, TzyArgs a)
{
    typedef typename OpOf<T>::type Op;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), g = lane >> 4, c = lane & 15;
    const long long slab = blockIdx.x;
    const int Ny = a.Ny, Nz = a.Nz, Nt = a.Nt, Kz = a.Kz, Kt = a.Kt;
    const T *xs = x + slab * (long long)Ny * Nz * Nt;

    // LDS: z-basis fragments (hi [+ lo where the z step uses it]) then the T1 chunk [col][k] with
    // row stride ldk.
    // RING: then each wave's slot for the first plane of its current pair, [z block][lane][t chunk]
    // (a lane's two fragments side by side: one 16-byte access).
    constexpr bool TS = SPLIT && FNO_TZY_TZ_SPLIT;
    constexpr bool RING = tzy_ring(sizeof(T), NTT, MY, NBW);
    const int nzf = a.NZB * a.MZ * 64;
    Op *zl = reinterpret_cast<Op *>(smem);
    T *tl = reinterpret_cast<T *>(smem + sizeof(Op) * nzf * (TS ? 2 : 1));
    const int ldk = 2 * a.Yc + 4;
    const int ncol = Kz * Kt;
    constexpr int NW = tzy_nw<T>();
    Op *ring0 = reinterpret_cast<Op *>(smem + tzy_ring_offset(nzf * (TS ? 2 : 1) * (int)sizeof(Op),
                                                              Kz * Kt * ldk * (int)sizeof(T)));
    Op *ring = ring0 + (size_t)w * a.NZB * 2 * 64;
    // RING: then two buffers of one chunk's y-basis fragments [hi, lo][K chunk][row tile][lane], the
    // next chunk's loaded one chunk ahead (no global load in the loop but the planes')
    const int nyc1 = a.QY * MY * 64;  // fragments of one chunk (hi or lo)
    Op *ybuf = ring0 + (size_t)NW * a.NZB * 2 * 64;
    if (RING)
        for (int i = threadIdx.x; i < nyc1; i += 64 * NW) {
            ybuf[i] = tabY[i];
            ybuf[nyc1 + i] = tabY_lo[i];
        }
    for (int i = threadIdx.x; i < nzf; i += 64 * NW) {
        zl[i] = tabZ[i];
        if (TS) zl[nzf + i] = tabZ_lo[i];
    }
    Op tb[2][NTT], tbl[2][NTT];
#pragma unroll
    for (int q = 0; q < 2; q++)
#pragma unroll
        for (int nt = 0; nt < NTT; nt++) {
            tb[q][nt] = q < a.NQ ? tabT[(q * NTT + nt) * 64 + lane] : op_zero<T>();
            if (SPLIT && FNO_TZY_TZ_SPLIT) tbl[q][nt] = q < a.NQ ? tabT_lo[(q * NTT + nt) * 64 + lane] : op_zero<T>();
        }

    f4v acc[NBW][MY];  // y-step tiles: column block w + NW nbi, row block mb (re rows < MY/2 <= im rows)
#pragma unroll
    for (int nbi = 0; nbi < NBW; nbi++)
#pragma unroll
        for (int mb = 0; mb < MY; mb++) acc[nbi][mb] = f4_zero();
    const int NT2 = (ncol + 15) / 16;
    const int per_wave = a.Yc / NW;  // planes per wave per chunk

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
    // YP: a wave's planes of a chunk are consecutive in y (yl = per_wave w + slot), so that a pair's
    // T1 values are neighbours; else interleaved over the waves (yl = NW slot + w)
    constexpr bool YP = FNO_TZY_YPAIR;
    auto plane_yl = [&](int s) { return YP ? w * per_wave + s % per_wave : (s % per_wave) * NW + w; };
    auto plane_y = [&](int s) { return (s / per_wave) * a.Yc + plane_yl(s); };
    // t and z steps of two planes (s, s + 1) at once: every z-basis fragment read
    // from LDS feeds both planes, and the two independent MFMA chains overlap.
    // Planes beyond Ny have zero input (guarded loads), hence a zero spectrum.
    // fx(u, zb, q): fragment [zb][q] of plane s + u
    auto do_pair = [&](int s, auto &&fx) {
        // keep the LDS basis reads inside the plane loop (no hoisting into registers)
        asm volatile("" ::: "memory");
        f4v Pc[2][MAXKB][NTT], Ps[2][MAXKB][NTT];  // [plane][kz block][n tile]: cos rows, sin rows
#pragma unroll
        for (int u = 0; u < 2; u++)
#pragma unroll
            for (int kb = 0; kb < MAXKB; kb++)
#pragma unroll
                for (int nt = 0; nt < NTT; nt++) Pc[u][kb][nt] = Ps[u][kb][nt] = f4_zero();
#pragma unroll
        for (int zb = 0; zb < NZBM; zb++) {
            if (zb < a.NZB) {
                Op bz[2][NTT];
#pragma unroll
                for (int nt = 0; nt < NTT; nt++) {
                    f4v c0 = f4_zero(), c1 = f4_zero();
                    if constexpr (SPLIT && !FNO_TZY_TZ_SPLIT && FNO_TZY_T_X32) {
                        // both t chunks in one 16x16x32 product (a chunk past Nt is zero in the
                        // fragments and in the basis)
                        c0 = mma32(fx(0, zb, 0), fx(0, zb, 1), tb[0][nt], tb[1][nt], c0);
                        c1 = mma32(fx(1, zb, 0), fx(1, zb, 1), tb[0][nt], tb[1][nt], c1);
                    } else {
#pragma unroll
                        for (int q = 0; q < 2; q++)
                            if (q < a.NQ) {
                                const Op xa = fx(0, zb, q), xb = fx(1, zb, q);
                                c0 = mma16(xa, tb[q][nt], c0);
                                c1 = mma16(xb, tb[q][nt], c1);
                                if (SPLIT && FNO_TZY_TZ_SPLIT) {
                                    c0 = mma16(xa, tbl[q][nt], c0);
                                    c1 = mma16(xb, tbl[q][nt], c1);
                                }
                            }
                    }
                    bz[0][nt] = to_op<T>(c0);
                    bz[1][nt] = to_op<T>(c1);
                }
#pragma unroll
                for (int kb = 0; kb < MAXKB; kb++)
                    if (kb < a.KB) {
                        const int ic = (zb * a.MZ + kb) * 64 + lane, is = (zb * a.MZ + a.KB + kb) * 64 + lane;
                        const Op zc = zl[ic], zs = zl[is];
                        Op zcl, zsl;
                        if (SPLIT && FNO_TZY_TZ_SPLIT) {
                            zcl = zl[nzf + ic];
                            zsl = zl[nzf + is];
                        }
#pragma unroll
                        for (int u = 0; u < 2; u++)
#pragma unroll
                            for (int nt = 0; nt < NTT; nt++) {
                                Pc[u][kb][nt] = mma16(zc, bz[u][nt], Pc[u][kb][nt]);
                                Ps[u][kb][nt] = mma16(zs, bz[u][nt], Ps[u][kb][nt]);
                                if (SPLIT && FNO_TZY_TZ_SPLIT) {
                                    Pc[u][kb][nt] = mma16(zcl, bz[u][nt], Pc[u][kb][nt]);
                                    Ps[u][kb][nt] = mma16(zsl, bz[u][nt], Ps[u][kb][nt]);
                                }
                            }
                    }
            }
        }
        // combine cos/sin halves into the complex spectrum and stage it in LDS; with YP the two
        // planes are neighbours in y and their values go out as one pair
        auto combine = [&](int u, int kb, int nt, f4v &v) {
            if (NTT == 1) {
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const float ps = row_ror8(Ps[u][kb][0][r]);
                    v[r] = c < 8 ? Pc[u][kb][0][r] + ps : Pc[u][kb][0][r] - ps;
                }
            } else {
#pragma unroll
                for (int r = 0; r < 4; r++)
                    v[r] = nt == 0 ? Pc[u][kb][0][r] + Ps[u][kb][NTT - 1][r] : Pc[u][kb][NTT - 1][r] - Ps[u][kb][0][r];
            }
        };
        const int ri_l = NTT == 1 ? (c >> 3) : 0, kt = NTT == 1 ? (c & 7) : c;
        if constexpr (YP) {
            const int yl = plane_yl(s);  // even: the pair (yl, yl + 1)
#pragma unroll
            for (int kb = 0; kb < MAXKB; kb++) {
                if (kb < a.KB) {
#pragma unroll
                    for (int nt = 0; nt < NTT; nt++) {
                        f4v v0, v1;
                        combine(0, kb, nt, v0);
                        combine(1, kb, nt, v1);
                        const int ri = NTT == 1 ? ri_l : nt;
#pragma unroll
                        for (int r = 0; r < 4; r++) {
                            const int kz = kb * 16 + 4 * g + r;
                            if (kz < Kz && kt < Kt) st_pair_t(tl + (kz * Kt + kt) * ldk + ri * a.Yc + yl, v0[r], v1[r]);
                        }
                    }
                }
            }
        } else {
#pragma unroll
            for (int u = 0; u < 2; u++) {
                const int yl = plane_yl(s + u);
#pragma unroll
                for (int kb = 0; kb < MAXKB; kb++) {
                    if (kb < a.KB) {
#pragma unroll
                        for (int nt = 0; nt < NTT; nt++) {
                            f4v v;
                            combine(u, kb, nt, v);
                            const int ri = NTT == 1 ? ri_l : nt;
#pragma unroll
                            for (int r = 0; r < 4; r++) {
                                const int kz = kb * 16 + 4 * g + r;
                                if (kz < Kz && kt < Kt) tl[(kz * Kt + kt) * ldk + ri * a.Yc + yl] = from_f32<T>(v[r]);
                            }
                        }
                    }
                }
            }
        }
    };
    // end of a chunk of Yc planes: the y step on the staged T1
    auto chunk_end = [&](int s) {
        if ((s + 1) % per_wave == 0) {
            // chunk complete: y step over its 2*Yc K values
            const int ych = s / per_wave;
            __syncthreads();
            for (int q = 0; q < a.QY; q++) {
                Op ay[MY], ayl[MY];
#pragma unroll
                for (int mb = 0; mb < MY; mb++) {
                    if (RING) {
                        const Op *yb = ybuf + (size_t)(ych & 1) * 2 * nyc1 + (q * MY + mb) * 64 + lane;
                        ay[mb] = yb[0];
                        ayl[mb] = yb[nyc1];
                    } else {
                        const int ti = ((ych * a.QY + q) * MY + mb) * 64 + lane;
                        ay[mb] = tabY[ti];
                        if (SPLIT) ayl[mb] = tabY_lo[ti];
                    }
                }
#pragma unroll
                for (int nbi = 0; nbi < NBW; nbi++) {
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
        }
    };

    if constexpr (RING) {
        // the first plane of the loaded pair goes to this wave's LDS slot (each lane reads back
        // only what it wrote, so no barrier), the second stays in registers, and the next pair's
        // loads are issued at once: they have the whole transform of this pair to arrive
        // The next chunk's y-basis fragments (this wave's share) are requested at a chunk's first
        // pair, before that pair's plane loads, and stored at its last pair, once those planes
        // have arrived (loads complete in order).
        constexpr int YV = 4;  // fragments per lane: 2 nyc1 / (64 NW) with the 8-wave, 32-plane chunks
        static_assert(NW == 8, "the plane-slot variant takes 8 waves (4 planes per wave and chunk)");
        Op yv[YV];
        Op xr[2][NZBM][2];
        load_plane(plane_y(0), xr[0]);
        load_plane(plane_y(1), xr[1]);
        for (int s = 0; s < nplanes; s += 2) {  // nplanes is even
            const int ych = s / per_wave;
            const bool first = s % per_wave == 0, last = (s + 2) % per_wave == 0;
#pragma unroll
            for (int zb = 0; zb < NZBM; zb++)
                if (zb < a.NZB)
#pragma unroll
                    for (int q = 0; q < 2; q++) ring[(zb * 64 + lane) * 2 + q] = xr[0][zb][q];
            if (last && ych + 1 < a.NYC) {
                Op *yb = ybuf + (size_t)((ych + 1) & 1) * 2 * nyc1;
#pragma unroll
                for (int k = 0; k < YV; k++) {
                    const int e = (w * YV + k) * 64 + lane;
                    if (e < 2 * nyc1) yb[e] = yv[k];
                }
            }
            if (first && ych + 1 < a.NYC) {
#pragma unroll
                for (int k = 0; k < YV; k++) {
                    const int e = (w * YV + k) * 64 + lane;
                    if (e < 2 * nyc1)
                        yv[k] = e < nyc1 ? tabY[(size_t)(ych + 1) * nyc1 + e] : tabY_lo[(size_t)(ych + 1) * nyc1 + e - nyc1];
                }
            }
            Op x2[NZBM][2];
#pragma unroll
            for (int zb = 0; zb < NZBM; zb++)
#pragma unroll
                for (int q = 0; q < 2; q++) x2[zb][q] = xr[1][zb][q];
            if (s + 2 < nplanes) {
                load_plane(plane_y(s + 2), xr[0]);
                load_plane(plane_y(s + 3), xr[1]);
            }
            do_pair(s, [&](int u, int zb, int q) { return u == 0 ? ring[(zb * 64 + lane) * 2 + q] : x2[zb][q]; });
            chunk_end(s + 1);
        }
    } else {
        // rotating register buffers: DEPTH planes are in flight while a pair is processed
        constexpr int DEPTH = FNO_TZY_DEPTH;
        Op xb[DEPTH][NZBM][2];
#pragma unroll
        for (int k = 0; k < DEPTH; k++) load_plane(plane_y(k), xb[k]);
        for (int s0 = 0; s0 < nplanes; s0 += DEPTH) {  // nplanes is a multiple of DEPTH
#pragma unroll
            for (int k = 0; k < DEPTH; k += 2) {
                const int s = s0 + k;
                do_pair(s, [&](int u, int zb, int q) { return xb[k + u][zb][q]; });
                chunk_end(s + 1);
                if (s + DEPTH < nplanes) load_plane(plane_y(s + DEPTH), xb[k]);
                if (s + 1 + DEPTH < nplanes) load_plane(plane_y(s + 1 + DEPTH), xb[k + 1]);
            }
        }
    }

    // write T2[slab][ky][(kz, kt)] as (re, im): row block mb holds re rows, mb + MY/2 the matching im rows
#pragma unroll
    for (int nbi = 0; nbi < NBW; nbi++) {
        const int nb = w + NW * nbi;
        if (nb < NT2) {
            const int col = nb * 16 + c;
#pragma unroll
            for (int mb = 0; mb < MY / 2; mb++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int ky = mb * 16 + 4 * g + r;
                    if (ky < a.Ky && col < ncol)
                        t2[(slab * a.Ky + ky) * (long long)ncol + col] = make_float2(acc[nbi][mb][r], acc[nbi][mb + MY / 2][r]);
                }
        }
    }
}

// ---------------------------------------------------------------- launcher

size_t tzy_lds_bytes(const TzyArgs &a, int elem, bool split, int my, int nbw)
{
    const size_t zf = (size_t)a.NZB * a.MZ * 64 * 4 * elem * ((split && FNO_TZY_TZ_SPLIT) ? 2 : 1);
    const size_t tl = (size_t)a.Kz * a.Kt * (2 * a.Yc + 4) * elem;
    if (tzy_ring(elem, a.Kt <= 8 ? 1 : 2, my, nbw))  // the waves' plane slots, two chunks' y basis (hi, lo)
        return (size_t)tzy_ring_offset((int)zf, (int)tl) +
               ((size_t)FNO_TZY_NW_BF16 * a.NZB * 2 + (size_t)2 * 2 * (2 * a.Yc / 16) * my) * 64 * 4 * elem;
    return zf + tl;
}

template <typename T, int NTT, int MY, int NBW>
static hipError_t launch_tzy_t(const T *x, float2 *t2, long long slabs, const TzyTabs &tb, const TzyArgs &a,
                               hipStream_t st)
{
    typedef typename OpOf<T>::type Op;
    constexpr bool SPLIT = sizeof(T) == 2;  // bfloat16 kernels use the hi/lo basis
    const size_t lds = tzy_lds_bytes(a, sizeof(T), SPLIT, MY, NBW);
    auto kern = k_tzy_fwd<T, NTT, SPLIT, MY, NBW, 8, 2>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)slabs), dim3(64 * tzy_nw<T>()), lds, st, x, t2, (const Op *)tb.t, (const Op *)tb.t_lo,
                       (const Op *)tb.z, (const Op *)tb.z_lo, (const Op *)tb.y, (const Op *)tb.y_lo, a);
    return hipGetLastError();
}

// (row tiles, column tiles per wave) of the y step
// nw: waves per workgroup of the kernel that will run
static void tzy_tiles(const Dims &d, int nw, int &MY, int &NBW)
{
    MY = 2 * ((d.K[1] + 15) / 16);
    const int NT2 = (d.K[2] * d.K[3] + 15) / 16;
    NBW = (NT2 + nw - 1) / nw;
}

// Whether the MFMA path covers these dimensions.
bool tzy_supported(const Dims &d, int dtype)
{
    if ((FNO_TZY_USE & (dtype == FNO_BF16 ? 1 : 2)) == 0) return false;
    const int Nt = d.N[3], Nz = d.N[2];
    if (Nt % 4 != 0 || Nt > 32 || Nz > 128 || d.K[3] > 16 || d.K[2] > 32) return false;
    int MY, NBW;
    tzy_tiles(d, dtype == FNO_BF16 ? FNO_TZY_NW_BF16 : FNO_TZY_NW_F32, MY, NBW);
    if (MY > 4 || NBW > 8) return false;
    TzyArgs a{};
    a.NZB = (Nz + 15) / 16;
    a.MZ = 2 * ((d.K[2] + 15) / 16);
    a.Kz = d.K[2];
    a.Kt = d.K[3];
    a.Yc = dtype == FNO_BF16 ? 32 : 16;
    const int nbw_t = NBW <= 2 ? 2 : NBW <= 4 ? 4 : 8;  // the instantiated column tiles per wave
    return tzy_lds_bytes(a, dtype == FNO_BF16 ? 2 : 4, dtype == FNO_BF16, MY, nbw_t) <= 160 * 1024;
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

template <typename T, int NTT>
static hipError_t launch_tzy_n(const T *x, float2 *t2, long long slabs, const TzyTabs &tb, const TzyArgs &a, int MY,
                               int NBW, hipStream_t st)
{
    if (MY == 2) return NBW <= 2   ? launch_tzy_t<T, NTT, 2, 2>(x, t2, slabs, tb, a, st)
                       : NBW <= 4 ? launch_tzy_t<T, NTT, 2, 4>(x, t2, slabs, tb, a, st)
                                  : launch_tzy_t<T, NTT, 2, 8>(x, t2, slabs, tb, a, st);
    return NBW <= 2   ? launch_tzy_t<T, NTT, 4, 2>(x, t2, slabs, tb, a, st)
           : NBW <= 4 ? launch_tzy_t<T, NTT, 4, 4>(x, t2, slabs, tb, a, st)
                      : launch_tzy_t<T, NTT, 4, 8>(x, t2, slabs, tb, a, st);
}

template <typename T>
hipError_t launch_tzy(const T *x, float2 *t2, long long slabs, const TzyTabs &tb, const Dims &d, hipStream_t st)
{
    const int dtype = sizeof(T) == 2 ? FNO_BF16 : FNO_F32;
    const TzyArgs a = tzy_args(d, dtype);
    int MY, NBW;
    tzy_tiles(d, tzy_nw<T>(), MY, NBW);
    if (d.K[3] <= 8) return launch_tzy_n<T, 1>(x, t2, slabs, tb, a, MY, NBW, st);
    return launch_tzy_n<T, 2>(x, t2, slabs, tb, a, MY, NBW, st);
}

template hipError_t launch_tzy<float>(const float *, float2 *, long long, const TzyTabs &, const Dims &, hipStream_t);
template hipError_t launch_tzy<__bf16>(const __bf16 *, float2 *, long long, const TzyTabs &, const Dims &,
                                       hipStream_t);

}  // namespace fno
