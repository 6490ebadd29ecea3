// zt_epi.h -- synthesis over z and t of one (b, x, y) plane for all
// channels at once, on the matrix cores, fused with the epilogue that needs
// every channel at a point:
//   EPI_PLAIN  out[c] = S_c                                     (Alg. 2, line 3)
//   EPI_BLOCK  out[o] = GELU(S_o + sum_i W_pw[o][i] x[i] + b[o])   (Alg. 1, FNO block)
//   EPI_BWD    z = S_o + sum_i W_pw[o][i] x[i] + b[o] recomputed, out[o] = gz = gy GELU'(z),
//              and partial sums of gz x^T and gz for the pointwise-weight gradients
//   EPI_ADJ    out[i] (+)= S_i + sum_o W_pw[o][i] gz[o]         (adjoint of the block input)
// S_c[z][t] = sum_kt w_kt Re(V_c[z][kt] exp(+i 2 pi kt t / Nt)),  V_c[z][kt] = sum_kz exp(+i theta(kz, z)) U_c[kz][kt],
// with w_kt = c(kt)/N for the real inverse and 1 for the adjoint.
//
// Per plane (one workgroup of NW waves), for each chunk of 16 values of z:
//   phase 1  V^T_c[(re/im, kt)][z] = Au_c[(re/im, kt)][(re/im', kz)] Ez[(re/im', kz)][z]   for every channel c
//            (Au holds [[Ur, -Ui], [Ui, Ur]], Ez [cos; sin]) -> LDS as V[z][c][(re/im, kt)].
//            U is staged as [c][kz / 4][kt][kz % 4] so the 16 rows (re/im, kt) of an operand
//            fragment fall in distinct banks.
//   phase 2  output columns are (z, channel) pairs, z major: a group of ZG consecutive z holds
//            ZG Cs columns, a multiple of 16, so no matrix-core column is padding whatever the
//            channel count.  For one 16-column tile:
//              Out^T[t][(z, co)] = Tb^T[t][k] V[k][(z, co)] + sum_(z', ci) xT[t][(z', ci)] Wd[(z', ci)][(z, co)]
//            with Wd[(z', ci)][(z, co)] = W[co][ci] if z' = z else 0 (block diagonal over z): the
//            synthesis and the pointwise 1x1 land in one accumulator, four consecutive t per lane.
//            Wave w always computes tile j = w mod NT (of groups w / NT, w / NT + R, ...), so its
//            column map, pointwise-weight fragments and EPI_BWD accumulators stay in registers.
//   bfloat16: in EPI_BLOCK / EPI_ADJ phase 1 takes the chunk's z-basis fragments from registers
//            (one round of loads per chunk instead of a dependent load per K step); the
//            accumulating adjoint loads each tile's accumulated output one z chunk ahead (across
//            planes at the last chunk), EPI_BWD its gy one tile ahead.
//   EPI_BWD  the gradient tile is then the B operand of
//              C[(z', i)][(z, o)] += sum_t x[z'][i][t] gz[z][o][t];
//            its z' = z entries, summed over z, are the pointwise-weight gradient.
#pragma once
#include "fno_internal.h"
#include "mfma_common.h"

namespace fno {

// ZEPI_ADJ_ACC: EPI_ADJ adding into the existing output (a kernel of its own, so that the plain
// adjoint holds no operand registers for it)
enum { ZEPI_PLAIN = 0, ZEPI_BLOCK = 1, ZEPI_BWD = 2, ZEPI_ADJ = 3, ZEPI_ADJ_ACC = 4 };

// Tuning knobs of the launch (defaults are the measured best on MI355X).
#ifndef FNO_ZT_AHEAD_BWD
#define FNO_ZT_AHEAD_BWD 0  // bfloat16 BWD: epilogue operands one z chunk ahead (else one tile)
#endif
#ifndef FNO_ZT_TZREG_BLOCK
#define FNO_ZT_TZREG_BLOCK 1  // bfloat16 BLOCK: z-basis fragments in registers
#endif
#ifndef FNO_ZT_TZREG_BWD
#define FNO_ZT_TZREG_BWD 0  // bfloat16 BWD: z-basis fragments in registers
#endif
#ifndef FNO_ZT_ZC_BF16
#define FNO_ZT_ZC_BF16 16  // z values per chunk in the bfloat16 kernels (8 or 16; 8 measured slower)
#endif
#ifndef FNO_ZT_FILL_ONE
#define FNO_ZT_FILL_ONE 1  // a workgroup alone on its CU (LDS) takes up to 16 waves
#endif
#ifndef FNO_ZT_P1_IM
#define FNO_ZT_P1_IM 2  // bfloat16 z synthesis without register-resident basis: items per wave at a time
#endif
#ifndef FNO_ZT_P1_SPLIT
#define FNO_ZT_P1_SPLIT 0  // bfloat16 z synthesis with the hi + lo basis (0: hi only)
#endif
#ifndef FNO_ZT_P2_SPLIT_BWD
#define FNO_ZT_P2_SPLIT_BWD 0  // bfloat16 BWD t synthesis with the hi + lo basis (0: hi only; frees its registers)
#endif
#ifndef FNO_ZT_GEN_VEC1
#define FNO_ZT_GEN_VEC1 1  // t-sliced kernels, even Nt: runs of 4 t as one dword-aligned access (else pairs)
#endif
#ifndef FNO_ZT_X32
#define FNO_ZT_X32 1  // bfloat16: paired K chunks as 16x16x32 products in the z and t synthesis
#endif
#ifndef FNO_ZT_X32_GW
#define FNO_ZT_X32_GW 1  // the same for the BWD weight-gradient products (both t tiles per product)
#endif
#ifndef FNO_ZT_GELU_BWD
#define FNO_ZT_GELU_BWD 1  // bfloat16 BWD GELU': 0 A&S 7.1.26, 1 logistic Phi + exact phi, 2 logistic derivative
#endif
#ifndef FNO_ZT_SBATCH
#define FNO_ZT_SBATCH 2  // source staging items loaded together per thread
#endif
#ifndef FNO_ZT_SBATCH_EXT
#define FNO_ZT_SBATCH_EXT 1  // the same for the bfloat16 accumulating ADJ kernel
#endif
#ifndef FNO_ZT_UBATCH
#define FNO_ZT_UBATCH 2  // bfloat16 U staging items loaded together per thread (float: half)
#endif
#ifndef FNO_ZT_WAVES_BLOCK
#define FNO_ZT_WAVES_BLOCK 5  // waves per SIMD the bfloat16 BLOCK kernel is compiled for
#endif
#ifndef FNO_ZT_WAVES_ADJ
#define FNO_ZT_WAVES_ADJ 5  // the same for the bfloat16 ADJ and PLAIN kernels
#endif
#ifndef FNO_ZT_WAVES_BWD
#define FNO_ZT_WAVES_BWD 5  // the same for the bfloat16 BWD kernel
#endif
#ifndef FNO_ZT_WAVES_F32
#define FNO_ZT_WAVES_F32 3  // the same for every float kernel
#endif
// waves per workgroup aimed at (rounded to a multiple of the tile count), per epilogue
#ifndef FNO_ZT_TARGET_BLOCK
#define FNO_ZT_TARGET_BLOCK 4
#endif
#ifndef FNO_ZT_TARGET_BWD
#define FNO_ZT_TARGET_BWD 4
#endif
#ifndef FNO_ZT_TARGET_ADJ
#define FNO_ZT_TARGET_ADJ 4  // also PLAIN
#endif
#ifndef FNO_ZT_TARGET_F32
#define FNO_ZT_TARGET_F32 8  // every float epilogue
#endif

constexpr int kZtMaxWaves = 16;
constexpr int kZtMaxSpan = 4;

struct ZtArgs {
    int B, Nx, Ny, Nz, Nt, Kz, Kt, Kzp;
    int Cs;    // spectral (= output) channels
    int Csrc;  // pointwise source channels (0: none)
    int Csp;   // Csrc rounded up to a multiple of 4: columns of one z in the transposed source
    int QZ;    // K chunks of the z synthesis: 2 Kzp / 16
    int NTQ;   // t tiles per slice: 1 (Nt <= 16) or 2
    int ZG;    // z values per column group: 16 / gcd(Cs, 16)
    int ZC;    // z values per chunk: 8 or 16 (a multiple of ZG)
    int NT;    // 16-column tiles per group: ZG Cs / 16
    int R;     // waves per tile index: NW = NT R
    int SPAN;  // source K chunks per tile (2 or 4; 1 with no source)
    int ldT;   // row stride (elements) of the transposed source chunk [t][(z, ci)]
    int uim_off;       // element offset of the U imaginary plane (its bank offset is 16 words)
    int off_v, off_x;  // LDS byte offsets of the V chunk and the transposed source chunk
    int NS;    // t slices of 16 NTQ values (1 unless the general kernel)
    int al;    // alignment of a lane's t run in memory (general kernel): 2 whole run, 1 runs of 4, 0 none
    int pr;    // general kernel, al == 0: Nt even, so pairs of t are 2-element aligned
    int accumulate;
};

// Sign flip of an operand fragment when `neg` (lane-dependent).
__device__ __forceinline__ f4v op_sign(f4v v, bool neg) { return neg ? -v : v; }
__device__ __forceinline__ s4v op_sign(s4v v, bool neg)
{
    const short m = neg ? (short)0x8000 : (short)0;
    return s4v{(short)(v[0] ^ m), (short)(v[1] ^ m), (short)(v[2] ^ m), (short)(v[3] ^ m)};
}

// (re, im) of an intermediate spectrum element into two LDS slots of type T (bits unchanged for bfloat16).
__device__ __forceinline__ void cplx_put(float *re, float *im, float2 v)
{
    *re = v.x;
    *im = v.y;
}
__device__ __forceinline__ void cplx_put(__bf16 *re, __bf16 *im, s2v v)
{
    *reinterpret_cast<short *>(re) = v[0];
    *reinterpret_cast<short *>(im) = v[1];
}

// Four consecutive spectrum elements (re, im pairs) in one register group, and their scatter into
// the real and imaginary U planes at element stride 4 (consecutive kt of one kz).
struct F8 {
    f4v a, b;
};
template <typename T> struct U4Of;
template <> struct U4Of<float> { typedef F8 type; };
template <> struct U4Of<__bf16> { typedef s8v type; };
__device__ __forceinline__ void u4_load(const float2 *p, F8 &v)
{
    v.a = *reinterpret_cast<const f4v *>(p);
    v.b = *reinterpret_cast<const f4v *>(p + 2);
}
__device__ __forceinline__ void u4_load(const s2v *p, s8v &v) { v = *reinterpret_cast<const s8v *>(p); }
__device__ __forceinline__ void u4_put(float *re, float *im, const F8 &v)
{
    re[0] = v.a[0];
    im[0] = v.a[1];
    re[4] = v.a[2];
    im[4] = v.a[3];
    re[8] = v.b[0];
    im[8] = v.b[1];
    re[12] = v.b[2];
    im[12] = v.b[3];
}
__device__ __forceinline__ void u4_put(__bf16 *re_, __bf16 *im_, const s8v &v)
{
    short *re = reinterpret_cast<short *>(re_), *im = reinterpret_cast<short *>(im_);
    re[0] = v[0];
    im[0] = v[1];
    re[4] = v[2];
    im[4] = v[3];
    re[8] = v[4];
    im[8] = v[5];
    re[12] = v[6];
    im[12] = v[7];
}

// Operand fragment from four scalars of storage type T at four addresses (bits unchanged).
__device__ __forceinline__ f4v op_gather4(const float *p0, const float *p1, const float *p2, const float *p3)
{
    return f4v{*p0, *p1, *p2, *p3};
}
__device__ __forceinline__ s4v op_gather4(const __bf16 *p0, const __bf16 *p1, const __bf16 *p2, const __bf16 *p3)
{
    return s4v{*reinterpret_cast<const short *>(p0), *reinterpret_cast<const short *>(p1),
               *reinterpret_cast<const short *>(p2), *reinterpret_cast<const short *>(p3)};
}

// Operand fragment from four scalars of storage type T, `stride` elements apart (bits unchanged).
__device__ __forceinline__ f4v op_gather(const float *p, int stride)
{
    return f4v{p[0], p[stride], p[2 * stride], p[3 * stride]};
}
__device__ __forceinline__ s4v op_gather(const __bf16 *p, int stride)
{
    const short *q = reinterpret_cast<const short *>(p);
    return s4v{q[0], q[stride], q[2 * stride], q[3 * stride]};
}

template <int EPI> constexpr bool has_src_c() { return EPI != ZEPI_PLAIN; }

// Two consecutive values of storage type T as floats (one 4- or 8-byte access; p 2-element aligned).
__device__ __forceinline__ float2 ld_pair(const float *p) { return *reinterpret_cast<const float2 *>(p); }
__device__ __forceinline__ float2 ld_pair(const __bf16 *p)
{
    const unsigned u = *reinterpret_cast<const unsigned *>(p);
    return make_float2(__uint_as_float(u << 16), __uint_as_float(u & 0xffff0000u));
}
__device__ __forceinline__ void st_pair(float *p, float a, float b) { *reinterpret_cast<float2 *>(p) = make_float2(a, b); }
__device__ __forceinline__ void st_pair(__bf16 *p, float a, float b)
{
    *reinterpret_cast<unsigned *>(p) = (unsigned)(unsigned short)bf16_bits(a) | ((unsigned)(unsigned short)bf16_bits(b) << 16);
}

// phase 2 for the current z chunk (and t slice): every tile of this wave.  With AHEAD, group j
// of this wave has its epilogue operand loaded one z chunk ahead (gi is hidden from the
// optimiser, or the LDS addresses of all JM tiles are hoisted out of the chunk loop and held
// in registers throughout); otherwise the next tile's operand is loaded before each tile.
// (A macro rather than a lambda: called through a lambda, the loop compiled into the tuned
// kernels with more register copies and waits per tile, and ran about 10% slower.)
#define FNO_ZT_PHASE2()                                                                \
    do {                                                                               \
            if constexpr (AHEAD) {                                                     \
_Pragma("unroll")                                                                      \
                for (int j = 0; j < JM; j++) {                                         \
                    int gi = tr + j * R;                                               \
                    asm volatile("" : "+s"(gi));                                       \
                    if (gi < ngroups) {                                                \
                        const int z0 = zc0 + gi * ZG;                                  \
                        if (z0 < Nz) tile(gi, z0, ext[j]);                             \
                        if (zc0 + ZC < Nz) load_ext(ecol, z0 + ZC, ext[j]);            \
                        else load_ext(ecol_n, has_next ? gi * ZG : Nz, ext[j]);        \
                    }                                                                  \
                }                                                                      \
            } else {                                                                   \
                for (int gi = tr; gi < ngroups; gi += R) {                             \
                    const int z0 = zc0 + gi * ZG;                                      \
                    if (z0 >= Nz) break;                                               \
                    Op en[NTQ];                                                        \
                    if (EXT) load_ext(ecol, gi + R < ngroups ? z0 + R * ZG : Nz, en);  \
                    tile(gi, z0, ext[0]);                                              \
                    if (EXT) {                                                         \
_Pragma("unroll")                                                                      \
                        for (int mt = 0; mt < NTQ; mt++) ext[0][mt] = en[mt];          \
                    }                                                                  \
                }                                                                      \
            }                                                                          \
    } while (0)


// NTT: (re/im, kt) tiles (1: Kt <= 8, 2: Kt <= 16).  NTQ: t tiles (1: Nt <= 16, 2: Nt <= 32).
// SPAN: source K chunks every tile multiplies (weight fragments beyond a tile's own chunks are zero).
// The workgroup has NW = NT R waves (<= MAXW).
// GEN: any Nt.  t is then taken in slices of 16 NTQ values: per z chunk, phase 1 once, then per
// slice the source rows of that slice are staged, the slice's t-basis fragments loaded and phase 2
// run; a lane's t run is read and written with vector accesses only where Nt makes it aligned
// (a.al), else element by element, and values at t >= Nt are zero (loads) or skipped (stores).
template <typename T, int EPI, int NTT, int NTQ, int SPAN, bool SPLIT, bool GEN>
__device__ __forceinline__ void zt_epi_body(const typename CplxOf<T>::type *__restrict__ u, T *__restrict__ out,
                                            const T *__restrict__ src, const T *__restrict__ gy,
                                            const float *__restrict__ wpw, const float *__restrict__ bpw,
                                            float *__restrict__ part,
                                            const typename OpOf<T>::type *__restrict__ tabZ,
                                            const typename OpOf<T>::type *__restrict__ tabZ_lo,
                                            const typename OpOf<T>::type *__restrict__ tabT,
                                            const typename OpOf<T>::type *__restrict__ tabT_lo, const ZtArgs &a)
{
    typedef typename OpOf<T>::type Op;
    constexpr bool PW = EPI != ZEPI_PLAIN;
    // bfloat16: two K chunks of one accumulator per 16x16x32 product: in the z synthesis (X32P1)
    // and in the tiles (X32; not in the t-sliced BWD kernel, where the paired operands cost spills)
    constexpr bool X32P1 = sizeof(T) == 2 && FNO_ZT_X32;
    constexpr bool X32 = X32P1 && !(GEN && EPI == ZEPI_BWD);
    constexpr bool ADJ = EPI == ZEPI_ADJ || EPI == ZEPI_ADJ_ACC;
    const int ZC = a.ZC, LZC = ZC == 8 ? 3 : 4;  // z values per chunk (8 or 16), log2
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int NTH = blockDim.x, NW = NTH >> 6;
    // the wave index is uniform: keep it (and the tile indices derived from it) in scalar registers
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), g = lane >> 4, c = lane & 15;
    const int Nz = a.Nz, Nt = a.Nt, Kt = a.Kt, Kzp = a.Kzp, Cs = a.Cs, Csrc = a.Csrc, Csp = a.Csp;
    const int ZG = a.ZG, NT = a.NT, R = a.R, ldT = a.ldT, KK = a.Kz * Kt;
    // BLOCK and BWD always have a pointwise source (the host checks); ADJ may have none
    const bool has_src = PW && (EPI == ZEPI_BLOCK || EPI == ZEPI_BWD || Csrc > 0);
    const long long nxy = (long long)a.Nx * a.Ny, plane = (long long)Nz * Nt, ncell = nxy * plane;

    // V rows hold 16 NTT values; the 4-value chunks of row r are stored XOR-swizzled by vswz(r)
    // so that 16 consecutive rows read at one chunk position fall in distinct banks
    constexpr int ldv = 16 * NTT;
    auto vswz = [](int r) { return (r >> (sizeof(T) == 2 ? 2 : 1)) & 3; };
    T *ure = reinterpret_cast<T *>(smem);
    T *uim = ure + a.uim_off;
    T *vl = reinterpret_cast<T *>(smem + a.off_v);
    T *xt = reinterpret_cast<T *>(smem + a.off_x);
    // transposed source: element (t, k) sits in row t at column xsw(t, k): bits 2-3 of k (the
    // 4-value chunk within each 16-column block) are XORed with bits of t, so that the 16 rows
    // one fragment read touches fall in distinct banks
    auto xsw = [](int t, int k) { return k ^ (((t >> (NTQ == 2 ? 3 : 2)) & 3) << 2); };

    // ---- one-time set-up: zero U (padding kz >= Kz stays zero) and the transposed source
    // (rows t >= Nt, channels ci >= Csrc and the over-read pad stay zero)
    for (int i = threadIdx.x; i < a.uim_off + Cs * Kt * Kzp; i += NTH) ure[i] = from_f32<T>(0.f);
    if (has_src)
        for (int i = threadIdx.x; i < 16 * NTQ * ldT; i += NTH) xt[i] = from_f32<T>(0.f);

    // ---- this wave's tile: j = w mod NT, groups r, r + R, ...
    const int tj = w % NT, tr = w / NT;
    // lane column n = 16 tj + c is (zr, co) = divmod(n, Cs)
    const int zr = (16 * tj + c) / Cs, co = 16 * tj + c - zr * Cs;
    // the tile's z values zlo..zhi cover source K entries [zlo Csp, (zhi + 1) Csp): chunks qlo .. qlo + nq - 1
    const int zlo = (16 * tj) / Cs, zhi = (16 * tj + 15) / Cs;
    const int qlo = (zlo * Csp) / 16;
    const int nq = has_src ? ((zhi + 1) * Csp + 15) / 16 - qlo : 0;
    // block-diagonal pointwise weights wd[s][jj] = Wd[k = 16 (qlo + s) + 4 g + jj][n]
    Op wd[SPAN];
#pragma unroll
    for (int s = 0; s < SPAN; s++) {
        float v[4];
#pragma unroll
        for (int jj = 0; jj < 4; jj++) {
            const int k = 16 * (qlo + s) + 4 * g + jj, zs = k / (Csp > 0 ? Csp : 1), ci = k - zs * Csp;
            float x = 0.f;
            if (s < nq && zs == zr && ci < Csrc)
                // BLOCK/BWD: co = o, ci = i: W_pw[o][i];  ADJ: co = i, ci = o: W_pw[o][i]
                x = ADJ ? wpw[ci * Cs + co] : wpw[co * Csrc + ci];
            v[jj] = x;
        }
        wd[s] = op_from4<T>(v[0], v[1], v[2], v[3]);
    }
    const float bj = (bpw && (EPI == ZEPI_BLOCK || EPI == ZEPI_BWD)) ? bpw[co] : 0.f;
    // t basis (A of the synthesis part); the bfloat16 BWD kernel takes it without the lo term
    constexpr bool P2S = SPLIT && (EPI != ZEPI_BWD || FNO_ZT_P2_SPLIT_BWD);
    Op ta[NTQ][NTT], tal[NTQ][NTT];
    auto load_ta = [&](int ts) {
#pragma unroll
        for (int mt = 0; mt < NTQ; mt++)
#pragma unroll
            for (int q = 0; q < NTT; q++) {
                const int ti = ((ts * NTQ + mt) * NTT + q) * 64 + lane;
                ta[mt][q] = tabT[ti];
                if (P2S) tal[mt][q] = tabT_lo[ti];
            }
    };
    load_ta(0);
    // GEN: first t of the current slice (0 otherwise)
    int tofs = 0;
    // EPI_BWD: C tiles [s] (rows (z', i) = 16 (qlo + s) + 4 g + r, column n) and the bias gradient of column n
    constexpr int NGW = EPI == ZEPI_BWD ? SPAN : 1;
    f4v gwacc[NGW];
    float gbacc = 0.f;
#pragma unroll
    for (int s = 0; s < NGW; s++) gwacc[s] = f4_zero();

    // U staging: thread -> fixed (kz, kt) entry r, channels strided by u_cstep
    const bool u_one = KK <= NTH;
    const int u_cstep = u_one ? NTH / KK : 1;
    const int u_r0 = u_one ? (int)threadIdx.x % KK : (int)threadIdx.x;
    const int u_c0 = u_one ? (int)threadIdx.x / KK : 0;
    const bool u_ok = u_one ? (int)threadIdx.x < u_cstep * KK : true;
    // vector staging when Kt % 4 == 0: 16-byte (bfloat16) or 32-byte (float) items (not in the
    // bfloat16 accumulating EPI_ADJ kernel, whose register budget it overruns)
    constexpr bool U_VEC = !(sizeof(T) == 2 && EPI == ZEPI_ADJ_ACC);
    const bool u_vec = U_VEC && Kt % 4 == 0;
    const int KK4 = KK / 4, nu4 = Cs * KK4;
    // source staging: item (channel quad cq, z zl, t quad t4) loads 4 consecutive t of channels
    // 4 cq .. 4 cq + 3, transposes them in registers and writes 4 rows t of 4 channels to LDS.
    // Items run over 4 NTQ t quads (a power of two; quads at or past Nt idle), so the item index
    // splits by shifts; SB items per thread have their loads issued before their writes.
    constexpr int LT4 = NTQ == 2 ? 3 : 2;
    constexpr int SB = (sizeof(T) == 2 && EPI == ZEPI_ADJ_ACC) ? FNO_ZT_SBATCH_EXT : FNO_ZT_SBATCH;
    const int nitem = ((Csrc + 3) / 4) << (LT4 + LZC);
    auto put_item = [&](int cq, int zl, int t4, const Op (&v)[4]) {
        Op r[4];
        op_transpose4(v, r);
#pragma unroll
        for (int jj = 0; jj < 4; jj++) {
            const int t = 4 * t4 + jj;
            *reinterpret_cast<Op *>(xt + (size_t)t * ldT + xsw(t, zl * Csp + 4 * cq)) = r[jj];
        }
    };
    const int ngroups = ZC / ZG;
    const int QH = a.QZ / 2;
    // bfloat16: the z-basis K chunks of a z chunk are held in registers when 2 Kzp / 16 <= QZM
    constexpr int QZM = 4;
    const bool tz_reg = sizeof(T) == 2 && (EPI != ZEPI_BWD || FNO_ZT_TZREG_BWD) &&
                        (EPI != ZEPI_BLOCK || FNO_ZT_TZREG_BLOCK) && a.QZ <= QZM;
    __syncthreads();

    const long long nplanes = (long long)a.B * nxy;
    // element offset of this lane's column (zr, co) at z = 0 and its first t = 4 NTQ g, in plane pl
    auto col_of = [&](long long pl) {
        const long long bb = pl / nxy;
        return (bb * Cs + co) * ncell + (pl - bb * nxy) * plane + (long long)zr * Nt + 4 * NTQ * g;
    };
    // The epilogue operand (gy for EPI_BWD, the accumulated output for EPI_ADJ).  bfloat16 (AHEAD):
    // group j of this wave has its operand loaded one z chunk ahead into ext[j] (the host keeps
    // the groups per wave within JM); float: one tile ahead.
    constexpr bool EXT = EPI == ZEPI_BWD || EPI == ZEPI_ADJ_ACC;
    constexpr bool AHEAD = !GEN && EXT && sizeof(T) == 2 && (EPI != ZEPI_BWD || FNO_ZT_AHEAD_BWD);
    constexpr int JM = AHEAD ? 4 : 1;
    Op ext[JM][NTQ];
    // GEN: the lane's run of 4 NTQ values of one row starting at p, its first t t0; zero at t >= Nt
    auto gen_load = [&](const T *p, bool ok, int t0, Op(&e)[NTQ]) {
#pragma unroll
        for (int mt = 0; mt < NTQ; mt++) e[mt] = op_zero<T>();
        if (!ok || t0 >= Nt) return;
        if (a.al == 2 && t0 + 4 * NTQ <= Nt) {
            if constexpr (NTQ == 2) load8(p, e[0], e[1]);
            else e[0] = *reinterpret_cast<const Op *>(p);
            return;
        }
#pragma unroll
        for (int mt = 0; mt < NTQ; mt++) {
            const int tm = t0 + 4 * mt;
            if (a.al >= 1 && tm + 4 <= Nt) {
                e[mt] = *reinterpret_cast<const Op *>(p + 4 * mt);
            } else if (FNO_ZT_GEN_VEC1 && a.pr && tm + 4 <= Nt) {
                e[mt] = ld_dword_aligned<Op>(p + 4 * mt);  // Nt even: the run starts on 4 bytes
            } else if (tm < Nt) {
                float v[4];
                if (a.pr) {  // Nt and tm even: whole pairs in or out
#pragma unroll
                    for (int j = 0; j < 4; j += 2) {
                        const float2 f = tm + j < Nt ? ld_pair(p + 4 * mt + j) : make_float2(0.f, 0.f);
                        v[j] = f.x;
                        v[j + 1] = f.y;
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < 4; j++) v[j] = tm + j < Nt ? to_f32(p[4 * mt + j]) : 0.f;
                }
                e[mt] = op_from4<T>(v[0], v[1], v[2], v[3]);
            }
        }
    };
    auto gen_store = [&](T *p, bool ok, int t0, const float (&v)[NTQ][4]) {
        if (!ok || t0 >= Nt) return;
        if (a.al == 2 && t0 + 4 * NTQ <= Nt) {
            if constexpr (NTQ == 2) store8(p, v);
            else store4(p, v[0]);
            return;
        }
#pragma unroll
        for (int mt = 0; mt < NTQ; mt++) {
            const int tm = t0 + 4 * mt;
            if (a.al >= 1 && tm + 4 <= Nt) {
                store4(p + 4 * mt, v[mt]);
            } else if (FNO_ZT_GEN_VEC1 && a.pr && tm + 4 <= Nt) {
                st_dword_aligned(p + 4 * mt, op_from4<T>(v[mt][0], v[mt][1], v[mt][2], v[mt][3]));
            } else if (a.pr) {
#pragma unroll
                for (int j = 0; j < 4; j += 2)
                    if (tm + j < Nt) st_pair(p + 4 * mt + j, v[mt][j], v[mt][j + 1]);
            } else {
#pragma unroll
                for (int j = 0; j < 4; j++)
                    if (tm + j < Nt) p[4 * mt + j] = from_f32<T>(v[mt][j]);
            }
        }
    };
    auto load_ext = [&](long long ec, int z0, Op(&e)[NTQ]) {
        const T *base = EPI == ZEPI_BWD ? gy : out;
        constexpr bool want = EXT;
        const bool zin = z0 < Nz && z0 + zr < Nz;
        if constexpr (GEN) {
            gen_load(base + ec + (long long)z0 * Nt + tofs, want && zin, tofs + 4 * NTQ * g, e);
            return;
        }
        const long long ei = ec + (long long)z0 * Nt;
#pragma unroll
        for (int mt = 0; mt < NTQ; mt++) e[mt] = op_zero<T>();
        // wave-uniform fast path (z0 is uniform): the whole group lies inside the grid
        if (want && z0 + ZG <= Nz && 16 * NTQ == Nt) {
            if constexpr (NTQ == 2) load8(base + ei, e[0], e[1]);
            else e[0] = *reinterpret_cast<const Op *>(base + ei);
            return;
        }
        bool whole = false;
        if constexpr (NTQ == 2) {
            whole = want && zin && 8 * g + 8 <= Nt;
            if (whole) load8(base + ei, e[0], e[1]);
        }
        if (!whole) {
#pragma unroll
            for (int mt = 0; mt < NTQ; mt++)
                if (want && zin && 4 * NTQ * g + 4 * mt < Nt) e[mt] = *reinterpret_cast<const Op *>(base + ei + 4 * mt);
        }
    };
    if (AHEAD && (long long)blockIdx.x < nplanes) {
        const long long ec0 = col_of(blockIdx.x);
#pragma unroll
        for (int j = 0; j < JM; j++)
            if (tr + j * R < ngroups) load_ext(ec0, (tr + j * R) * ZG, ext[j]);
    }
    for (long long pl = blockIdx.x; pl < nplanes; pl += gridDim.x) {
        const int b = (int)(pl / nxy);
        const long long xy = pl % nxy;
        const T *srcp = src + (long long)b * Csrc * ncell + xy * plane;
        const bool has_next = pl + gridDim.x < nplanes;
        const long long ecol = col_of(pl), ecol_n = has_next ? col_of(pl + gridDim.x) : ecol;
        __syncthreads();  // previous plane's readers of U are done
        // ---- phase 0: U of every channel, to [c][kz / 4][kt][kz % 4]
        if (u_vec) {
            // items (channel, 4 consecutive kt of one kz); a batch's loads all precede its writes
            constexpr int UB = sizeof(T) == 2 ? FNO_ZT_UBATCH : (FNO_ZT_UBATCH + 1) / 2;
            const typename CplxOf<T>::type *ub = u + ((long long)b * Cs * nxy + xy) * KK;
            for (int i0 = threadIdx.x; i0 < nu4; i0 += UB * NTH) {
                typename U4Of<T>::type v[UB];
#pragma unroll
                for (int k = 0; k < UB; k++) {
                    const int it = i0 + k * NTH;
                    if (it < nu4) {
                        const int cs = it / KK4, r = 4 * (it - cs * KK4);
                        u4_load(ub + (long long)cs * nxy * KK + r, v[k]);
                    }
                }
#pragma unroll
                for (int k = 0; k < UB; k++) {
                    const int it = i0 + k * NTH;
                    if (it < nu4) {
                        const int cs = it / KK4, r = 4 * (it - cs * KK4), kz = r / Kt, kt = r - kz * Kt;
                        const size_t ul = (size_t)cs * Kt * Kzp + ((size_t)(kz >> 2) * Kt + kt) * 4 + (kz & 3);
                        u4_put(ure + ul, uim + ul, v[k]);
                    }
                }
            }
        } else if (u_ok)
            for (int r = u_r0; r < KK; r += (u_one ? KK : NTH)) {
                const int kz = r / Kt, kt = r - kz * Kt;
                const typename CplxOf<T>::type *up = u + ((long long)b * Cs * nxy + xy) * KK + r;
                const size_t ul = ((size_t)(kz >> 2) * Kt + kt) * 4 + (kz & 3);
                T *ur = ure + ul, *ui = uim + ul;
                for (int cs = u_c0; cs < Cs; cs += u_cstep) {
                    const typename CplxOf<T>::type v = up[(long long)cs * nxy * KK];
                    cplx_put(ur + (size_t)cs * Kt * Kzp, ui + (size_t)cs * Kt * Kzp, v);
                }
            }
        for (int zc0 = 0; zc0 < Nz; zc0 += ZC) {
            __syncthreads();  // U staged / previous chunk's V and source consumed
            if (!GEN && EXT && !AHEAD) load_ext(ecol, zc0 + tr * ZG, ext[0]);
            // source chunk -> LDS transposed [t][(zl, ci)] (GEN: per t slice, below)
            if (!GEN && has_src) {
                for (int e0 = threadIdx.x; e0 < nitem; e0 += SB * NTH) {
                    Op v[SB][4];
#pragma unroll
                    for (int m = 0; m < SB; m++) {
                        const int e = e0 + m * NTH, t4 = e & (4 * NTQ - 1), zl = (e >> LT4) & (ZC - 1),
                                  cq = e >> (LT4 + LZC);
                        const T *sp = srcp + (long long)(zc0 + zl) * Nt + 4 * t4;
                        const bool ok = e < nitem && 4 * t4 < Nt && zc0 + zl < Nz;
#pragma unroll
                        for (int k = 0; k < 4; k++) {
                            const int ci = 4 * cq + k;
                            v[m][k] = (ok && ci < Csrc) ? *reinterpret_cast<const Op *>(sp + (long long)ci * ncell)
                                                        : op_zero<T>();
                        }
                    }
#pragma unroll
                    for (int m = 0; m < SB; m++) {
                        const int e = e0 + m * NTH, t4 = e & (4 * NTQ - 1), zl = (e >> LT4) & (ZC - 1),
                                  cq = e >> (LT4 + LZC);
                        if (e < nitem && 4 * t4 < Nt) put_item(cq, zl, t4, v[m]);
                    }
                }
            }
            // GEN: the source rows of the current t slice -> LDS transposed [t][(zl, ci)]; every
            // item is written, zeros at t >= Nt, so no row keeps an earlier slice's values.  (The
            // other kernels stage inline: as a lambda the same loop costs them registers.)
            auto stage_src = [&]() {
                const int t_of = tofs;
                for (int e0 = threadIdx.x; e0 < nitem; e0 += SB * NTH) {
                    Op v[SB][4];
#pragma unroll
                    for (int m = 0; m < SB; m++) {
                        const int e = e0 + m * NTH, t4 = e & (4 * NTQ - 1), zl = (e >> LT4) & (ZC - 1),
                                  cq = e >> (LT4 + LZC);
                        const int tq = t_of + 4 * t4;
                        const T *sp = srcp + (long long)(zc0 + zl) * Nt + tq;
                        const bool ok = e < nitem && tq < Nt && zc0 + zl < Nz;
#pragma unroll
                        for (int k = 0; k < 4; k++) {
                            const int ci = 4 * cq + k;
                            const bool okc = ok && ci < Csrc;
                            if (a.al >= 1 && tq + 4 <= Nt) {
                                v[m][k] = okc ? *reinterpret_cast<const Op *>(sp + (long long)ci * ncell) : op_zero<T>();
                            } else if (FNO_ZT_GEN_VEC1 && a.pr && tq + 4 <= Nt) {
                                v[m][k] = okc ? ld_dword_aligned<Op>(sp + (long long)ci * ncell) : op_zero<T>();
                            } else if (a.pr) {
                                float f[4];
#pragma unroll
                                for (int j = 0; j < 4; j += 2) {
                                    const float2 q = (okc && tq + j < Nt) ? ld_pair(sp + (long long)ci * ncell + j)
                                                                          : make_float2(0.f, 0.f);
                                    f[j] = q.x;
                                    f[j + 1] = q.y;
                                }
                                v[m][k] = op_from4<T>(f[0], f[1], f[2], f[3]);
                            } else {
                                float f[4];
#pragma unroll
                                for (int j = 0; j < 4; j++)
                                    f[j] = (okc && tq + j < Nt) ? to_f32(sp[(long long)ci * ncell + j]) : 0.f;
                                v[m][k] = op_from4<T>(f[0], f[1], f[2], f[3]);
                            }
                        }
                    }
#pragma unroll
                    for (int m = 0; m < SB; m++) {
                        const int e = e0 + m * NTH, t4 = e & (4 * NTQ - 1), zl = (e >> LT4) & (ZC - 1),
                                  cq = e >> (LT4 + LZC);
                        if (e < nitem) put_item(cq, zl, t4, v[m]);
                    }
                }
            };
            // ---- phase 1: V^T tiles (channel cs, (re/im, kt) tile mt) of this z tile into LDS
            // z-basis fragments of this chunk (cos rows, then sin rows), loaded once per wave for
            // all of its items
            const int zg = zc0 / 16;
            Op tzc[QZM / 2], tzs[QZM / 2], tzcl[QZM / 2], tzsl[QZM / 2];
            if (tz_reg) {
#pragma unroll
                for (int q = 0; q < QZM / 2; q++)
                    if (q < QH) {
                        const int ti = (zg * a.QZ + q) * 64 + lane, si = ti + QH * 64;
                        tzc[q] = tabZ[ti];
                        tzs[q] = tabZ[si];
                        if (SPLIT && FNO_ZT_P1_SPLIT) {
                            tzcl[q] = tabZ_lo[ti];
                            tzsl[q] = tabZ_lo[si];
                        }
                    }
            }
            // without register-resident z basis: IM items of the wave at a time, so that each z-basis
            // fragment is loaded once for all of them and IM independent product chains wait on it
            constexpr int IM = sizeof(T) == 2 ? FNO_ZT_P1_IM : 1;
            if (!tz_reg && IM > 1) {
                for (int it0 = w; it0 < Cs * NTT; it0 += NW * IM) {
                    f4v acc[IM];
                    const T *pcs[IM], *psn[IM];
                    bool kr[IM], neg[IM];
#pragma unroll
                    for (int i = 0; i < IM; i++) {
                        const int item = it0 + i * NW;
                        const int cs = NTT == 1 ? item : item >> 1, mt = NTT == 1 ? 0 : item & 1;
                        const int ri = NTT == 1 ? (c >> 3) : mt;
                        const int kt = NTT == 1 ? (c & 7) : c;
                        kr[i] = kt < Kt && item < Cs * NTT;
                        neg[i] = ri == 0;
                        const size_t roff = ((size_t)(item < Cs * NTT ? cs : 0) * Kt * Kzp) +
                                            ((size_t)g * Kt + (kt < Kt ? kt : 0)) * 4;
                        pcs[i] = (ri == 0 ? ure : uim) + roff;
                        psn[i] = (ri == 0 ? uim : ure) + roff;
                        acc[i] = f4_zero();
                    }
                    const int qstep = 16 * Kt;
                    for (int q = 0; q < QH; q++) {
                        const int ti = (zg * a.QZ + q) * 64 + lane, si = ti + QH * 64;
                        const Op zcv = tabZ[ti], zsv = tabZ[si];
                        Op zcl, zsl;
                        if (SPLIT && FNO_ZT_P1_SPLIT) {
                            zcl = tabZ_lo[ti];
                            zsl = tabZ_lo[si];
                        }
#pragma unroll
                        for (int i = 0; i < IM; i++) {
                            const Op ac = kr[i] ? *reinterpret_cast<const Op *>(pcs[i] + qstep * q) : op_zero<T>();
                            const Op as =
                                kr[i] ? op_sign(*reinterpret_cast<const Op *>(psn[i] + qstep * q), neg[i]) : op_zero<T>();
                            if (X32P1 && !FNO_ZT_P1_SPLIT) {
                                acc[i] = mma32(ac, as, zcv, zsv, acc[i]);
                            } else {
                                acc[i] = mma16(ac, zcv, acc[i]);
                                if (SPLIT && FNO_ZT_P1_SPLIT) acc[i] = mma16(ac, zcl, acc[i]);
                                acc[i] = mma16(as, zsv, acc[i]);
                                if (SPLIT && FNO_ZT_P1_SPLIT) acc[i] = mma16(as, zsl, acc[i]);
                            }
                        }
                    }
#pragma unroll
                    for (int i = 0; i < IM; i++) {
                        const int item = it0 + i * NW;
                        const int cs = NTT == 1 ? item : item >> 1, mt = NTT == 1 ? 0 : item & 1;
                        const int zc = c - (zc0 & 15);
                        if (item < Cs * NTT && zc >= 0 && zc < ZC) {
                            float v[4] = {acc[i][0], acc[i][1], acc[i][2], acc[i][3]};
                            const int vr = zc * Cs + cs;
                            store4(vl + (size_t)vr * ldv + 16 * mt + 4 * (g ^ vswz(vr)), v);
                        }
                    }
                }
            }
            for (int item = w; item < ((!tz_reg && IM > 1) ? 0 : Cs * NTT); item += NW) {
                const int cs = NTT == 1 ? item : item >> 1, mt = NTT == 1 ? 0 : item & 1;
                const int ri = NTT == 1 ? (c >> 3) : mt;
                const int kt = NTT == 1 ? (c & 7) : c;
                const bool krow = kt < Kt;
                // row (ri, kt), K entries kz = 16 q + 4 g + jj: one 4-vector at [cs][4 q + g][kt][.]
                const size_t roff = ((size_t)cs * Kt * Kzp) + ((size_t)g * Kt + (krow ? kt : 0)) * 4;
                const T *p_cos = (ri == 0 ? ure : uim) + roff;  // multiplies cos
                const T *p_sin = (ri == 0 ? uim : ure) + roff;  // multiplies sin (negated for ri = 0)
                const int qstep = 16 * Kt;
                f4v acc = f4_zero();
                if (tz_reg) {
#pragma unroll
                    for (int q = 0; q < QZM / 2; q++)
                        if (q < QH) {
                            const Op ac = krow ? *reinterpret_cast<const Op *>(p_cos + qstep * q) : op_zero<T>();
                            const Op as = krow ? op_sign(*reinterpret_cast<const Op *>(p_sin + qstep * q), ri == 0)
                                               : op_zero<T>();
                            if (X32P1 && !FNO_ZT_P1_SPLIT) {
                                acc = mma32(ac, as, tzc[q], tzs[q], acc);
                            } else {
                                acc = mma16(ac, tzc[q], acc);
                                if (SPLIT && FNO_ZT_P1_SPLIT) acc = mma16(ac, tzcl[q], acc);
                                acc = mma16(as, tzs[q], acc);
                                if (SPLIT && FNO_ZT_P1_SPLIT) acc = mma16(as, tzsl[q], acc);
                            }
                        }
                } else {
                    for (int q = 0; q < QH; q++) {
                        const Op av = krow ? *reinterpret_cast<const Op *>(p_cos + qstep * q) : op_zero<T>();
                        const int ti = (zg * a.QZ + q) * 64 + lane;
                        acc = mma16(av, tabZ[ti], acc);
                        if (SPLIT) acc = mma16(av, tabZ_lo[ti], acc);
                    }
                    for (int q = 0; q < QH; q++) {
                        const Op av =
                            krow ? op_sign(*reinterpret_cast<const Op *>(p_sin + qstep * q), ri == 0) : op_zero<T>();
                        const int ti = (zg * a.QZ + QH + q) * 64 + lane;
                        acc = mma16(av, tabZ[ti], acc);
                        if (SPLIT) acc = mma16(av, tabZ_lo[ti], acc);
                    }
                }
                // acc[r] = V^T[(ri, kt) = 16 mt + 4 g + r][z = zc0 + c]
                // column c is z = 16 zg + c; the chunk keeps z = zc0 .. zc0 + ZC - 1
                float v[4] = {acc[0], acc[1], acc[2], acc[3]};
                const int zc = c - (zc0 & 15);
                if (zc >= 0 && zc < ZC) {
                    const int vr = zc * Cs + cs;
                    store4(vl + (size_t)vr * ldv + 16 * mt + 4 * (g ^ vswz(vr)), v);
                }
            }
            // ---- phase 2: this wave's tile of group gi (first z0), epilogue operand ext_c
            auto tile = [&](int gi, int z0, const Op(&ext_c)[NTQ]) {
                // operands: V columns (B of the synthesis) and the transposed source (A of the 1x1)
                const int vrow = gi * ZG * Cs + 16 * tj + c;
                Op bv[NTT];
#pragma unroll
                for (int q = 0; q < NTT; q++)
                    bv[q] = *reinterpret_cast<const Op *>(vl + (size_t)vrow * ldv + 16 * q + 4 * (g ^ vswz(vrow)));
                // A[t][k = 16 (qlo + s) + 4 g + jj] for row c of t tile mt: t = 4 NTQ (c / 4) + 4 mt + c % 4
                const int xrow = 4 * NTQ * (c >> 2) + (c & 3), xk = gi * ZG * Csp + 16 * qlo + 4 * g;
                Op av[has_src_c<EPI>() ? SPAN : 1][NTQ];
                if (PW) {
#pragma unroll
                    for (int s = 0; s < SPAN; s++)
#pragma unroll
                        for (int mt = 0; mt < NTQ; mt++)
                            av[s][mt] = has_src ? *reinterpret_cast<const Op *>(
                                                      xt + (size_t)(xrow + 4 * mt) * ldT + xsw(xrow + 4 * mt, xk + 16 * s))
                                                : op_zero<T>();
                }
                f4v acc[NTQ];
#pragma unroll
                for (int mt = 0; mt < NTQ; mt++) {
                    acc[mt] = f4_zero();
                    if constexpr (X32) {
                        // the synthesis and pointwise K chunks of this accumulator, two per product
                        // (a zero partner for an odd count: one product shape per chain)
                        constexpr int NP = NTT * (P2S ? 2 : 1) + (PW ? SPAN : 0);
                        Op pa[NP + 1], pb[NP + 1];
                        int n = 0;
#pragma unroll
                        for (int q = 0; q < NTT; q++) {
                            pa[n] = ta[mt][q];
                            pb[n++] = bv[q];
                            if (P2S) {
                                pa[n] = tal[mt][q];
                                pb[n++] = bv[q];
                            }
                        }
                        if (PW) {
#pragma unroll
                            for (int s = 0; s < SPAN; s++) {
                                pa[n] = av[s][mt];
                                pb[n++] = wd[s];
                            }
                        }
                        pa[NP] = op_zero<T>();
                        pb[NP] = op_zero<T>();
#pragma unroll
                        for (int i = 0; i < NP; i += 2) acc[mt] = mma32(pa[i], pa[i + 1], pb[i], pb[i + 1], acc[mt]);
                    } else {
#pragma unroll
                        for (int q = 0; q < NTT; q++) {
                            acc[mt] = mma16(ta[mt][q], bv[q], acc[mt]);
                            if (P2S) acc[mt] = mma16(tal[mt][q], bv[q], acc[mt]);
                        }
                        if (PW) {
#pragma unroll
                            for (int s = 0; s < SPAN; s++) acc[mt] = mma16(av[s][mt], wd[s], acc[mt]);
                        }
                    }
                }
                // epilogue: acc[mt][r] is (t = 4 NTQ g + 4 mt + r, column n)
                const bool zok = z0 + zr < Nz;
                float v[NTQ][4];
#pragma unroll
                for (int mt = 0; mt < NTQ; mt++) {
#pragma unroll
                    for (int r = 0; r < 4; r++) v[mt][r] = acc[mt][r];
                    if (EPI == ZEPI_BLOCK) {
#pragma unroll
                        for (int r = 0; r < 4; r++)
                            v[mt][r] = sizeof(T) == 2 ? gelu_lg(v[mt][r] + bj) : gelu_fast(v[mt][r] + bj);
                    } else if (EPI == ZEPI_BWD) {
#pragma unroll
                        for (int r = 0; r < 4; r++) {
                            // gy is zero outside the grid (load_ext), so no select is needed
                            const float u = v[mt][r] + bj;
                            v[mt][r] = op_get(ext_c[mt], r) * (sizeof(T) == 4 || FNO_ZT_GELU_BWD == 0 ? gelu_grad_fast(u)
                                                               : FNO_ZT_GELU_BWD == 1                ? gelu_grad_lg(u)
                                                                                                      : gelu_grad_lgd(u));
                            gbacc += v[mt][r];
                        }
                        acc[mt] = f4v{v[mt][0], v[mt][1], v[mt][2], v[mt][3]};  // gradient tile, B of the product below
                    } else if (EPI == ZEPI_ADJ_ACC) {
#pragma unroll
                        for (int r = 0; r < 4; r++) v[mt][r] += op_get(ext_c[mt], r);
                    }
                }
                T *op = out + ecol + (long long)z0 * Nt;
                if constexpr (GEN) {
                    gen_store(op + tofs, zok, tofs + 4 * NTQ * g, v);
                } else if (z0 + ZG <= Nz && 16 * NTQ == Nt) {  // wave-uniform: the whole group is in the grid
                    if constexpr (NTQ == 2) store8(op, v);
                    else store4(op, v[0]);
                } else {
                    bool whole = false;
                    if constexpr (NTQ == 2) {
                        whole = zok && 8 * g + 8 <= Nt;
                        if (whole) store8(op, v);
                    }
                    if (!whole) {
#pragma unroll
                        for (int mt = 0; mt < NTQ; mt++)
                            if (zok && 4 * NTQ * g + 4 * mt < Nt) store4(op + 4 * mt, v[mt]);
                    }
                }
                if (EPI == ZEPI_BWD) {
                    // C[(z', i) = 16 (qlo + s) + 4 g + r][n] += sum_t x[z'][i][t] gz[n][t]; K chunk = t tile mt
                    const int grow = 4 * NTQ * g, gk = gi * ZG * Csp + 16 * qlo + c;
                    auto gather_x = [&](int mt, int s) {
                        const int r0 = grow + 4 * mt, k = gk + 16 * s;
                        const T *xg = xt + (size_t)r0 * ldT;
                        return op_gather4(xg + xsw(r0, k), xg + ldT + xsw(r0 + 1, k), xg + 2 * ldT + xsw(r0 + 2, k),
                                          xg + 3 * ldT + xsw(r0 + 3, k));
                    };
                    if constexpr (X32 && FNO_ZT_X32_GW && NTQ == 2) {
                        // both t tiles (K chunks) of each weight-gradient accumulator in one product
                        const Op bg0 = to_op<T>(acc[0]), bg1 = to_op<T>(acc[1]);
#pragma unroll
                        for (int s = 0; s < NGW; s++) gwacc[s] = mma32(gather_x(0, s), gather_x(1, s), bg0, bg1, gwacc[s]);
                    } else {
#pragma unroll
                        for (int mt = 0; mt < NTQ; mt++) {
                            const Op bg = to_op<T>(acc[mt]);
#pragma unroll
                            for (int s = 0; s < NGW; s++) gwacc[s] = mma16(gather_x(mt, s), bg, gwacc[s]);
                        }
                    }
                }
            };
            if constexpr (GEN) {
                for (int ts = 0; ts < a.NS; ts++) {
                    tofs = 16 * NTQ * ts;
                    if (ts > 0) __syncthreads();  // the previous slice's readers of the source rows are done
                    if (has_src) stage_src();
                    load_ta(ts);
                    if (EXT) load_ext(ecol, zc0 + tr * ZG, ext[0]);
                    __syncthreads();  // V and the slice's source rows staged
                    FNO_ZT_PHASE2();
                }
            } else {
                __syncthreads();  // V staged
                FNO_ZT_PHASE2();
            }
        }
    }
    if (EPI == ZEPI_BWD) {
        // gw[o][i] = sum over waves and z of the z' = z entries of the C tiles, gb[o] likewise.
        // The slots go to LDS as [wave][s][r][lane] (gb: [wave][lane] after the sum over g), then
        // one thread per (o, i) adds its slots in a fixed order: waves, then z.
        const int Ci = Csrc, Co = Cs;
        float *slots = reinterpret_cast<float *>(smem);
        float *gbs = slots + (size_t)NW * SPAN * 4 * 64;
        gbacc += __shfl_xor(gbacc, 16);
        gbacc += __shfl_xor(gbacc, 32);
        __syncthreads();
#pragma unroll
        for (int s = 0; s < SPAN; s++)
#pragma unroll
            for (int r = 0; r < 4; r++) slots[((size_t)(w * SPAN + s) * 4 + r) * 64 + lane] = gwacc[s][r];
        gbs[w * 64 + lane] = gbacc;
        __syncthreads();
        float *pw = part + (size_t)blockIdx.x * Co * (Ci + 1);
        for (int e = threadIdx.x; e < Co * (Ci + 1); e += NTH) {
            const int o = e / (Ci + 1), i = e - o * (Ci + 1);
            float sum = 0.f;
            for (int ww = 0; ww < NW; ww++) {
                const int j = ww % NT;
                const int q0 = ((16 * j) / Cs * Csp) / 16;
                for (int zz = 0; zz < ZG; zz++) {
                    const int cc = zz * Cs + o - 16 * j;  // lane column of (zz, o) in tile j
                    if (cc < 0 || cc >= 16) continue;
                    if (i == Ci) {
                        sum += gbs[ww * 64 + cc];
                    } else {
                        const int k = zz * Csp + i, sq = k / 16 - q0, gg = (k % 16) / 4, rr = k % 4;
                        sum += slots[((size_t)(ww * SPAN + sq) * 4 + rr) * 64 + 16 * gg + cc];
                    }
                }
            }
            pw[e] = sum;
        }
    }
}


// One kernel name per epilogue, so that traces and counters tell them apart.
#define FNO_ZT_KERNEL(NAME, EPI)                                                                                  \
    template <typename T, int NTT, int NTQ, int SPAN, bool SPLIT, int MAXW, bool GEN>                              \
    __global__ void __launch_bounds__(64 * MAXW)                                                                   \
        __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4          ? FNO_ZT_WAVES_F32                           \
                                           : EPI == ZEPI_BWD   ? FNO_ZT_WAVES_BWD                                   \
                                           : EPI == ZEPI_BLOCK ? FNO_ZT_WAVES_BLOCK                                 \
                                                               : FNO_ZT_WAVES_ADJ)))                                \
        NAME(const typename CplxOf<T>::type *__restrict__ u, T *__restrict__ out, const T *__restrict__ src,       \
             const T *__restrict__ gy,                                                                             \
             const float *__restrict__ wpw, const float *__restrict__ bpw, float *__restrict__ part,                \
             const typename OpOf<T>::type *__restrict__ tabZ, const typename OpOf<T>::type *__restrict__ tabZ_lo,   \
             const typename OpOf<T>::type *__restrict__ tabT, const typename OpOf<T>::type *__restrict__ tabT_lo,   \
             ZtArgs a)                                                                                             \
    {                                                                                                              \
        zt_epi_body<T, EPI, NTT, NTQ, SPAN, SPLIT, GEN>(u, out, src, gy, wpw, bpw, part, tabZ, tabZ_lo, tabT, tabT_lo, \
                                                        a);                                                        \
    }
FNO_ZT_KERNEL(k_zt_plain, ZEPI_PLAIN)
FNO_ZT_KERNEL(k_zt_block, ZEPI_BLOCK)
FNO_ZT_KERNEL(k_zt_bwd, ZEPI_BWD)
FNO_ZT_KERNEL(k_zt_adj, ZEPI_ADJ)
FNO_ZT_KERNEL(k_zt_adj_acc, ZEPI_ADJ_ACC)
#undef FNO_ZT_KERNEL

template <int EPI, typename T, int NTT, int NTQ, int SPAN, bool SPLIT, int MAXW, bool GEN> struct ZtKernel;
#define FNO_ZT_PICK(NAME, EPI)                                                                                    \
    template <typename T, int NTT, int NTQ, int SPAN, bool SPLIT, int MAXW, bool GEN>                              \
    struct ZtKernel<EPI, T, NTT, NTQ, SPAN, SPLIT, MAXW, GEN> {                                                     \
        static const void *get()                                                                                   \
        {                                                                                                          \
            return reinterpret_cast<const void *>(NAME<T, NTT, NTQ, SPAN, SPLIT, MAXW, GEN>);                       \
        }                                                                                                          \
    };
FNO_ZT_PICK(k_zt_plain, ZEPI_PLAIN)
FNO_ZT_PICK(k_zt_block, ZEPI_BLOCK)
FNO_ZT_PICK(k_zt_bwd, ZEPI_BWD)
FNO_ZT_PICK(k_zt_adj, ZEPI_ADJ)
FNO_ZT_PICK(k_zt_adj_acc, ZEPI_ADJ_ACC)
#undef FNO_ZT_PICK

// ---------------------------------------------------------------- launcher
struct ZtTabs {
    const void *z, *z_lo, *t, *t_lo;
};

static int gcd_int(int a, int b)
{
    while (b) {
        const int t = a % b;
        a = b;
        b = t;
    }
    return a;
}

static size_t al16(size_t v) { return (v + 15) / 16 * 16; }

// Geometry and LDS carve-up of one launch; returns the LDS bytes (0: shape not supported).
static bool zt_ext(int epi) { return epi == ZEPI_BWD || epi == ZEPI_ADJ_ACC; }

static int zt_target_waves(int epi, int elem)
{
    if (elem == 4) return FNO_ZT_TARGET_F32;
    return epi == ZEPI_BLOCK ? FNO_ZT_TARGET_BLOCK : epi == ZEPI_BWD ? FNO_ZT_TARGET_BWD : FNO_ZT_TARGET_ADJ;
}

// ext: the epilogue reads an operand per output tile (EPI_BWD, EPI_ADJ); for bfloat16 the kernel
// keeps it one z chunk ahead for at most 4 groups per wave.
int zt_grid(const Dims &d);

// Shapes the t-sliced general kernels take: Nt beyond one slice of 32, or rows not 4-aligned.
static bool zt_is_gen(const Dims &d) { return d.N[3] > 32 || d.N[3] % 4 != 0; }

static size_t zt_layout_zc(const Dims &d, int Cs, int Csrc, int elem, int target, bool ext, int zc, ZtArgs &a);

// Layout with 16-z chunks (the bfloat16 default may be 8), or with 8-z chunks where 16 would need
// more LDS than a workgroup has (wide float planes: the V chunk and the transposed source halve).
// Where the LDS admits a single workgroup per CU (float planes at width 20, the batched block's
// width-32 planes), that workgroup takes up to 16 waves instead of the target (the tile indices
// per group allow it): with 4 or 5 waves the CU had one wave per SIMD to hide every latency with.
static size_t zt_layout(const Dims &d, int Cs, int Csrc, int elem, int target, bool ext, ZtArgs &a)
{
    const int zg = 16 / gcd_int(Cs, 16);
    int zc = (elem == 2 && zg <= FNO_ZT_ZC_BF16) ? FNO_ZT_ZC_BF16 : 16;
    size_t lds = zt_layout_zc(d, Cs, Csrc, elem, target, ext, zc, a);
    if ((lds == 0 || lds > 160 * 1024) && zc == 16 && zg <= 8) {
        ZtArgs a8;
        const size_t lds8 = zt_layout_zc(d, Cs, Csrc, elem, target, ext, 8, a8);
        if (lds8 != 0 && lds8 <= 160 * 1024) {
            a = a8;
            lds = lds8;
            zc = 8;
        }
    }
    if (FNO_ZT_FILL_ONE && lds != 0 && lds <= 160 * 1024 && 2 * lds > 160 * 1024 && a.NT * a.R < kZtMaxWaves) {
        ZtArgs aw;
        const size_t ldsw = zt_layout_zc(d, Cs, Csrc, elem, kZtMaxWaves, ext, zc, aw);
        if (ldsw != 0 && ldsw <= 160 * 1024) {
            a = aw;
            lds = ldsw;
        }
    }
    return lds;
}

static size_t zt_layout_zc(const Dims &d, int Cs, int Csrc, int elem, int target, bool ext, int zc, ZtArgs &a)
{
    const bool gen = zt_is_gen(d);
    a = ZtArgs{};
    a.B = d.B;
    a.Nx = d.N[0];
    a.Ny = d.N[1];
    a.Nz = d.N[2];
    a.Nt = d.N[3];
    a.Kz = d.K[2];
    a.Kt = d.K[3];
    a.Kzp = (d.K[2] + 15) / 16 * 16;
    a.Cs = Cs;
    a.Csrc = Csrc;
    a.Csp = (Csrc + 3) / 4 * 4;
    a.QZ = 2 * a.Kzp / 16;
    a.NTQ = d.N[3] > 16 ? 2 : 1;
    a.NS = (d.N[3] + 16 * a.NTQ - 1) / (16 * a.NTQ);
    if (elem == 4) a.al = d.N[3] % 4 == 0 ? 2 : 0;
    else a.al = d.N[3] % 8 == 0 ? 2 : d.N[3] % 4 == 0 ? (a.NTQ == 1 ? 2 : 1) : 0;
    a.pr = d.N[3] % 2 == 0;
    a.ZG = 16 / gcd_int(Cs, 16);
    a.ZC = zc;
    a.NT = a.ZG * Cs / 16;
    if (a.NT > kZtMaxWaves) return 0;
    // waves per tile index: about `target` waves in all (at most 16), never more than there are groups
    a.R = std::max(1, std::min(a.ZC / a.ZG, (target + a.NT - 1) / a.NT));
    const bool ahead = ext && elem == 2 && !gen;
    if (ahead) a.R = std::max(a.R, (a.ZC / a.ZG + 3) / 4);
    while (a.NT * a.R > kZtMaxWaves) a.R--;
    if (ahead && (a.ZC / a.ZG + a.R - 1) / a.R > 4) return 0;
    int span = 1;
    for (int j = 0; j < a.NT && Csrc > 0; j++) {
        const int zlo = (16 * j) / Cs, zhi = (16 * j + 15) / Cs;
        const int qlo = (zlo * a.Csp) / 16, qhi = ((zhi + 1) * a.Csp + 15) / 16 - 1;
        span = std::max(span, qhi - qlo + 1);
    }
    if (span > kZtMaxSpan) return 0;
    a.SPAN = Csrc == 0 ? 1 : std::max(2, span);
    // row stride of the transposed source: every tile reads SPAN chunks from its first one, so
    // the last group's tiles read up to 16 (qlo + SPAN) columns past that group's start
    int reach = a.ZC * a.Csp;
    for (int j = 0; j < a.NT && Csrc > 0; j++) {
        const int qlo = ((16 * j) / Cs * a.Csp) / 16;
        reach = std::max(reach, (a.ZC - a.ZG) * a.Csp + 16 * (qlo + a.SPAN));
    }
    // rows cover whole 16-column blocks (the chunk swizzle stays inside a block), and the row
    // stride is 8 words mod 32 (see the kernel's xsw)
    a.ldT = (reach + 15) / 16 * 16;
    while ((a.ldT * elem / 4) % 32 != 8) a.ldT += 4;
    const int ntt = d.K[3] <= 8 ? 1 : 2;
    // imaginary plane at a word offset = 16 (mod 32) from the real one
    a.uim_off = Cs * a.Kt * a.Kzp;
    while (((size_t)a.uim_off * elem / 4) % 32 != 16) a.uim_off += 16 / elem;
    size_t off = al16(((size_t)a.uim_off + (size_t)Cs * a.Kt * a.Kzp) * elem);
    a.off_v = (int)off;
    off += al16((size_t)a.ZC * Cs * (16 * ntt) * elem);
    a.off_x = (int)off;
    if (Csrc) off += al16((size_t)16 * a.NTQ * a.ldT * elem);
    // the BWD reduction at the end reuses the front: [waves][span][4][64] slots + [waves][64]
    return std::max(off, (size_t)a.NT * a.R * (a.SPAN * 4 + 1) * 64 * sizeof(float));
}

static bool zt_pair_ok(const Dims &d, int Cs, int Csrc, int elem)
{
    for (int epi = ZEPI_PLAIN; epi <= ZEPI_ADJ_ACC; epi++) {
        ZtArgs a;
        const size_t lds = zt_layout(d, Cs, Csrc, elem, zt_target_waves(epi, elem), zt_ext(epi), a);
        if (lds == 0 || lds > 160 * 1024) return false;
    }
    return true;
}


template <typename T, int EPI, int NTT, int NTQ, int SPAN, int MAXW, bool GEN = false>
static hipError_t launch_zt_t(const Dims &d, int Cs, int Csrc, int accumulate, const void *u_, T *out,
                              const T *src, const T *gy, const float *wpw, const float *bpw, float *part,
                              const ZtTabs &tb, hipStream_t st, int *rows_used)
{
    typedef typename OpOf<T>::type Op;
    constexpr bool split = sizeof(T) == 2;
    ZtArgs a;
    const size_t lds = zt_layout(d, Cs, Csrc, sizeof(T), zt_target_waves(EPI, sizeof(T)), zt_ext(EPI), a);
    if (lds == 0) return hipErrorInvalidValue;
    a.accumulate = accumulate;
    const int nth = 64 * a.NT * a.R;
    if (a.NT * a.R > MAXW || a.NTQ != NTQ || GEN != zt_is_gen(d) ||
        (EPI != ZEPI_PLAIN && a.SPAN != SPAN && Csrc > 0) ||
        ((EPI == ZEPI_BLOCK || EPI == ZEPI_BWD) && Csrc <= 0))
        return hipErrorInvalidValue;
    const void *kern = ZtKernel<EPI, T, NTT, NTQ, SPAN, split, MAXW, GEN>::get();
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    // persistent grid: as many workgroups as can be resident at once (at most one per plane)
    int grid = zt_grid(d);
    int per_cu = 0, dev = 0, ncu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, nth, lds) ==
            hipSuccess &&
        hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && per_cu > 0)
        grid = std::min(grid, per_cu * ncu);
    if (rows_used) *rows_used = grid;
    const Op *tz = (const Op *)tb.z, *tzl = (const Op *)tb.z_lo, *tt = (const Op *)tb.t, *ttl = (const Op *)tb.t_lo;
    const typename CplxOf<T>::type *u = reinterpret_cast<const typename CplxOf<T>::type *>(u_);
    void *args[] = {&u, &out, &src, &gy, &wpw, &bpw, &part, &tz, &tzl, &tt, &ttl, &a};
    e = hipLaunchKernel(kern, dim3(grid), dim3(nth), args, lds, st);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

// Launch of epilogue E (the kernel variant picked from the shape).  Instantiated per epilogue in
// zt_epi_*.hip, so that the variants compile in parallel.
template <int E, typename T>
hipError_t launch_zt_epi(const Dims &d, int Cs, int Csrc, const void *u, T *out, const T *src, const T *gy,
                         const float *wpw, const float *bpw, float *part, const ZtTabs &tb, int accumulate,
                         hipStream_t st, int *rows_used)
{
    ZtArgs a;
    if (zt_layout(d, Cs, Csrc, sizeof(T), zt_target_waves(E, sizeof(T)), zt_ext(E), a) == 0)
        return hipErrorInvalidValue;
    const bool w8 = a.NT * a.R <= 8, gen = zt_is_gen(d);
    const int sel = (d.K[3] <= 8 ? 0 : 6) + (a.NTQ == 1 ? 0 : 3) + std::min(2, std::max(0, a.SPAN - 2));
    // general (t-sliced) kernels are built for the largest workgroup only
#define FNO_ZT_W(E, NTT_, NTQ_, SPAN_)                                                                              \
    return gen ? launch_zt_t<T, E, NTT_, NTQ_, SPAN_, kZtMaxWaves, true>(d, Cs, Csrc, accumulate, u, out, src, gy,  \
                                                                        wpw, bpw, part, tb, st, rows_used)          \
           : w8 ? launch_zt_t<T, E, NTT_, NTQ_, SPAN_, 8>(d, Cs, Csrc, accumulate, u, out, src, gy, wpw, bpw, part,  \
                                                          tb, st, rows_used)                                        \
                : launch_zt_t<T, E, NTT_, NTQ_, SPAN_, kZtMaxWaves>(d, Cs, Csrc, accumulate, u, out, src, gy, wpw,  \
                                                                    bpw, part, tb, st, rows_used)
#define FNO_ZT(E)                                                                                                   \
    switch (E == ZEPI_PLAIN ? sel - sel % 3 : sel) {                                                                \
    case 0: FNO_ZT_W(E, 1, 1, 2);                                                                                   \
    case 1: FNO_ZT_W(E, 1, 1, 3);                                                                                   \
    case 2: FNO_ZT_W(E, 1, 1, 4);                                                                                   \
    case 3: FNO_ZT_W(E, 1, 2, 2);                                                                                   \
    case 4: FNO_ZT_W(E, 1, 2, 3);                                                                                   \
    case 5: FNO_ZT_W(E, 1, 2, 4);                                                                                   \
    case 6: FNO_ZT_W(E, 2, 1, 2);                                                                                   \
    case 7: FNO_ZT_W(E, 2, 1, 3);                                                                                   \
    case 8: FNO_ZT_W(E, 2, 1, 4);                                                                                   \
    case 9: FNO_ZT_W(E, 2, 2, 2);                                                                                   \
    case 10: FNO_ZT_W(E, 2, 2, 3);                                                                                  \
    default: FNO_ZT_W(E, 2, 2, 4);                                                                                  \
    }
    FNO_ZT(E);
#undef FNO_ZT_W
#undef FNO_ZT
}

#define FNO_ZT_INSTANTIATE(E)                                                                                      \
    template hipError_t launch_zt_epi<E, float>(const Dims &, int, int, const void *, float *, const float *,      \
                                                const float *, const float *, const float *, float *,             \
                                                const ZtTabs &, int, hipStream_t, int *);                         \
    template hipError_t launch_zt_epi<E, __bf16>(const Dims &, int, int, const void *, __bf16 *, const __bf16 *,   \
                                                 const __bf16 *, const float *, const float *, float *,           \
                                                 const ZtTabs &, int, hipStream_t, int *);
#define FNO_ZT_EXTERN(E)                                                                                           \
    extern template hipError_t launch_zt_epi<E, float>(const Dims &, int, int, const void *, float *,             \
                                                       const float *, const float *, const float *, const float *, \
                                                       float *, const ZtTabs &, int, hipStream_t, int *);         \
    extern template hipError_t launch_zt_epi<E, __bf16>(const Dims &, int, int, const void *, __bf16 *,           \
                                                        const __bf16 *, const __bf16 *, const float *,            \
                                                        const float *, float *, const ZtTabs &, int, hipStream_t, \
                                                        int *);

}  // namespace fno
