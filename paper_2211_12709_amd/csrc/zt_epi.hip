// zt_epi.hip -- synthesis over z and t of one (b, x, y) plane for all
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
//            (Au holds [[Ur, -Ui], [Ui, Ur]], Ez [cos; sin]) -> LDS as V[z][c][(re/im, kt)]
//   phase 2  output columns are (z, channel) pairs, z major: a group of ZG consecutive z holds
//            ZG Cs columns, a multiple of 16, so no matrix-core column is padding whatever the
//            channel count.  For one 16-column tile:
//              Out^T[t][(z, co)] = Tb^T[t][k] V[k][(z, co)] + sum_(z', ci) xT[t][(z', ci)] Wd[(z', ci)][(z, co)]
//            with Wd[(z', ci)][(z, co)] = W[co][ci] if z' = z else 0 (block diagonal over z): the
//            synthesis and the pointwise 1x1 land in one accumulator, four consecutive t per lane.
//            (group, tile) pairs are spread over the waves; per-tile column maps live in LDS.
//   EPI_BWD  after the chunk, per z: gW^T[i][o] += sum_t x[i][t] gz[o][t] from the chunk's
//            source and gradient, read back in their natural [c][z][t] layout.
#include "fno_internal.h"
#include "mfma_common.h"

namespace fno {

enum { ZEPI_PLAIN = 0, ZEPI_BLOCK = 1, ZEPI_BWD = 2, ZEPI_ADJ = 3 };

struct ZtArgs {
    int B, Nx, Ny, Nz, Nt, Kz, Kt, Kzp;
    int Cs;    // spectral (= output) channels
    int Csrc;  // pointwise source channels (0: none)
    int Csp;   // Csrc rounded up to a multiple of 4: columns of one z in the transposed source
    int QZ;    // K chunks of the z synthesis: 2 Kzp / 16
    int NTQ;   // t tiles: ceil(Nt / 16)
    int ZG;    // z values per column group: 16 / gcd(Cs, 16)
    int NT;    // 16-column tiles per group: ZG Cs / 16
    int SPAN;  // most 16-deep source K chunks one tile covers
    int ldT;   // row stride (elements) of the transposed source chunk [t][(z, ci)]
    // LDS byte offsets
    int off_v, off_x, off_wd, off_tcol, off_tzr, off_tb, off_tq;
    int accumulate;
};

// Sign flip of an operand fragment when `neg` (lane-dependent).
__device__ __forceinline__ f4v op_sign(f4v v, bool neg) { return neg ? -v : v; }
__device__ __forceinline__ s4v op_sign(s4v v, bool neg)
{
    const short m = neg ? (short)0x8000 : (short)0;
    return s4v{(short)(v[0] ^ m), (short)(v[1] ^ m), (short)(v[2] ^ m), (short)(v[3] ^ m)};
}

// NTT: (re/im, kt) tiles (1: Kt <= 8, 2: Kt <= 16).  NW: waves per workgroup.
// MAXC: 16-channel tiles of the BWD weight-gradient product (channels <= 16 MAXC).
template <typename T, int EPI, int NTT, bool SPLIT, int NW, int MAXC>
__global__ void __launch_bounds__(64 * NW) k_zt_epi(const float2 *__restrict__ u, T *__restrict__ out,
                                                    const T *__restrict__ src, const T *__restrict__ gy,
                                                    const float *__restrict__ wpw, const float *__restrict__ bpw,
                                                    float *__restrict__ part,
                                                    const typename OpOf<T>::type *__restrict__ tabZ,
                                                    const typename OpOf<T>::type *__restrict__ tabZ_lo,
                                                    const typename OpOf<T>::type *__restrict__ tabT,
                                                    const typename OpOf<T>::type *__restrict__ tabT_lo, ZtArgs a)
{
    typedef typename OpOf<T>::type Op;
    constexpr bool PW = EPI != ZEPI_PLAIN;
    constexpr int ZC = 16;  // z values per chunk
    constexpr int NTH = 64 * NW;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, c = lane & 15;
    const int Nz = a.Nz, Nt = a.Nt, Kt = a.Kt, Kzp = a.Kzp, Cs = a.Cs, Csrc = a.Csrc, Csp = a.Csp;
    const int ZG = a.ZG, NT = a.NT, ldT = a.ldT, KK = a.Kz * Kt;
    const long long nxy = (long long)a.Nx * a.Ny, plane = (long long)Nz * Nt, ncell = nxy * plane;

    const int ldv = 16 * NTT + 4;
    T *ure = reinterpret_cast<T *>(smem);
    T *uim = ure + (size_t)Cs * Kt * Kzp;
    T *vl = reinterpret_cast<T *>(smem + a.off_v);
    T *xt = reinterpret_cast<T *>(smem + a.off_x);
    Op *wdl = reinterpret_cast<Op *>(smem + a.off_wd);
    long long *tcol = reinterpret_cast<long long *>(smem + a.off_tcol);
    int *tzr = reinterpret_cast<int *>(smem + a.off_tzr);
    float *tb = reinterpret_cast<float *>(smem + a.off_tb);
    int *tq = reinterpret_cast<int *>(smem + a.off_tq);

    // ---- one-time set-up: zero U (padding kz >= Kz stays zero) and the transposed source
    // (rows t >= Nt, channels ci >= Csrc and the over-read pad stay zero); tile tables
    for (int i = threadIdx.x; i < 2 * Cs * Kt * Kzp; i += NTH) ure[i] = from_f32<T>(0.f);
    if (PW && Csrc > 0)
        for (int i = threadIdx.x; i < 16 * a.NTQ * ldT; i += NTH) xt[i] = from_f32<T>(0.f);
    for (int e = threadIdx.x; e < NT * 16; e += NTH) {
        // column n = 16 j + cc of a group is (zr, co) = divmod(n, Cs)
        const int zr = e / Cs, co = e - zr * Cs;
        tcol[e] = (long long)co * ncell + (long long)zr * Nt;
        tzr[e] = zr;
        tb[e] = (bpw && (EPI == ZEPI_BLOCK || EPI == ZEPI_BWD)) ? bpw[co] : 0.f;
    }
    for (int j = threadIdx.x; j < NT; j += NTH) {
        // tile j's z values zlo..zhi cover source K entries [zlo Csp, (zhi + 1) Csp): chunks qlo..qhi
        const int zlo = (16 * j) / Cs, zhi = (16 * j + 15) / Cs;
        const int qlo = (zlo * Csp) / 16, qhi = ((zhi + 1) * Csp + 15) / 16 - 1;
        tq[j] = qlo | (PW && Csrc > 0 ? (qhi - qlo + 1) << 16 : 0);
    }
    // block-diagonal pointwise weights: wdl[(j SPAN + s) 64 + lane][jj] = Wd[k = 16 (qlo_j + s) + 4 g + jj][16 j + c]
    if (PW && Csrc > 0)
        for (int e = threadIdx.x; e < NT * a.SPAN * 64; e += NTH) {
            const int el = e & 63, js = e >> 6, j = js / a.SPAN, s = js - j * a.SPAN;
            const int eg = el >> 4, ec = el & 15;
            const int n = 16 * j + ec, zr = n / Cs, co = n - zr * Cs;
            const int zlo = (16 * j) / Cs, zhi = (16 * j + 15) / Cs;
            const int q = (zlo * Csp) / 16 + s, qh = ((zhi + 1) * Csp + 15) / 16 - 1;
            float v[4];
#pragma unroll
            for (int jj = 0; jj < 4; jj++) {
                const int k = 16 * q + 4 * eg + jj, zs = k / Csp, ci = k - zs * Csp;
                float x = 0.f;
                if (q <= qh && zs == zr && ci < Csrc)
                    // BLOCK/BWD: co = o, ci = i: W_pw[o][i];  ADJ: co = i, ci = o: W_pw[o][i]
                    x = EPI == ZEPI_ADJ ? wpw[ci * Cs + co] : wpw[co * Csrc + ci];
                v[jj] = x;
            }
            wdl[e] = op_from4<T>(v[0], v[1], v[2], v[3]);
        }

    // constant fragments: t basis (A of the synthesis part)
    Op ta[2][NTT], tal[2][NTT];
#pragma unroll
    for (int mt = 0; mt < 2; mt++)
#pragma unroll
        for (int q = 0; q < NTT; q++) {
            ta[mt][q] = mt < a.NTQ ? tabT[(mt * NTT + q) * 64 + lane] : op_zero<T>();
            if (SPLIT) tal[mt][q] = mt < a.NTQ ? tabT_lo[(mt * NTT + q) * 64 + lane] : op_zero<T>();
        }
    // EPI_BWD: gW^T tiles [mi][nc] (rows i, columns o) and per-lane bias-gradient partials
    f4v gwacc[EPI == ZEPI_BWD ? MAXC : 1][EPI == ZEPI_BWD ? MAXC : 1];
    float gbacc[EPI == ZEPI_BWD ? MAXC : 1];
    if (EPI == ZEPI_BWD) {
#pragma unroll
        for (int mi = 0; mi < MAXC; mi++)
#pragma unroll
            for (int nc = 0; nc < MAXC; nc++) gwacc[mi][nc] = f4_zero();
#pragma unroll
        for (int nc = 0; nc < MAXC; nc++) gbacc[nc] = 0.f;
    }

    // U staging: thread -> fixed (kz, kt) entry r, channels strided by u_cstep
    const bool u_one = KK <= NTH;
    const int u_cstep = u_one ? NTH / KK : 1;
    const int u_r0 = u_one ? (int)threadIdx.x % KK : (int)threadIdx.x;
    const int u_c0 = u_one ? (int)threadIdx.x / KK : 0;
    const bool u_ok = u_one ? (int)threadIdx.x < u_cstep * KK : true;
    // source staging: thread -> fixed (zl, t4) pair (4 consecutive t), channels strided
    const int nt4 = Nt / 4, npair = ZC * nt4;
    const int sp_cstep = NTH / npair;  // threads per pair (>= 2 since Nt <= 32)
    const bool sp_ok = (int)threadIdx.x < sp_cstep * npair;
    const int sp_pair = threadIdx.x % npair, sp_c0 = threadIdx.x / npair;
    const int sp_zl = sp_pair / nt4, sp_t4 = sp_pair % nt4;
    const int ngroups = ZC / ZG, npairs = ngroups * NT;
    const int QH = a.QZ / 2;
    __syncthreads();

    const long long nplanes = (long long)a.B * nxy;
    for (long long pl = blockIdx.x; pl < nplanes; pl += gridDim.x) {
        const int b = (int)(pl / nxy);
        const long long xy = pl % nxy;
        const T *srcp = src + (long long)b * Csrc * ncell + xy * plane;
        const long long obase = (long long)b * Cs * ncell + xy * plane;
        __syncthreads();  // previous plane's readers of U are done
        // ---- phase 0: U of every channel, transposed to [c][kt][kz]
        if (u_ok)
            for (int r = u_r0; r < KK; r += (u_one ? KK : NTH)) {
                const int kz = r / Kt, kt = r - kz * Kt;
                const float2 *up = u + ((long long)b * Cs * nxy + xy) * KK + r;
                T *ur = ure + (size_t)kt * Kzp + kz, *ui = uim + (size_t)kt * Kzp + kz;
                for (int cs = u_c0; cs < Cs; cs += u_cstep) {
                    const float2 v = up[(long long)cs * nxy * KK];
                    ur[(size_t)cs * Kt * Kzp] = from_f32<T>(v.x);
                    ui[(size_t)cs * Kt * Kzp] = from_f32<T>(v.y);
                }
            }
        for (int zc0 = 0; zc0 < Nz; zc0 += ZC) {
            __syncthreads();  // U staged / previous chunk's V and source consumed
            // source chunk -> LDS transposed [t][(zl, ci)]: thread owns pair (zl, t4), strides over channels
            if (PW && Csrc > 0 && sp_ok) {
                const bool zin = zc0 + sp_zl < Nz;
                const T *sp = srcp + (long long)(zc0 + sp_zl) * Nt + 4 * sp_t4;
                T *dl = xt + (size_t)(4 * sp_t4) * ldT + sp_zl * Csp;
                for (int ci0 = sp_c0; ci0 < Csrc; ci0 += 4 * sp_cstep) {
                    Op vv[4];
#pragma unroll
                    for (int k = 0; k < 4; k++) {
                        const int ci = ci0 + k * sp_cstep;
                        vv[k] = (zin && ci < Csrc) ? *reinterpret_cast<const Op *>(sp + (long long)ci * ncell)
                                                   : op_zero<T>();
                    }
#pragma unroll
                    for (int k = 0; k < 4; k++) {
                        const int ci = ci0 + k * sp_cstep;
                        if (ci < Csrc) {
#pragma unroll
                            for (int jj = 0; jj < 4; jj++) op_put(dl + (size_t)jj * ldT + ci, vv[k], jj);
                        }
                    }
                }
            }
            // ---- phase 1: V^T tiles (channel cs, (re/im, kt) tile mt) of this z tile into LDS
            const int zg = zc0 / 16;
            for (int item = w; item < Cs * NTT; item += NW) {
                const int cs = NTT == 1 ? item : item >> 1, mt = NTT == 1 ? 0 : item & 1;
                const int ri = NTT == 1 ? (c >> 3) : mt;
                const int kt = NTT == 1 ? (c & 7) : c;
                const bool krow = kt < Kt;
                const size_t roff = ((size_t)cs * Kt + (krow ? kt : 0)) * Kzp + 4 * g;
                const T *p_cos = (ri == 0 ? ure : uim) + roff;  // multiplies cos
                const T *p_sin = (ri == 0 ? uim : ure) + roff;  // multiplies sin (negated for ri = 0)
                f4v acc = f4_zero();
                for (int q = 0; q < QH; q++) {
                    const Op av = krow ? *reinterpret_cast<const Op *>(p_cos + 16 * q) : op_zero<T>();
                    const int ti = (zg * a.QZ + q) * 64 + lane;
                    acc = mma16(av, tabZ[ti], acc);
                    if (SPLIT) acc = mma16(av, tabZ_lo[ti], acc);
                }
                for (int q = 0; q < QH; q++) {
                    const Op av =
                        krow ? op_sign(*reinterpret_cast<const Op *>(p_sin + 16 * q), ri == 0) : op_zero<T>();
                    const int ti = (zg * a.QZ + QH + q) * 64 + lane;
                    acc = mma16(av, tabZ[ti], acc);
                    if (SPLIT) acc = mma16(av, tabZ_lo[ti], acc);
                }
                // acc[r] = V^T[(ri, kt) = 16 mt + 4 g + r][z = zc0 + c]
                float v[4] = {acc[0], acc[1], acc[2], acc[3]};
                store4(vl + ((size_t)c * Cs + cs) * ldv + 16 * mt + 4 * g, v);
            }
            __syncthreads();
            // ---- phase 2: (group gi, tile j) pairs p = gi NT + j, spread over the waves
            int gi = w / NT, j = w - (w / NT) * NT;
            for (int p = w; p < npairs; p += NW) {
                const int z0 = zc0 + gi * ZG;
                if (z0 < Nz) {
                    const int tqv = tq[j], qlo = tqv & 0xffff, nq = tqv >> 16;
                    const long long e0 = obase + tcol[16 * j + c] + (long long)z0 * Nt + 4 * g;
                    const bool zok = z0 + tzr[16 * j + c] < Nz;
                    const float bj = tb[16 * j + c];
                    // early loads of the epilogue's second operand (gy, or the accumulated output)
                    Op ext[2];
#pragma unroll
                    for (int mt = 0; mt < 2; mt++) {
                        ext[mt] = op_zero<T>();
                        const bool ok = zok && mt < a.NTQ && 16 * mt + 4 * g < Nt;
                        if (EPI == ZEPI_BWD && ok) ext[mt] = *reinterpret_cast<const Op *>(gy + e0 + 16 * mt);
                        if (EPI == ZEPI_ADJ && ok && a.accumulate)
                            ext[mt] = *reinterpret_cast<const Op *>(out + e0 + 16 * mt);
                    }
                    f4v acc[2] = {f4_zero(), f4_zero()};
                    const int vrow = gi * ZG * Cs + 16 * j + c;
#pragma unroll
                    for (int q = 0; q < NTT; q++) {
                        const Op bv = *reinterpret_cast<const Op *>(vl + (size_t)vrow * ldv + 16 * q + 4 * g);
#pragma unroll
                        for (int mt = 0; mt < 2; mt++)
                            if (mt < a.NTQ) {
                                acc[mt] = mma16(ta[mt][q], bv, acc[mt]);
                                if (SPLIT) acc[mt] = mma16(tal[mt][q], bv, acc[mt]);
                            }
                    }
                    if (PW && nq > 0) {
                        const T *xa = xt + (size_t)c * ldT + gi * ZG * Csp + 16 * qlo + 4 * g;
                        const Op *wa = wdl + (size_t)j * a.SPAN * 64 + lane;
                        for (int s = 0; s < nq; s++) {
                            const Op wv = wa[s * 64];
#pragma unroll
                            for (int mt = 0; mt < 2; mt++)
                                if (mt < a.NTQ) {
                                    // A[t = 16 mt + c][k = 16 (qlo + s) + 4 g + jj]
                                    const Op av = *reinterpret_cast<const Op *>(xa + (size_t)16 * mt * ldT + 16 * s);
                                    acc[mt] = mma16(av, wv, acc[mt]);
                                }
                        }
                    }
                    // epilogue: acc[mt][r] is (t = 16 mt + 4 g + r, column 16 j + c)
#pragma unroll
                    for (int mt = 0; mt < 2; mt++) {
                        const bool ok = zok && mt < a.NTQ && 16 * mt + 4 * g < Nt;
                        float v[4];
#pragma unroll
                        for (int r = 0; r < 4; r++) v[r] = acc[mt][r];
                        if (EPI == ZEPI_BLOCK) {
#pragma unroll
                            for (int r = 0; r < 4; r++) v[r] = gelu_fast(v[r] + bj);
                        } else if (EPI == ZEPI_BWD) {
#pragma unroll
                            for (int r = 0; r < 4; r++) v[r] = op_get(ext[mt], r) * gelu_grad_fast(v[r] + bj);
                        } else if (EPI == ZEPI_ADJ) {
#pragma unroll
                            for (int r = 0; r < 4; r++) v[r] += op_get(ext[mt], r);
                        }
                        if (ok) store4(out + e0 + 16 * mt, v);
                    }
                }
                j += NW;
                while (j >= NT) {
                    j -= NT;
                    gi++;
                }
            }
            if (EPI == ZEPI_BWD) {
                // weight-gradient product of this chunk, one z per wave at a time:
                // gW^T[i][o] += sum_t x[i][z][t] gz[o][z][t]  (A rows i, B columns o, K = t)
                __syncthreads();  // the chunk's gz is written
                const int Ci = Csrc, Co = Cs;
                for (int zl = w; zl < ZC && zc0 + zl < Nz; zl += NW) {
                    const long long zo = xy * plane + (long long)(zc0 + zl) * Nt + 4 * g;
#pragma unroll
                    for (int mt = 0; mt < 2; mt++) {
                        if (mt < a.NTQ && 16 * mt + 4 * g < Nt) {
                            Op ax[MAXC], bz[MAXC];
#pragma unroll
                            for (int m = 0; m < MAXC; m++) {
                                const int ch = 16 * m + c;
                                ax[m] = ch < Ci ? *reinterpret_cast<const Op *>(src + ((long long)b * Ci + ch) * ncell +
                                                                                 zo + 16 * mt)
                                                : op_zero<T>();
                                bz[m] = ch < Co ? *reinterpret_cast<const Op *>(out + ((long long)b * Co + ch) * ncell +
                                                                                 zo + 16 * mt)
                                                : op_zero<T>();
                            }
#pragma unroll
                            for (int nc = 0; nc < MAXC; nc++) {
                                gbacc[nc] += (op_get(bz[nc], 0) + op_get(bz[nc], 1)) + (op_get(bz[nc], 2) + op_get(bz[nc], 3));
#pragma unroll
                                for (int mi = 0; mi < MAXC; mi++) gwacc[mi][nc] = mma16(ax[mi], bz[nc], gwacc[mi][nc]);
                            }
                        }
                    }
                }
            }
        }
    }
    if (EPI == ZEPI_BWD) {
        // partial sums of this wave: part[(block NW + w)][o][0..Ci-1] = gw, [o][Ci] = gb
        const int Ci = Csrc, Co = Cs;
        float *pw = part + ((size_t)blockIdx.x * NW + w) * Co * (Ci + 1);
#pragma unroll
        for (int mi = 0; mi < MAXC; mi++)
#pragma unroll
            for (int nc = 0; nc < MAXC; nc++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int i = 16 * mi + 4 * g + r, o = 16 * nc + c;
                    if (i < Ci && o < Co) pw[o * (Ci + 1) + i] = gwacc[mi][nc][r];
                }
#pragma unroll
        for (int nc = 0; nc < MAXC; nc++) {
            float s = gbacc[nc];
            s += __shfl_xor(s, 16);
            s += __shfl_xor(s, 32);
            const int o = 16 * nc + c;
            if (g == 0 && o < Co) pw[o * (Ci + 1) + Ci] = s;
        }
    }
}

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

// Geometry and LDS carve-up of one launch; returns the LDS bytes.
static size_t zt_layout(const Dims &d, int Cs, int Csrc, int elem, ZtArgs &a)
{
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
    a.NTQ = (d.N[3] + 15) / 16;
    a.ZG = 16 / gcd_int(Cs, 16);
    a.NT = a.ZG * Cs / 16;
    a.SPAN = 1;
    for (int j = 0; j < a.NT; j++) {
        const int zlo = (16 * j) / Cs, zhi = (16 * j + 15) / Cs;
        const int qlo = (zlo * a.Csp) / 16, qhi = ((zhi + 1) * a.Csp + 15) / 16 - 1;
        a.SPAN = std::max(a.SPAN, qhi - qlo + 1);
    }
    a.ldT = 16 * a.Csp + 12;  // + over-read of the last group's last K chunk
    const int ntt = d.K[3] <= 8 ? 1 : 2;
    size_t off = al16((size_t)2 * Cs * a.Kt * a.Kzp * elem);
    a.off_v = (int)off;
    off += al16((size_t)16 * Cs * (16 * ntt + 4) * elem);
    a.off_x = (int)off;
    if (Csrc) off += al16((size_t)16 * a.NTQ * a.ldT * elem);
    a.off_wd = (int)off;
    if (Csrc) off += (size_t)a.NT * a.SPAN * 64 * 4 * elem;
    a.off_tcol = (int)off;
    off += al16((size_t)a.NT * 16 * 8);
    a.off_tzr = (int)off;
    off += al16((size_t)a.NT * 16 * 4);
    a.off_tb = (int)off;
    off += al16((size_t)a.NT * 16 * 4);
    a.off_tq = (int)off;
    off += al16((size_t)a.NT * 4);
    return off;
}

static bool zt_pair_ok(const Dims &d, int Cs, int Csrc, int elem)
{
    ZtArgs a;
    return zt_layout(d, Cs, Csrc, elem, a) <= 160 * 1024;
}

bool zt_supported(const Dims &d, int dtype)
{
    if (d.N[3] % 4 != 0 || d.N[3] > 32 || d.K[3] > 16) return false;
    if (d.Ci > 64 || d.Co > 64) return false;
    const int elem = dtype == FNO_BF16 ? 2 : 4;
    // every (output, source) channel pair the entry points use
    return zt_pair_ok(d, d.Co, 0, elem) && zt_pair_ok(d, d.Co, d.Ci, elem) && zt_pair_ok(d, d.Ci, d.Co, elem) &&
           zt_pair_ok(d, d.Ci, 0, elem);
}

constexpr int kZtWaves = 8;

int zt_grid(const Dims &d) { return (int)std::min<long long>((long long)d.B * d.N[0] * d.N[1], 2048); }
int zt_partial_rows(const Dims &d) { return zt_grid(d) * kZtWaves; }

template <typename T, int EPI, int NTT, int MAXC>
static hipError_t launch_zt_t(const Dims &d, int Cs, int Csrc, int accumulate, const float2 *u, T *out,
                              const T *src, const T *gy, const float *wpw, const float *bpw, float *part,
                              const ZtTabs &tb, hipStream_t st, int *rows_used)
{
    typedef typename OpOf<T>::type Op;
    constexpr bool split = sizeof(T) == 2;
    constexpr int NW = kZtWaves;
    ZtArgs a;
    const size_t lds = zt_layout(d, Cs, Csrc, sizeof(T), a);
    a.accumulate = accumulate;
    auto kern = k_zt_epi<T, EPI, NTT, split, NW, MAXC>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    // persistent grid: as many workgroups as can be resident at once (at most one per plane)
    int grid = zt_grid(d);
    int per_cu = 0, dev = 0, ncu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(kern), 64 * NW, lds) ==
            hipSuccess &&
        hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && per_cu > 0)
        grid = std::min(grid, per_cu * ncu);
    if (rows_used) *rows_used = grid * NW;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * NW), lds, st, u, out, src, gy, wpw, bpw, part, (const Op *)tb.z,
                       (const Op *)tb.z_lo, (const Op *)tb.t, (const Op *)tb.t_lo, a);
    return hipGetLastError();
}

template <typename T, int EPI>
static hipError_t launch_zt_e(const Dims &d, int Cs, int Csrc, int accumulate, const float2 *u, T *out, const T *src,
                              const T *gy, const float *wpw, const float *bpw, float *part, const ZtTabs &tb,
                              hipStream_t st, int *rows_used)
{
    const bool ntt1 = d.K[3] <= 8;
    const bool c2 = std::max(Cs, Csrc) <= 32;
    if (EPI != ZEPI_BWD) {
        return ntt1 ? launch_zt_t<T, EPI, 1, 1>(d, Cs, Csrc, accumulate, u, out, src, gy, wpw, bpw, part, tb, st, rows_used)
                    : launch_zt_t<T, EPI, 2, 1>(d, Cs, Csrc, accumulate, u, out, src, gy, wpw, bpw, part, tb, st, rows_used);
    }
    if (ntt1)
        return c2 ? launch_zt_t<T, EPI, 1, 2>(d, Cs, Csrc, accumulate, u, out, src, gy, wpw, bpw, part, tb, st, rows_used)
                  : launch_zt_t<T, EPI, 1, 4>(d, Cs, Csrc, accumulate, u, out, src, gy, wpw, bpw, part, tb, st, rows_used);
    return c2 ? launch_zt_t<T, EPI, 2, 2>(d, Cs, Csrc, accumulate, u, out, src, gy, wpw, bpw, part, tb, st, rows_used)
              : launch_zt_t<T, EPI, 2, 4>(d, Cs, Csrc, accumulate, u, out, src, gy, wpw, bpw, part, tb, st, rows_used);
}

// epi: ZEPI_*; Cs = output/spectral channels, Csrc = pointwise source channels.
// rows_used (nullable) receives the number of BWD partial-sum rows written.
template <typename T>
hipError_t launch_zt(int epi, const Dims &d, int Cs, int Csrc, const float2 *u, T *out, const T *src, const T *gy,
                     const float *wpw, const float *bpw, float *part, const ZtTabs &tb, int accumulate, hipStream_t st,
                     int *rows_used)
{
    switch (epi) {
    case ZEPI_PLAIN: return launch_zt_e<T, ZEPI_PLAIN>(d, Cs, Csrc, accumulate, u, out, src, gy, wpw, bpw, part, tb, st, rows_used);
    case ZEPI_BLOCK: return launch_zt_e<T, ZEPI_BLOCK>(d, Cs, Csrc, accumulate, u, out, src, gy, wpw, bpw, part, tb, st, rows_used);
    case ZEPI_BWD: return launch_zt_e<T, ZEPI_BWD>(d, Cs, Csrc, accumulate, u, out, src, gy, wpw, bpw, part, tb, st, rows_used);
    default: return launch_zt_e<T, ZEPI_ADJ>(d, Cs, Csrc, accumulate, u, out, src, gy, wpw, bpw, part, tb, st, rows_used);
    }
}

template hipError_t launch_zt<float>(int, const Dims &, int, int, const float2 *, float *, const float *,
                                     const float *, const float *, const float *, float *, const ZtTabs &, int,
                                     hipStream_t, int *);
template hipError_t launch_zt<__bf16>(int, const Dims &, int, int, const float2 *, __bf16 *, const __bf16 *,
                                      const __bf16 *, const float *, const float *, float *, const ZtTabs &, int,
                                      hipStream_t, int *);

}  // namespace fno
