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
// Per plane (one workgroup, 4 waves), for each chunk of ZC values of z:
//   phase 1  V^T_c[(re/im, kt)][z] = Au_c[(re/im, kt)][(re/im', kz)] Ez[(re/im', kz)][z]   for every channel c
//            (Au holds [[Ur, -Ui], [Ui, Ur]], Ez [cos; sin]) -> LDS as V[z][c][(re/im, kt)]
//   phase 2  per z:  Out^T[t][co] = [Tb^T | src_z^T][t][k] [V_z^T ; Wm][k][co]
//            K = (re/im, kt) then the pointwise source channels; the output lands with four
//            consecutive t per lane, so loads of gy and stores of the result are vectors.
// For EPI_BWD the gradient tile is then reused as the B operand of
//   gWpw^T[i][o] += sum_t x_z[i][t] gz^T[t][o]
// without moving data between lanes.
#include "fno_internal.h"
#include "mfma_common.h"

namespace fno {

enum { ZEPI_PLAIN = 0, ZEPI_BLOCK = 1, ZEPI_BWD = 2, ZEPI_ADJ = 3 };

struct ZtArgs {
    int B, Nx, Ny, Nz, Nt, Kz, Kt, Kzp;
    int Cs;    // spectral (= output) channels
    int Csrc;  // pointwise source channels
    int QZ;    // K chunks of the z synthesis: 2 Kzp / 16
    int NTQ;   // t tiles: ceil(Nt / 16)
    int ZC;    // z values per chunk
    int accumulate;
};

// NTT: (re/im, kt) tiles (1: Kt <= 8, 2: Kt <= 16).  MAXC: channel tiles (channels <= 16 MAXC).
template <typename T, int EPI, int NTT, bool SPLIT, int MAXC>
__global__ void __launch_bounds__(256) k_zt_epi(const float2 *__restrict__ u, T *__restrict__ out,
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
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, c = lane & 15;
    const int Nz = a.Nz, Nt = a.Nt, Kz = a.Kz, Kt = a.Kt, Kzp = a.Kzp, Cs = a.Cs, Csrc = a.Csrc;
    const long long nxy = (long long)a.Nx * a.Ny, plane = (long long)Nz * Nt, ncell = nxy * plane;

    // LDS: U planes [Cs][Kt][Kzp] re then im; V chunk [ZC][Cs][ldv]; source chunk [ci][ZC][Ntp]
    const int ldv = 16 * NTT + 4;
    const int Ntp = 16 * a.NTQ;
    const int ldxc = ZC * Ntp + 4;  // source channel stride (padded against bank conflicts)
    T *ure = reinterpret_cast<T *>(smem);
    T *uim = ure + (size_t)Cs * Kt * Kzp;
    T *vl = uim + (size_t)Cs * Kt * Kzp;
    T *xl = vl + (size_t)ZC * Cs * ldv;
    for (int i = threadIdx.x; i < 2 * Cs * Kt * Kzp; i += 256) ure[i] = from_f32<T>(0.f);
    if (PW)
        for (int i = threadIdx.x; i < Csrc * ldxc; i += 256) xl[i] = from_f32<T>(0.f);

    // constant fragments: t basis (A of phase 2), pointwise weights (B of phase 2)
    Op ta[2][NTT], tal[2][NTT];
#pragma unroll
    for (int mt = 0; mt < 2; mt++)
#pragma unroll
        for (int q = 0; q < NTT; q++) {
            ta[mt][q] = mt < a.NTQ ? tabT[(mt * NTT + q) * 64 + lane] : op_zero<T>();
            if (SPLIT) tal[mt][q] = mt < a.NTQ ? tabT_lo[(mt * NTT + q) * 64 + lane] : op_zero<T>();
        }
    Op wb[MAXC][MAXC];  // wb[qi][nc]: Wm[ci = 16 qi + 4 g + j][co = 16 nc + c]
#pragma unroll
    for (int qi = 0; qi < MAXC; qi++)
#pragma unroll
        for (int nc = 0; nc < MAXC; nc++) {
            float v[4];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int ci = 16 * qi + 4 * g + j, co = 16 * nc + c;
                float x = 0.f;
                if (PW && ci < Csrc && co < Cs) {
                    // BLOCK/BWD: co = o, ci = i: W_pw[o][i];  ADJ: co = i, ci = o: W_pw[o][i]
                    x = EPI == ZEPI_ADJ ? wpw[ci * Cs + co] : wpw[co * Csrc + ci];
                }
                v[j] = x;
            }
            wb[qi][nc] = op_from4<T>(v[0], v[1], v[2], v[3]);
        }
    float bias[MAXC];
#pragma unroll
    for (int nc = 0; nc < MAXC; nc++) {
        const int co = 16 * nc + c;
        bias[nc] = (bpw && co < Cs && (EPI == ZEPI_BLOCK || EPI == ZEPI_BWD)) ? bpw[co] : 0.f;
    }
    // EPI_BWD accumulators: gw^T[i][o] tiles [mi][nc] and per-lane gb partial for o = 16 nc + c
    f4v gwacc[MAXC][MAXC];
    float gbacc[MAXC];
#pragma unroll
    for (int mi = 0; mi < MAXC; mi++)
#pragma unroll
        for (int nc = 0; nc < MAXC; nc++) gwacc[mi][nc] = f4_zero();
#pragma unroll
    for (int nc = 0; nc < MAXC; nc++) gbacc[nc] = 0.f;

    // source chunk staging: thread -> fixed (zl, t4) pair (4 consecutive t), channels strided
    const int nt4 = Nt / 4, npair = ZC * nt4;
    const int sp_cstep = 256 / npair;  // threads per pair (>= 2 since Nt <= 32)
    const bool sp_ok = (int)threadIdx.x < sp_cstep * npair;
    const int sp_pair = threadIdx.x % npair, sp_c0 = threadIdx.x / npair;
    const int sp_zl = sp_pair / nt4, sp_t4 = sp_pair % nt4;
    const long long nplanes = (long long)a.B * nxy;
    for (long long pl = blockIdx.x; pl < nplanes; pl += gridDim.x) {
        const int b = (int)(pl / nxy);
        const long long xy = pl % nxy;
        const T *srcp = src + (long long)b * Csrc * ncell + xy * plane;
        __syncthreads();  // previous plane's readers of U are done
        // ---- phase 0: U of every channel, transposed to [c][kt][kz]; thread owns fixed (kz, kt) pairs
        for (int r = threadIdx.x; r < Kz * Kt; r += 256) {
            const int kz = r / Kt, kt = r - (r / Kt) * Kt;
            const float2 *up = u + ((long long)b * Cs * nxy + xy) * Kz * Kt + r;
            T *ur = ure + (size_t)kt * Kzp + kz, *ui = uim + (size_t)kt * Kzp + kz;
            for (int cs = 0; cs < Cs; cs++) {
                const float2 v = up[(long long)cs * nxy * Kz * Kt];
                ur[(size_t)cs * Kt * Kzp] = from_f32<T>(v.x);
                ui[(size_t)cs * Kt * Kzp] = from_f32<T>(v.y);
            }
        }
        for (int zc0 = 0; zc0 < Nz; zc0 += ZC) {
            __syncthreads();  // U staged / previous chunk's V and source consumed
            // source chunk -> LDS [ci][zl][t]: thread owns pair (zl, t4), strides over channels
            if (PW && sp_ok && zc0 + sp_zl < Nz) {
                const T *sp = srcp + (long long)(zc0 + sp_zl) * Nt + 4 * sp_t4;
                T *dl = xl + sp_zl * Ntp + 4 * sp_t4;
                for (int ci0 = sp_c0; ci0 < Csrc; ci0 += 4 * sp_cstep) {
                    Op vv[4];
#pragma unroll
                    for (int k = 0; k < 4; k++) {
                        const int ci = ci0 + k * sp_cstep;
                        vv[k] = ci < Csrc ? *reinterpret_cast<const Op *>(sp + (long long)ci * ncell) : op_zero<T>();
                    }
#pragma unroll
                    for (int k = 0; k < 4; k++) {
                        const int ci = ci0 + k * sp_cstep;
                        if (ci < Csrc) *reinterpret_cast<Op *>(dl + (size_t)ci * ldxc) = vv[k];
                    }
                }
            } else if (PW && sp_ok) {
                // z beyond the grid: zeros
                T *dl = xl + sp_zl * Ntp + 4 * sp_t4;
                for (int ci = sp_c0; ci < Csrc; ci += sp_cstep)
                    *reinterpret_cast<Op *>(dl + (size_t)ci * ldxc) = op_zero<T>();
            }
            // ---- phase 1: V^T tiles (channel cs) of this z tile into LDS
            const int zg = zc0 / 16;
            for (int cs = w; cs < Cs; cs += 4) {
#pragma unroll
                for (int mt = 0; mt < NTT; mt++) {
                    const int ri = NTT == 1 ? (c >> 3) : mt;
                    const int kt = NTT == 1 ? (c & 7) : c;
                    f4v acc = f4_zero();
                    for (int q = 0; q < a.QZ; q++) {
                        const int ri2 = (16 * q) / Kzp, kz0 = (16 * q) % Kzp + 4 * g;
                        Op av = op_zero<T>();
                        if (kt < Kt) {
                            const size_t off = ((size_t)cs * Kt + kt) * Kzp + kz0;
                            // Au = [[Ur, -Ui], [Ui, Ur]]
                            if (ri == 0) av = ri2 == 0 ? *reinterpret_cast<const Op *>(ure + off)
                                                       : op_neg<T>(*reinterpret_cast<const Op *>(uim + off));
                            else av = ri2 == 0 ? *reinterpret_cast<const Op *>(uim + off)
                                               : *reinterpret_cast<const Op *>(ure + off);
                        }
                        const int ti = (zg * a.QZ + q) * 64 + lane;
                        acc = mma16(av, tabZ[ti], acc);
                        if (SPLIT) acc = mma16(av, tabZ_lo[ti], acc);
                    }
                    // acc[r] = V^T[(ri, kt) = 16 mt + 4 g + r][z = zc0 + c]
                    float v[4] = {acc[0], acc[1], acc[2], acc[3]};
                    store4(vl + ((size_t)c * Cs + cs) * ldv + 16 * mt + 4 * g, v);
                }
            }
            __syncthreads();
            // ---- phase 2: per z, Out^T[t][co] and the epilogue (two z in flight per wave)
#pragma unroll 2
            for (int zl = w; zl < ZC && zc0 + zl < Nz; zl += 4) {
                const int z = zc0 + zl;
                f4v acc[2][MAXC];
#pragma unroll
                for (int mt = 0; mt < 2; mt++)
#pragma unroll
                    for (int nc = 0; nc < MAXC; nc++) acc[mt][nc] = f4_zero();
#pragma unroll
                for (int q = 0; q < NTT; q++)
#pragma unroll
                    for (int nc = 0; nc < MAXC; nc++) {
                        const int co = 16 * nc + c;
                        const Op bv = co < Cs ? *reinterpret_cast<const Op *>(vl + ((size_t)zl * Cs + co) * ldv + 16 * q + 4 * g)
                                              : op_zero<T>();
#pragma unroll
                        for (int mt = 0; mt < 2; mt++)
                            if (mt < a.NTQ) {
                                acc[mt][nc] = mma16(ta[mt][q], bv, acc[mt][nc]);
                                if (SPLIT) acc[mt][nc] = mma16(tal[mt][q], bv, acc[mt][nc]);
                            }
                    }
                if (PW) {
#pragma unroll
                    for (int qi = 0; qi < MAXC; qi++) {
                        if (16 * qi < Csrc) {
#pragma unroll
                            for (int mt = 0; mt < 2; mt++) {
                                if (mt < a.NTQ) {
                                    // A[t = 16 mt + c][ci = 16 qi + 4 g + j]
                                    const int ci0 = 16 * qi + 4 * g;
                                    const T *xr = xl + (size_t)ci0 * ldxc + zl * Ntp + 16 * mt + c;
                                    float xv[4];
#pragma unroll
                                    for (int j = 0; j < 4; j++) xv[j] = ci0 + j < Csrc ? to_f32(xr[j * ldxc]) : 0.f;
                                    const Op av = op_from4<T>(xv[0], xv[1], xv[2], xv[3]);
#pragma unroll
                                    for (int nc = 0; nc < MAXC; nc++) acc[mt][nc] = mma16(av, wb[qi][nc], acc[mt][nc]);
                                }
                            }
                        }
                    }
                }
                // epilogue: acc[mt][nc][r] is (t = 16 mt + 4 g + r, co = 16 nc + c)
#pragma unroll
                for (int mt = 0; mt < 2; mt++) {
#pragma unroll
                    for (int nc = 0; nc < MAXC; nc++) {
                        const int co = 16 * nc + c, t0 = 16 * mt + 4 * g;
                        const bool ok = mt < a.NTQ && co < Cs && t0 < Nt;
                        const long long idx = ((long long)b * Cs + co) * ncell + xy * plane + (long long)z * Nt + t0;
                        float v[4];
#pragma unroll
                        for (int r = 0; r < 4; r++) v[r] = acc[mt][nc][r];
                        if (EPI == ZEPI_BLOCK) {
#pragma unroll
                            for (int r = 0; r < 4; r++) v[r] = gelu_fast(v[r] + bias[nc]);
                        } else if (EPI == ZEPI_BWD) {
                            float gv[4] = {0.f, 0.f, 0.f, 0.f};
                            if (ok) load4(gy + idx, gv);
#pragma unroll
                            for (int r = 0; r < 4; r++) {
                                v[r] = ok ? gv[r] * gelu_grad_fast(v[r] + bias[nc]) : 0.f;
                                gbacc[nc] += v[r];
                            }
                            // keep the gradient tile for the weight-gradient product
                            acc[mt][nc] = f4v{v[0], v[1], v[2], v[3]};
                        } else if (EPI == ZEPI_ADJ) {
                            if (ok && a.accumulate) {
                                float o4[4];
                                load4(out + idx, o4);
#pragma unroll
                                for (int r = 0; r < 4; r++) v[r] += o4[r];
                            }
                        }
                        if (ok) store4(out + idx, v);
                    }
                }
                if (EPI == ZEPI_BWD) {
                    // gw^T[i][o] += sum_t x_z[i][t] gz^T[t][o]: K chunk = t tile mt
#pragma unroll
                    for (int mt = 0; mt < 2; mt++) {
                        if (mt < a.NTQ) {
                            Op bg[MAXC];
#pragma unroll
                            for (int nc = 0; nc < MAXC; nc++) bg[nc] = to_op<T>(acc[mt][nc]);
#pragma unroll
                            for (int mi = 0; mi < MAXC; mi++) {
                                // A[i = 16 mi + c][t = 16 mt + 4 g + j] from the staged source (zero beyond Csrc)
                                const Op ax = 16 * mi + c < Csrc
                                                  ? *reinterpret_cast<const Op *>(xl + (size_t)(16 * mi + c) * ldxc +
                                                                                  zl * Ntp + 16 * mt + 4 * g)
                                                  : op_zero<T>();
#pragma unroll
                                for (int nc = 0; nc < MAXC; nc++) gwacc[mi][nc] = mma16(ax, bg[nc], gwacc[mi][nc]);
                            }
                        }
                    }
                }
            }
        }
    }
    if (EPI == ZEPI_BWD) {
        // partial sums of this wave: part[(block * 4 + w)][o][0..Ci-1] = gw, [o][Ci] = gb
        const int Ci = Csrc, Co = Cs;
        float *pw = part + ((size_t)blockIdx.x * 4 + w) * Co * (Ci + 1);
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

static size_t zt_lds_bytes(const ZtArgs &a, int elem, int ntt)
{
    const int ZC = 16, Ntp = 16 * ((a.Nt + 15) / 16);
    return ((size_t)2 * a.Cs * a.Kt * a.Kzp + (size_t)ZC * a.Cs * (16 * ntt + 4) +
            (size_t)a.Csrc * (ZC * Ntp + 4)) * elem;
}

bool zt_supported(const Dims &d, int dtype)
{
    if (d.N[3] % 4 != 0 || d.N[3] > 32 || d.K[3] > 16) return false;
    if (d.Ci > 64 || d.Co > 64) return false;
    ZtArgs a{};
    a.Cs = std::max(d.Ci, d.Co);
    a.Kt = d.K[3];
    a.Nt = d.N[3];
    a.Kzp = (d.K[2] + 15) / 16 * 16;
    a.Csrc = std::max(d.Ci, d.Co);
    a.ZC = 16;
    return zt_lds_bytes(a, dtype == FNO_BF16 ? 2 : 4, d.K[3] <= 8 ? 1 : 2) <= 160 * 1024;
}

int zt_grid(const Dims &d) { return (int)std::min<long long>((long long)d.B * d.N[0] * d.N[1], 2048); }

template <typename T, int EPI, int NTT, int MAXC>
static hipError_t launch_zt_t(const ZtArgs &a, const float2 *u, T *out, const T *src, const T *gy, const float *wpw,
                              const float *bpw, float *part, const ZtTabs &tb, int grid, hipStream_t st,
                              int *grid_used)
{
    typedef typename OpOf<T>::type Op;
    constexpr bool split = sizeof(T) == 2;
    const size_t lds = zt_lds_bytes(a, sizeof(T), NTT);
    auto kern = k_zt_epi<T, EPI, NTT, split, MAXC>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    // persistent grid: as many workgroups as can be resident at once (at most `grid`)
    int per_cu = 0, dev = 0, ncu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(kern), 256, lds) ==
            hipSuccess &&
        hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && per_cu > 0)
        grid = std::min(grid, per_cu * ncu);
    if (grid_used) *grid_used = grid;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(256), lds, st, u, out, src, gy, wpw, bpw, part, (const Op *)tb.z,
                       (const Op *)tb.z_lo, (const Op *)tb.t, (const Op *)tb.t_lo, a);
    return hipGetLastError();
}

template <typename T, int EPI>
static hipError_t launch_zt_e(const ZtArgs &a, int ntt, int maxc, const float2 *u, T *out, const T *src, const T *gy,
                              const float *wpw, const float *bpw, float *part, const ZtTabs &tb, int grid,
                              hipStream_t st, int *grid_used)
{
    if (ntt == 1) {
        if (maxc <= 2) return launch_zt_t<T, EPI, 1, 2>(a, u, out, src, gy, wpw, bpw, part, tb, grid, st, grid_used);
        return launch_zt_t<T, EPI, 1, 4>(a, u, out, src, gy, wpw, bpw, part, tb, grid, st, grid_used);
    }
    if (maxc <= 2) return launch_zt_t<T, EPI, 2, 2>(a, u, out, src, gy, wpw, bpw, part, tb, grid, st, grid_used);
    return launch_zt_t<T, EPI, 2, 4>(a, u, out, src, gy, wpw, bpw, part, tb, grid, st, grid_used);
}

// epi: ZEPI_*; Cs = output/spectral channels, Csrc = pointwise source channels.
// grid_used (nullable) receives the number of workgroups launched (rows of BWD partial sums / 4).
template <typename T>
hipError_t launch_zt(int epi, const Dims &d, int Cs, int Csrc, const float2 *u, T *out, const T *src, const T *gy,
                     const float *wpw, const float *bpw, float *part, const ZtTabs &tb, int accumulate, hipStream_t st,
                     int *grid_used)
{
    ZtArgs a{};
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
    a.QZ = 2 * a.Kzp / 16;
    a.NTQ = (d.N[3] + 15) / 16;
    a.ZC = 16;
    a.accumulate = accumulate;
    const int ntt = d.K[3] <= 8 ? 1 : 2;
    const int maxc = (std::max(Cs, Csrc) + 15) / 16;
    const int grid = zt_grid(d);
    switch (epi) {
    case ZEPI_PLAIN: return launch_zt_e<T, ZEPI_PLAIN>(a, ntt, maxc, u, out, src, gy, wpw, bpw, part, tb, grid, st, grid_used);
    case ZEPI_BLOCK: return launch_zt_e<T, ZEPI_BLOCK>(a, ntt, maxc, u, out, src, gy, wpw, bpw, part, tb, grid, st, grid_used);
    case ZEPI_BWD: return launch_zt_e<T, ZEPI_BWD>(a, ntt, maxc, u, out, src, gy, wpw, bpw, part, tb, grid, st, grid_used);
    default: return launch_zt_e<T, ZEPI_ADJ>(a, ntt, maxc, u, out, src, gy, wpw, bpw, part, tb, grid, st, grid_used);
    }
}

template hipError_t launch_zt<float>(int, const Dims &, int, int, const float2 *, float *, const float *,
                                     const float *, const float *, const float *, float *, const ZtTabs &, int,
                                     hipStream_t, int *);
template hipError_t launch_zt<__bf16>(int, const Dims &, int, int, const float2 *, __bf16 *, const __bf16 *,
                                      const __bf16 *, const float *, const float *, float *, const ZtTabs &, int,
                                      hipStream_t, int *);

}  // namespace fno
