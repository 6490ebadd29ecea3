// tables.hip -- basis tables of the MFMA kernels, stored directly in MFMA
// fragment order (see mfma_common.h): entry [tile...][lane][j] is the value a
// lane feeds to the matrix core.  Every value is computed in FP64 on the GPU
// (phase k*n reduced modulo N exactly in 64-bit integers), then rounded once
// to float and, for the bfloat16 kernels, split into hi = bf16(v) and
// lo = bf16(v - hi) so that hi + lo carries about 16 significant bits.
//
// Retained frequencies follow the truncation of Alg. 2 (Sec. IV-C): compact
// index j < m is frequency j and j >= m is N - 2m + j on x, y, z; on t it is j.
#include "fno_internal.h"
#include "mfma_common.h"

namespace fno {

__device__ __forceinline__ double ang(long long k, long long n, long long N)
{
    return 6.283185307179586476925286766559 * (double)((k * n) % N) / (double)N;
}

__device__ __forceinline__ long long freq(int j, int m, int N) { return j < m ? j : (long long)N - 2 * m + j; }

__device__ __forceinline__ double ct_weight(int kt, int Nt, double inv_ncell, int kind)
{
    if (kind == 0) return 1.0;
    const double c = (kt == 0 || (Nt % 2 == 0 && 2 * kt == Nt)) ? 1.0 : 2.0;
    return c * inv_ncell;
}

// kind: TAB_T_FWD / TAB_T_BWD (t-step B operand, weights 1 or c(kt)/N),
//       TAB_Z_FWD (z-step A operand), TAB_Y_FWD (y-step A operand).
//       TAB_ZI (z-synthesis B operand), TAB_TI_INV / TAB_TI_ADJ (t-synthesis A
//       operand with weights c(kt)/N or 1).
//       TAB_AXF / TAB_AXI (one-axis contraction A operand, forward / inverse,
//       for the axis described by the ax* fields).
enum {
    TAB_T_FWD = 0, TAB_T_BWD = 1, TAB_Z_FWD = 2, TAB_Y_FWD = 3, TAB_ZI = 4, TAB_TI_INV = 5, TAB_TI_ADJ = 6,
    TAB_AXF = 7, TAB_AXI = 8
};

struct TabGeom {
    int Nt, Kt, NTT, NQ;
    int Nz, Kz, mz, Kzp, NZB, MZ;
    int Ny, Ky, my, Kyp, MY, Yc, QY, NYC;
    double inv_ncell;
    int axN, axm, axNin, axNout, axNinp, axNoutp;  // one-axis contraction
};

__global__ void k_gen_tab(int kind, TabGeom G, long long n, float *__restrict__ f32, short *__restrict__ hi,
                          short *__restrict__ lo)
{
    long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int j = (int)(e & 3), lane = (int)((e >> 2) & 63);
    const int g = lane >> 4, c = lane & 15;
    long long tile = e >> 8;
    double v = 0.0;
    if (kind == TAB_T_FWD || kind == TAB_T_BWD) {
        const int nt = (int)(tile % G.NTT), q = (int)(tile / G.NTT);
        const int t = 16 * q + 4 * g + j;
        const int ri = G.NTT == 1 ? c / 8 : nt;
        const int kt = G.NTT == 1 ? c % 8 : c;
        if (t < G.Nt && kt < G.Kt) {
            const double th = ang(kt, t, G.Nt);
            const double w = ct_weight(kt, G.Nt, G.inv_ncell, kind == TAB_T_BWD);
            v = ri == 0 ? w * cos(th) : -w * sin(th);
        }
    } else if (kind == TAB_Z_FWD) {
        const int mb = (int)(tile % G.MZ), zb = (int)(tile / G.MZ);
        const int m = mb * 16 + c, z = zb * 16 + 4 * g + j;
        const int h = m < G.Kzp ? 0 : 1, kz = m < G.Kzp ? m : m - G.Kzp;
        if (z < G.Nz && kz < G.Kz) {
            const double th = ang(freq(kz, G.mz, G.Nz), z, G.Nz);
            v = h == 0 ? cos(th) : sin(th);
        }
    } else if (kind == TAB_Y_FWD) {
        const int mb = (int)(tile % G.MY);
        const long long r1 = tile / G.MY;
        const int q = (int)(r1 % G.QY), ych = (int)(r1 / G.QY);
        const int row = mb * 16 + c, ro = row / G.Kyp, ky = row % G.Kyp;
        const int k = 16 * q + 4 * g + j, ri = k / G.Yc, y = ych * G.Yc + k % G.Yc;
        if (ky < G.Ky && y < G.Ny) {
            const double th = ang(freq(ky, G.my, G.Ny), y, G.Ny);
            const double cs = cos(th), sn = sin(th);
            // [[cos, sin], [-sin, cos]]: (Re, Im) out from (Re, Im) in for exp(-i theta)
            v = ro == 0 ? (ri == 0 ? cs : sn) : (ri == 0 ? -sn : cs);
        }
    } else if (kind == TAB_ZI) {
        // B[(ri, kz)][z] for z tile zt and K chunk q: cos (ri = 0) / sin (ri = 1) of theta(kz, z)
        const int q = (int)(tile % (2 * G.Kzp / 16)), zt = (int)(tile / (2 * G.Kzp / 16));
        const int k = 16 * q + 4 * g + j, ri = k / G.Kzp, kz = k % G.Kzp, z = zt * 16 + c;
        if (z < G.Nz && kz < G.Kz) {
            const double th = ang(freq(kz, G.mz, G.Nz), z, G.Nz);
            v = ri == 0 ? cos(th) : sin(th);
        }
    } else if (kind == TAB_TI_INV || kind == TAB_TI_ADJ) {
        // A[t][(ri, kt)] for t tile mt of t slice ts and K chunk q: w cos (ri = 0) / -w sin (ri = 1) of
        // 2 pi kt t / Nt.  A slice is NTQ t tiles (NTQ = 1 for Nt <= 16, else 2: 32 t); row c of tile mt
        // of slice ts is t = 16 NTQ ts + 4 NTQ (c / 4) + 4 mt + c % 4, so that an output lane 16 g' + c'
        // holds the 4 NTQ consecutive t = 16 NTQ ts + 4 NTQ g' .. of column c' across the slice's tiles.
        const int q = (int)(tile % G.NTT), st = (int)(tile / G.NTT);
        const int ntq = G.Nt > 16 ? 2 : 1, ts = st / ntq, mt = st % ntq;
        const int t = 16 * ntq * ts + 4 * ntq * (c >> 2) + 4 * mt + (c & 3), k = 16 * q + 4 * g + j;
        const int ri = G.NTT == 1 ? k / 8 : q;
        const int kt = G.NTT == 1 ? k % 8 : k - 16 * q;
        if (t < G.Nt && kt < G.Kt) {
            const double th = ang(kt, t, G.Nt);
            const double w = ct_weight(kt, G.Nt, G.inv_ncell, kind == TAB_TI_INV);
            v = ri == 0 ? w * cos(th) : -w * sin(th);
        }
    } else if (kind == TAB_AXF || kind == TAB_AXI) {
        const int QK = 2 * G.axNinp / 16;
        const int q = (int)(tile % QK), mt = (int)(tile / QK);
        const int row = mt * 16 + c, ro = row / G.axNoutp, jj = row % G.axNoutp;
        const int k = 16 * q + 4 * g + j, ri = k / G.axNinp, nn = k % G.axNinp;
        if (jj < G.axNout && nn < G.axNin) {
            const bool fwd = kind == TAB_AXF;
            // forward: jj retained frequency, nn grid point; inverse: jj grid point, nn retained frequency
            const double th = fwd ? ang(freq(jj, G.axm, G.axN), nn, G.axN) : ang(freq(nn, G.axm, G.axN), jj, G.axN);
            const double cs = cos(th), sn = fwd ? sin(th) : -sin(th);
            // [[cos, s], [-s, cos]] with s = sin (exp(-i theta)) or -sin (exp(+i theta))
            v = ro == 0 ? (ri == 0 ? cs : sn) : (ri == 0 ? -sn : cs);
        }
    }
    const float vf = (float)v;
    f32[e] = vf;
    if (hi) {
        const __bf16 h = (__bf16)vf;
        const float rem = (float)(v - (double)(float)h);
        hi[e] = __builtin_bit_cast(short, h);
        lo[e] = __builtin_bit_cast(short, (__bf16)rem);
    }
}

void fill_geom(const Dims &d, int dtype, TabGeom &G)
{
    G.Nt = d.N[3];
    G.Kt = d.K[3];
    G.NTT = d.K[3] <= 8 ? 1 : 2;
    G.NQ = (d.N[3] + 15) / 16;
    G.Nz = d.N[2];
    G.Kz = d.K[2];
    G.mz = d.m[2];
    G.Kzp = (d.K[2] + 15) / 16 * 16;
    G.NZB = (d.N[2] + 15) / 16;
    G.MZ = 2 * G.Kzp / 16;
    G.Ny = d.N[1];
    G.Ky = d.K[1];
    G.my = d.m[1];
    G.Kyp = (d.K[1] + 15) / 16 * 16;
    G.MY = 2 * G.Kyp / 16;
    G.Yc = dtype == FNO_BF16 ? 32 : 16;
    G.QY = 2 * G.Yc / 16;
    G.NYC = (d.N[1] + G.Yc - 1) / G.Yc;
    G.inv_ncell = 1.0 / (double)d.ncell;
}

long long tab_values(int kind, const TabGeom &G)
{
    switch (kind) {
    case TAB_T_FWD:
    case TAB_T_BWD: return (long long)G.NQ * G.NTT * 256;
    case TAB_Z_FWD: return (long long)G.NZB * G.MZ * 256;
    case TAB_Y_FWD: return (long long)G.NYC * G.QY * G.MY * 256;
    case TAB_ZI: return (long long)G.NZB * (2 * G.Kzp / 16) * 256;
    case TAB_TI_INV:
    case TAB_TI_ADJ: {
        const int ntq = G.Nt > 16 ? 2 : 1;  // t tiles per slice; slices cover Nt
        return (long long)((G.Nt + 16 * ntq - 1) / (16 * ntq)) * ntq * G.NTT * 256;
    }
    case TAB_AXF:
    case TAB_AXI: return (long long)(2 * G.axNoutp / 16) * (2 * G.axNinp / 16) * 256;
    }
    return 0;
}

void gen_tab(int kind, const TabGeom &G, float *f32, short *hi, short *lo, hipStream_t st)
{
    const long long n = tab_values(kind, G);
    hipLaunchKernelGGL(k_gen_tab, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, kind, G, n, f32, hi, lo);
}

}  // namespace fno

namespace fno {

TabGeom *new_geom(const Dims &d, int dtype)
{
    TabGeom *g = new TabGeom();
    fill_geom(d, dtype, *g);
    return g;
}

// Geometry of the one-axis contraction along axis a (0 = x, 1 = y), forward
// (grid -> retained) or inverse (retained -> grid).
TabGeom *new_axis_geom(const Dims &d, int a, bool forward)
{
    TabGeom *g = new TabGeom();
    fill_geom(d, FNO_F32, *g);
    g->axN = d.N[a];
    g->axm = d.m[a];
    g->axNin = forward ? d.N[a] : d.K[a];
    g->axNout = forward ? d.K[a] : d.N[a];
    g->axNinp = (g->axNin + 15) / 16 * 16;
    g->axNoutp = (g->axNout + 15) / 16 * 16;
    return g;
}

void free_geom(TabGeom *g) { delete g; }

long long tab_count(int kind, const TabGeom &G) { return tab_values(kind, G); }

void gen_frag(int kind, const TabGeom &G, const Tables::Frag &f, hipStream_t st) { gen_tab(kind, G, f.f, f.hi, f.lo, st); }

}  // namespace fno
