/*
 * fno_oracle.c -- plain FP64 CPU oracle for the 4-D spectral-convolution FNO
 * block (arXiv 2211.12709, "SciAI4Industry", Sec. IV-C, Alg. 1 and Alg. 2).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only tests/, the smoke check in __graft_entry__.py and the
 * cpu_baseline leg of bench.py use it.  It shares no code, header, table or
 * constant with the HIP library; it is written from the paper's definitions.
 *
 * Everything is double precision, explicit loops, direct DFT sums (no FFT),
 * OpenMP only over independent outer loops.
 *
 * Notation (Sec. IV-C): data tensor X[b][c][x][y][z][t] (t fastest), spectral
 * tensor X^[b][c][kx][ky][kz][kt], weights W[ci][co][kx][ky][kz][kt].
 * Complex numbers are stored as interleaved (re, im) doubles.
 *
 * Readings where the paper is silent (each is listed in the design doc):
 *  - Retained set K (Sec. IV-C "most frequencies are truncated"): on x, y, z
 *    the m lowest non-negative and the m lowest negative frequencies; the
 *    compact index j maps to frequency j (j < m) or N - 2m + j (j >= m).  On t
 *    (the real-transformed, last axis) the m_t lowest non-negative ones.
 *  - Forward transform unnormalised with sign -1; the inverse carries 1/N and
 *    the real-output weight c(kt) (1 for kt = 0 and for the Nyquist bin of an
 *    even N_t, 2 otherwise) and keeps the real part, i.e. it is the real
 *    inverse of the zero-padded truncated spectrum.
 *  - sigma is GELU in its erf form; the block adds a pointwise 1x1 channel
 *    linear with bias beside the spectral convolution, inside sigma.
 *
 * Dimension vector used by every entry point ("d"):
 *   d[0]=B, d[1]=C_in, d[2]=C_out, d[3..6]=N_x,N_y,N_z,N_t, d[7..10]=m_x,m_y,m_z,m_t
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PI_D 3.14159265358979323846264338327950288

typedef struct {
    long B, Ci, Co;
    long N[4];   /* x, y, z, t */
    long m[4];   /* modes per axis; for t the count of non-negative bins */
    long K[4];   /* retained count per axis: 2m for x,y,z and m_t for t */
    long ncell;  /* Nx*Ny*Nz*Nt */
    long nmode;  /* Kx*Ky*Kz*Kt */
} dims_t;

static int get_dims(const int *d, dims_t *s)
{
    s->B = d[0]; s->Ci = d[1]; s->Co = d[2];
    for (int a = 0; a < 4; a++) { s->N[a] = d[3 + a]; s->m[a] = d[7 + a]; }
    for (int a = 0; a < 3; a++) s->K[a] = 2 * s->m[a];
    s->K[3] = s->m[3];
    if (s->B < 1 || s->Ci < 1 || s->Co < 1) return -1;
    for (int a = 0; a < 4; a++) if (s->N[a] < 1 || s->m[a] < 1) return -1;
    for (int a = 0; a < 3; a++) if (2 * s->m[a] > s->N[a]) return -1;
    if (s->m[3] > s->N[3] / 2 + 1) return -1;
    s->ncell = s->N[0] * s->N[1] * s->N[2] * s->N[3];
    s->nmode = s->K[0] * s->K[1] * s->K[2] * s->K[3];
    return 0;
}

int oracle_check_dims(const int *d) { dims_t s; return get_dims(d, &s); }

/* Grid frequency (in [0, N)) of compact index j on axis a. */
static long freq_of(const dims_t *s, int a, long j)
{
    if (a == 3) return j;
    return j < s->m[a] ? j : s->N[a] - 2 * s->m[a] + j;
}

/* Angle 2*pi*((k*n) mod N)/N with the product reduced exactly in integers. */
static double angle(long k, long n, long N)
{
    long r = (k * n) % N;
    return 2.0 * PI_D * (double)r / (double)N;
}

/* Real-output weight of the t bin kt (irfft convention). */
double oracle_ct(long kt, long Nt)
{
    if (kt == 0) return 1.0;
    if (Nt % 2 == 0 && 2 * kt == Nt) return 1.0;
    return 2.0;
}

/* cos/sin tables for one axis: tab[(j*N + n)*2 + {0,1}] = cos, sin of the
 * angle of retained frequency j at grid point n. */
static double *axis_table(const dims_t *s, int a)
{
    long N = s->N[a], K = s->K[a];
    double *t = (double *)malloc(sizeof(double) * 2 * K * N);
    for (long j = 0; j < K; j++)
        for (long n = 0; n < N; n++) {
            double th = angle(freq_of(s, a, j), n, N);
            t[(j * N + n) * 2 + 0] = cos(th);
            t[(j * N + n) * 2 + 1] = sin(th);
        }
    return t;
}

/* ------------------------------------------------------------------------ */
/* Forward truncated DFT (Alg. 2, first line): S_x F_x R S_yzt F_yzt.
 * out[b][c][k] = wt[kt] * sum_n in[b][c][n] * exp(-i theta(k, n)).
 * The sum is taken one axis at a time in the order of Alg. 2: t, z, y (the
 * non-partitioned dimensions), then x; only retained frequencies are ever
 * evaluated, which is what truncation after the transform keeps.
 * wt may be NULL (all ones).  C is the channel count of "in".             */
void oracle_dft_fwd(const int *d, int C, const double *in, const double *wt, double *out)
{
    dims_t s; if (get_dims(d, &s)) return;
    const long Nx = s.N[0], Ny = s.N[1], Nz = s.N[2], Nt = s.N[3];
    const long Kx = s.K[0], Ky = s.K[1], Kz = s.K[2], Kt = s.K[3];
    double *ex = axis_table(&s, 0), *ey = axis_table(&s, 1), *ez = axis_table(&s, 2), *et = axis_table(&s, 3);
    const long nslab = s.B * C * Nx;
    /* T2[b][c][x][ky][kz][kt] complex: result of the y, z, t stages */
    double *T2 = (double *)calloc((size_t)nslab * Ky * Kz * Kt * 2, sizeof(double));

    #pragma omp parallel
    {
        double *A = (double *)malloc(sizeof(double) * Ny * Nz * Kt * 2);  /* [y][z][kt]  */
        double *Bz = (double *)malloc(sizeof(double) * Ny * Kz * Kt * 2); /* [y][kz][kt] */
        #pragma omp for schedule(dynamic)
        for (long sl = 0; sl < nslab; sl++) {
            const double *xs = in + (size_t)sl * Ny * Nz * Nt;
            /* t: real -> complex, A = sum_t x * (cos - i sin) */
            for (long y = 0; y < Ny; y++)
                for (long z = 0; z < Nz; z++) {
                    const double *row = xs + (y * Nz + z) * Nt;
                    for (long kt = 0; kt < Kt; kt++) {
                        double re = 0, im = 0;
                        for (long t = 0; t < Nt; t++) {
                            re += row[t] * et[(kt * Nt + t) * 2 + 0];
                            im -= row[t] * et[(kt * Nt + t) * 2 + 1];
                        }
                        A[((y * Nz + z) * Kt + kt) * 2 + 0] = re;
                        A[((y * Nz + z) * Kt + kt) * 2 + 1] = im;
                    }
                }
            /* z: Bz[y][kz][kt] = sum_z exp(-i th) A[y][z][kt] */
            for (long y = 0; y < Ny; y++)
                for (long kz = 0; kz < Kz; kz++)
                    for (long kt = 0; kt < Kt; kt++) {
                        double re = 0, im = 0;
                        for (long z = 0; z < Nz; z++) {
                            double c = ez[(kz * Nz + z) * 2], sn = ez[(kz * Nz + z) * 2 + 1];
                            double ar = A[((y * Nz + z) * Kt + kt) * 2], ai = A[((y * Nz + z) * Kt + kt) * 2 + 1];
                            /* (c - i sn)(ar + i ai) */
                            re += c * ar + sn * ai;
                            im += c * ai - sn * ar;
                        }
                        Bz[((y * Kz + kz) * Kt + kt) * 2 + 0] = re;
                        Bz[((y * Kz + kz) * Kt + kt) * 2 + 1] = im;
                    }
            /* y: T2[ky][kz][kt] = sum_y exp(-i th) Bz[y][kz][kt] */
            double *t2 = T2 + (size_t)sl * Ky * Kz * Kt * 2;
            for (long ky = 0; ky < Ky; ky++)
                for (long q = 0; q < Kz * Kt; q++) {
                    double re = 0, im = 0;
                    for (long y = 0; y < Ny; y++) {
                        double c = ey[(ky * Ny + y) * 2], sn = ey[(ky * Ny + y) * 2 + 1];
                        double br = Bz[(y * Kz * Kt + q) * 2], bi = Bz[(y * Kz * Kt + q) * 2 + 1];
                        re += c * br + sn * bi;
                        im += c * bi - sn * br;
                    }
                    t2[(ky * Kz * Kt + q) * 2 + 0] = re;
                    t2[(ky * Kz * Kt + q) * 2 + 1] = im;
                }
        }
        free(A); free(Bz);
    }
    /* x: out[b][c][kx][q] = wt[kt] * sum_x exp(-i th) T2[b][c][x][q] */
    const long Q = Ky * Kz * Kt;
    #pragma omp parallel for collapse(2) schedule(static)
    for (long bc = 0; bc < s.B * C; bc++)
        for (long kx = 0; kx < Kx; kx++)
            for (long q = 0; q < Q; q++) {
                double re = 0, im = 0;
                for (long x = 0; x < Nx; x++) {
                    double c = ex[(kx * Nx + x) * 2], sn = ex[(kx * Nx + x) * 2 + 1];
                    const double *p = T2 + (((size_t)bc * Nx + x) * Q + q) * 2;
                    re += c * p[0] + sn * p[1];
                    im += c * p[1] - sn * p[0];
                }
                double w = wt ? wt[q % Kt] : 1.0;
                out[(((size_t)bc * Kx + kx) * Q + q) * 2 + 0] = w * re;
                out[(((size_t)bc * Kx + kx) * Q + q) * 2 + 1] = w * im;
            }
    free(T2); free(ex); free(ey); free(ez); free(et);
}

/* ------------------------------------------------------------------------ */
/* Synthesis from retained modes (Alg. 2, third line, and its adjoint use):
 * out[b][c][n] = sum_{k in K} wt[kt] * Re( F[b][c][k] * exp(+i theta(k, n)) ).
 * With wt[kt] = c(kt)/N this is the real inverse DFT of the zero-padded
 * spectrum; with wt = 1 it is the adjoint of oracle_dft_fwd.
 * Axis order is the reverse of the forward: x, then y, z, t.             */
void oracle_synth(const int *d, int C, const double *F, const double *wt, double *out)
{
    dims_t s; if (get_dims(d, &s)) return;
    const long Nx = s.N[0], Ny = s.N[1], Nz = s.N[2], Nt = s.N[3];
    const long Kx = s.K[0], Ky = s.K[1], Kz = s.K[2], Kt = s.K[3];
    double *ex = axis_table(&s, 0), *ey = axis_table(&s, 1), *ez = axis_table(&s, 2), *et = axis_table(&s, 3);
    const long Q = Ky * Kz * Kt;
    const long nslab = s.B * C * Nx;
    double *U2 = (double *)malloc(sizeof(double) * (size_t)nslab * Q * 2); /* [b][c][x][ky][kz][kt] */
    /* x: U2[b][c][x][q] = sum_kx exp(+i th) F[b][c][kx][q] */
    #pragma omp parallel for collapse(2) schedule(static)
    for (long bc = 0; bc < s.B * C; bc++)
        for (long x = 0; x < Nx; x++)
            for (long q = 0; q < Q; q++) {
                double re = 0, im = 0;
                for (long kx = 0; kx < Kx; kx++) {
                    double c = ex[(kx * Nx + x) * 2], sn = ex[(kx * Nx + x) * 2 + 1];
                    const double *p = F + (((size_t)bc * Kx + kx) * Q + q) * 2;
                    /* (c + i sn)(pr + i pi) */
                    re += c * p[0] - sn * p[1];
                    im += c * p[1] + sn * p[0];
                }
                U2[(((size_t)bc * Nx + x) * Q + q) * 2 + 0] = re;
                U2[(((size_t)bc * Nx + x) * Q + q) * 2 + 1] = im;
            }
    #pragma omp parallel
    {
        double *U1 = (double *)malloc(sizeof(double) * Ny * Kz * Kt * 2); /* [y][kz][kt] */
        double *V = (double *)malloc(sizeof(double) * Ny * Nz * Kt * 2);  /* [y][z][kt]  */
        #pragma omp for schedule(dynamic)
        for (long sl = 0; sl < nslab; sl++) {
            const double *u2 = U2 + (size_t)sl * Q * 2;
            /* y */
            for (long y = 0; y < Ny; y++)
                for (long q = 0; q < Kz * Kt; q++) {
                    double re = 0, im = 0;
                    for (long ky = 0; ky < Ky; ky++) {
                        double c = ey[(ky * Ny + y) * 2], sn = ey[(ky * Ny + y) * 2 + 1];
                        double pr = u2[(ky * Kz * Kt + q) * 2], pi = u2[(ky * Kz * Kt + q) * 2 + 1];
                        re += c * pr - sn * pi;
                        im += c * pi + sn * pr;
                    }
                    U1[(y * Kz * Kt + q) * 2 + 0] = re;
                    U1[(y * Kz * Kt + q) * 2 + 1] = im;
                }
            /* z */
            for (long y = 0; y < Ny; y++)
                for (long z = 0; z < Nz; z++)
                    for (long kt = 0; kt < Kt; kt++) {
                        double re = 0, im = 0;
                        for (long kz = 0; kz < Kz; kz++) {
                            double c = ez[(kz * Nz + z) * 2], sn = ez[(kz * Nz + z) * 2 + 1];
                            double pr = U1[((y * Kz + kz) * Kt + kt) * 2], pi = U1[((y * Kz + kz) * Kt + kt) * 2 + 1];
                            re += c * pr - sn * pi;
                            im += c * pi + sn * pr;
                        }
                        V[((y * Nz + z) * Kt + kt) * 2 + 0] = re;
                        V[((y * Nz + z) * Kt + kt) * 2 + 1] = im;
                    }
            /* t: keep the real part, weighted per kt */
            double *os = out + (size_t)sl * Ny * Nz * Nt;
            for (long y = 0; y < Ny; y++)
                for (long z = 0; z < Nz; z++)
                    for (long t = 0; t < Nt; t++) {
                        double acc = 0;
                        for (long kt = 0; kt < Kt; kt++) {
                            double c = et[(kt * Nt + t) * 2], sn = et[(kt * Nt + t) * 2 + 1];
                            double vr = V[((y * Nz + z) * Kt + kt) * 2], vi = V[((y * Nz + z) * Kt + kt) * 2 + 1];
                            double w = wt ? wt[kt] : 1.0;
                            acc += w * (vr * c - vi * sn);
                        }
                        os[(y * Nz + z) * Nt + t] = acc;
                    }
        }
        free(U1); free(V);
    }
    free(U2); free(ex); free(ey); free(ez); free(et);
}

/* ------------------------------------------------------------------------ */
/* Non-separable versions: one 4-D sum per output, for tiny grids and for
 * sampled outputs of large ones.                                          */

/* out[b][c][k] = sum_n in[b][c][n] exp(-i theta(k, n)) for every k in K. */
void oracle_dft_fwd_direct(const int *d, int C, const double *in, double *out)
{
    dims_t s; if (get_dims(d, &s)) return;
    const long BC = s.B * C, M = s.nmode;
    #pragma omp parallel for collapse(2) schedule(dynamic)
    for (long bc = 0; bc < BC; bc++)
        for (long mi = 0; mi < M; mi++) {
            long j[4], r = mi;
            for (int a = 3; a >= 0; a--) { j[a] = r % s.K[a]; r /= s.K[a]; }
            long k[4]; for (int a = 0; a < 4; a++) k[a] = freq_of(&s, a, j[a]);
            double re = 0, im = 0;
            for (long n = 0; n < s.ncell; n++) {
                long nn[4], q = n;
                for (int a = 3; a >= 0; a--) { nn[a] = q % s.N[a]; q /= s.N[a]; }
                /* theta = 2 pi sum_a k_a n_a / N_a, each term reduced exactly */
                double th = 0;
                for (int a = 0; a < 4; a++) th += angle(k[a], nn[a], s.N[a]);
                double v = in[(size_t)bc * s.ncell + n];
                re += v * cos(th);
                im -= v * sin(th);
            }
            out[((size_t)bc * M + mi) * 2 + 0] = re;
            out[((size_t)bc * M + mi) * 2 + 1] = im;
        }
}

/* Forward DFT at a list of retained modes: kidx holds 4 compact indices per
 * mode; out[(b*C + c)*nk + i] complex. */
void oracle_dft_fwd_modes(const int *d, int C, const double *in, long nk, const int *kidx, double *out)
{
    dims_t s; if (get_dims(d, &s)) return;
    const long BC = s.B * C;
    #pragma omp parallel for collapse(2) schedule(dynamic)
    for (long bc = 0; bc < BC; bc++)
        for (long i = 0; i < nk; i++) {
            long k[4]; for (int a = 0; a < 4; a++) k[a] = freq_of(&s, a, kidx[i * 4 + a]);
            double re = 0, im = 0;
            for (long n = 0; n < s.ncell; n++) {
                long nn[4], q = n;
                for (int a = 3; a >= 0; a--) { nn[a] = q % s.N[a]; q /= s.N[a]; }
                double th = 0;
                for (int a = 0; a < 4; a++) th += angle(k[a], nn[a], s.N[a]);
                double v = in[(size_t)bc * s.ncell + n];
                re += v * cos(th);
                im -= v * sin(th);
            }
            out[((size_t)bc * nk + i) * 2 + 0] = re;
            out[((size_t)bc * nk + i) * 2 + 1] = im;
        }
}

/* out[b][c][p] = sum_k wt[kt] Re(F[b][c][k] exp(+i theta(k, n_p))) at the
 * flat grid points pts[0..np).  Used for the full 4-D sum on tiny grids
 * (pts = every point) and for sampled outputs of large grids.            */
void oracle_synth_points(const int *d, int C, const double *F, const double *wt, long np, const long *pts, double *out)
{
    dims_t s; if (get_dims(d, &s)) return;
    const long BC = s.B * C, M = s.nmode;
    #pragma omp parallel for collapse(2) schedule(dynamic)
    for (long bc = 0; bc < BC; bc++)
        for (long p = 0; p < np; p++) {
            long nn[4], q = pts[p];
            for (int a = 3; a >= 0; a--) { nn[a] = q % s.N[a]; q /= s.N[a]; }
            double acc = 0;
            for (long mi = 0; mi < M; mi++) {
                long j[4], r = mi;
                for (int a = 3; a >= 0; a--) { j[a] = r % s.K[a]; r /= s.K[a]; }
                double th = 0;
                for (int a = 0; a < 4; a++) th += angle(freq_of(&s, a, j[a]), nn[a], s.N[a]);
                const double *f = F + ((size_t)bc * M + mi) * 2;
                double w = wt ? wt[j[3]] : 1.0;
                acc += w * (f[0] * cos(th) - f[1] * sin(th));
            }
            out[(size_t)bc * np + p] = acc;
        }
}

/* ------------------------------------------------------------------------ */
/* Spectral convolution (Alg. 2, second line; einsum rule of Sec. IV-C):
 * Y^[b][o][k] = sum_i X^[b][i][k] * W[i][o][k]  (complex, no conjugation). */
void oracle_mix(const int *d, const double *xh, const double *w, double *yh)
{
    dims_t s; if (get_dims(d, &s)) return;
    const long M = s.nmode;
    #pragma omp parallel for collapse(2) schedule(static)
    for (long b = 0; b < s.B; b++)
        for (long o = 0; o < s.Co; o++)
            for (long k = 0; k < M; k++) {
                double re = 0, im = 0;
                for (long i = 0; i < s.Ci; i++) {
                    const double *a = xh + (((size_t)b * s.Ci + i) * M + k) * 2;
                    const double *q = w + (((size_t)i * s.Co + o) * M + k) * 2;
                    re += a[0] * q[0] - a[1] * q[1];
                    im += a[0] * q[1] + a[1] * q[0];
                }
                yh[(((size_t)b * s.Co + o) * M + k) * 2 + 0] = re;
                yh[(((size_t)b * s.Co + o) * M + k) * 2 + 1] = im;
            }
}

/* Gradients of oracle_mix in the convention g = dL/dRe + i dL/dIm:
 * gX^[b][i][k] = sum_o gY^[b][o][k] * conj(W[i][o][k]);
 * gW[i][o][k]  = sum_b conj(X^[b][i][k]) * gY^[b][o][k].  Either output may be NULL. */
void oracle_mix_bwd(const int *d, const double *xh, const double *w, const double *gyh, double *gxh, double *gw)
{
    dims_t s; if (get_dims(d, &s)) return;
    const long M = s.nmode;
    if (gxh) {
        #pragma omp parallel for collapse(2) schedule(static)
        for (long b = 0; b < s.B; b++)
            for (long i = 0; i < s.Ci; i++)
                for (long k = 0; k < M; k++) {
                    double re = 0, im = 0;
                    for (long o = 0; o < s.Co; o++) {
                        const double *g = gyh + (((size_t)b * s.Co + o) * M + k) * 2;
                        const double *q = w + (((size_t)i * s.Co + o) * M + k) * 2;
                        /* g * conj(q) */
                        re += g[0] * q[0] + g[1] * q[1];
                        im += g[1] * q[0] - g[0] * q[1];
                    }
                    gxh[(((size_t)b * s.Ci + i) * M + k) * 2 + 0] = re;
                    gxh[(((size_t)b * s.Ci + i) * M + k) * 2 + 1] = im;
                }
    }
    if (gw) {
        #pragma omp parallel for collapse(2) schedule(static)
        for (long i = 0; i < s.Ci; i++)
            for (long o = 0; o < s.Co; o++)
                for (long k = 0; k < M; k++) {
                    double re = 0, im = 0;
                    for (long b = 0; b < s.B; b++) {
                        const double *a = xh + (((size_t)b * s.Ci + i) * M + k) * 2;
                        const double *g = gyh + (((size_t)b * s.Co + o) * M + k) * 2;
                        /* conj(a) * g */
                        re += a[0] * g[0] + a[1] * g[1];
                        im += a[0] * g[1] - a[1] * g[0];
                    }
                    gw[(((size_t)i * s.Co + o) * M + k) * 2 + 0] = re;
                    gw[(((size_t)i * s.Co + o) * M + k) * 2 + 1] = im;
                }
    }
}

/* Per-kt weights of the real inverse: c(kt)/N. */
static double *inverse_weights(const dims_t *s)
{
    double *w = (double *)malloc(sizeof(double) * s->K[3]);
    for (long kt = 0; kt < s->K[3]; kt++) w[kt] = oracle_ct(kt, s->N[3]) / (double)s->ncell;
    return w;
}

/* ------------------------------------------------------------------------ */
/* Spectral convolution layer (Alg. 2 as a whole): forward DFT + truncation,
 * mode mix, zero-padding + real inverse DFT.  y has C_out channels.
 * xh_out (nullable) receives X^ [B][Ci][modes] and yh_out (nullable) Y^.  */
void oracle_spectral_fwd(const int *d, const double *x, const double *w, double *y, double *xh_out, double *yh_out)
{
    dims_t s; if (get_dims(d, &s)) return;
    double *xh = (double *)malloc(sizeof(double) * 2 * s.B * s.Ci * s.nmode);
    double *yh = (double *)malloc(sizeof(double) * 2 * s.B * s.Co * s.nmode);
    double *wt = inverse_weights(&s);
    oracle_dft_fwd(d, (int)s.Ci, x, NULL, xh);
    oracle_mix(d, xh, w, yh);
    oracle_synth(d, (int)s.Co, yh, wt, y);
    if (xh_out) memcpy(xh_out, xh, sizeof(double) * 2 * s.B * s.Ci * s.nmode);
    if (yh_out) memcpy(yh_out, yh, sizeof(double) * 2 * s.B * s.Co * s.nmode);
    free(xh); free(yh); free(wt);
}

/* Backward of the spectral layer.  gx (nullable) = adjoint applied to gy;
 * gw (nullable) = complex weight gradient summed over the batch.
 * gY^ = (c(kt)/N) sum_n gy exp(-i theta)   (adjoint of the real inverse),
 * gX^ and gW from oracle_mix_bwd, gx = sum_k Re(gX^ exp(+i theta)).      */
void oracle_spectral_bwd(const int *d, const double *x, const double *w, const double *gy, double *gx, double *gw)
{
    dims_t s; if (get_dims(d, &s)) return;
    double *xh = (double *)malloc(sizeof(double) * 2 * s.B * s.Ci * s.nmode);
    double *gyh = (double *)malloc(sizeof(double) * 2 * s.B * s.Co * s.nmode);
    double *gxh = (double *)malloc(sizeof(double) * 2 * s.B * s.Ci * s.nmode);
    double *wt = inverse_weights(&s);
    oracle_dft_fwd(d, (int)s.Ci, x, NULL, xh);
    oracle_dft_fwd(d, (int)s.Co, gy, wt, gyh);
    oracle_mix_bwd(d, xh, w, gyh, gxh, gw);
    if (gx) oracle_synth(d, (int)s.Ci, gxh, NULL, gx);
    free(xh); free(gyh); free(gxh); free(wt);
}

/* ------------------------------------------------------------------------ */
/* GELU, erf form, and its derivative Phi(u) + u phi(u). */
double oracle_gelu(double u) { return 0.5 * u * (1.0 + erf(u / sqrt(2.0))); }
double oracle_gelu_grad(double u)
{
    return 0.5 * (1.0 + erf(u / sqrt(2.0))) + u * exp(-0.5 * u * u) / sqrt(2.0 * PI_D);
}

/* Pre-activation of the block: z = spectral(x) + W_pw x + b_pw.
 * w_pw is [C_out][C_in]; b_pw (nullable) is [C_out]. */
static void block_preact(const dims_t *s, const int *d, const double *x, const double *w,
                         const double *wpw, const double *bpw, double *z, double *xh_out)
{
    oracle_spectral_fwd(d, x, w, z, xh_out, NULL);
    const long n = s->ncell;
    #pragma omp parallel for collapse(2) schedule(static)
    for (long b = 0; b < s->B; b++)
        for (long o = 0; o < s->Co; o++) {
            double *zo = z + ((size_t)b * s->Co + o) * n;
            for (long p = 0; p < n; p++) {
                double acc = bpw ? bpw[o] : 0.0;
                for (long i = 0; i < s->Ci; i++) acc += wpw[o * s->Ci + i] * x[((size_t)b * s->Ci + i) * n + p];
                zo[p] += acc;
            }
        }
}

/* FNO block (Alg. 1, FNO-block line): y = sigma(spectral(x) + W_pw x + b_pw). */
void oracle_block_fwd(const int *d, const double *x, const double *w, const double *wpw, const double *bpw, double *y)
{
    dims_t s; if (get_dims(d, &s)) return;
    const size_t tot = (size_t)s.B * s.Co * s.ncell;
    block_preact(&s, d, x, w, wpw, bpw, y, NULL);
    #pragma omp parallel for schedule(static)
    for (size_t p = 0; p < tot; p++) y[p] = oracle_gelu(y[p]);
}

/* Backward of the FNO block, by hand: gz = gy * gelu'(z); gb = sum gz;
 * gW_pw[o][i] = sum gz[o] x[i]; gx = W_pw^T gz + spectral adjoint of gz;
 * gw = complex spectral weight gradient.  Outputs are written (not added);
 * any of them may be NULL except gx.                                      */
void oracle_block_bwd(const int *d, const double *x, const double *w, const double *wpw, const double *bpw,
                      const double *gy, double *gx, double *gw, double *gwpw, double *gb)
{
    dims_t s; if (get_dims(d, &s)) return;
    const long n = s.ncell;
    const size_t tot = (size_t)s.B * s.Co * n;
    double *z = (double *)malloc(sizeof(double) * tot);
    block_preact(&s, d, x, w, wpw, bpw, z, NULL);
    #pragma omp parallel for schedule(static)
    for (size_t p = 0; p < tot; p++) z[p] = gy[p] * oracle_gelu_grad(z[p]);   /* z now holds gz */
    if (gb) {
        for (long o = 0; o < s.Co; o++) {
            double acc = 0;
            for (long b = 0; b < s.B; b++) {
                const double *g = z + ((size_t)b * s.Co + o) * n;
                for (long p = 0; p < n; p++) acc += g[p];
            }
            gb[o] = acc;
        }
    }
    if (gwpw) {
        #pragma omp parallel for collapse(2) schedule(static)
        for (long o = 0; o < s.Co; o++)
            for (long i = 0; i < s.Ci; i++) {
                double acc = 0;
                for (long b = 0; b < s.B; b++) {
                    const double *g = z + ((size_t)b * s.Co + o) * n;
                    const double *xi = x + ((size_t)b * s.Ci + i) * n;
                    for (long p = 0; p < n; p++) acc += g[p] * xi[p];
                }
                gwpw[o * s.Ci + i] = acc;
            }
    }
    /* spectral part: gx <- adjoint(gz), gw */
    oracle_spectral_bwd(d, x, w, z, gx, gw);
    /* pointwise part: gx += W_pw^T gz */
    #pragma omp parallel for collapse(2) schedule(static)
    for (long b = 0; b < s.B; b++)
        for (long i = 0; i < s.Ci; i++) {
            double *gxi = gx + ((size_t)b * s.Ci + i) * n;
            for (long p = 0; p < n; p++) {
                double acc = 0;
                for (long o = 0; o < s.Co; o++) acc += wpw[o * s.Ci + i] * z[((size_t)b * s.Co + o) * n + p];
                gxi[p] += acc;
            }
        }
    free(z);
}

/* ------------------------------------------------------------------------ */
/* Network glue of Alg. 1: encoder (lifting), decoder (projection), loss.    */

/* Lifting (Alg. 1, encoder): y[b][o][n] = GELU(sum_i we[o][i] x[b][i][n] + be[o]).
 * we is [Co][Ci], be (nullable) [Co]; N is the number of grid points. */
void oracle_lift_fwd(int B, int Ci, int Co, long N, const double *x, const double *we, const double *be, double *y)
{
    #pragma omp parallel for collapse(2) schedule(static)
    for (long b = 0; b < B; b++)
        for (long o = 0; o < Co; o++)
            for (long p = 0; p < N; p++) {
                double acc = be ? be[o] : 0.0;
                for (long i = 0; i < Ci; i++) acc += we[o * Ci + i] * x[((size_t)b * Ci + i) * N + p];
                y[((size_t)b * Co + o) * N + p] = oracle_gelu(acc);
            }
}

/* Backward of the lifting layer; gx, gwe, gbe nullable (written, not added). */
void oracle_lift_bwd(int B, int Ci, int Co, long N, const double *x, const double *we, const double *be,
                     const double *gy, double *gx, double *gwe, double *gbe)
{
    double *gz = (double *)malloc(sizeof(double) * (size_t)B * Co * N);
    #pragma omp parallel for collapse(2) schedule(static)
    for (long b = 0; b < B; b++)
        for (long o = 0; o < Co; o++)
            for (long p = 0; p < N; p++) {
                double acc = be ? be[o] : 0.0;
                for (long i = 0; i < Ci; i++) acc += we[o * Ci + i] * x[((size_t)b * Ci + i) * N + p];
                gz[((size_t)b * Co + o) * N + p] = gy[((size_t)b * Co + o) * N + p] * oracle_gelu_grad(acc);
            }
    if (gx) {
        #pragma omp parallel for collapse(2) schedule(static)
        for (long b = 0; b < B; b++)
            for (long i = 0; i < Ci; i++)
                for (long p = 0; p < N; p++) {
                    double acc = 0;
                    for (long o = 0; o < Co; o++) acc += we[o * Ci + i] * gz[((size_t)b * Co + o) * N + p];
                    gx[((size_t)b * Ci + i) * N + p] = acc;
                }
    }
    if (gwe) {
        #pragma omp parallel for collapse(2) schedule(static)
        for (long o = 0; o < Co; o++)
            for (long i = 0; i < Ci; i++) {
                double acc = 0;
                for (long b = 0; b < B; b++)
                    for (long p = 0; p < N; p++) acc += gz[((size_t)b * Co + o) * N + p] * x[((size_t)b * Ci + i) * N + p];
                gwe[o * Ci + i] = acc;
            }
    }
    if (gbe) {
        for (long o = 0; o < Co; o++) {
            double acc = 0;
            for (long b = 0; b < B; b++)
                for (long p = 0; p < N; p++) acc += gz[((size_t)b * Co + o) * N + p];
            gbe[o] = acc;
        }
    }
    free(gz);
}

/* Projection (Alg. 1, decoder, two pointwise layers with GELU between them):
 * h = GELU(w1 x + b1) with H hidden channels, y = w2 h + b2.
 * w1 [H][Ci], b1 [H], w2 [Co][H], b2 [Co] (biases nullable). */
void oracle_proj_fwd(int B, int Ci, int H, int Co, long N, const double *x, const double *w1, const double *b1,
                     const double *w2, const double *b2, double *y)
{
    #pragma omp parallel
    {
        double *h = (double *)malloc(sizeof(double) * H);
        #pragma omp for collapse(2) schedule(static)
        for (long b = 0; b < B; b++)
            for (long p = 0; p < N; p++) {
                for (long k = 0; k < H; k++) {
                    double acc = b1 ? b1[k] : 0.0;
                    for (long i = 0; i < Ci; i++) acc += w1[k * Ci + i] * x[((size_t)b * Ci + i) * N + p];
                    h[k] = oracle_gelu(acc);
                }
                for (long o = 0; o < Co; o++) {
                    double acc = b2 ? b2[o] : 0.0;
                    for (long k = 0; k < H; k++) acc += w2[o * H + k] * h[k];
                    y[((size_t)b * Co + o) * N + p] = acc;
                }
            }
        free(h);
    }
}

/* Backward of the projection; every output nullable, written (not added).
 * The points are split into a fixed number of contiguous chunks; each chunk's
 * weight-gradient sums run over its points in order, and the chunk sums are
 * added in chunk order, so the result does not depend on the thread count. */
#define PROJ_CHUNKS 256
void oracle_proj_bwd(int B, int Ci, int H, int Co, long N, const double *x, const double *w1, const double *b1,
                     const double *w2, const double *b2, const double *gy, double *gx, double *gw1, double *gb1,
                     double *gw2, double *gb2)
{
    (void)b2;
    const long np = (long)B * N;
    const long per = (np + PROJ_CHUNKS - 1) / PROJ_CHUNKS;
    const long len = (long)H * Ci + H + (long)Co * H + Co; /* gw1, gb1, gw2, gb2 of one chunk */
    double *part = (double *)calloc((size_t)PROJ_CHUNKS * len, sizeof(double));
    #pragma omp parallel
    {
        double *z = (double *)malloc(sizeof(double) * H), *gh = (double *)malloc(sizeof(double) * H);
        #pragma omp for schedule(dynamic)
        for (long ch = 0; ch < PROJ_CHUNKS; ch++) {
            double *pw1 = part + (size_t)ch * len, *pb1 = pw1 + (size_t)H * Ci, *pw2 = pb1 + H, *pb2 = pw2 + (size_t)Co * H;
            const long end = (ch + 1) * per < np ? (ch + 1) * per : np;
            for (long e = ch * per; e < end; e++) {
                const long b = e / N, p = e % N;
                for (long k = 0; k < H; k++) {
                    double acc = b1 ? b1[k] : 0.0;
                    for (long i = 0; i < Ci; i++) acc += w1[k * Ci + i] * x[((size_t)b * Ci + i) * N + p];
                    z[k] = acc;
                }
                for (long k = 0; k < H; k++) {
                    double g = 0;
                    for (long o = 0; o < Co; o++) g += w2[o * H + k] * gy[((size_t)b * Co + o) * N + p];
                    gh[k] = g * oracle_gelu_grad(z[k]);
                }
                for (long o = 0; o < Co; o++) {
                    const double g = gy[((size_t)b * Co + o) * N + p];
                    pb2[o] += g;
                    for (long k = 0; k < H; k++) pw2[o * H + k] += g * oracle_gelu(z[k]);
                }
                for (long k = 0; k < H; k++) {
                    pb1[k] += gh[k];
                    for (long i = 0; i < Ci; i++) pw1[k * Ci + i] += gh[k] * x[((size_t)b * Ci + i) * N + p];
                }
                if (gx)
                    for (long i = 0; i < Ci; i++) {
                        double acc = 0;
                        for (long k = 0; k < H; k++) acc += w1[k * Ci + i] * gh[k];
                        gx[((size_t)b * Ci + i) * N + p] = acc;
                    }
            }
        }
        free(z);
        free(gh);
    }
    for (long j = 0; j < len; j++) {
        double acc = 0;
        for (long ch = 0; ch < PROJ_CHUNKS; ch++) acc += part[(size_t)ch * len + j];
        double *dst = j < (long)H * Ci ? (gw1 ? gw1 + j : NULL)
                      : j < (long)H * Ci + H ? (gb1 ? gb1 + (j - (long)H * Ci) : NULL)
                      : j < (long)H * Ci + H + (long)Co * H ? (gw2 ? gw2 + (j - (long)H * Ci - H) : NULL)
                      : (gb2 ? gb2 + (j - (long)H * Ci - H - (long)Co * H) : NULL);
        if (dst) *dst = acc;
    }
    free(part);
}

/* Mean-squared-error loss L = (1/n) sum (y - t)^2 and its gradient gy = 2 (y - t)/n (nullable). */
double oracle_mse(long n, const double *y, const double *t, double *gy)
{
    double acc = 0;
    for (long i = 0; i < n; i++) {
        const double d = y[i] - t[i];
        acc += d * d;
        if (gy) gy[i] = 2.0 * d / (double)n;
    }
    return acc / (double)n;
}
