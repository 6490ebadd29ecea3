// api.hip -- host side of the C-ABI declared in include/fno_mi355x.h:
// descriptor validation, plans (device basis tables), workspace and cache
// sizing, argument checks, and the launch sequences of the four entry points.
//
// Launch sequences (Alg. 2 of arXiv 2211.12709, truncation applied as each
// axis is transformed, t first, x last; the inverse runs in reverse order):
//   forward spectrum:  activations -t,z-> T1 -y-> T2 -x-> X^
//   mix:               Y^ = X^ W per retained mode
//   inverse:           Y^ -x-> U2 -y-> U1 -z,t + epilogue-> output
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "fno_internal.h"

namespace fno {

hipError_t generate_tables(const Dims &d, Tables &t, hipStream_t st);
void launch_axis(const float2 *in, float2 *out, const float2 *tab, long long outer, int Nin, int Nout,
                 long long inner, int N, int inverse, hipStream_t st);
void launch_mix_fwd(const float2 *xh, const float2 *w, const unsigned short *wq, const float *wscale, float2 *yh,
                    int B, int Ci, int Co, long long M, hipStream_t st);
void launch_mix_bwd(const float2 *xh, const float2 *w, const unsigned short *wq, const float *wscale,
                    const float2 *gyh, float2 *gxh, float2 *gw, int B, int Ci, int Co, long long M, int accumulate,
                    hipStream_t st);
bool mix_tiled(int B, int Ci, int Co);
size_t packed_weight_bytes(int Ci, int Co, long long M);
size_t packed_scale_offset(int Ci, int Co, long long M);
hipError_t launch_pack_w_fp8(const float2 *w, void *wq, int Ci, int Co, long long M, hipStream_t st);
int pw_wgrad_chunks(long long total);
template <typename T>
void launch_pw_wgrad(const float *gz, const T *x, float *part, float *gwpw, float *gb, int B, int Ci, int Co,
                     long long ncell, int accumulate, hipStream_t st);
template <typename T>
void launch_fwd_tz(const T *in, float2 *out, long long planes, const Dims &d, const Tables &tab, const float *wt,
                   hipStream_t st);
template <typename T>
void launch_inv_zt(int epi, const float2 *u, T *out, int C, const Dims &d, const Tables &tab, const float *wt,
                   const T *x, const float *wpw, const float *bpw, const float *gz, int Cx, int accumulate,
                   hipStream_t st);
template <typename T>
void launch_bwd_gz(const float2 *u, const T *x, const T *gy, float *gz, const Dims &d, const Tables &tab,
                   const float *wpw, const float *bpw, hipStream_t st);
size_t fwd_tz_lds(const Dims &d);
struct TabGeom;
bool tzy_supported(const Dims &d, int dtype);
bool tzy_gen_supported(const Dims &d, int dtype);
template <typename T>
hipError_t launch_tzy_gen(const T *x, float2 *t2, long long slabs, const TzyTabs &tb, const Dims &d, hipStream_t st);
struct ZtTabs {
    const void *z, *z_lo, *t, *t_lo;
};
enum { ZEPI_PLAIN = 0, ZEPI_BLOCK = 1, ZEPI_BWD = 2, ZEPI_ADJ = 3 };
bool zt_supported(const Dims &d, int dtype);
bool zt_t_sliced(const Dims &d);
int zt_grid(const Dims &d);
template <typename T>
hipError_t launch_zt(int epi, const Dims &d, int Cs, int Csrc, const void *u, T *out, const T *src, const T *gy,
                     const float *wpw, const float *bpw, float *part, const ZtTabs &tb, int accumulate, hipStream_t st,
                     int *rows_used = nullptr);
int zt_partial_rows(const Dims &d);
template <typename TC>
hipError_t launch_axis_mfma(const float2 *in, void *out, const void *tab, const void *tab_lo, long long outer,
                            int Nin, int Nout, long long cols, hipStream_t st, bool out16 = false);
size_t axis_lds_bytes(int Ninp, int elem);
TabGeom *new_axis_geom(const Dims &d, int a, bool forward);
void launch_pw_reduce(const float *part, float *gwpw, float *gb, int Ci, int Co, int nchunk, int accumulate,
                      hipStream_t st);
template <typename T>
hipError_t launch_tzy(const T *x, float2 *t2, long long slabs, const TzyTabs &tb, const Dims &d, hipStream_t st);
size_t inv_zt_lds(const Dims &d);

enum { EPI_PLAIN = 0, EPI_BLOCK = 1, EPI_ADJ = 2 };

TabGeom *new_geom(const Dims &d, int dtype);
void free_geom(TabGeom *g);
long long tab_count(int kind, const TabGeom &G);
void gen_frag(int kind, const TabGeom &G, const Tables::Frag &f, hipStream_t st);

static const int kMaxChannels = 64;
static const size_t kMaxLds = 65536;

static size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

// Brackets one kernel launch with events when the plan's timing is enabled.
class KernelTimer {
  public:
    KernelTimer(const fno_plan_t *p, const char *name, hipStream_t st) : p_(p), name_(name), st_(st)
    {
        if (p_->timing.on) {
            start_ = take();
            (void)hipEventRecord(start_, st_);
        }
    }
    ~KernelTimer()
    {
        if (p_->timing.on) {
            hipEvent_t stop = take();
            (void)hipEventRecord(stop, st_);
            p_->timing.recs.push_back({name_, start_, stop});
        }
    }

  private:
    hipEvent_t take()
    {
        auto &pool = p_->timing.pool;
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        (void)hipEventCreate(&e);
        return e;
    }
    const fno_plan_t *p_;
    const char *name_;
    hipStream_t st_;
    hipEvent_t start_ = nullptr;
};

#define FNO_TIMED(p, st, name, call) \
    do {                             \
        KernelTimer _kt(p, name, st); \
        call;                        \
    } while (0)


static int dims_from_desc(const fno_desc_t *s, Dims *d)
{
    if (!s) return FNO_ERR_INVALID_ARG;
    if (s->B < 1 || s->C_in < 1 || s->C_out < 1) return FNO_ERR_INVALID_ARG;
    for (int a = 0; a < 4; a++)
        if (s->grid[a] < 1 || s->modes[a] < 1) return FNO_ERR_INVALID_ARG;
    for (int a = 0; a < 3; a++)
        if (2LL * s->modes[a] > s->grid[a]) return FNO_ERR_INVALID_ARG;
    if (s->modes[3] > s->grid[3] / 2 + 1) return FNO_ERR_INVALID_ARG;
    if (s->dtype != FNO_F32 && s->dtype != FNO_BF16) return FNO_ERR_UNSUPPORTED;
    if (s->flags & ~(uint32_t)FNO_W_FP8) return FNO_ERR_UNSUPPORTED;
    d->B = s->B;
    d->Ci = s->C_in;
    d->Co = s->C_out;
    for (int a = 0; a < 4; a++) {
        d->N[a] = s->grid[a];
        d->m[a] = s->modes[a];
        d->K[a] = a < 3 ? 2 * s->modes[a] : s->modes[a];
    }
    d->ncell = (long long)d->N[0] * d->N[1] * d->N[2] * d->N[3];
    d->nmode = (long long)d->K[0] * d->K[1] * d->K[2] * d->K[3];
    d->plane = (long long)d->N[2] * d->N[3];
    d->kplane = (long long)d->K[2] * d->K[3];
    d->P = (long long)d->K[1] * d->K[2] * d->K[3];
    // limits of this implementation
    if (d->Ci > kMaxChannels || d->Co > kMaxChannels) return FNO_ERR_UNSUPPORTED;
    if (fwd_tz_lds(*d) > kMaxLds || inv_zt_lds(*d) > kMaxLds) return FNO_ERR_UNSUPPORTED;
    if ((long long)d->B * std::max(d->Ci, d->Co) * d->N[0] * d->N[1] > 0x7fffffffLL) return FNO_ERR_UNSUPPORTED;
    // packed weights are read by the tiled mix kernels only
    if ((s->flags & FNO_W_FP8) && !mix_tiled(d->B, d->Ci, d->Co)) return FNO_ERR_UNSUPPORTED;
    return FNO_OK;
}

// Workspace layout (bytes, each part 256-byte aligned).
struct WsPlan {
    size_t t1, t2, sp, sp2, sp3, gz, part, total;
};

static WsPlan ws_plan(const Dims &d, int op)
{
    const long long C = std::max(d.Ci, d.Co);
    WsPlan w{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align_up(bytes); return o; };
    w.t1 = take(sizeof(float2) * (size_t)(d.B * C * d.N[0] * d.N[1] * d.kplane));
    w.t2 = take(sizeof(float2) * (size_t)(d.B * C * d.N[0] * d.P));
    w.sp = take(sizeof(float2) * (size_t)(d.B * C * d.nmode));
    w.sp2 = take(sizeof(float2) * (size_t)(d.B * C * d.nmode));
    w.sp3 = take(sizeof(float2) * (size_t)(d.B * C * d.nmode));
    if (op == FNO_OP_BLOCK_BWD) {
        w.gz = take(sizeof(float) * (size_t)(d.B * d.Co * d.ncell));
        const size_t chunks = std::max<size_t>(pw_wgrad_chunks(d.B * d.ncell), (size_t)zt_partial_rows(d));
        w.part = take(sizeof(float) * chunks * d.Co * (d.Ci + 1));
    }
    w.total = off;
    return w;
}

// Forward cache: the retained spectrum X^ [B Ci][nmode] complex64, then the y-inverse U1 of Y^
// [B Co][Nx][Ny][Kz Kt] as the z,t synthesis reads it (bfloat16 pairs in the bfloat16 plan's
// matrix-core path, complex64 otherwise), so the backward recomputes the pre-activation from it
// without redoing the x and y inverses.
static size_t cache_xh_bytes(const Dims &d) { return align_up(sizeof(float2) * (size_t)(d.B * d.Ci * d.nmode)); }
static size_t cache_u1_elem(const fno_plan_t *p)
{
    return (p->desc.dtype == FNO_BF16 && zt_supported(p->d, FNO_BF16)) ? 4 : sizeof(float2);
}
static size_t cache_bytes(const fno_plan_t *p)
{
    const Dims &d = p->d;
    return cache_xh_bytes(d) + align_up(cache_u1_elem(p) * (size_t)(d.B * d.Co * d.N[0] * d.N[1] * d.kplane));
}

static bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

static int check_plan(const fno_plan_t *plan)
{
    if (!plan) return FNO_ERR_INVALID_ARG;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return FNO_ERR_HIP;
    if (dev != plan->device) return FNO_ERR_INVALID_ARG;
    return FNO_OK;
}

// First launch error of the current entry point on this host thread (launchers
// that return hipError_t report through it; finish() reports and clears it).
static thread_local hipError_t g_launch_err = hipSuccess;
static void note(hipError_t e)
{
    if (e != hipSuccess && g_launch_err == hipSuccess) g_launch_err = e;
}

static int finish()
{
    const hipError_t e = g_launch_err;
    g_launch_err = hipSuccess;
    const hipError_t last = hipGetLastError();
    return (e == hipSuccess && last == hipSuccess) ? FNO_OK : FNO_ERR_HIP;
}

#ifndef FNO_AXIS_X_BF16
#define FNO_AXIS_X_BF16 1  // bfloat16 plans: the x inverse on bfloat16 operands (float results)
#endif

// X^ of activations `in` (C channels) into xh, using t1/t2 as scratch.
// One-axis contraction of complex spectra along axis ax (0 = x, 1 = y) on the
// matrix cores (float operands): in [outer][Nin][cols] -> out [outer][Nout][cols].
// bf16: bfloat16 operands (spectrum rounded once, basis as a hi + lo pair) with float
// accumulation, result stored as bfloat16 (re, im) pairs -- used where the consumer
// rounds it to bfloat16 anyway (the z,t synthesis of the bfloat16 path).  ops16: bfloat16
// operands the same way, float result (the x inverse of the bfloat16 path, whose output the y
// inverse rounds to bfloat16 next; the x forward stays float: no faster on bfloat16 operands and
// it sets the precision of X^ and so of the weight gradient).
static void axis_stage(const fno_plan_t *p, int ax, bool forward, const float2 *in, float2 *out, long long outer,
                       long long cols, hipStream_t st, const char *name, bool bf16 = false, bool ops16 = false)
{
    const Dims &d = p->d;
    const int Nin = forward ? d.N[ax] : d.K[ax], Nout = forward ? d.K[ax] : d.N[ax];
    const Tables::Frag &tb = forward ? p->tab.ax_fwd[ax] : p->tab.ax_inv[ax];
    if ((bf16 || ops16) && axis_lds_bytes((Nin + 15) / 16 * 16, 2) <= 160 * 1024) {
        FNO_TIMED(p, st, name, note(launch_axis_mfma<__bf16>(in, out, tb.hi, tb.lo, outer, Nin, Nout, cols, st, bf16)));
    } else if (axis_lds_bytes((Nin + 15) / 16 * 16, 4) <= 160 * 1024) {
        FNO_TIMED(p, st, name, note(launch_axis_mfma<float>(in, out, tb.f, nullptr, outer, Nin, Nout, cols, st)));
    } else {
        FNO_TIMED(p, st, name, launch_axis(in, out, p->tab.cs[ax], outer, Nin, Nout, cols, d.N[ax], forward ? 0 : 1, st));
    }
}

// The spectral weights as the mix reads them: complex64, or (FNO_W_FP8 plans) the packed e4m3
// words and their per-channel-pair scales.
struct MixW {
    const float2 *w;
    const unsigned short *q;
    const float *scale;
};
static MixW mix_w(const fno_plan_t *p, const void *w)
{
    const Dims &d = p->d;
    if (p->desc.flags & FNO_W_FP8)
        return MixW{nullptr, (const unsigned short *)w,
                    (const float *)((const char *)w + packed_scale_offset(d.Ci, d.Co, d.nmode))};
    return MixW{(const float2 *)w, nullptr, nullptr};
}

template <typename T>
static TzyTabs tzy_tabs(const fno_plan_t *p, const float *wt)
{
    const Tables &tb = p->tab;
    const Tables::Frag &tt = (wt == tb.wt_inv) ? tb.t_bwd : tb.t_fwd;
    TzyTabs r;
    if (sizeof(T) == 2) {
        r = {tt.hi, tt.lo, tb.z_fwd.hi, tb.z_fwd.lo, tb.y_fwd_bf16.hi, tb.y_fwd_bf16.lo};
    } else {
        r = {tt.f, nullptr, tb.z_fwd.f, nullptr, tb.y_fwd_f32.f, nullptr};
    }
    return r;
}

// X^ of activations `in` (C channels) into xh, using t1/t2 as scratch.
// wt selects the t weights: wt_one (forward DFT) or wt_inv (c(kt)/N, adjoint of the real inverse).
template <typename T>
static void forward_spectrum(const fno_plan_t *p, const T *in, int C, const float *wt, float2 *t1, float2 *t2,
                             float2 *xh, hipStream_t st)
{
    const Dims &d = p->d;
    const int dt = sizeof(T) == 2 ? FNO_BF16 : FNO_F32;
    if (tzy_supported(d, dt)) {
        FNO_TIMED(p, st, sizeof(T) == 2 ? "tzy_fwd<bf16>" : "tzy_fwd<f32>",
                  note(launch_tzy<T>(in, t2, (long long)d.B * C * d.N[0], tzy_tabs<T>(p, wt), d, st)));
    } else if (tzy_gen_supported(d, dt)) {
        FNO_TIMED(p, st, sizeof(T) == 2 ? "tzy_gen<bf16>" : "tzy_gen<f32>",
                  note(launch_tzy_gen<T>(in, t2, (long long)d.B * C * d.N[0], tzy_tabs<T>(p, wt), d, st)));
    } else {
        FNO_TIMED(p, st, sizeof(T) == 2 ? "fwd_tz<bf16>" : "fwd_tz<f32>",
                  launch_fwd_tz<T>(in, t1, (long long)d.B * C * d.N[0] * d.N[1], d, p->tab, wt, st));
        axis_stage(p, 1, true, t1, t2, (long long)d.B * C * d.N[0], d.kplane, st, "axis_fwd_y");
    }
    axis_stage(p, 0, true, t2, xh, (long long)d.B * C, d.P, st, "axis_fwd_x");
}

template <typename T>
static ZtTabs zt_tabs(const fno_plan_t *p, bool adjoint)
{
    const Tables &tb = p->tab;
    const Tables::Frag &tt = adjoint ? tb.t_syn_adj : tb.t_syn_inv;
    if (sizeof(T) == 2) return ZtTabs{tb.z_syn.hi, tb.z_syn.lo, tt.hi, tt.lo};
    return ZtTabs{tb.z_syn.f, nullptr, tt.f, nullptr};
}

// Inverse x then y stage of a retained spectrum (C channels): spec -> u2 -> u1.
static void inverse_xy(const fno_plan_t *p, const float2 *spec, int C, float2 *u2, float2 *u1, hipStream_t st)
{
    const Dims &d = p->d;
    axis_stage(p, 0, false, spec, u2, (long long)d.B * C, d.P, st, "axis_inv_x", false,
               FNO_AXIS_X_BF16 && p->desc.dtype == FNO_BF16);
    // the y inverse feeds the z,t synthesis, which rounds it to the activation type
    axis_stage(p, 1, false, u2, u1, (long long)d.B * C * d.N[0], d.kplane, st, "axis_inv_y",
               p->desc.dtype == FNO_BF16 && zt_supported(d, FNO_BF16));
}

template <typename T>
static int spectral_or_block_fwd(const fno_plan_t *p, const void *x_, const void *w_, const void *wpw, const void *bpw,
                                 void *y_, void *cache, void *ws, size_t ws_bytes, void *stream, bool block)
{
    const Dims &d = p->d;
    const int op = block ? FNO_OP_BLOCK_FWD : FNO_OP_SPECTRAL_FWD;
    WsPlan wp = ws_plan(d, op);
    if (!x_ || !w_ || !y_ || !ws || (block && !wpw)) return FNO_ERR_INVALID_ARG;
    if (!aligned16(x_) || !aligned16(w_) || !aligned16(y_) || !aligned16(ws) || (cache && !aligned16(cache)) ||
        (wpw && !aligned16(wpw)) || (bpw && !aligned16(bpw)))
        return FNO_ERR_ALIGNMENT;
    if (ws_bytes < wp.total) return FNO_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    char *wb = (char *)ws;
    float2 *t1 = (float2 *)(wb + wp.t1), *t2 = (float2 *)(wb + wp.t2);
    float2 *xh = cache ? (float2 *)cache : (float2 *)(wb + wp.sp);
    // the y-inverse of Y^ (the z,t synthesis input) goes to the cache when there is one
    float2 *u1 = cache ? (float2 *)((char *)cache + cache_xh_bytes(d)) : t1;
    float2 *yh = (float2 *)(wb + wp.sp2);
    const T *x = (const T *)x_;
    forward_spectrum<T>(p, x, d.Ci, p->tab.wt_one, t1, t2, xh, st);
    const MixW mw = mix_w(p, w_);
    FNO_TIMED(p, st, "mix_fwd", launch_mix_fwd(xh, mw.w, mw.q, mw.scale, yh, d.B, d.Ci, d.Co, d.nmode, st));
    inverse_xy(p, yh, d.Co, t2, u1, st);
    if (zt_supported(d, sizeof(T) == 2 ? FNO_BF16 : FNO_F32)) {
        const bool gen = zt_t_sliced(d);
        FNO_TIMED(p, st, block ? (gen ? "zt_block_tsl" : "zt_block") : (gen ? "zt_plain_tsl" : "zt_plain"),
                  note(launch_zt<T>(block ? ZEPI_BLOCK : ZEPI_PLAIN, d, d.Co, block ? d.Ci : 0, u1, (T *)y_, x,
                                     nullptr, (const float *)wpw, (const float *)bpw, nullptr, zt_tabs<T>(p, false), 0,
                                     st)));
    } else {
        FNO_TIMED(p, st, block ? "inv_zt_block" : "inv_zt_plain",
                  launch_inv_zt<T>(block ? EPI_BLOCK : EPI_PLAIN, u1, (T *)y_, d.Co, d, p->tab, p->tab.wt_inv, x,
                                   (const float *)wpw, (const float *)bpw, nullptr, d.Ci, 0, st));
    }
    return finish();
}

template <typename T>
static int spectral_bwd_impl(const fno_plan_t *p, const void *x_, const void *cache, const void *w_, const void *gy_,
                             void *gx_, void *gw_, int accumulate, void *ws, size_t ws_bytes, void *stream)
{
    const Dims &d = p->d;
    WsPlan wp = ws_plan(d, FNO_OP_SPECTRAL_BWD);
    if (!w_ || !gy_ || !ws) return FNO_ERR_INVALID_ARG;
    if (gw_ && !cache && !x_) return FNO_ERR_INVALID_ARG;
    if (!aligned16(w_) || !aligned16(gy_) || !aligned16(ws) || (x_ && !aligned16(x_)) || (cache && !aligned16(cache)) ||
        (gx_ && !aligned16(gx_)) || (gw_ && !aligned16(gw_)))
        return FNO_ERR_ALIGNMENT;
    if (ws_bytes < wp.total) return FNO_ERR_WORKSPACE;
    if (!gx_ && !gw_) return FNO_OK;
    hipStream_t st = (hipStream_t)stream;
    char *wb = (char *)ws;
    float2 *t1 = (float2 *)(wb + wp.t1), *t2 = (float2 *)(wb + wp.t2);
    float2 *sp = (float2 *)(wb + wp.sp), *gyh = (float2 *)(wb + wp.sp2), *gxh = (float2 *)(wb + wp.sp3);
    const float2 *xh = nullptr;
    if (gw_) {
        if (cache) {
            xh = (const float2 *)cache;
        } else {
            forward_spectrum<T>(p, (const T *)x_, d.Ci, p->tab.wt_one, t1, t2, sp, st);
            xh = sp;
        }
    }
    // adjoint of the real inverse: gY^ = (c(kt)/N) sum_n gy exp(-i theta)
    forward_spectrum<T>(p, (const T *)gy_, d.Co, p->tab.wt_inv, t1, t2, gyh, st);
    FNO_TIMED(p, st, "mix_bwd",
              launch_mix_bwd(xh, mix_w(p, w_).w, mix_w(p, w_).q, mix_w(p, w_).scale, gyh, gx_ ? gxh : nullptr,
                             (float2 *)gw_, d.B, d.Ci, d.Co,
                             d.nmode, accumulate, st));
    if (gx_) {
        inverse_xy(p, gxh, d.Ci, t2, t1, st);
        if (zt_supported(d, sizeof(T) == 2 ? FNO_BF16 : FNO_F32)) {
            FNO_TIMED(p, st, zt_t_sliced(d) ? "zt_adj_tsl" : "zt_adj",
                      note(launch_zt<T>(ZEPI_ADJ, d, d.Ci, 0, t1, (T *)gx_, nullptr, nullptr, nullptr, nullptr,
                                         nullptr, zt_tabs<T>(p, true), accumulate, st)));
        } else {
            FNO_TIMED(p, st, "inv_zt_adj",
                      launch_inv_zt<T>(EPI_ADJ, t1, (T *)gx_, d.Ci, d, p->tab, p->tab.wt_one, nullptr, nullptr,
                                       nullptr, nullptr, d.Co, accumulate, st));
        }
    }
    return finish();
}

template <typename T>
static int block_bwd_impl(const fno_plan_t *p, const void *x_, const void *cache, const void *w_, const void *wpw_,
                          const void *bpw_, const void *gy_, void *gx_, void *gw_, void *gwpw_, void *gb_,
                          int accumulate, void *ws, size_t ws_bytes, void *stream)
{
    const Dims &d = p->d;
    WsPlan wp = ws_plan(d, FNO_OP_BLOCK_BWD);
    if (!x_ || !cache || !w_ || !wpw_ || !gy_ || !gx_ || !ws) return FNO_ERR_INVALID_ARG;
    if (!aligned16(x_) || !aligned16(cache) || !aligned16(w_) || !aligned16(wpw_) || (bpw_ && !aligned16(bpw_)) ||
        !aligned16(gy_) || !aligned16(gx_) || (gw_ && !aligned16(gw_)) || (gwpw_ && !aligned16(gwpw_)) ||
        (gb_ && !aligned16(gb_)) || !aligned16(ws))
        return FNO_ERR_ALIGNMENT;
    if (ws_bytes < wp.total) return FNO_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    char *wb = (char *)ws;
    float2 *t1 = (float2 *)(wb + wp.t1), *t2 = (float2 *)(wb + wp.t2);
    float2 *gyh = (float2 *)(wb + wp.sp2), *gxh = (float2 *)(wb + wp.sp3);
    float *gz = (float *)(wb + wp.gz), *part = (float *)(wb + wp.part);
    const float2 *xh = (const float2 *)cache;
    const float2 *u1 = (const float2 *)((const char *)cache + cache_xh_bytes(d));
    const T *x = (const T *)x_;
    const float *wpw = (const float *)wpw_, *bpw = (const float *)bpw_;
    // recompute the pre-activation from x and the cached y-inverse of Y^, then gz
    if (zt_supported(d, sizeof(T) == 2 ? FNO_BF16 : FNO_F32)) {
        T *gzt = (T *)gz;  // gz stored in the activation type
        int rows_used = zt_partial_rows(d);
        const bool gen = zt_t_sliced(d);
        FNO_TIMED(p, st, gen ? "zt_bwd_tsl" : "zt_bwd",
                  note(launch_zt<T>(ZEPI_BWD, d, d.Co, d.Ci, u1, gzt, x, (const T *)gy_, wpw, bpw, part,
                                     zt_tabs<T>(p, false), 0, st, &rows_used)));
        if (gwpw_ || gb_)
            FNO_TIMED(p, st, "pw_reduce",
                      launch_pw_reduce(part, (float *)gwpw_, (float *)gb_, d.Ci, d.Co, rows_used, accumulate, st));
        forward_spectrum<T>(p, gzt, d.Co, p->tab.wt_inv, t1, t2, gyh, st);
        FNO_TIMED(p, st, "mix_bwd",
                  launch_mix_bwd(xh, mix_w(p, w_).w, mix_w(p, w_).q, mix_w(p, w_).scale, gyh, gxh, (float2 *)gw_, d.B,
                                 d.Ci, d.Co, d.nmode, accumulate,
                                 st));
        inverse_xy(p, gxh, d.Ci, t2, t1, st);
        FNO_TIMED(p, st, gen ? "zt_adj_tsl" : "zt_adj",
                  note(launch_zt<T>(ZEPI_ADJ, d, d.Ci, d.Co, t1, (T *)gx_, gzt, nullptr, wpw, nullptr, nullptr,
                                     zt_tabs<T>(p, true), accumulate, st)));
        return finish();
    }
    FNO_TIMED(p, st, "bwd_gz", launch_bwd_gz<T>(u1, x, (const T *)gy_, gz, d, p->tab, wpw, bpw, st));
    if (gwpw_ || gb_)
        FNO_TIMED(p, st, "pw_wgrad",
                  launch_pw_wgrad<T>(gz, x, part, (float *)gwpw_, (float *)gb_, d.B, d.Ci, d.Co, d.ncell, accumulate,
                                     st));
    // spectral part: gY^ = (c/N) DFT(gz), then the mix gradients and the adjoint
    forward_spectrum<float>(p, gz, d.Co, p->tab.wt_inv, t1, t2, gyh, st);
    FNO_TIMED(p, st, "mix_bwd",
              launch_mix_bwd(xh, mix_w(p, w_).w, mix_w(p, w_).q, mix_w(p, w_).scale, gyh, gxh, (float2 *)gw_, d.B, d.Ci,
                             d.Co, d.nmode, accumulate,
                             st));
    inverse_xy(p, gxh, d.Ci, t2, t1, st);
    FNO_TIMED(p, st, "inv_zt_adj",
              launch_inv_zt<T>(EPI_ADJ, t1, (T *)gx_, d.Ci, d, p->tab, p->tab.wt_one, nullptr, wpw, nullptr, gz, d.Co,
                               accumulate, st));
    return finish();
}

}  // namespace fno

// ---------------------------------------------------------------- network glue
namespace fno {
int glue_blocks();
size_t proj_part_len(int Ci, int H);
int proj_part_chunks();
void launch_sum_rows(const float *part, float *out, int len, size_t stride, int nchunk, int accumulate, hipStream_t st);
template <typename T>
hipError_t launch_lift_fwd(const T *x, T *y, const float *w, const float *b, int B, int Ci, int Co, long long N,
                           hipStream_t st);
template <typename T>
hipError_t launch_lift_bwd(const T *x, const T *gy, const float *w, const float *b, float *part, float *gw, float *gb,
                           int B, int Ci, int Co, long long N, int accumulate, hipStream_t st);
template <typename T>
hipError_t launch_proj(bool bwd, int B, int Ci, int H, int Co, long long N, const T *x, const T *gy, T *y_or_gx,
                       const float *w1, const float *b1, const float *w2, const float *b2, float *part, int accumulate,
                       hipStream_t st, int *nchunk);
template <typename T>
hipError_t launch_mse(const T *y, const T *t, T *gy, float *part, float *loss, long long n, hipStream_t st);

static size_t glue_ws(int Ci, int H, int Co)
{
    const size_t lift = (size_t)glue_blocks() * Co * (Ci + 1) * sizeof(float);
    const size_t proj = (size_t)proj_part_chunks() * proj_part_len(Ci, H) * sizeof(float);
    const size_t mse = (size_t)glue_blocks() * sizeof(float);
    return std::max(std::max(lift, proj), mse);
}
static bool al16(const void *p) { return ((uintptr_t)p & 15u) == 0; }
}  // namespace fno

using namespace fno;

extern "C" {

int fno_desc_validate(const fno_desc_t *desc)
{
    Dims d;
    return dims_from_desc(desc, &d);
}

int fno_plan_create(fno_plan_t **out, const fno_desc_t *desc)
{
    if (!out) return FNO_ERR_INVALID_ARG;
    *out = nullptr;
    Dims d;
    int rc = dims_from_desc(desc, &d);
    if (rc != FNO_OK) return rc;
    fno_plan_t *p = new (std::nothrow) fno_plan_t();
    if (!p) return FNO_ERR_OOM;
    p->desc = *desc;
    p->d = d;
    if (hipGetDevice(&p->device) != hipSuccess) { delete p; return FNO_ERR_HIP; }
    // basis tables: per-axis (cos, sin), inverse weights, and the MFMA fragment tables
    TabGeom *G32 = new_geom(d, FNO_F32), *G16 = new_geom(d, FNO_BF16);
    const long long n_t = tab_count(0, *G32), n_z = tab_count(2, *G32);
    const long long n_y32 = tab_count(3, *G32), n_y16 = tab_count(3, *G16);
    const long long n_zs = tab_count(4, *G32), n_ts = tab_count(5, *G32);
    TabGeom *GA[2][2];
    long long n_ax[2][2];
    for (int ax = 0; ax < 2; ax++)
        for (int f = 0; f < 2; f++) {
            GA[ax][f] = new_axis_geom(d, ax, f == 0);
            n_ax[ax][f] = tab_count(f == 0 ? 7 : 8, *GA[ax][f]);
        }
    size_t off = 0;
    size_t o_cs[4];
    for (int a = 0; a < 4; a++) { o_cs[a] = off; off += align_up(sizeof(float2) * (size_t)d.K[a] * d.N[a]); }
    const size_t o_wi = off; off += align_up(sizeof(float) * d.K[3]);
    const size_t o_wo = off; off += align_up(sizeof(float) * d.K[3]);
    auto frag_bytes = [](long long n) { return align_up(sizeof(float) * n) + 2 * align_up(sizeof(short) * n); };
    const size_t o_tf = off; off += frag_bytes(n_t);
    const size_t o_tb = off; off += frag_bytes(n_t);
    const size_t o_zf = off; off += frag_bytes(n_z);
    const size_t o_y32 = off; off += frag_bytes(n_y32);
    const size_t o_y16 = off; off += frag_bytes(n_y16);
    const size_t o_zs = off; off += frag_bytes(n_zs);
    const size_t o_tsi = off; off += frag_bytes(n_ts);
    const size_t o_tsa = off; off += frag_bytes(n_ts);
    size_t o_ax[2][2];
    for (int ax = 0; ax < 2; ax++)
        for (int f = 0; f < 2; f++) { o_ax[ax][f] = off; off += frag_bytes(n_ax[ax][f]); }
    if (hipMalloc(&p->table_mem, off) != hipSuccess) {
        (void)hipGetLastError();
        free_geom(G32);
        free_geom(G16);
        for (int ax = 0; ax < 2; ax++)
            for (int f = 0; f < 2; f++) free_geom(GA[ax][f]);
        delete p;
        return FNO_ERR_OOM;
    }
    char *base = (char *)p->table_mem;
    for (int a = 0; a < 4; a++) p->tab.cs[a] = (float2 *)(base + o_cs[a]);
    p->tab.wt_inv = (float *)(base + o_wi);
    p->tab.wt_one = (float *)(base + o_wo);
    auto frag_at = [&](size_t o, long long n) {
        Tables::Frag f;
        f.f = (float *)(base + o);
        f.hi = (short *)(base + o + align_up(sizeof(float) * n));
        f.lo = (short *)(base + o + align_up(sizeof(float) * n) + align_up(sizeof(short) * n));
        return f;
    };
    p->tab.t_fwd = frag_at(o_tf, n_t);
    p->tab.t_bwd = frag_at(o_tb, n_t);
    p->tab.z_fwd = frag_at(o_zf, n_z);
    p->tab.y_fwd_f32 = frag_at(o_y32, n_y32);
    p->tab.y_fwd_bf16 = frag_at(o_y16, n_y16);
    p->tab.z_syn = frag_at(o_zs, n_zs);
    p->tab.t_syn_inv = frag_at(o_tsi, n_ts);
    p->tab.t_syn_adj = frag_at(o_tsa, n_ts);
    for (int ax = 0; ax < 2; ax++) {
        p->tab.ax_fwd[ax] = frag_at(o_ax[ax][0], n_ax[ax][0]);
        p->tab.ax_inv[ax] = frag_at(o_ax[ax][1], n_ax[ax][1]);
    }
    hipError_t ge = generate_tables(d, p->tab, nullptr);
    if (ge == hipSuccess) {
        gen_frag(0, *G32, p->tab.t_fwd, nullptr);
        gen_frag(1, *G32, p->tab.t_bwd, nullptr);
        gen_frag(2, *G32, p->tab.z_fwd, nullptr);
        gen_frag(3, *G32, p->tab.y_fwd_f32, nullptr);
        gen_frag(3, *G16, p->tab.y_fwd_bf16, nullptr);
        gen_frag(4, *G32, p->tab.z_syn, nullptr);
        gen_frag(5, *G32, p->tab.t_syn_inv, nullptr);
        gen_frag(6, *G32, p->tab.t_syn_adj, nullptr);
        for (int ax = 0; ax < 2; ax++) {
            gen_frag(7, *GA[ax][0], p->tab.ax_fwd[ax], nullptr);
            gen_frag(8, *GA[ax][1], p->tab.ax_inv[ax], nullptr);
        }
        ge = hipGetLastError();
    }
    free_geom(G32);
    free_geom(G16);
    for (int ax = 0; ax < 2; ax++)
        for (int f = 0; f < 2; f++) free_geom(GA[ax][f]);
    if (ge != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        (void)hipFree(p->table_mem);
        delete p;
        return FNO_ERR_HIP;
    }
    *out = p;
    return FNO_OK;
}

int fno_plan_destroy(fno_plan_t *plan)
{
    if (!plan) return FNO_ERR_INVALID_ARG;
    int rc = FNO_OK;
    for (auto &r : plan->timing.recs) {
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    for (auto e : plan->timing.pool) (void)hipEventDestroy(e);
    if (plan->table_mem && hipFree(plan->table_mem) != hipSuccess) rc = FNO_ERR_HIP;
    delete plan;
    return rc;
}

int fno_workspace_bytes(const fno_plan_t *plan, int op, size_t *out)
{
    if (!plan || !out || op < FNO_OP_SPECTRAL_FWD || op > FNO_OP_BLOCK_BWD) return FNO_ERR_INVALID_ARG;
    *out = ws_plan(plan->d, op).total;
    return FNO_OK;
}

int fno_cache_bytes(const fno_plan_t *plan, size_t *out)
{
    if (!plan || !out) return FNO_ERR_INVALID_ARG;
    *out = cache_bytes(plan);
    return FNO_OK;
}

int fno_packed_weight_bytes(const fno_plan_t *plan, size_t *out)
{
    if (!plan || !out) return FNO_ERR_INVALID_ARG;
    *out = packed_weight_bytes(plan->d.Ci, plan->d.Co, plan->d.nmode);
    return FNO_OK;
}

int fno_pack_weights(const fno_plan_t *plan, const void *w, void *wq, size_t wq_bytes, void *stream)
{
    int rc = check_plan(plan);
    if (rc) return rc;
    if (!w || !wq) return FNO_ERR_INVALID_ARG;
    if (!aligned16(w) || !aligned16(wq)) return FNO_ERR_ALIGNMENT;
    const Dims &d = plan->d;
    if (wq_bytes < packed_weight_bytes(d.Ci, d.Co, d.nmode)) return FNO_ERR_WORKSPACE;
    hipError_t e = hipSuccess;
    FNO_TIMED(plan, (hipStream_t)stream, "pack_w_fp8",
              e = launch_pack_w_fp8((const float2 *)w, wq, d.Ci, d.Co, d.nmode, (hipStream_t)stream));
    return e == hipSuccess ? FNO_OK : FNO_ERR_HIP;
}

int fno_spectral_fwd(const fno_plan_t *plan, const void *x, const void *w, void *y, void *cache, void *ws,
                     size_t ws_bytes, void *stream)
{
    int rc = check_plan(plan);
    if (rc) return rc;
    if (plan->desc.dtype == FNO_BF16)
        return spectral_or_block_fwd<__bf16>(plan, x, w, nullptr, nullptr, y, cache, ws, ws_bytes, stream, false);
    return spectral_or_block_fwd<float>(plan, x, w, nullptr, nullptr, y, cache, ws, ws_bytes, stream, false);
}

int fno_spectral_bwd(const fno_plan_t *plan, const void *x, const void *cache, const void *w, const void *gy, void *gx,
                     void *gw, int accumulate, void *ws, size_t ws_bytes, void *stream)
{
    int rc = check_plan(plan);
    if (rc) return rc;
    if (plan->desc.dtype == FNO_BF16)
        return spectral_bwd_impl<__bf16>(plan, x, cache, w, gy, gx, gw, accumulate, ws, ws_bytes, stream);
    return spectral_bwd_impl<float>(plan, x, cache, w, gy, gx, gw, accumulate, ws, ws_bytes, stream);
}

// ---- the allocation-free variant of fno_spectral_fwd
// Its workspace is a file-scope device array.  In host code the array's name is only a stand-in
// for the symbol: its device address comes from hipGetSymbolAddress, taken once per device (that
// GPU's own copy) and kept in g_scratch_ptr; only that pointer is ever handed to a kernel.
static __device__ __align__(256) char scratch[FNO_NOALLOC_SCRATCH_BYTES];
static const int kMaxDevices = 64;
static void *g_scratch_ptr[kMaxDevices];
static std::mutex g_scratch_mu;

static int scratch_ptr(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices) return FNO_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return FNO_ERR_HIP;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return FNO_OK;
}

int fno_spectral_fwd_noalloc(const fno_plan_t *plan, const void *x, const void *w, void *y, void *cache, void *stream)
{
    int rc = check_plan(plan);
    if (rc) return rc;
    const size_t need = ws_plan(plan->d, FNO_OP_SPECTRAL_FWD).total;
    if (need > (size_t)FNO_NOALLOC_SCRATCH_BYTES) return FNO_ERR_WORKSPACE;
    void *ws = nullptr;
    rc = scratch_ptr(plan->device, &ws);
    if (rc) return rc;
    if (plan->desc.dtype == FNO_BF16)
        return spectral_or_block_fwd<__bf16>(plan, x, w, nullptr, nullptr, y, cache, ws, need, stream, false);
    return spectral_or_block_fwd<float>(plan, x, w, nullptr, nullptr, y, cache, ws, need, stream, false);
}

int fno_block_fwd(const fno_plan_t *plan, const void *x, const void *w, const void *w_pw, const void *b_pw, void *y,
                  void *cache, void *ws, size_t ws_bytes, void *stream)
{
    int rc = check_plan(plan);
    if (rc) return rc;
    if (plan->desc.dtype == FNO_BF16)
        return spectral_or_block_fwd<__bf16>(plan, x, w, w_pw, b_pw, y, cache, ws, ws_bytes, stream, true);
    return spectral_or_block_fwd<float>(plan, x, w, w_pw, b_pw, y, cache, ws, ws_bytes, stream, true);
}

int fno_block_bwd(const fno_plan_t *plan, const void *x, const void *cache, const void *w, const void *w_pw,
                  const void *b_pw, const void *gy, void *gx, void *gw, void *gw_pw, void *gb_pw, int accumulate,
                  void *ws, size_t ws_bytes, void *stream)
{
    int rc = check_plan(plan);
    if (rc) return rc;
    if (plan->desc.dtype == FNO_BF16)
        return block_bwd_impl<__bf16>(plan, x, cache, w, w_pw, b_pw, gy, gx, gw, gw_pw, gb_pw, accumulate, ws,
                                      ws_bytes, stream);
    return block_bwd_impl<float>(plan, x, cache, w, w_pw, b_pw, gy, gx, gw, gw_pw, gb_pw, accumulate, ws, ws_bytes,
                                 stream);
}


int fno_glue_workspace_bytes(int32_t C_in, int32_t H, int32_t C_out, size_t *out)
{
    if (!out || C_in < 1 || H < 1 || C_out < 1) return FNO_ERR_INVALID_ARG;
    *out = glue_ws(C_in, std::max(H, 1), C_out);
    return FNO_OK;
}

int fno_lift_fwd(int32_t dtype, int32_t B, int32_t C_in, int32_t C_out, int64_t N, const void *x, const float *w,
                 const float *b, void *y, void *stream)
{
    if (B < 1 || C_in < 1 || C_out < 1 || N < 1 || !x || !w || !y) return FNO_ERR_INVALID_ARG;
    if (dtype != FNO_F32 && dtype != FNO_BF16) return FNO_ERR_UNSUPPORTED;
    if (C_in > 8 || C_out > 64) return FNO_ERR_UNSUPPORTED;
    if (!al16(x) || !al16(w) || !al16(y) || (b && !al16(b))) return FNO_ERR_ALIGNMENT;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = dtype == FNO_BF16
                       ? launch_lift_fwd<__bf16>((const __bf16 *)x, (__bf16 *)y, w, b, B, C_in, C_out, N, st)
                       : launch_lift_fwd<float>((const float *)x, (float *)y, w, b, B, C_in, C_out, N, st);
    return e == hipSuccess ? FNO_OK : FNO_ERR_HIP;
}

int fno_lift_bwd(int32_t dtype, int32_t B, int32_t C_in, int32_t C_out, int64_t N, const void *x, const float *w,
                 const float *b, const void *gy, float *gw, float *gb, int accumulate, void *ws, size_t ws_bytes,
                 void *stream)
{
    if (B < 1 || C_in < 1 || C_out < 1 || N < 1 || !x || !w || !gy || !ws) return FNO_ERR_INVALID_ARG;
    if (dtype != FNO_F32 && dtype != FNO_BF16) return FNO_ERR_UNSUPPORTED;
    if (C_in > 8 || C_out > 64) return FNO_ERR_UNSUPPORTED;
    if (!al16(x) || !al16(w) || !al16(gy) || !al16(ws) || (b && !al16(b)) || (gw && !al16(gw)) || (gb && !al16(gb)))
        return FNO_ERR_ALIGNMENT;
    if (ws_bytes < glue_ws(C_in, 1, C_out)) return FNO_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = dtype == FNO_BF16
                       ? launch_lift_bwd<__bf16>((const __bf16 *)x, (const __bf16 *)gy, w, b, (float *)ws, gw, gb, B,
                                                 C_in, C_out, N, accumulate, st)
                       : launch_lift_bwd<float>((const float *)x, (const float *)gy, w, b, (float *)ws, gw, gb, B, C_in,
                                                C_out, N, accumulate, st);
    return e == hipSuccess ? FNO_OK : FNO_ERR_HIP;
}

int fno_proj_fwd(int32_t dtype, int32_t B, int32_t C_in, int32_t H, int32_t C_out, int64_t N, const void *x,
                 const float *w1, const float *b1, const float *w2, const float *b2, void *y, void *stream)
{
    if (B < 1 || C_in < 1 || H < 1 || C_out < 1 || N < 1 || !x || !w1 || !w2 || !y) return FNO_ERR_INVALID_ARG;
    if (dtype != FNO_F32 && dtype != FNO_BF16) return FNO_ERR_UNSUPPORTED;
    if (C_in > 32 || H > 128 || C_out != 1 || N > (int64_t)INT32_MAX - 16) return FNO_ERR_UNSUPPORTED;
    if (!al16(x) || !al16(w1) || !al16(w2) || !al16(y) || (b1 && !al16(b1)) || (b2 && !al16(b2)))
        return FNO_ERR_ALIGNMENT;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = dtype == FNO_BF16
                       ? launch_proj<__bf16>(false, B, C_in, H, C_out, N, (const __bf16 *)x, nullptr, (__bf16 *)y, w1,
                                             b1, w2, b2, nullptr, 0, st, nullptr)
                       : launch_proj<float>(false, B, C_in, H, C_out, N, (const float *)x, nullptr, (float *)y, w1, b1,
                                            w2, b2, nullptr, 0, st, nullptr);
    return e == hipSuccess ? FNO_OK : FNO_ERR_HIP;
}

int fno_proj_bwd(int32_t dtype, int32_t B, int32_t C_in, int32_t H, int32_t C_out, int64_t N, const void *x,
                 const float *w1, const float *b1, const float *w2, const float *b2, const void *gy, void *gx,
                 float *gw1, float *gb1, float *gw2, float *gb2, int accumulate, void *ws, size_t ws_bytes,
                 void *stream)
{
    (void)b2;
    if (B < 1 || C_in < 1 || H < 1 || C_out < 1 || N < 1 || !x || !w1 || !w2 || !gy || !gx || !ws)
        return FNO_ERR_INVALID_ARG;
    if (dtype != FNO_F32 && dtype != FNO_BF16) return FNO_ERR_UNSUPPORTED;
    if (C_in > 32 || H > 128 || C_out != 1 || N > (int64_t)INT32_MAX - 16) return FNO_ERR_UNSUPPORTED;
    if (!al16(x) || !al16(w1) || !al16(w2) || !al16(gy) || !al16(gx) || !al16(ws) || (b1 && !al16(b1)) ||
        (gw1 && !al16(gw1)) || (gb1 && !al16(gb1)) || (gw2 && !al16(gw2)) || (gb2 && !al16(gb2)))
        return FNO_ERR_ALIGNMENT;
    if (ws_bytes < glue_ws(C_in, H, C_out)) return FNO_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    float *part = (float *)ws;
    int nchunk = 0;
    hipError_t e = dtype == FNO_BF16
                       ? launch_proj<__bf16>(true, B, C_in, H, C_out, N, (const __bf16 *)x, (const __bf16 *)gy,
                                             (__bf16 *)gx, w1, b1, w2, b2, part, accumulate, st, &nchunk)
                       : launch_proj<float>(true, B, C_in, H, C_out, N, (const float *)x, (const float *)gy,
                                            (float *)gx, w1, b1, w2, b2, part, accumulate, st, &nchunk);
    if (e != hipSuccess) return FNO_ERR_HIP;
    const size_t row = proj_part_len(C_in, H);
    launch_sum_rows(part, gw1, H * C_in, row, nchunk, accumulate, st);
    launch_sum_rows(part + (size_t)H * C_in, gb1, H, row, nchunk, accumulate, st);
    launch_sum_rows(part + (size_t)H * C_in + H, gw2, H, row, nchunk, accumulate, st);
    launch_sum_rows(part + (size_t)H * C_in + 2 * H, gb2, 1, row, nchunk, accumulate, st);
    return hipGetLastError() == hipSuccess ? FNO_OK : FNO_ERR_HIP;
}

int fno_mse(int32_t dtype, int64_t n, const void *y, const void *target, float *loss, void *gy, void *ws,
            size_t ws_bytes, void *stream)
{
    if (n < 1 || !y || !target || !loss || !ws) return FNO_ERR_INVALID_ARG;
    if (dtype != FNO_F32 && dtype != FNO_BF16) return FNO_ERR_UNSUPPORTED;
    if (!al16(y) || !al16(target) || !al16(ws) || (gy && !al16(gy))) return FNO_ERR_ALIGNMENT;
    if (ws_bytes < (size_t)glue_blocks() * sizeof(float)) return FNO_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = dtype == FNO_BF16 ? launch_mse<__bf16>((const __bf16 *)y, (const __bf16 *)target, (__bf16 *)gy,
                                                          (float *)ws, loss, n, st)
                                     : launch_mse<float>((const float *)y, (const float *)target, (float *)gy,
                                                         (float *)ws, loss, n, st);
    return e == hipSuccess ? FNO_OK : FNO_ERR_HIP;
}

int fno_timing_enable(fno_plan_t *plan, int enable)
{
    if (!plan) return FNO_ERR_INVALID_ARG;
    plan->timing.on = enable != 0;
    return FNO_OK;
}

int fno_timing_read(fno_plan_t *plan, char *buf, size_t buf_bytes)
{
    if (!plan || !buf || buf_bytes == 0) return FNO_ERR_INVALID_ARG;
    Timing &t = plan->timing;
    std::vector<std::pair<std::string, std::pair<long, double>>> agg;
    int rc = FNO_OK;
    for (auto &r : t.recs) {
        float ms = 0.f;
        if (hipEventSynchronize(r.stop) != hipSuccess || hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess)
            rc = FNO_ERR_HIP;
        bool found = false;
        for (auto &a : agg)
            if (a.first == r.name) { a.second.first += 1; a.second.second += ms; found = true; break; }
        if (!found) agg.push_back({r.name, {1, (double)ms}});
        t.pool.push_back(r.start);
        t.pool.push_back(r.stop);
    }
    t.recs.clear();
    std::string js = "{";
    for (size_t i = 0; i < agg.size(); i++) {
        char item[256];
        snprintf(item, sizeof item, "%s\"%s\": [%ld, %.6f]", i ? ", " : "", agg[i].first.c_str(), agg[i].second.first,
                 agg[i].second.second);
        js += item;
    }
    js += "}";
    if (js.size() + 1 > buf_bytes) return FNO_ERR_WORKSPACE;
    memcpy(buf, js.c_str(), js.size() + 1);
    return rc;
}

const char *fno_status_str(int status)
{
    switch (status) {
    case FNO_OK: return "FNO_OK";
    case FNO_ERR_INVALID_ARG: return "FNO_ERR_INVALID_ARG: null pointer, bad size or mode count out of range";
    case FNO_ERR_UNSUPPORTED: return "FNO_ERR_UNSUPPORTED: valid request beyond this implementation's limits";
    case FNO_ERR_ALIGNMENT: return "FNO_ERR_ALIGNMENT: tensor pointer not 16-byte aligned";
    case FNO_ERR_WORKSPACE: return "FNO_ERR_WORKSPACE: workspace or cache too small";
    case FNO_ERR_HIP: return "FNO_ERR_HIP: HIP runtime or launch error";
    case FNO_ERR_OOM: return "FNO_ERR_OOM: device allocation failed";
    default: return "unknown fno status";
    }
}

}  // extern "C"
