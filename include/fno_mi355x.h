/*
 * fno_mi355x.h -- C-ABI of the MI355X (gfx950) 4-D spectral-convolution FNO
 * block library, libfno_mi355x.so.
 *
 * The operation is the FNO block of arXiv 2211.12709 ("SciAI4Industry"),
 * Sec. IV-C, Alg. 1 (encoder, FNO blocks, decoder) and Alg. 2 (distributed FNO
 * block): a truncated forward real DFT over x, y, z, t, a per-retained-mode
 * complex channel mix (einsum over c_in, elementwise over k), a zero-padded
 * inverse DFT, and, for the block, the pointwise 1x1 channel linear plus bias
 * beside it, inside the activation sigma (GELU, erf form).
 *
 * Definitions (n = (x, y, z, t) grid point, k = (kx, ky, kz, kt) retained mode,
 * theta(k, n) = 2*pi*(kx x/Nx + ky y/Ny + kz z/Nz + kt t/Nt), N = Nx Ny Nz Nt):
 *   retained set K: on x, y, z the m lowest non-negative and the m lowest
 *     negative frequencies (compact index j -> frequency j for j < m and
 *     N_d - 2m + j for j >= m); on t the m_t lowest non-negative bins.
 *   X^[b,i,k]  = sum_n x[b,i,n] exp(-i theta(k,n))                 (Alg. 2, line 1)
 *   Y^[b,o,k]  = sum_i X^[b,i,k] W[i,o,k]                          (Alg. 2, line 2)
 *   S[b,o,n]   = (1/N) sum_k c(kt) Re(Y^[b,o,k] exp(+i theta(k,n))) (Alg. 2, line 3)
 *     with c(0) = 1, c(Nt/2) = 1 for even Nt, c = 2 otherwise (real inverse of
 *     the zero-padded spectrum).
 *   block:  y = GELU(S + W_pw x + b_pw),  GELU(u) = u/2 (1 + erf(u/sqrt 2)) (Alg. 1)
 * Gradients use the convention g = dL/dRe + i dL/dIm for complex tensors.
 *
 * Layouts (all dense, C order, device memory, 16-byte aligned):
 *   x, gx          [B][C_in ][Nx][Ny][Nz][Nt]   activation dtype (desc.dtype)
 *   y, gy          [B][C_out][Nx][Ny][Nz][Nt]   activation dtype
 *   w, gw          [C_in][C_out][2mx][2my][2mz][mt] complex float (re, im interleaved)
 *   w_pw, gw_pw    [C_out][C_in] float
 *   b_pw, gb_pw    [C_out] float
 *   activation dtype: FNO_F32 = float, FNO_BF16 = bfloat16 (round-to-nearest-even)
 *
 * Ownership: the caller allocates and owns every tensor, the workspace and the
 * cache; the library owns only the plan and its device basis tables.  All
 * work is enqueued on `stream` (a hipStream_t, NULL = default stream) without
 * host synchronisation.  No C++ exception crosses this interface.
 *
 * Errors: every entry point returns an fno_status_t.  Argument, alignment and
 * workspace checks happen on the host before anything is launched; a HIP
 * launch error is returned as FNO_ERR_HIP.  Calls on distinct workspaces and
 * caches may run concurrently on different streams with one plan.
 */
#ifndef FNO_MI355X_H
#define FNO_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FNO_OK = 0,
    FNO_ERR_INVALID_ARG = 1, /* null pointer, non-positive size, mode count out of range  */
    FNO_ERR_UNSUPPORTED = 2, /* valid but not implemented (dtype, sizes beyond limits)    */
    FNO_ERR_ALIGNMENT = 3,   /* a tensor pointer not 16-byte aligned                       */
    FNO_ERR_WORKSPACE = 4,   /* ws_bytes smaller than fno_workspace_bytes (or a too small text buffer) */
    FNO_ERR_HIP = 5,         /* HIP runtime or launch error                                */
    FNO_ERR_OOM = 6          /* device allocation failed (plan creation only)              */
} fno_status_t;

enum { FNO_F32 = 0, FNO_BF16 = 1 };

/* Descriptor flags.
 * FNO_W_FP8: the spectral weights `w` taken by fno_spectral_fwd/bwd and fno_block_fwd/bwd are the
 *   packed 8-bit form written by fno_pack_weights (OCP E4M3 values with one power-of-two scale
 *   per (c_in, c_out) pair) instead of complex float; the mode mix (Alg. 2, line 2) reads 2 bytes
 *   per complex weight instead of 8.  Weight gradients stay complex float.  Requires batch <= 8
 *   and a mode tile of the mix that fits in LDS (FNO_ERR_UNSUPPORTED otherwise). */
enum { FNO_W_FP8 = 1u << 0 };

enum {
    FNO_OP_SPECTRAL_FWD = 0,
    FNO_OP_SPECTRAL_BWD = 1,
    FNO_OP_BLOCK_FWD = 2,
    FNO_OP_BLOCK_BWD = 3
};

/* Problem descriptor: the arguments of the layer in Sec. IV-C -- batch,
 * channels, grid (x, y, z, t), retained modes per axis.
 * Requires B, C_in, C_out, grid[d], modes[d] >= 1; 2*modes[d] <= grid[d] for
 * d = x, y, z; modes[3] <= grid[3]/2 + 1.  flags: 0 or FNO_W_FP8. */
typedef struct {
    int32_t B, C_in, C_out;
    int32_t grid[4];  /* Nx, Ny, Nz, Nt */
    int32_t modes[4]; /* mx, my, mz, mt */
    int32_t dtype;    /* FNO_F32 or FNO_BF16: storage/compute type of activations */
    uint32_t flags;
} fno_desc_t;

typedef struct fno_plan fno_plan_t;

/* Host-only check of a descriptor (no HIP call).  FNO_OK or FNO_ERR_INVALID_ARG
 * (or FNO_ERR_UNSUPPORTED for a dtype/flag the library does not provide). */
int fno_desc_validate(const fno_desc_t *desc);

/* Create a plan on the current HIP device: validates `desc`, allocates the
 * basis tables and generates them in FP64 (exact integer phase reduction),
 * rounded once to the kernel types.  Synchronises the device before return.
 * *out is NULL on failure. */
int fno_plan_create(fno_plan_t **out, const fno_desc_t *desc);
int fno_plan_destroy(fno_plan_t *plan);

/* Workspace bytes one call of operation `op` (FNO_OP_*) needs. */
int fno_workspace_bytes(const fno_plan_t *plan, int op, size_t *out);
/* Bytes of the forward cache (the retained spectrum X^ and the y-inverse of Y^,
 * i.e. the input of the z,t synthesis) written by fno_spectral_fwd /
 * fno_block_fwd and read by the backward calls.
 * Precondition of every entry point that takes a non-NULL `cache`: it points to
 * at least this many bytes of device memory.  The entry points take no cache
 * size, so the library cannot check this; a shorter buffer is written or read
 * out of bounds on the device. */
int fno_cache_bytes(const fno_plan_t *plan, size_t *out);

/* Bytes of the packed 8-bit form of a plan's spectral weights:
 * [C_in][C_out][2mx][2my][2mz][mt] 16-bit words (low byte the real part, high byte the imaginary
 * part, each an OCP E4M3 value), then, at the next 256-byte boundary, [C_in][C_out] float scales,
 * then scratch that fno_pack_weights uses for its per-chunk sums. */
int fno_packed_weight_bytes(const fno_plan_t *plan, size_t *out);
/* Packs complex float weights w ([C_in][C_out][modes], as for the other entry points) into wq:
 * for every (c_in, c_out) pair, s = 2^round(log2 RMS) over the real and imaginary parts of its
 * weights, and each part stored as the E4M3 value nearest to part / s (ties to even, magnitudes
 * above 448 saturating).  Enqueued on `stream`; FNO_ERR_WORKSPACE if wq_bytes is smaller than
 * fno_packed_weight_bytes.  Any plan can pack; FNO_W_FP8 plans consume the result. */
int fno_pack_weights(const fno_plan_t *plan, const void *w, void *wq, size_t wq_bytes, void *stream);

/* Spectral convolution layer (Alg. 2): y = S(x; w).  cache (nullable)
 * receives what the backward needs. */
int fno_spectral_fwd(const fno_plan_t *plan, const void *x, const void *w, void *y,
                     void *cache, void *ws, size_t ws_bytes, void *stream);

/* Backward of the spectral layer: gx = adjoint of x -> y applied to gy
 * (nullable: skipped); gw = sum_b conj(X^) * (c(kt)/N) DFT(gy)  (nullable:
 * skipped).  gw needs the spectrum of x: from `cache` if non-NULL (as written
 * by fno_spectral_fwd with the same x), else recomputed from `x`.
 * accumulate != 0 adds into gx / gw instead of overwriting. */
int fno_spectral_bwd(const fno_plan_t *plan, const void *x, const void *cache, const void *w,
                     const void *gy, void *gx, void *gw, int accumulate,
                     void *ws, size_t ws_bytes, void *stream);

/* Allocation-free variant of fno_spectral_fwd, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same operation, arguments and layouts as
 * fno_spectral_fwd, without the workspace: the intermediates live in a static
 * device array of FNO_NOALLOC_SCRATCH_BYTES that the library holds on every
 * GPU it runs on until the process ends.  Returns FNO_ERR_WORKSPACE, before
 * anything is launched, when the plan's spectral-forward workspace
 * (fno_workspace_bytes(plan, FNO_OP_SPECTRAL_FWD)) exceeds that size.  The
 * array needs no clearing between calls (every call writes each intermediate
 * before reading it).  All calls on one GPU share the array: calls that
 * overlap on one GPU (other streams, other host threads) race and must be
 * serialised by the caller.  Calls no allocating routine. */
#define FNO_NOALLOC_SCRATCH_BYTES (32u << 20)
int fno_spectral_fwd_noalloc(const fno_plan_t *plan, const void *x, const void *w, void *y, void *cache, void *stream);

/* FNO block (Alg. 1, block line): y = GELU(S(x; w) + w_pw x + b_pw).
 * b_pw may be NULL (no bias).  cache (nullable) receives what fno_block_bwd
 * needs to recompute the pre-activation (the full-size pre-activation itself
 * is never stored). */
int fno_block_fwd(const fno_plan_t *plan, const void *x, const void *w, const void *w_pw,
                  const void *b_pw, void *y, void *cache, void *ws, size_t ws_bytes, void *stream);

/* Backward of the FNO block with recomputation of the pre-activation from x
 * and `cache` (required, written by fno_block_fwd with the same x, w).
 * Outputs gx (required), gw, gw_pw, gb_pw (each nullable).  accumulate != 0
 * adds into every output instead of overwriting. */
int fno_block_bwd(const fno_plan_t *plan, const void *x, const void *cache, const void *w,
                  const void *w_pw, const void *b_pw, const void *gy, void *gx, void *gw,
                  void *gw_pw, void *gb_pw, int accumulate, void *ws, size_t ws_bytes, void *stream);

/* ---- Network glue of Alg. 1 (encoder, decoder, loss).  These act pointwise
 * on the grid, so they take the number of grid points N instead of a plan.
 * Activations are [B][C][N] in `dtype` (FNO_F32 / FNO_BF16), weights float,
 * all device pointers 16-byte aligned; work is enqueued on `stream`.
 * Weight gradients are deterministic (fixed-order two-stage sums). */

/* Encoder (Alg. 1, lifting): y = GELU(w x + b), w [C_out][C_in], b [C_out]
 * (nullable).  Limits: C_in <= 8, C_out <= 64. */
int fno_lift_fwd(int32_t dtype, int32_t B, int32_t C_in, int32_t C_out, int64_t N, const void *x, const float *w,
                 const float *b, void *y, void *stream);
/* Weight gradients of the encoder: gw [C_out][C_in], gb [C_out] (each nullable);
 * no input gradient (the encoder's input is data).  accumulate != 0 adds. */
int fno_lift_bwd(int32_t dtype, int32_t B, int32_t C_in, int32_t C_out, int64_t N, const void *x, const float *w,
                 const float *b, const void *gy, float *gw, float *gb, int accumulate, void *ws, size_t ws_bytes,
                 void *stream);
/* Decoder (Alg. 1, two pointwise layers): y = w2 GELU(w1 x + b1) + b2 with
 * H hidden channels that are never stored; w1 [H][C_in], b1 [H], w2 [C_out][H],
 * b2 [C_out] (biases nullable).  Limits: C_in <= 32, H <= 128, C_out == 1,
 * N < 2^31 - 16 (FNO_ERR_UNSUPPORTED otherwise). */
int fno_proj_fwd(int32_t dtype, int32_t B, int32_t C_in, int32_t H, int32_t C_out, int64_t N, const void *x,
                 const float *w1, const float *b1, const float *w2, const float *b2, void *y, void *stream);
/* Backward of the decoder: gx (required) and gw1, gb1, gw2, gb2 (nullable).
 * accumulate != 0 adds into every output. */
int fno_proj_bwd(int32_t dtype, int32_t B, int32_t C_in, int32_t H, int32_t C_out, int64_t N, const void *x,
                 const float *w1, const float *b1, const float *w2, const float *b2, const void *gy, void *gx,
                 float *gw1, float *gb1, float *gw2, float *gb2, int accumulate, void *ws, size_t ws_bytes,
                 void *stream);
/* Mean-squared error over n elements: *loss (device float) = mean((y - t)^2),
 * gy (nullable) = 2 (y - t) / n. */
int fno_mse(int32_t dtype, int64_t n, const void *y, const void *target, float *loss, void *gy, void *ws,
            size_t ws_bytes, void *stream);
/* Workspace bytes that fno_lift_bwd, fno_proj_bwd and fno_mse need (the
 * largest of the three for these channel counts). */
int fno_glue_workspace_bytes(int32_t C_in, int32_t H, int32_t C_out, size_t *out);

/* Per-kernel timing (diagnostic, for benchmarks and profiles).  While enabled
 * on a plan, every kernel the plan launches is bracketed by two HIP events
 * recorded on the launch stream.  fno_timing_read waits for the recorded
 * events, writes a NUL-terminated JSON object {"kernel": [launches, total_ms],
 * ...} into buf (FNO_ERR_WORKSPACE if buf_bytes is too small) and clears the
 * records.  Not thread-safe: enable it only where one thread drives the plan. */
int fno_timing_enable(fno_plan_t *plan, int enable);
int fno_timing_read(fno_plan_t *plan, char *buf, size_t buf_bytes);

/* Static description of a status code. */
const char *fno_status_str(int status);

#ifdef __cplusplus
}
#endif
#endif /* FNO_MI355X_H */
