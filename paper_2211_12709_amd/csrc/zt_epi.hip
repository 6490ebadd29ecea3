// zt_epi.hip -- host side of the z,t synthesis epilogue kernels declared in
// zt_epi.h: which shapes they take, the persistent grid size, and the launch
// of the variant an epilogue needs (the variants are compiled per epilogue in
// zt_epi_plain.hip, zt_epi_block.hip, zt_epi_bwd.hip and zt_epi_adj.hip).
#include "zt_epi.h"

namespace fno {

FNO_ZT_EXTERN(ZEPI_PLAIN)
FNO_ZT_EXTERN(ZEPI_BLOCK)
FNO_ZT_EXTERN(ZEPI_BWD)
FNO_ZT_EXTERN(ZEPI_ADJ)
FNO_ZT_EXTERN(ZEPI_ADJ_ACC)

bool zt_supported(const Dims &d, int dtype)
{
    if (d.K[3] > 16) return false;
    if (d.Ci > 64 || d.Co > 64) return false;
    const int elem = dtype == FNO_BF16 ? 2 : 4;
    // every (output, source) channel pair the entry points use
    return zt_pair_ok(d, d.Co, 0, elem) && zt_pair_ok(d, d.Co, d.Ci, elem) && zt_pair_ok(d, d.Ci, d.Co, elem) &&
           zt_pair_ok(d, d.Ci, 0, elem);
}

bool zt_t_sliced(const Dims &d) { return zt_is_gen(d); }

int zt_grid(const Dims &d) { return (int)std::min<long long>((long long)d.B * d.N[0] * d.N[1], 2048); }
int zt_partial_rows(const Dims &d) { return zt_grid(d); }

// epi: ZEPI_*; Cs = output/spectral channels, Csrc = pointwise source channels.
// u: the y-inverse spectrum [B Cs][Nx][Ny][Kz Kt] of CplxOf<T> elements (bfloat16 pairs for T = bf16).
// rows_used (nullable) receives the number of BWD partial-sum rows written.
template <typename T>
hipError_t launch_zt(int epi, const Dims &d, int Cs, int Csrc, const void *u, T *out, const T *src, const T *gy,
                     const float *wpw, const float *bpw, float *part, const ZtTabs &tb, int accumulate, hipStream_t st,
                     int *rows_used)
{
    if (epi == ZEPI_ADJ && accumulate) epi = ZEPI_ADJ_ACC;
    switch (epi) {
    case ZEPI_PLAIN:
        return launch_zt_epi<ZEPI_PLAIN, T>(d, Cs, Csrc, u, out, src, gy, wpw, bpw, part, tb, accumulate, st, rows_used);
    case ZEPI_BLOCK:
        return launch_zt_epi<ZEPI_BLOCK, T>(d, Cs, Csrc, u, out, src, gy, wpw, bpw, part, tb, accumulate, st, rows_used);
    case ZEPI_BWD:
        return launch_zt_epi<ZEPI_BWD, T>(d, Cs, Csrc, u, out, src, gy, wpw, bpw, part, tb, accumulate, st, rows_used);
    case ZEPI_ADJ:
        return launch_zt_epi<ZEPI_ADJ, T>(d, Cs, Csrc, u, out, src, gy, wpw, bpw, part, tb, accumulate, st, rows_used);
    default:
        return launch_zt_epi<ZEPI_ADJ_ACC, T>(d, Cs, Csrc, u, out, src, gy, wpw, bpw, part, tb, accumulate, st,
                                              rows_used);
    }
}

template hipError_t launch_zt<float>(int, const Dims &, int, int, const void *, float *, const float *,
                                     const float *, const float *, const float *, float *, const ZtTabs &, int,
                                     hipStream_t, int *);
template hipError_t launch_zt<__bf16>(int, const Dims &, int, int, const void *, __bf16 *, const __bf16 *,
                                      const __bf16 *, const float *, const float *, float *, const ZtTabs &, int,
                                      hipStream_t, int *);

}  // namespace fno
