// basis.hip -- generation of the Fourier basis tables of a plan.
//
// The retained frequencies follow the truncation S of Alg. 2 (Sec. IV-C): on
// x, y, z the compact index j < m is frequency j and j >= m is N - 2m + j
// (the m lowest negative frequencies); on t it is j itself.  Every entry is
// computed in FP64 on the GPU with the product k*n reduced modulo N exactly in
// 64-bit integers, then rounded once to float.
#include "fno_internal.h"

namespace fno {

__global__ void k_basis_cs(float2 *__restrict__ out, int N, int K, int m, int is_t)
{
    long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)K * N) return;
    const int j = (int)(e / N), n = (int)(e % N);
    const long long k = is_t ? j : (j < m ? j : (long long)N - 2 * m + j);
    const long long r = (k * (long long)n) % N;
    const double th = 6.283185307179586476925286766559 * (double)r / (double)N;
    double s, c;
    sincos(th, &s, &c);
    out[e] = make_float2((float)c, (float)s);
}

__global__ void k_basis_wt(float *__restrict__ wt_inv, float *__restrict__ wt_one, int Kt, int Nt, double inv_ncell)
{
    int kt = blockIdx.x * blockDim.x + threadIdx.x;
    if (kt >= Kt) return;
    // real-output weight c(kt): 1 for the zero bin and the Nyquist bin of an even Nt, else 2
    double c = (kt == 0 || (Nt % 2 == 0 && 2 * kt == Nt)) ? 1.0 : 2.0;
    wt_inv[kt] = (float)(c * inv_ncell);
    wt_one[kt] = 1.0f;
}

hipError_t generate_tables(const Dims &d, Tables &t, hipStream_t st)
{
    for (int a = 0; a < 4; a++) {
        long long tot = (long long)d.K[a] * d.N[a];
        int blocks = (int)((tot + 255) / 256);
        hipLaunchKernelGGL(k_basis_cs, dim3(blocks), dim3(256), 0, st, t.cs[a], d.N[a], d.K[a], d.m[a], a == 3 ? 1 : 0);
    }
    hipLaunchKernelGGL(k_basis_wt, dim3((d.K[3] + 63) / 64), dim3(64), 0, st, t.wt_inv, t.wt_one, d.K[3], d.N[3],
                       1.0 / (double)d.ncell);
    return hipGetLastError();
}

}  // namespace fno
