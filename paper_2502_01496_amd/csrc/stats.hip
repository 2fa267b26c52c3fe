// Momentum diagnostics of the paper (Secs. 5-6): with F_i = m_i a_i,
//   sumF = sum F_i,  sumAbsF = sum |F_i|,  ratio = |sumF| / sumAbsF,
//   M = sum m_i,  x_com = sum m_i x_i / M,  P = sum m_i v_i,  L = sum m_i x_i x v_i.
// FP64 throughout (also for FP32 accelerations).  The grid size depends on n
// only and every reduction runs in a fixed order, so the result is bitwise
// reproducible from run to run.
#include <mutex>

#include "fmm_internal.h"

namespace fmm {

constexpr int ST_THREADS = 256;
constexpr int ST_MAX_BLOCKS = 512;
constexpr int NSTAT = 15;

template <typename TA>
__global__ __launch_bounds__(ST_THREADS) void k_stats_partial(const double *__restrict__ x,
                                                              const double *__restrict__ v,
                                                              const double *__restrict__ m,
                                                              const TA *__restrict__ a, int64_t n,
                                                              double *part)
{
    __shared__ double sh[NSTAT][ST_THREADS];
    double acc[NSTAT];
#pragma unroll
    for (int k = 0; k < NSTAT; ++k)
        acc[k] = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)ST_THREADS + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * ST_THREADS) {
        const double mi = m[i];
        const double a0 = (double)a[3 * i], a1 = (double)a[3 * i + 1], a2 = (double)a[3 * i + 2];
        const double x0 = x[3 * i], x1 = x[3 * i + 1], x2 = x[3 * i + 2];
        acc[0] += mi * a0;
        acc[1] += mi * a1;
        acc[2] += mi * a2;
        acc[3] += mi * sqrt(a0 * a0 + a1 * a1 + a2 * a2);
        acc[4] += mi;
        acc[5] += mi * x0;
        acc[6] += mi * x1;
        acc[7] += mi * x2;
        if (v) {
            const double v0 = v[3 * i], v1 = v[3 * i + 1], v2 = v[3 * i + 2];
            acc[8] += mi * v0;
            acc[9] += mi * v1;
            acc[10] += mi * v2;
            acc[11] += mi * (x1 * v2 - x2 * v1);
            acc[12] += mi * (x2 * v0 - x0 * v2);
            acc[13] += mi * (x0 * v1 - x1 * v0);
        }
    }
#pragma unroll
    for (int k = 0; k < NSTAT; ++k)
        sh[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = ST_THREADS / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
#pragma unroll
            for (int k = 0; k < NSTAT; ++k)
                sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < NSTAT)
        part[blockIdx.x * 16 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(ST_THREADS) void k_stats_final(const double *__restrict__ part, int nb,
                                                            double *out)
{
    __shared__ double sh[NSTAT][ST_THREADS];
    double acc[NSTAT];
#pragma unroll
    for (int k = 0; k < NSTAT; ++k)
        acc[k] = 0.0;
    for (int b = threadIdx.x; b < nb; b += ST_THREADS)
#pragma unroll
        for (int k = 0; k < NSTAT; ++k)
            acc[k] += part[b * 16 + k];
#pragma unroll
    for (int k = 0; k < NSTAT; ++k)
        sh[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = ST_THREADS / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
#pragma unroll
            for (int k = 0; k < NSTAT; ++k)
                sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double F0 = sh[0][0], F1 = sh[1][0], F2 = sh[2][0], Fa = sh[3][0], M = sh[4][0];
        out[0] = F0;
        out[1] = F1;
        out[2] = F2;
        out[3] = Fa;
        out[4] = sqrt(F0 * F0 + F1 * F1 + F2 * F2) / Fa;
        out[5] = M;
        out[6] = sh[5][0] / M;
        out[7] = sh[6][0] / M;
        out[8] = sh[7][0] / M;
        for (int k = 0; k < 6; ++k)
            out[9 + k] = sh[8 + k][0];
        out[15] = 0.0;
    }
}

// Partial sums in red + 16; the 16 results to d_out (device) if given, else
// to red, then copied to h_out with the stream synchronised.  With h_out ==
// nullptr nothing waits.
hipError_t launch_stats(const double *x, const double *v, const double *m, const void *a,
                        int a_fp32, int64_t n, double *red, double *d_out, double *h_out,
                        hipStream_t s)
{
    int nb = (int)std::min<int64_t>((n + ST_THREADS - 1) / ST_THREADS, ST_MAX_BLOCKS);
    double *part = red + 16;
    if (a_fp32)
        k_stats_partial<float><<<nb, ST_THREADS, 0, s>>>(x, v, m, (const float *)a, n, part);
    else
        k_stats_partial<double><<<nb, ST_THREADS, 0, s>>>(x, v, m, (const double *)a, n, part);
    k_stats_final<<<1, ST_THREADS, 0, s>>>(part, nb, d_out ? d_out : red);
    if (!h_out)
        return hipGetLastError();
    hipError_t e = hipMemcpyAsync(h_out, red, 16 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess)
        return e;
    return hipStreamSynchronize(s);
}

// ---------------------------------------------------------------- no-allocation form
// fmm_momentum_stats_noalloc keeps its partial sums in this array instead of
// an allocated buffer: 16 doubles of results after 16 x ST_MAX_BLOCKS
// per-block partials, one copy per device in the library's code object
// (64.1 KiB, held until the process ends).  Every partial the final
// reduction reads is written by the same call first, so nothing needs
// clearing; calls that overlap on one device race for it.
constexpr int NOALLOC_DOUBLES = 16 + 16 * ST_MAX_BLOCKS;
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

// Device address of `scratch` on the current device, looked up once per
// device (the host-side name is only a stand-in for the symbol).
hipError_t stats_noalloc_scratch(double **ptr)
{
    static std::mutex mu;
    static double *addr[64] = {};
    int d = 0;
    hipError_t e = hipGetDevice(&d);
    if (e != hipSuccess)
        return e;
    if (d < 0 || d >= 64)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[d]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        addr[d] = (double *)p;
    }
    *ptr = addr[d];
    return hipSuccess;
}

}  // namespace fmm
