// Leapfrog update used by the kick-drift-kick integration of the workloads:
// v += kick * a, then x += drift * v (FP64 state; a may be FP32).
#include "fmm_internal.h"

namespace fmm {

template <typename TA>
__global__ void k_kick_drift(double *__restrict__ x, double *__restrict__ v,
                             const TA *__restrict__ a, int64_t n3, double kick, double drift)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n3;
         i += (int64_t)gridDim.x * blockDim.x) {
        double vi = v[i] + kick * (double)a[i];
        v[i] = vi;
        x[i] = x[i] + drift * vi;
    }
}

hipError_t launch_kick_drift(double *x, double *v, const void *a, int a_fp32, int64_t n,
                             double kick, double drift, hipStream_t s)
{
    int64_t n3 = 3 * n;
    int gs = (int)std::min<int64_t>((n3 + 255) / 256, 8192);
    if (a_fp32)
        k_kick_drift<float><<<gs, 256, 0, s>>>(x, v, (const float *)a, n3, kick, drift);
    else
        k_kick_drift<double><<<gs, 256, 0, s>>>(x, v, (const double *)a, n3, kick, drift);
    return hipGetLastError();
}

}  // namespace fmm
