// Pointwise kernels: the Anscombe transform that starts the scheme and the
// closed-form inverse that ends it (eq. 2.3 and eq. 2.4).
#include "fe_internal.h"

namespace fe {
namespace {

// v = 2 sqrt(y + 3/8) (eq. 2.3); the iteration starts from u^0 = u^{-1} = v.
__global__ void anscombe_init_kernel(const float *__restrict__ counts,
                                     float *__restrict__ u0,
                                     float *__restrict__ u1, long n)
{
    const long stride = (long)gridDim.x * blockDim.x;
    for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        const float v = 2.0f * sqrtf(counts[p] + 0.375f);
        u0[p] = v;
        u1[p] = v;
    }
}

// Closed-form unbiased inverse (eq. 2.4):
//   I_C(z) = z^2/4 + sqrt(3/2)/4 z^-1 - 11/8 z^-2 + 5/8 sqrt(3/2) z^-3 - 1/8,
// used for z >= sqrt(3/2) (where it is exactly zero); 0 below.
__device__ __forceinline__ float inverse_anscombe(float z)
{
    const float c = 1.2247448713915890f;  // sqrt(3/2)
    if (!(z >= c)) return 0.0f;
    const float iz = 1.0f / z;
    const float iz2 = iz * iz;
    return 0.25f * z * z + 0.25f * c * iz - 1.375f * iz2
           + 0.625f * c * iz2 * iz - 0.125f;
}

__global__ void inverse_anscombe_kernel(const float *__restrict__ u,
                                        float *__restrict__ out,
                                        float *__restrict__ out_anscombe,
                                        long n)
{
    const long stride = (long)gridDim.x * blockDim.x;
    for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        const float z = u[p];
        if (out) out[p] = inverse_anscombe(z);
        if (out_anscombe) out_anscombe[p] = z;
    }
}

int grid_for(long n)
{
    long b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return (int)b;
}

}  // namespace

hipError_t launch_anscombe_init(const float *counts, float *u0, float *u1,
                                long n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    anscombe_init_kernel<<<grid_for(n), 256, 0, s>>>(counts, u0, u1, n);
    return hipGetLastError();
}

hipError_t launch_inverse_anscombe(const float *u, float *out,
                                   float *out_anscombe, long n, hipStream_t s)
{
    if (n <= 0 || (!out && !out_anscombe)) return hipSuccess;
    inverse_anscombe_kernel<<<grid_for(n), 256, 0, s>>>(u, out, out_anscombe, n);
    return hipGetLastError();
}

}  // namespace fe
