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

__device__ __forceinline__ int sym1(int i, int n)
{
    if (i < 0) i = -1 - i;
    if (i >= n) i = 2 * n - 1 - i;
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// Binning (Section 4): sums of the non-overlapping 3 x 3 blocks of the
// symmetrically extended image; binned image ceil(H/3) x ceil(W/3).
__global__ void bin3_kernel(const float *__restrict__ y, int H, int W,
                            float *__restrict__ yb, int Hb, int Wb)
{
    const long n = (long)Hb * Wb;
    const long stride = (long)gridDim.x * blockDim.x;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
        const int i = (int)(q / Wb), j = (int)(q - (long)i * Wb);
        float s = 0.0f;
        for (int a = 0; a < 3; ++a) {
            const long row = (long)sym1(3 * i + a, H) * W;
            for (int b = 0; b < 3; ++b) s += y[row + sym1(3 * j + b, W)];
        }
        yb[q] = s;
    }
}

// Bilinear upscaling of xb / 9 (the binned estimate of nine pixels'
// intensity) from the bin centres (3i + 1, 3j + 1) to H x W; constant beyond
// the outermost centres.
__global__ void upsample3_kernel(const float *__restrict__ xb, int Hb, int Wb,
                                 float *__restrict__ x, int H, int W)
{
    const long n = (long)H * W;
    const long stride = (long)gridDim.x * blockDim.x;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
        const int yy = (int)(q / W), xx = (int)(q - (long)yy * W);
        float fy = fminf(fmaxf((yy - 1) / 3.0f, 0.0f), (float)(Hb - 1));
        float fx = fminf(fmaxf((xx - 1) / 3.0f, 0.0f), (float)(Wb - 1));
        const int i0 = min((int)floorf(fy), Hb - 1), j0 = min((int)floorf(fx), Wb - 1);
        const int i1 = min(i0 + 1, Hb - 1), j1 = min(j0 + 1, Wb - 1);
        const float wy = fy - i0, wx = fx - j0;
        const float top = (1.0f - wx) * xb[(long)i0 * Wb + j0] + wx * xb[(long)i0 * Wb + j1];
        const float bot = (1.0f - wx) * xb[(long)i1 * Wb + j0] + wx * xb[(long)i1 * Wb + j1];
        x[q] = ((1.0f - wy) * top + wy * bot) / 9.0f;
    }
}

// Flags (sets *bad = 1) if any count is negative, NaN or infinite.
__global__ void check_counts_kernel(const float *__restrict__ y, long n, int *bad)
{
    const long stride = (long)gridDim.x * blockDim.x;
    bool any = false;
    for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        const float v = y[p];
        any |= !(v >= 0.0f && v <= 3.0e38f);
    }
    if (any) atomicOr(bad, 1);
}

__global__ void zero_ints_kernel(int *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

int grid_for(long n)
{
    long b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return (int)b;
}

}  // namespace

hipError_t launch_check_counts(const float *y, long n, int *bad, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    check_counts_kernel<<<grid_for(n), 256, 0, s>>>(y, n, bad);
    return hipGetLastError();
}

hipError_t launch_zero_ints(int *p, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    zero_ints_kernel<<<(n + 255) / 256, 256, 0, s>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_bin3(const float *y, int H, int W, float *yb, hipStream_t s)
{
    const int Hb = (H + 2) / 3, Wb = (W + 2) / 3;
    bin3_kernel<<<grid_for((long)Hb * Wb), 256, 0, s>>>(y, H, W, yb, Hb, Wb);
    return hipGetLastError();
}

hipError_t launch_upsample3(const float *xb, int Hb, int Wb, float *x, int H, int W,
                            hipStream_t s)
{
    upsample3_kernel<<<grid_for((long)H * W), 256, 0, s>>>(xb, Hb, Wb, x, H, W);
    return hipGetLastError();
}

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
