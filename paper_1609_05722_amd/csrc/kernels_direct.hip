// Direct filter-bank kernels: one thread per pixel, no matrix cores.
//
// These compute the prior's gradient of eq. 3.2 in two passes through HBM:
// the forward pass writes psi_i = alpha_i rho'(K_i u) for every filter, the
// adjoint pass gathers sum_i K_i^T psi_i per pixel.  They serve the energy
// and gradient entry point (which also needs the Student-t energy of
// eq. 2.5/2.6) and any filter shape the fused matrix-core step is not built
// for.
#include "fe_internal.h"
#include "fe_math.h"

namespace fe {
namespace {

constexpr int kBX = 16, kBY = 16;

// Operand rounding of the contractions: FE_PREC_FP32 keeps the value,
// FE_PREC_BF16 / FE_PREC_FP16 round it to nearest even in that format (the
// products are then accumulated in FP32).
template <int PREC>
__device__ __forceinline__ float operand(float x)
{
    if constexpr (PREC == 1) return (float)(__bf16)x;
    else if constexpr (PREC == 2) return (float)(_Float16)x;
    else return x;
}

// Half-sample symmetric index (u(-1-i) = u(i), u(n+i) = u(n-1-i)), one
// reflection, then clamped so that even an unused far ghost stays in bounds.
__device__ __forceinline__ int sym(int i, int n)
{
    if (i < 0) i = -1 - i;
    if (i >= n) i = 2 * n - 1 - i;
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

__device__ float block_sum(float v, float *red)
{
    const int t = threadIdx.y * kBX + threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int w = kBX * kBY / 2; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    const float r = red[0];
    __syncthreads();
    return r;
}

template <int M, int PREC>
__global__ __launch_bounds__(kBX * kBY)
void forward_kernel(const float *__restrict__ taps,
                    const float *__restrict__ alpha2,
                    const float *__restrict__ alpha, int nf,
                    const float *__restrict__ u, int H, int W,
                    float *__restrict__ psi, float *__restrict__ rho_partial,
                    float *__restrict__ data_partial,
                    const float *__restrict__ counts, float lambda,
                    int data_term)
{
    constexpr int R = (M - 1) / 2;
    __shared__ float red[kBX * kBY];
    const int x = blockIdx.x * kBX + threadIdx.x;
    const int y = blockIdx.y * kBY + threadIdx.y;
    const bool in = (x < W) && (y < H);
    float e[M * M];
    if (in) {
#pragma unroll
        for (int a = 0; a < M; ++a) {
            const int yy = sym(y + a - R, H);
#pragma unroll
            for (int b = 0; b < M; ++b)
                e[a * M + b] = operand<PREC>(u[(long)yy * W + sym(x + b - R, W)]);
        }
    }
    float rho_acc = 0.0f;
    const long plane = (long)H * W;
    for (int i = 0; i < nf; ++i) {
        if (!in) break;
        const float *k = taps + i * M * M;
        float z = 0.0f;
#pragma unroll
        for (int t = 0; t < M * M; ++t) z = fmaf(operand<PREC>(k[t]), e[t], z);
        psi[i * plane + (long)y * W + x] = influence(z, alpha2[i]);
        if (rho_partial) rho_acc += alpha[i] * log1pf(z * z);
    }
    if (rho_partial) {
        const int blk = blockIdx.y * gridDim.x + blockIdx.x;
        const float s = block_sum(rho_acc, red);
        float d = 0.0f;
        if (in && counts) {
            const float uc = u[(long)y * W + x];
            d = data_energy(uc, anscombe(counts[(long)y * W + x]), data_term);
        }
        const float sd = block_sum(d, red);
        if (threadIdx.x == 0 && threadIdx.y == 0) {
            rho_partial[blk] = s;
            data_partial[blk] = lambda * sd;
        }
    }
}

// sum_i K_i^T psi_i at pixel (y, x): the transpose of "extend, then
// correlate".  The extended position s = (sy, sx) receives
//   G(s) = sum_i sum_{a,b} k_i[a][b] psi_i(sy - a + R, sx - b + R)
// (psi = 0 outside the image), and every extended position mirroring
// (y, x) adds onto it: the pixel itself, plus the ghost row -1-y (y < R) or
// 2H-1-y (y >= H-R), likewise for columns.
template <int M, int PREC>
__device__ float adjoint_at(const float *__restrict__ taps, int nf,
                            const float *__restrict__ psi, int H, int W,
                            int y, int x)
{
    constexpr int R = (M - 1) / 2;
    int rows[3], cols[3];
    int nr = 0, nc = 0;
    if (y < R) rows[nr++] = -1 - y;
    rows[nr++] = y;
    if (y >= H - R) rows[nr++] = 2 * H - 1 - y;
    if (x < R) cols[nc++] = -1 - x;
    cols[nc++] = x;
    if (x >= W - R) cols[nc++] = 2 * W - 1 - x;
    const long plane = (long)H * W;
    float g = 0.0f;
    for (int ir = 0; ir < nr; ++ir) {
        for (int ic = 0; ic < nc; ++ic) {
            const int sy = rows[ir], sx = cols[ic];
            float acc = 0.0f;
            for (int i = 0; i < nf; ++i) {
                const float *k = taps + i * M * M;
                const float *p = psi + i * plane;
#pragma unroll
                for (int a = 0; a < M; ++a) {
                    const int qy = sy - a + R;
                    if (qy < 0 || qy >= H) continue;
#pragma unroll
                    for (int b = 0; b < M; ++b) {
                        const int qx = sx - b + R;
                        if (qx < 0 || qx >= W) continue;
                        acc = fmaf(operand<PREC>(k[a * M + b]),
                                   operand<PREC>(p[(long)qy * W + qx]), acc);
                    }
                }
            }
            g += acc;
        }
    }
    return g;
}

template <int M>
__global__ __launch_bounds__(kBX * kBY)
void adjoint_step_kernel(const float *__restrict__ taps, int nf,
                         const float *__restrict__ psi,
                         const float *__restrict__ u,
                         const float *u_prev, const float *__restrict__ counts,
                         float *u_next, int H, int W, StepParams prm)
{
    const int x = blockIdx.x * kBX + threadIdx.x;
    const int y = blockIdx.y * kBY + threadIdx.y;
    if (x >= W || y >= H) return;
    const long p = (long)y * W + x;
    const float g = adjoint_at<M, 0>(taps, nf, psi, H, W, y, x);
    const float uc = u[p];
    const float ut = inertial_step(uc, u_prev[p], g, prm.tau, prm.gamma);
    u_next[p] = prox(ut, anscombe(counts[p]), prm.tau_lambda, prm.data_term);
}

template <int M, int PREC>
__global__ __launch_bounds__(kBX * kBY)
void adjoint_grad_kernel(const float *__restrict__ taps, int nf,
                         const float *__restrict__ psi,
                         const float *__restrict__ u,
                         const float *__restrict__ counts,
                         float *__restrict__ grad, int H, int W, float lambda,
                         int data_term)
{
    const int x = blockIdx.x * kBX + threadIdx.x;
    const int y = blockIdx.y * kBY + threadIdx.y;
    if (x >= W || y >= H) return;
    const long p = (long)y * W + x;
    const float g = adjoint_at<M, PREC>(taps, nf, psi, H, W, y, x);
    grad[p] = g + lambda * data_gradient(u[p], anscombe(counts[p]), data_term);
}

dim3 grid2d(int H, int W) { return dim3((W + kBX - 1) / kBX, (H + kBY - 1) / kBY); }

}  // namespace

int direct_forward_blocks(int H, int W)
{
    const dim3 g = grid2d(H, W);
    return (int)(g.x * g.y);
}

#define FE_DISPATCH_M(m, CALL) \
    switch (m) {               \
    case 3: CALL(3); break;    \
    case 5: CALL(5); break;    \
    case 7: CALL(7); break;    \
    default: return hipErrorInvalidValue; }

#define FE_DISPATCH_MP(m, prec, CALL)                                        \
    switch ((m) * 10 + (prec)) {                                             \
    case 30: CALL(3, 0); break;                                              \
    case 31: CALL(3, 1); break;                                              \
    case 32: CALL(3, 2); break;                                              \
    case 50: CALL(5, 0); break;                                              \
    case 51: CALL(5, 1); break;                                              \
    case 52: CALL(5, 2); break;                                              \
    case 70: CALL(7, 0); break;                                              \
    case 71: CALL(7, 1); break;                                              \
    case 72: CALL(7, 2); break;                                              \
    default: return hipErrorInvalidValue; }

hipError_t launch_direct_forward(const DeviceBank &bank, const float *u,
                                 int H, int W, float *psi,
                                 float *rho_partial, float *data_partial,
                                 const float *counts, float lambda,
                                 int data_term, int precision, int *n_blocks,
                                 hipStream_t s)
{
    const dim3 g = grid2d(H, W), b(kBX, kBY);
    if (n_blocks) *n_blocks = (int)(g.x * g.y);
#define FE_CALL(MM, PP)                                                      \
    forward_kernel<MM, PP><<<g, b, 0, s>>>(bank.taps, bank.alpha2, bank.alpha, \
                                           bank.nf, u, H, W, psi, rho_partial, \
                                           data_partial, counts, lambda, data_term)
    FE_DISPATCH_MP(bank.m, precision, FE_CALL)
#undef FE_CALL
    return hipGetLastError();
}

hipError_t launch_direct_adjoint_step(const DeviceBank &bank, const float *psi,
                                      const float *u, const float *u_prev,
                                      const float *counts, float *u_next,
                                      int H, int W, StepParams p,
                                      hipStream_t s)
{
    const dim3 g = grid2d(H, W), b(kBX, kBY);
#define FE_CALL(MM)                                                          \
    adjoint_step_kernel<MM><<<g, b, 0, s>>>(bank.taps, bank.nf, psi, u,       \
                                            u_prev, counts, u_next, H, W, p)
    FE_DISPATCH_M(bank.m, FE_CALL)
#undef FE_CALL
    return hipGetLastError();
}

hipError_t launch_direct_adjoint_grad(const DeviceBank &bank, const float *psi,
                                      const float *u, const float *counts,
                                      float *grad, int H, int W, float lambda,
                                      int data_term, int precision, hipStream_t s)
{
    const dim3 g = grid2d(H, W), b(kBX, kBY);
#define FE_CALL(MM, PP)                                                      \
    adjoint_grad_kernel<MM, PP><<<g, b, 0, s>>>(bank.taps, bank.nf, psi, u,   \
                                                counts, grad, H, W, lambda,   \
                                                data_term)
    FE_DISPATCH_MP(bank.m, precision, FE_CALL)
#undef FE_CALL
    return hipGetLastError();
}

}  // namespace fe
