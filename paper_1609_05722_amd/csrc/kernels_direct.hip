// Direct filter-bank kernels of the energy and gradient entry point: one
// thread per pixel, no matrix cores.
//
// The prior's gradient (eq. 3.2) takes two passes through HBM: the forward
// pass writes psi_i = alpha_i rho'(K_i u) for every filter (and the
// Student-t energy of eq. 2.5/2.6 when asked), the adjoint pass gathers
// sum_i K_i^T psi_i per pixel from LDS tiles of psi.
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
        const float *k = taps + i * M * M;   // already rounded to the precision
        float z = 0.0f;
#pragma unroll
        for (int t = 0; t < M * M; ++t) z = fmaf(k[t], e[t], z);
        psi[i * plane + (long)y * W + x] = alpha2[i] * z * __builtin_amdgcn_rcpf(fmaf(z, z, 1.0f));
        // log(1 + z^2) as ln 2 * log2 on the hardware logarithm (about 1 ulp;
        // the rounding of 1 + z^2 costs at most 6e-8 absolute per term)
        if (rho_partial)
            rho_acc += alpha[i] * (0.693147181f * __builtin_amdgcn_logf(fmaf(z, z, 1.0f)));
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

// grad E at pixel (y, x): the transpose of "extend, then correlate" plus the
// data term.  The extended position s = (sy, sx) receives
//   G(s) = sum_i sum_{a,b} k_i[a][b] psi_i(sy - a + R, sx - b + R)
// (psi = 0 outside the image), and every extended position mirroring
// (y, x) adds onto it: the pixel itself, plus the ghost row -1-y (y < R) and
// the ghost row 2H-1-y (y >= H-R), likewise for columns.
//
// Per filter, the workgroup stages psi_i on rows y0 - 2R .. y0 + kBY + 3R - 1
// (and the same columns) in LDS, zero off the image, so the tap loop reads
// LDS only and needs no bounds tests.  That window holds every q a pixel of
// the block reaches: a mirrored row s lies in [y0 - R, y0 + kBY + 2R)
// (s = -1-y only occurs with y0 = 0; s = 2H-1-y <= H+R-1, and a block holding
// a row y >= H-R has H < y0 + kBY + R), and q = s - a + R with 0 <= a < m.
// The tile's rows are TS floats apart, 16 mod 32, so that the four 16-lane
// rows of a wave read disjoint banks (a stride of kBX + 5R itself, -1 mod 32
// for 7 x 7, put them on nearly the same banks).  Tiles alternate between two
// LDS buffers and the next filter's tile is loaded into registers while the
// current one is summed: one barrier per filter (a thread storing tile i + 1
// has passed the barrier of tile i, which every thread reached after summing
// tile i - 1, the buffer it overwrites).
template <int M, int PREC>
__global__ __launch_bounds__(kBX * kBY)
void adjoint_grad_kernel(const float *__restrict__ taps, int nf,
                         const float *__restrict__ psi,
                         const float *__restrict__ u,
                         const float *__restrict__ counts,
                         float *__restrict__ grad, int H, int W, float lambda,
                         int data_term)
{
    constexpr int R = (M - 1) / 2;
    constexpr int TH = kBY + 5 * R, TW = kBX + 5 * R, TN = TH * TW;
    constexpr int TS = (TW + 16 + 31) / 32 * 32 - 16;   // >= TW, 16 mod 32
    constexpr int NT = kBX * kBY;
    constexpr int LPT = (TN + NT - 1) / NT;   // tile elements per thread
    __shared__ float tile[2][TH * TS];
    const int y0 = blockIdx.y * kBY, x0 = blockIdx.x * kBX;
    const int y = y0 + threadIdx.y, x = x0 + threadIdx.x;
    const int tid = threadIdx.y * kBX + threadIdx.x;
    const bool in = (x < W) && (y < H);
    // this thread's tile elements: LDS slot, and plane offset or -1 off the
    // image (slot -1: beyond the tile)
    int goff[LPT], slot[LPT];
#pragma unroll
    for (int j = 0; j < LPT; ++j) {
        const int t = tid + j * NT;
        const int ty = t / TW, tx = t % TW;
        const int qy = y0 - 2 * R + ty, qx = x0 - 2 * R + tx;
        slot[j] = t < TN ? ty * TS + tx : -1;
        goff[j] = (t < TN && qy >= 0 && qy < H && qx >= 0 && qx < W) ? qy * W + qx : -1;
    }
    // mirrored extended positions: slot 0 the pixel, 1 the low ghost, 2 the high
    const int sy[3] = {y, -1 - y, 2 * H - 1 - y}, sx[3] = {x, -1 - x, 2 * W - 1 - x};
    const bool vy[3] = {in, in && y < R, in && y >= H - R};
    const bool vx[3] = {true, x < R, x >= W - R};
    const long plane = (long)H * W;
    float pf[LPT];
#pragma unroll
    for (int j = 0; j < LPT; ++j) pf[j] = goff[j] >= 0 ? operand<PREC>(psi[goff[j]]) : 0.0f;
    float g = 0.0f;
    for (int i = 0; i < nf; ++i) {
        float *tb = tile[i & 1];
#pragma unroll
        for (int j = 0; j < LPT; ++j)
            if (slot[j] >= 0) tb[slot[j]] = pf[j];
        __syncthreads();
        if (i + 1 < nf) {
            const float *p = psi + (i + 1) * plane;
#pragma unroll
            for (int j = 0; j < LPT; ++j)
                pf[j] = goff[j] >= 0 ? operand<PREC>(p[goff[j]]) : 0.0f;
        }
        const float *k = taps + i * M * M;   // already rounded to the precision
#pragma unroll
        for (int ir = 0; ir < 3; ++ir) {
#pragma unroll
            for (int ic = 0; ic < 3; ++ic) {
                if (!(vy[ir] && vx[ic])) continue;
                // tile element of q = (s - a + R, s - b + R) at a = b = 0
                const float *tp = tb + (sy[ir] - y0 + 3 * R) * TS + (sx[ic] - x0 + 3 * R);
                float acc = 0.0f;
#pragma unroll
                for (int a = 0; a < M; ++a)
#pragma unroll
                    for (int b = 0; b < M; ++b) acc = fmaf(k[a * M + b], tp[-a * TS - b], acc);
                g += acc;
            }
        }
    }
    if (!in) return;
    const long q = (long)y * W + x;
    grad[q] = g + lambda * data_gradient(u[q], anscombe(counts[q]), data_term);
}

dim3 grid2d(int H, int W) { return dim3((W + kBX - 1) / kBX, (H + kBY - 1) / kBY); }

}  // namespace

int direct_forward_blocks(int H, int W)
{
    const dim3 g = grid2d(H, W);
    return (int)(g.x * g.y);
}

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
    forward_kernel<MM, PP><<<g, b, 0, s>>>(bank.taps_for(PP), bank.alpha2,      \
                                           bank.alpha,                         \
                                           bank.nf, u, H, W, psi, rho_partial, \
                                           data_partial, counts, lambda, data_term)
    FE_DISPATCH_MP(bank.m, precision, FE_CALL)
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
    adjoint_grad_kernel<MM, PP><<<g, b, 0, s>>>(bank.taps_for(PP), bank.nf,   \
                                                psi, u,                       \
                                                counts, grad, H, W, lambda,   \
                                                data_term)
    FE_DISPATCH_MP(bank.m, precision, FE_CALL)
#undef FE_CALL
    return hipGetLastError();
}

}  // namespace fe
