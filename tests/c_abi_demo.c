/* A plain C client of libfe.so: no Python, no PyTorch.  Reads a problem
 * from a binary file, denoises it on device 0 through the C ABI, writes
 * x_hat and u_hat, and checks an argument error on the way.
 *
 *   c_abi_demo IN OUT
 *   IN : int32 H, W, m, n_filters, iterations, data_term;
 *        float32 lambda, tau, gamma; float32 counts[H*W];
 *        float32 filters[n_filters*m*m]; float32 weights[n_filters]
 *   OUT: float32 x_hat[H*W], u_hat[H*W]
 * Exit status 0 on success. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "fe.h"

#define HIP_OK(call)                                                          \
    do {                                                                      \
        hipError_t e_ = (call);                                               \
        if (e_ != hipSuccess) {                                               \
            fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));        \
            return 2;                                                         \
        }                                                                     \
    } while (0)

static int read_all(FILE *f, void *p, size_t bytes)
{
    return fread(p, 1, bytes, f) == bytes;
}

int main(int argc, char **argv)
{
    if (argc != 3) {
        fprintf(stderr, "usage: c_abi_demo IN OUT\n");
        return 1;
    }
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 1;
    int32_t hdr[6];
    float prm[3];
    if (!read_all(f, hdr, sizeof hdr) || !read_all(f, prm, sizeof prm)) return 1;
    const int H = hdr[0], W = hdr[1], m = hdr[2], nf = hdr[3];
    const size_t npx = (size_t)H * W, ntap = (size_t)nf * m * m;
    float *counts = malloc(npx * 4), *taps = malloc(ntap * 4), *w = malloc((size_t)nf * 4);
    float *x = malloc(npx * 4), *u = malloc(npx * 4);
    if (!counts || !taps || !w || !x || !u) return 1;
    if (!read_all(f, counts, npx * 4) || !read_all(f, taps, ntap * 4) ||
        !read_all(f, w, (size_t)nf * 4))
        return 1;
    fclose(f);

    fe_prior prior = {m, nf, taps, w};
    fe_ctx *ctx = NULL;
    fe_status st = fe_create(&prior, 0, &ctx);
    if (st != FE_OK) {
        fprintf(stderr, "fe_create: %s\n", fe_last_error());
        return 3;
    }
    float *d_counts, *d_x, *d_u;
    HIP_OK(hipMalloc((void **)&d_counts, npx * 4));
    HIP_OK(hipMalloc((void **)&d_x, npx * 4));
    HIP_OK(hipMalloc((void **)&d_u, npx * 4));
    HIP_OK(hipMemcpy(d_counts, counts, npx * 4, hipMemcpyHostToDevice));

    fe_job job;
    memset(&job, 0, sizeof job);
    job.height = H;
    job.width = W;
    job.counts = d_counts;
    job.out = d_x;
    job.out_anscombe = d_u;
    job.lambda = prm[0];
    job.iterations = hdr[4];
    job.data_term = hdr[5];
    job.tau = prm[1];
    job.gamma = prm[2];
    job.precision = FE_PREC_FP32;

    /* an argument error is reported before anything is enqueued */
    fe_job bad = job;
    bad.lambda = -1.0f;
    size_t ws_bytes = 0;
    if (fe_workspace_size(ctx, &bad, 1, &ws_bytes) != FE_ERR_INVALID ||
        strlen(fe_last_error()) == 0) {
        fprintf(stderr, "negative lambda was not rejected\n");
        return 4;
    }
    st = fe_workspace_size(ctx, &job, 1, &ws_bytes);
    if (st != FE_OK) return 3;
    void *ws = NULL;
    HIP_OK(hipMalloc(&ws, ws_bytes));
    hipStream_t s;
    HIP_OK(hipStreamCreate(&s));
    st = fe_denoise(ctx, &job, 1, ws, ws_bytes, s);
    if (st != FE_OK) {
        fprintf(stderr, "fe_denoise: %s\n", fe_last_error());
        return 3;
    }
    HIP_OK(hipStreamSynchronize(s));
    HIP_OK(hipMemcpy(x, d_x, npx * 4, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(u, d_u, npx * 4, hipMemcpyDeviceToHost));
    HIP_OK(hipStreamDestroy(s));
    HIP_OK(hipFree(ws));
    HIP_OK(hipFree(d_counts));
    HIP_OK(hipFree(d_x));
    HIP_OK(hipFree(d_u));
    fe_destroy(ctx);

    FILE *o = fopen(argv[2], "wb");
    if (!o || fwrite(x, 4, npx, o) != npx || fwrite(u, 4, npx, o) != npx) return 1;
    fclose(o);
    free(counts);
    free(taps);
    free(w);
    free(x);
    free(u);
    printf("OK\n");
    return 0;
}
