// Internal declarations shared by the host runtime and the kernel files of
// the gfx950 FoE Poisson denoiser.  Not part of the public ABI (include/fe.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "fe.h"

namespace fe {

constexpr int kMaxM = 7;         // largest filter side built
constexpr int kMaxFilters = 64;  // largest filter count built

// Filter bank on the device, in the layouts the kernels read.
struct DeviceBank {
    int m = 0, nf = 0;
    float *taps = nullptr;     // [nf][m*m] correlation taps
    float *taps_r[2] = {};     // the same rounded to BF16, FP16 (held as float)
    float *alpha2 = nullptr;   // [nf] 2 * alpha_i (the influence's factor)
    float *alpha = nullptr;    // [nf] alpha_i
    // the taps as the contractions of a precision (FE_PREC_*) use them
    const float *taps_for(int precision) const
    {
        return precision == 1 ? taps_r[0] : precision == 2 ? taps_r[1] : taps;
    }
};

// ---- elementwise kernels (kernels_pointwise.hip) --------------------------
hipError_t launch_anscombe_init(const float *counts, float *u0, float *u1,
                                long n, hipStream_t s);
hipError_t launch_inverse_anscombe(const float *u, float *out,
                                   float *out_anscombe, long n, hipStream_t s);
hipError_t launch_bin3(const float *y, int H, int W, float *yb, hipStream_t s);
// Debug validation: bad[0] |= 1 if any of y[0..n) is negative, NaN or
// infinite; launch_zero_ints clears n flags first.
hipError_t launch_check_counts(const float *y, long n, int *bad, hipStream_t s);
hipError_t launch_zero_ints(int *p, int n, hipStream_t s);
hipError_t launch_upsample3(const float *xb, int Hb, int Wb, float *x, int H, int W,
                            hipStream_t s);

// ---- debug validation of counts (fe_runtime.cpp) -------------------------
// With FE_VALIDATE=1 in the environment: FE_ERR_INVALID (and the message in
// fe_last_error) if any job's counts hold a negative, NaN or infinite
// value; synchronous, on the null stream of `device`.  FE_OK otherwise.
fe_status validate_job_counts(int device, const fe_job *jobs, int n);

// ---- direct (non-MFMA) FP32 kernels (kernels_direct.hip) ------------------
// psi_i = alpha_i rho'(K_i u) for all filters, written as nf planes of H*W.
// If rho_partial != NULL every block also writes its FP32 partial sum of
// alpha_i rho(K_i u) (and data_partial the data-term sum when counts != NULL).
// precision (FE_PREC_*) rounds the operands of K_i u (FP32 accumulation).
hipError_t launch_direct_forward(const DeviceBank &bank, const float *u,
                                 int H, int W, float *psi,
                                 float *rho_partial, float *data_partial,
                                 const float *counts, float lambda,
                                 int data_term, int precision, int *n_blocks,
                                 hipStream_t s);
// grad = sum_i K_i^T psi_i + grad D(u, v); precision rounds the operands
// of K_i^T psi_i (FP32 accumulation).
hipError_t launch_direct_adjoint_grad(const DeviceBank &bank, const float *psi,
                                      const float *u, const float *counts,
                                      float *grad, int H, int W, float lambda,
                                      int data_term, int precision, hipStream_t s);
int direct_forward_blocks(int H, int W);

// ---- allocation-free stepping (fe_noalloc.hip) ----------------------------
// Size of the file-scope device array that holds the job table of
// fe_advance_noalloc (one copy per device, kept until the process ends).
constexpr size_t kNoallocScratchBytes = 256 * 1024;
// Resolves the array's address on `device`, which must be current; once per
// device (later calls return at once).  Called by fe_create.
hipError_t noalloc_setup(int device);
// The array's device address on `device`, or NULL before noalloc_setup.
void *noalloc_scratch(int device);

}  // namespace fe
