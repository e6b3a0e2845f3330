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

// ---- allocation-free stepping (fe_noalloc.hip) ----------------------------
// Size of the file-scope device array that holds the job table of
// fe_advance_noalloc (one copy per device, kept until the process ends).
constexpr size_t kNoallocScratchBytes = 256 * 1024;
// Resolves the array's address on `device`, which must be current; once per
// device (later calls return at once; devices 64 and up keep none).  Called
// by fe_create.
hipError_t noalloc_setup(int device);
// The array's device address on `device`, or NULL before noalloc_setup.
void *noalloc_scratch(int device);

}  // namespace fe
