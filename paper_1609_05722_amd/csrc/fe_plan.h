// Launch plan of the fused matrix-core step: how a batch of images is cut
// into workgroup tiles, and the device tables the step kernel reads.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "fe.h"

namespace fe {

constexpr int kMaxTileRows = 128;  // largest tile height a plan may pick

// Matrix-core operand tables of one filter bank (see kernels_fused.hip).
struct FusedBank {
    int m = 0, nf = 0, nfb = 0;  // nfb: filter blocks of 16 after zero-padding
    float *fwd = nullptr;        // forward A operands          [kf][nfb][64]
    float *adj = nullptr;        // adjoint B operands x 2alpha [nfb][4][ntb][64]
    float *lastf = nullptr;      // last tap, forward           [nfb][4][64]
    float *lasta = nullptr;      // last tap x 2alpha, adjoint  [nfb][4][64]
};

// How a batch is cut into workgroup tiles: every job's image is split into
// a grid of ntx x nty nearly equal tiles of at most tile_w x tile_h pixels.
struct Plan {
    int tile_w = 0, tile_h = 0;
    int njobs = 0, ntiles = 0;
    std::vector<int> jobs_ntx, jobs_nty;
    size_t device_bytes() const;  // job table in the workspace
};

bool fused_supported(int m, int nf);
hipError_t fused_upload(const float *taps, const float *alpha, int m, int nf,
                        FusedBank *out);
void fused_release(FusedBank *b);
void make_plan(int m, const fe_job *jobs, int n, Plan *plan);
// Runs every job's iterations; on return ua[i] holds job i's last iterate
// (the pointers are swapped as needed).
hipError_t run_fused(const FusedBank &bank, const Plan &plan, const fe_job *jobs,
                     int n, float **ua, float **ub, void *plan_ws, hipStream_t s);

}  // namespace fe
