// Launch plan of the fused matrix-core step: how a batch of images is cut
// into workgroup tiles, and the device tables the step kernel reads.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "fe.h"

namespace fe {

// Matrix-core operand tables of one filter bank (see kernels_fused.hip).
struct FusedBank {
    int m = 0, nf = 0, nfb = 0;  // nfb: filter blocks of 16 after zero-padding
    float *fwd = nullptr;        // forward A operands   [kf][nfb][64]
    float *adj = nullptr;        // adjoint B operands   [nfb][4][ntb][64]
    float *last = nullptr;       // last tap per filter  [nfb][4][64]
    float *alpha2 = nullptr;     // 2 alpha per filter   [nfb][4][64]
};

// One workgroup's share of an image: output rows [y0, y0 + ty) and
// columns [x0, x0 + tx) of job `job`.
struct Tile {
    int job, y0, x0, ty, tx;
};

struct Plan {
    std::vector<Tile> tiles;
    int tile_w = 0, tile_h = 0;
    size_t device_bytes() const { return tiles.size() * sizeof(Tile); }
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
