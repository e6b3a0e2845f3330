// Launch plan of the fused matrix-core step: how a batch of images is cut
// into workgroup tiles, and the device tables the step kernel reads.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fe.h"

namespace fe {

constexpr int kMaxTileRows = 128;  // largest tile height a plan may pick
constexpr int kMinTileRows = 8;    // smallest tile height a plan or a tuning file may pick

// Matrix-core operand tables of one filter bank (see kernels_fused.hip).
struct FusedBank {
    int m = 0, nf = 0, nfb = 0;  // nfb: filter blocks of 16 after zero-padding
    float *fwd = nullptr;        // forward A operands          [kf][nfb][64]
    float *adj = nullptr;        // adjoint B operands x 2alpha [nfb][4][ntb][64]
    float *lastf = nullptr;      // last tap, forward           [nfb][4][64]
    float *lasta = nullptr;      // last tap x 2alpha, adjoint  [nfb][4][64]
    void *bf_fwd = nullptr, *bf_adj = nullptr;  // bfloat16 operand tables
    void *h_fwd = nullptr, *h_adj = nullptr;    // float16 operand tables
    float *alpha = nullptr;      // alpha_i, zero-padded to 64 (energy)
};

// How a batch is cut into workgroup tiles: every job's image is split into
// a grid of ntx x nty nearly equal tiles of at most tile_w x tile_h pixels,
// each run by a workgroup of `waves` waves.
struct Plan {
    int tile_w = 0, tile_h = 0, waves = 0;
    int njobs = 0;
    long ntiles = 0;
    std::vector<int> jobs_ntx, jobs_nty;
    size_t device_bytes() const;  // job table in the workspace
};

// One job of an fe_advance batch: its description, its state (two planes
// u^n / u^{n-1}, u^n in plane done % 2), iterations done and to apply.
struct AdvanceItem {
    const fe_job *job;
    float *state;
    int done, count;
};

// Workgroup shape of the step: waves per workgroup and tile height.
struct TileChoice {
    int waves = 0, ty = 0;   // 0: not chosen (default waves, cost-model height)
};

// Measured tile shapes: batch signature (precision and job sizes) -> waves
// and tile height.  Filled by fe_autotune, consulted by every plan.
struct TuneTable {
    mutable std::mutex mu;
    std::map<std::string, TileChoice> tab;
    TileChoice lookup(const std::string &key) const
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = tab.find(key);
        return it == tab.end() ? TileChoice{} : it->second;
    }
    void store(const std::string &key, TileChoice v)
    {
        std::lock_guard<std::mutex> lk(mu);
        tab[key] = v;
    }
};

// Signature of one precision group of a batch: precision and the multiset
// of image sizes of the jobs that advance.
std::string batch_key(int prec, const AdvanceItem *items, int n);
// Tile heights worth measuring for a group run with nw waves per
// workgroup, best cost-model estimate first.
std::vector<int> tile_candidates(const FusedBank &bank, int prec, const AdvanceItem *items,
                                 int n, int nw, int max_n);
// Waves per workgroup the step is built for: default_waves(prec) unless a
// measured choice says otherwise; wave_options lists every variant.
int default_waves(int prec);
// default_waves(prec) where its variant exists for the bank, else the other one
int bank_default_waves(const FusedBank &bank, int prec);
// the waves a batch runs with when no measured choice exists (FP32: 12 on
// tiles of at least six pipeline steps, else 8)
int plan_waves(const FusedBank &bank, int prec, const AdvanceItem *items, int n);
std::vector<int> wave_options(int prec);
// Tallest tile the variant's LDS allows (0 if no such variant).
int max_tile_rows(const FusedBank &bank, int prec, int nw);

bool fused_supported(int m, int nf);
hipError_t fused_upload(const float *taps, const float *alpha, int m, int nf,
                        FusedBank *out);
void fused_release(FusedBank *b);
// forced_ty > 0 imposes the tile height (clamped to the variant's range);
// otherwise the cost model picks it.
void make_plan(const FusedBank &bank, int prec, const AdvanceItem *items, int n, Plan *plan,
               int nw, int forced_ty = 0);
size_t fused_table_bytes(int n);
// Enqueues the job table and max(count) step launches per precision group;
// job i is advanced by items[i].count iterations.
// tune: measured tile shapes (may be NULL); only_prec >= 0 restricts the
// launch to one precision group and `forced` imposes its shape (used while
// tuning).
hipError_t run_fused(const FusedBank &bank, const AdvanceItem *items, int n, void *plan_ws,
                     hipStream_t s, const TuneTable *tune = nullptr, int only_prec = -1,
                     TileChoice forced = TileChoice{});

// One image of a gradient launch: grad E(u) (eq. 3.2 plus the data term's
// gradient) into grad (NULL: not stored), E(u) (eq. 2.5 with eq. 3.4 / 3.6)
// on request.
struct GradItem {
    int height, width;
    const float *counts, *u;
    float *grad;
    float lambda;
    int data_term;   // FE_DATA_QUADRATIC or FE_DATA_IDIV
};
// One fused launch over every tile of the images (contractions in precision
// prec); with `energy`, the energies are summed by a second, deterministic
// pass into n device doubles whose address goes to *energy_dev.  ws:
// DEVICE, 256-byte aligned, grad_workspace_bytes.
size_t grad_workspace_bytes(const FusedBank &bank, const GradItem *items, int n);
hipError_t run_grad(const FusedBank &bank, const GradItem *items, int n, int prec, bool energy,
                    void *ws, double **energy_dev, hipStream_t s);

}  // namespace fe
