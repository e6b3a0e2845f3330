// Host-only checks of the step's launch planner (tile grid, tile heights
// within each variant's LDS limit, tuning candidates, batch signatures).
// Linked against libfe.so by tests/test_plan_cpu.py; touches no device.
// Prints "OK" and exits 0 on success.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <vector>

#include "fe_plan.h"

#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c);    \
            std::exit(1);                                               \
        }                                                               \
    } while (0)

static fe::FusedBank bank(int m, int nf)
{
    fe::FusedBank b;
    b.m = m;
    b.nf = nf;
    b.nfb = (nf + 15) / 16;
    return b;
}

static void limits()
{
    // 48 filters of 7 x 7: 12-wave FP32 keeps 15 KB of tables in LDS;
    // BF16 / FP16 keep 12 psi scratches of 70 q-positions x 112 bytes
    const fe::FusedBank b7 = bank(7, 48);
    CHECK(fe::max_tile_rows(b7, FE_PREC_FP32, 8) == fe::kMaxTileRows);
    CHECK(fe::max_tile_rows(b7, FE_PREC_FP32, 12) == 96);
    CHECK(fe::max_tile_rows(b7, FE_PREC_BF16, 12) == 97);
    CHECK(fe::max_tile_rows(b7, FE_PREC_FP16, 12) == 97);
    CHECK(fe::max_tile_rows(b7, FE_PREC_BF16, 8) == 0);     // not built
    CHECK(fe::max_tile_rows(b7, FE_PREC_FP32, 10) == 0);
    // 64 filters of 7 x 7 do not fit three waves per SIMD in FP32
    CHECK(fe::max_tile_rows(bank(7, 64), FE_PREC_FP32, 12) == 0);
    CHECK(fe::max_tile_rows(bank(7, 64), FE_PREC_FP32, 8) > 0);
    CHECK(fe::default_waves(FE_PREC_FP32) == 12 && fe::default_waves(FE_PREC_FP16) == 12);
    // where the 12-wave FP32 variant does not fit, the default falls back to 8
    CHECK(fe::bank_default_waves(b7, FE_PREC_FP32) == 12);
    CHECK(fe::bank_default_waves(bank(7, 64), FE_PREC_FP32) == 8);
    // FP32 runs 12 waves on tall tiles (4 x 512^2: 74 rows, 7 steps), 8 on
    // short ones (one 512^2 image spread over the CUs); BF16 / FP16 always 12
    {
        std::vector<fe_job> jb(4);
        std::vector<fe::AdvanceItem> it(4);
        for (int i = 0; i < 4; ++i) {
            jb[i] = fe_job{};
            jb[i].height = jb[i].width = 512;
            it[i] = {&jb[i], nullptr, 0, 10};
        }
        CHECK(fe::plan_waves(b7, FE_PREC_FP32, it.data(), 4) == 12);
        CHECK(fe::plan_waves(b7, FE_PREC_FP32, it.data(), 1) == 8);
        CHECK(fe::plan_waves(b7, FE_PREC_BF16, it.data(), 1) == 12);
        CHECK(fe::plan_waves(bank(7, 64), FE_PREC_FP32, it.data(), 4) == 8);
    }
    const std::vector<int> w = fe::wave_options(FE_PREC_FP32);
    CHECK(w.size() == 2 && std::count(w.begin(), w.end(), 8) == 1 &&
          std::count(w.begin(), w.end(), 12) == 1);
}

static void random_batches()
{
    std::mt19937 rng(12345);
    const int ms[3] = {3, 5, 7};
    for (int trial = 0; trial < 400; ++trial) {
        const int m = ms[trial % 3], r = (m - 1) / 2;
        const fe::FusedBank b = bank(m, 8 + (int)(rng() % 57));
        const int n = 1 + (int)(rng() % 40);
        std::vector<fe_job> jobs(n);
        std::vector<fe::AdvanceItem> items(n);
        for (int i = 0; i < n; ++i) {
            jobs[i] = fe_job{};
            jobs[i].height = r + (int)(rng() % (trial % 5 == 0 ? 3000 : 400));
            jobs[i].width = r + (int)(rng() % (trial % 7 == 0 ? 3000 : 400));
            items[i] = {&jobs[i], nullptr, 0, (int)(rng() % 4) == 0 ? 0 : 1 + (int)(rng() % 9)};
        }
        for (int prec = FE_PREC_FP32; prec <= FE_PREC_FP16; ++prec) {
            for (int nw : fe::wave_options(prec)) {
                const int hi = fe::max_tile_rows(b, prec, nw);
                if (hi <= 0) continue;
                fe::Plan p;
                fe::make_plan(b, prec, items.data(), n, &p, nw);
                CHECK(p.waves == nw && p.tile_w == 64 - 2 * r);
                CHECK(p.tile_h >= fe::kMinTileRows && p.tile_h <= hi);
                long tiles = 0;
                for (int i = 0; i < n; ++i) {
                    const fe_job &j = jobs[i];
                    if (items[i].count <= 0) {
                        CHECK(p.jobs_ntx[i] == 0 && p.jobs_nty[i] == 0);
                        continue;
                    }
                    // every tile of the balanced split fits the tile shape
                    CHECK(p.jobs_ntx[i] == (j.width + p.tile_w - 1) / p.tile_w);
                    CHECK(p.jobs_nty[i] == (j.height + p.tile_h - 1) / p.tile_h);
                    CHECK((j.height + p.jobs_nty[i] - 1) / p.jobs_nty[i] <= p.tile_h);
                    CHECK((j.width + p.jobs_ntx[i] - 1) / p.jobs_ntx[i] <= p.tile_w);
                    tiles += (long)p.jobs_ntx[i] * p.jobs_nty[i];
                }
                CHECK(tiles == p.ntiles);
                // candidates: distinct, in range, the plan's own choice first
                const std::vector<int> c = fe::tile_candidates(b, prec, items.data(), n, nw, 6);
                CHECK(!c.empty() && c.size() <= 6 && c[0] == p.tile_h);
                CHECK(std::set<int>(c.begin(), c.end()).size() == c.size());
                for (int ty : c) CHECK(ty >= fe::kMinTileRows && ty <= hi);
                // a forced height is clamped to the variant's range
                fe::Plan q;
                fe::make_plan(b, prec, items.data(), n, &q, nw, 100000);
                CHECK(q.tile_h == hi);
                fe::make_plan(b, prec, items.data(), n, &q, nw, 3);
                CHECK(q.tile_h == fe::kMinTileRows);
            }
        }
    }
}

static void keys()
{
    fe_job a{}, c{}, d{};
    a.height = 10; a.width = 20;
    c.height = 30; c.width = 5;
    d.height = 7;  d.width = 7;
    fe::AdvanceItem x[3] = {{&a, nullptr, 0, 2}, {&c, nullptr, 4, 2}, {&d, nullptr, 0, 0}};
    fe::AdvanceItem y[3] = {{&d, nullptr, 0, 0}, {&c, nullptr, 0, 6}, {&a, nullptr, 2, 8}};
    // the multiset of advancing sizes decides; order, counts and idle jobs do not
    CHECK(fe::batch_key(FE_PREC_FP32, x, 3) == fe::batch_key(FE_PREC_FP32, y, 3));
    CHECK(fe::batch_key(FE_PREC_FP32, x, 3) == "p0:10x20,30x5,");
    CHECK(fe::batch_key(FE_PREC_BF16, x, 3) != fe::batch_key(FE_PREC_FP32, x, 3));
    fe::AdvanceItem z[2] = {{&a, nullptr, 0, 2}, {&a, nullptr, 0, 2}};
    CHECK(fe::batch_key(FE_PREC_FP32, z, 2) == "p0:10x20,10x20,");
}

// The largest jobs: tile counts in 64-bit arithmetic, beyond one launch's
// 2^21 workgroups for a 3-row image of 2^31 - 2 pixels (the step then splits
// its launches over tile ranges), and a batch of them beyond 2^31 tiles.
static void huge()
{
    const fe::FusedBank b7 = bank(7, 48);
    fe_job thin{};
    thin.height = 3;
    thin.width = 715827882;
    thin.precision = FE_PREC_FP32;
    fe::AdvanceItem one[1] = {{&thin, nullptr, 0, 4}};
    fe::Plan p;
    fe::make_plan(b7, FE_PREC_FP32, one, 1, &p, 8);
    CHECK(p.jobs_ntx[0] == (715827882 + 57) / 58 && p.jobs_nty[0] == 1);
    CHECK(p.ntiles == 12341861L && p.ntiles > (1L << 21));
    std::vector<fe::AdvanceItem> many(200, fe::AdvanceItem{&thin, nullptr, 0, 4});
    fe::make_plan(b7, FE_PREC_FP32, many.data(), 200, &p, 8);
    CHECK(p.ntiles == 200L * 12341861L && p.ntiles > 2147483647L);
}

int main()
{
    limits();
    random_batches();
    keys();
    huge();
    std::printf("OK\n");
    return 0;
}
