// Host-only checks of the serving scheduler (admission by memory budget,
// arrival order, per-tick iteration counts, deferred release).  Built with
// g++ by tests/test_sched_cpu.py; prints "OK" and exits 0 on success.
#include <cstdio>
#include <cstdlib>

#include "fe_sched.h"

#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c);    \
            std::exit(1);                                               \
        }                                                               \
    } while (0)

static void arena_tests()
{
    fe::Arena a(10 * 256);
    size_t o1, o2, o3, o4;
    CHECK(a.alloc(300, &o1) && o1 == 0);        // rounds up to 512
    CHECK(a.alloc(256, &o2) && o2 == 512);
    CHECK(a.alloc(1000, &o3) && o3 == 768);     // 1024 bytes
    CHECK(a.used() == 512 + 256 + 1024);
    CHECK(!a.alloc(1024, &o4));                 // only 768 left
    a.release(o2, 256);
    CHECK(a.largest_free() == 768);
    a.release(o1, 300);                         // merges with the freed 256
    CHECK(a.largest_free() == 768);
    CHECK(a.alloc(768, &o4) && o4 == 0);        // first fit at the merged hole
    a.release(o4, 768);
    a.release(o3, 1000);
    CHECK(a.used() == 0 && a.largest_free() == 10 * 256);
}

static void scheduler_tests()
{
    // budget for two 1 KiB jobs
    fe::Scheduler s(2048, 10, 100);
    CHECK(s.fits_ever(2048) && !s.fits_ever(2049));
    const uint64_t a = s.submit(1024, 25, 0.0);
    const uint64_t b = s.submit(1024, 10, 0.1);
    const uint64_t c = s.submit(512, 5, 0.2);   // must wait behind a and b
    fe::TickPlan t = s.plan(1.0);
    CHECK(t.admitted.size() == 2 && t.admitted[0] == a && t.admitted[1] == b);
    CHECK(t.active.size() == 2 && t.count[0] == 10 && t.count[1] == 10);
    CHECK(t.done_before[0] == 0 && t.done_before[1] == 0);
    CHECK(t.finishing.size() == 1 && t.finishing[0] == b);
    CHECK(s.pending() == 1 && s.active() == 1 && s.retiring() == 1);
    // b's memory is not reusable until its tick completed
    t = s.plan(2.0);
    CHECK(t.admitted.empty() && t.active.size() == 1 && t.count[0] == 10);
    CHECK(t.done_before[0] == 10 && t.finishing.empty());
    s.retire({b});
    t = s.plan(3.0);
    CHECK(t.admitted.size() == 1 && t.admitted[0] == c);
    CHECK(t.active.size() == 2 && t.count[0] == 5 && t.count[1] == 5);
    CHECK(t.finishing.size() == 2);
    const fe::SchedJob *jc = s.find(c);
    CHECK(jc && jc->t_admit == 3.0 && jc->t_submit == 0.2);
    s.retire({a, c});
    CHECK(s.active() == 0 && s.pending() == 0 && s.arena().used() == 0);
}

static void order_and_caps()
{
    // a large head blocks smaller later jobs (arrival order is kept)
    fe::Scheduler s(4096, 7, 100);
    const uint64_t small1 = s.submit(1024, 7, 0);
    const uint64_t big = s.submit(4096, 7, 0);
    const uint64_t small2 = s.submit(1024, 7, 0);
    fe::TickPlan t = s.plan(0);
    CHECK(t.admitted.size() == 1 && t.admitted[0] == small1);
    s.retire(t.finishing);
    t = s.plan(0);
    CHECK(t.admitted.size() == 1 && t.admitted[0] == big);
    s.retire(t.finishing);
    t = s.plan(0);
    CHECK(t.admitted.size() == 1 && t.admitted[0] == small2);
    // the active cap
    fe::Scheduler s2(1 << 20, 3, 2);
    for (int i = 0; i < 5; ++i) s2.submit(1024, 9, 0);
    t = s2.plan(0);
    CHECK(t.admitted.size() == 2 && s2.pending() == 3);
    // zero-iteration jobs are admitted and finish in the same tick
    fe::Scheduler s3(4096, 3, 10);
    const uint64_t z = s3.submit(256, 0, 0);
    t = s3.plan(0);
    CHECK(t.admitted.size() == 1 && t.count[0] == 0 && t.finishing.size() == 1 &&
          t.finishing[0] == z);
}

static void tick_budget()
{
    // work budget 1000 pixel-iterations per tick, 10 iterations per job
    fe::Scheduler s(1 << 20, 10, 100, 1000);
    const uint64_t big = s.submit(4096, 30, 0.0, 200);    // 2000 px-it per tick alone
    const uint64_t a = s.submit(1024, 10, 0.1, 50);
    const uint64_t b = s.submit(1024, 10, 0.2, 50);
    fe::TickPlan t = s.plan(1.0);
    // all admitted; the oldest (over budget on its own) advances, the rest wait
    CHECK(t.admitted.size() == 3);
    CHECK(t.active.size() == 3 && t.active[0] == big);
    CHECK(t.count[0] == 10 && t.count[1] == 0 && t.count[2] == 0);
    CHECK(t.finishing.empty());
    t = s.plan(2.0);
    CHECK(t.count[0] == 10 && t.count[1] == 0 && t.done_before[0] == 10);
    t = s.plan(3.0);
    CHECK(t.count[0] == 10 && t.finishing.size() == 1 && t.finishing[0] == big);
    s.retire(t.finishing);
    // the two small ones fit one budget together: both advance and finish
    t = s.plan(4.0);
    CHECK(t.active.size() == 2 && t.count[0] == 10 && t.count[1] == 10);
    CHECK(t.finishing.size() == 2 && t.finishing[0] == a && t.finishing[1] == b);
    s.retire(t.finishing);
    CHECK(s.active() == 0 && s.arena().used() == 0);
    // the budget is reached part-way: the jobs after the one that reaches it wait
    fe::Scheduler s2(1 << 20, 4, 100, 1000);
    for (int i = 0; i < 5; ++i) s2.submit(256, 8, 0.0, 100);   // 400 px-it per tick each
    t = s2.plan(0.0);
    CHECK(t.active.size() == 5);
    CHECK(t.count[0] == 4 && t.count[1] == 4 && t.count[2] == 4);   // 1200 >= 1000
    CHECK(t.count[3] == 0 && t.count[4] == 0);
    // without a budget every resident job advances (processor sharing)
    fe::Scheduler s3(1 << 20, 4, 100, 0);
    for (int i = 0; i < 5; ++i) s3.submit(256, 8, 0.0, 100);
    t = s3.plan(0.0);
    for (size_t i = 0; i < t.count.size(); ++i) CHECK(t.count[i] == 4);
}

int main()
{
    arena_tests();
    scheduler_tests();
    order_and_caps();
    tick_budget();
    std::printf("OK\n");
    return 0;
}
