// Host-only checks of the solve server's admission policy (compiled with g++ by
// test_server_policy.py; no device involved).
#include <cassert>
#include <cstdio>
#include <map>
#include <random>
#include <string>
#include <vector>

#include "policy.h"

using qrvie::sched::Policy;

#define EXPECT(c)                                                        \
    do {                                                                 \
        if (!(c)) {                                                      \
            std::fprintf(stderr, "line %d: failed: %s\n", __LINE__, #c); \
            return 1;                                                    \
        }                                                                \
    } while (0)

static int fifo_and_slots() {
    Policy p(2, 100, 0);
    std::vector<uint64_t> adm;
    std::vector<std::string> ev;
    EXPECT(p.enqueue(1, "a", 10, 5));
    EXPECT(p.enqueue(2, "b", 10, 5));
    EXPECT(p.enqueue(3, "c", 10, 5));
    p.admit(&adm, &ev);
    EXPECT(adm.size() == 2 && adm[0] == 1 && adm[1] == 2);      // two slots, arrival order
    EXPECT(p.running() == 2 && p.in_use() == 20 && p.queued() == 1);
    adm.clear();
    EXPECT(!p.finish(1, true, &ev));                             // op_cache = 0: not kept
    p.admit(&adm, &ev);
    EXPECT(adm.size() == 1 && adm[0] == 3);
    return 0;
}

static int no_head_of_line_blocking() {
    Policy p(4, 100, 0);
    std::vector<uint64_t> adm;
    std::vector<std::string> ev;
    EXPECT(p.enqueue(1, "a", 60, 40));
    EXPECT(p.enqueue(2, "b", 60, 40));                           // does not fit next to 1
    EXPECT(p.enqueue(3, "c", 30, 20));                           // fits: must not wait behind 2
    p.admit(&adm, &ev);
    EXPECT(adm.size() == 2 && adm[0] == 1 && adm[1] == 3);
    EXPECT(p.in_use() == 90 && p.queued() == 1);
    adm.clear();
    p.finish(1, true, &ev);
    p.admit(&adm, &ev);
    EXPECT(adm.size() == 1 && adm[0] == 2);
    EXPECT(p.peak() == 90);
    return 0;
}

static int refuses_what_can_never_fit() {
    Policy p(2, 100, 2);
    EXPECT(!p.enqueue(1, "a", 101, 50));
    EXPECT(!p.enqueue(2, "b", 10, 20));                          // inconsistent sizes
    EXPECT(p.enqueue(3, "c", 100, 50));
    return 0;
}

static int cache_hits_pin_and_lru_eviction() {
    Policy p(2, 100, 2);
    std::vector<uint64_t> adm;
    std::vector<std::string> ev;
    // request on "a" builds its operator (40 B) and keeps it
    EXPECT(p.enqueue(1, "a", 50, 40));
    p.admit(&adm, &ev);
    EXPECT(p.finish(1, true, &ev) && p.cached("a") && p.in_use() == 40);
    // a second request on "a" needs only its solver bytes and pins the entry
    adm.clear();
    EXPECT(p.enqueue(2, "a", 50, 40));
    p.admit(&adm, &ev);
    EXPECT(adm.size() == 1 && p.in_use() == 50 && p.hits() == 1);
    // a big request cannot evict the pinned entry: it waits
    EXPECT(p.enqueue(3, "b", 70, 40));                          // 50 in use + 70 > 100
    adm.clear();
    p.admit(&adm, &ev);
    EXPECT(adm.empty() && ev.empty());
    // once the hit finishes, the entry is unpinned and evicted for the big request
    EXPECT(!p.finish(2, false, &ev));
    p.admit(&adm, &ev);
    EXPECT(adm.size() == 1 && adm[0] == 3 && ev.size() == 1 && ev[0] == "a" && !p.cached("a"));
    EXPECT(p.in_use() == 70 && p.evictions() == 1);
    return 0;
}

static int cache_capacity_is_bounded() {
    Policy p(1, 1000, 2);
    std::vector<uint64_t> adm;
    std::vector<std::string> ev;
    const char* keys[] = {"a", "b", "c"};
    for (uint64_t t = 0; t < 3; ++t) {
        EXPECT(p.enqueue(t, keys[t], 20, 10));
        adm.clear();
        p.admit(&adm, &ev);
        EXPECT(adm.size() == 1);
        p.finish(t, true, &ev);
    }
    EXPECT(p.cache_size() == 2 && !p.cached("a") && p.cached("b") && p.cached("c"));
    EXPECT(ev.size() == 1 && ev[0] == "a" && p.in_use() == 20);
    ev.clear();
    p.clear(&ev);
    EXPECT(ev.size() == 2 && p.in_use() == 0);
    return 0;
}

static int bypass_limit_prevents_starvation() {
    Policy p(4, 100, 0, 2);
    std::vector<uint64_t> adm;
    std::vector<std::string> ev;
    EXPECT(p.enqueue(1, "a", 60, 40));
    p.admit(&adm, &ev);                                          // 1 runs (60)
    EXPECT(p.enqueue(2, "big", 80, 40));                         // waits for 1
    EXPECT(p.enqueue(3, "s1", 10, 5));
    EXPECT(p.enqueue(4, "s2", 10, 5));
    EXPECT(p.enqueue(5, "s3", 10, 5));
    adm.clear();
    p.admit(&adm, &ev);
    EXPECT(adm.size() == 2 && adm[0] == 3 && adm[1] == 4);       // two overtakes, then 2 blocks
    EXPECT(p.queued() == 2);
    adm.clear();
    p.finish(3, true, &ev);
    p.admit(&adm, &ev);
    EXPECT(adm.empty());                                         // 5 would fit but must wait behind 2
    p.finish(4, true, &ev);
    p.finish(1, true, &ev);
    p.admit(&adm, &ev);
    EXPECT(adm.size() == 2 && adm[0] == 2 && adm[1] == 5);       // 2 first, then 5 next to it
    // without a limit the small request is admitted ahead of the big one
    Policy q(4, 100, 0);
    std::vector<uint64_t> a2;
    EXPECT(q.enqueue(1, "a", 60, 40));
    q.admit(&a2, &ev);
    EXPECT(q.enqueue(2, "big", 80, 40));
    for (uint64_t t = 3; t < 6; ++t) EXPECT(q.enqueue(t, "s", 10, 5));
    a2.clear();
    q.admit(&a2, &ev);
    EXPECT(a2.size() == 3);
    return 0;
}

static int cache_hit_never_evicts_its_own_operator() {
    Policy p(2, 100, 2);
    std::vector<uint64_t> adm;
    std::vector<std::string> ev;
    EXPECT(p.enqueue(1, "a", 50, 40));
    p.admit(&adm, &ev);
    EXPECT(p.finish(1, true, &ev) && p.cached("a") && p.in_use() == 40);
    EXPECT(p.enqueue(2, "x", 50, 10));
    p.admit(&adm, &ev);
    EXPECT(p.in_use() == 90 && p.running() == 1);
    // a hit on "a" needs 20 more bytes; the only evictable entry is its own operator
    EXPECT(p.enqueue(3, "a", 60, 40));
    adm.clear();
    p.admit(&adm, &ev);
    EXPECT(adm.empty() && ev.empty() && p.cached("a") && p.in_use() == 90);
    EXPECT(p.finish(2, true, &ev) && p.in_use() == 50);          // "x" kept (10 B)
    p.admit(&adm, &ev);
    EXPECT(adm.size() == 1 && adm[0] == 3 && ev.empty() && p.hits() == 1 && p.in_use() == 70);
    return 0;
}

static int no_eviction_for_a_request_that_still_waits() {
    Policy p(2, 100, 2);
    std::vector<uint64_t> adm;
    std::vector<std::string> ev;
    EXPECT(p.enqueue(1, "a", 30, 20));
    p.admit(&adm, &ev);
    EXPECT(p.finish(1, true, &ev) && p.in_use() == 20);
    EXPECT(p.enqueue(2, "x", 70, 10));
    p.admit(&adm, &ev);
    EXPECT(p.in_use() == 90);
    // even with "a" evicted, 70 + 50 > 100: "a" stays cached
    EXPECT(p.enqueue(3, "b", 50, 20));
    adm.clear();
    p.admit(&adm, &ev);
    EXPECT(adm.empty() && ev.empty() && p.cached("a"));

    // a request held back by the bypass limit evicts nothing either
    Policy q(3, 100, 2, 1);
    adm.clear();
    EXPECT(q.enqueue(1, "a", 30, 20));
    q.admit(&adm, &ev);
    EXPECT(q.finish(1, true, &ev) && q.in_use() == 20);
    EXPECT(q.enqueue(2, "x", 50, 10));
    q.admit(&adm, &ev);
    EXPECT(q.in_use() == 70);
    EXPECT(q.enqueue(3, "b", 60, 20));                           // 130 > 100 + 20: waits
    EXPECT(q.enqueue(4, "y", 10, 5));                            // fits: overtakes 3 once
    EXPECT(q.enqueue(5, "c", 30, 20));                           // fits only by evicting "a"
    adm.clear();
    q.admit(&adm, &ev);
    EXPECT(adm.size() == 1 && adm[0] == 4 && ev.empty() && q.cached("a") && q.in_use() == 80);
    return 0;
}

static int a_miss_stays_unpinned_when_its_key_is_cached_later() {
    Policy p(3, 100, 2);
    std::vector<uint64_t> adm;
    std::vector<std::string> ev;
    EXPECT(p.enqueue(1, "a", 40, 20));
    EXPECT(p.enqueue(2, "a", 40, 20));
    p.admit(&adm, &ev);                                          // both miss and build
    EXPECT(adm.size() == 2 && !p.pinned(1) && !p.pinned(2));
    EXPECT(p.finish(1, true, &ev) && p.cached("a") && p.in_use() == 60);
    EXPECT(!p.pinned(2));                                        // still charged as a miss
    // so the entry may be evicted while 2 runs: 2 must keep using the operator it built
    EXPECT(p.enqueue(3, "b", 50, 20));
    adm.clear();
    p.admit(&adm, &ev);
    EXPECT(adm.size() == 1 && adm[0] == 3 && ev.size() == 1 && ev[0] == "a" && p.in_use() == 90);
    EXPECT(p.finish(2, true, &ev) && p.cached("a"));             // its own operator is kept now
    // a request admitted on a cached key is pinned until it finishes
    EXPECT(p.enqueue(4, "a", 30, 20));
    adm.clear();
    p.admit(&adm, &ev);
    EXPECT(adm.size() == 1 && p.pinned(4));
    EXPECT(!p.finish(4, false, &ev) && !p.pinned(4));
    return 0;
}

// Random submissions and completions against a shadow model of what the policy must keep:
// bytes in use = needs of the running requests + bytes of the cached operators, within the
// budget; at most `slots` running; a running cache hit keeps its operator cached; no waiting
// request overtaken more than max_bypass times.
static int random_sequences_keep_the_invariants() {
    const size_t budget = 100;
    const int slots = 3, op_cache = 2, max_bypass = 3;
    for (uint32_t seed = 1; seed <= 20; ++seed) {
        Policy p(slots, budget, op_cache, max_bypass);
        std::mt19937 rng(seed);
        auto op_bytes = [](int k) { return (size_t)(5 + 3 * k); };
        struct Sh { int key; size_t fp; bool running; int bypass; };
        std::map<uint64_t, Sh> jobs;                              // ordered by ticket = arrival
        std::vector<uint64_t> adm;
        std::vector<std::string> ev;
        uint64_t next = 1;
        for (int step = 0; step < 20000; ++step) {
            std::vector<uint64_t> run;
            for (auto& kv : jobs)
                if (kv.second.running) run.push_back(kv.first);
            if (run.empty() || (p.queued() < 12 && rng() % 2 == 0)) {   // bounded queue
                const int k = (int)(rng() % 6);
                const size_t fp = op_bytes(k) + 1 + rng() % 40;
                if (p.enqueue(next, "k" + std::to_string(k), fp, op_bytes(k))) jobs[next] = Sh{k, fp, false, 0};
                ++next;
            } else {
                const uint64_t t = run[rng() % run.size()];
                p.finish(t, !p.pinned(t), &ev);
                jobs.erase(t);
            }
            adm.clear();
            p.admit(&adm, &ev);
            for (uint64_t t : adm) {
                jobs.at(t).running = true;
                for (auto& kv : jobs)                             // every earlier request still queued
                    if (kv.first < t && !kv.second.running) ++kv.second.bypass;
            }
            size_t expect = 0;
            int nrun = 0;
            size_t nq = 0;
            for (auto& kv : jobs) {
                const Sh& j = kv.second;
                const std::string key = "k" + std::to_string(j.key);
                if (j.running) {
                    ++nrun;
                    const bool pin = p.pinned(kv.first);
                    expect += pin ? j.fp - op_bytes(j.key) : j.fp;
                    EXPECT(!pin || p.cached(key));
                } else {
                    ++nq;
                    EXPECT(j.bypass <= max_bypass);
                }
            }
            for (int k = 0; k < 6; ++k)
                if (p.cached("k" + std::to_string(k))) expect += op_bytes(k);
            EXPECT(p.in_use() == expect && p.in_use() <= budget);
            EXPECT(p.running() == nrun && nrun <= slots && p.queued() == nq);
            EXPECT((int)p.cache_size() <= op_cache);
        }
    }
    return 0;
}

int main() {
    int (*tests[])() = {fifo_and_slots, no_head_of_line_blocking, refuses_what_can_never_fit,
                        cache_hits_pin_and_lru_eviction, cache_capacity_is_bounded,
                        bypass_limit_prevents_starvation, cache_hit_never_evicts_its_own_operator,
                        no_eviction_for_a_request_that_still_waits,
                        a_miss_stays_unpinned_when_its_key_is_cached_later,
                        random_sequences_keep_the_invariants};
    for (auto t : tests)
        if (t()) return 1;
    std::printf("ok\n");
    return 0;
}
