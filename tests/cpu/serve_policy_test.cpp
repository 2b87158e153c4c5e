// CPU checks of the query server's host policy (serve_policy.h), built with
// the address and undefined-behaviour sanitizers by tests/test_serve_policy_cpu.py:
//   1. the arena allocator against a brute-force model of first fit;
//   2. admission driven by a fake executor (no GPU): at most one heavy query
//      runs, heavy queries start in arrival order, light ones in arrival order
//      among themselves, memory is never over-committed, every query finishes,
//      and a heavy query waits for no light query that arrived after it.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <deque>
#include <random>
#include <vector>

#include "serve_policy.h"

using sgwb::serve::Arena;

static int failures = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            if (++failures > 20) exit(1);                                     \
        }                                                                     \
    } while (0)

// ---------------------------------------------------------------- arena
struct Block {
    size_t off, len;
};

static void check_arena(const Arena &a, const std::vector<Block> &model, size_t size)
{
    // live blocks equal the model's, in order
    const auto &live = a.live();
    CHECK(live.size() == model.size());
    size_t used = 0;
    auto it = live.begin();
    for (const Block &b : model) {
        if (it == live.end()) break;
        CHECK(it->first == b.off && it->second == b.len);
        used += b.len;
        ++it;
    }
    CHECK(a.used() == used);
    // free ranges and live blocks tile [0, size): no gap, no overlap, coalesced
    size_t pos = 0;
    auto f = a.free_ranges().begin();
    auto l = live.begin();
    bool prev_free = false;
    while (pos < size) {
        if (f != a.free_ranges().end() && f->first == pos) {
            CHECK(!prev_free);  // two adjacent free ranges were not merged
            CHECK(f->second > 0);
            pos += f->second;
            prev_free = true;
            ++f;
        } else if (l != live.end() && l->first == pos) {
            pos += l->second;
            prev_free = false;
            ++l;
        } else {
            CHECK(false && "hole in the arena");
            return;
        }
    }
    CHECK(pos == size);
    CHECK(f == a.free_ranges().end() && l == live.end());
}

// first fit in the model: lowest offset whose gap holds n
static bool model_first_fit(const std::vector<Block> &model, size_t size, size_t n, size_t *off)
{
    size_t pos = 0;
    for (const Block &b : model) {
        if (b.off - pos >= n) {
            *off = pos;
            return true;
        }
        pos = b.off + b.len;
    }
    if (size - pos >= n) {
        *off = pos;
        return true;
    }
    return false;
}

static void test_arena(unsigned seed)
{
    std::mt19937_64 rng(seed);
    const size_t size = 256 * (size_t)(1000 + rng() % 5000);
    static char base_storage[1];
    char *base = base_storage;  // addresses are only compared, never dereferenced
    Arena a;
    a.init(base, size);
    std::vector<Block> model;
    check_arena(a, model, size);
    CHECK(!a.release(nullptr));
    for (int step = 0; step < 4000; ++step) {
        const bool do_alloc = model.empty() || (rng() % 100) < 55;
        if (do_alloc) {
            const size_t req = (rng() % 4 == 0) ? (size_t)(rng() % 300) : (size_t)(rng() % (size / 8));
            const size_t n = Arena::granule(req);
            size_t off = 0;
            const bool ok = model_first_fit(model, size, n, &off);
            CHECK(a.fits(req) == ok);
            char *p = a.alloc(req);
            CHECK((p != nullptr) == ok);
            if (p) {
                CHECK((size_t)(p - base) == off);
                CHECK(off % 256 == 0 && n % 256 == 0 && n >= req && n > 0);
                Block b{off, n};
                model.insert(std::upper_bound(model.begin(), model.end(), b,
                                              [](const Block &x, const Block &y) { return x.off < y.off; }),
                             b);
            }
        } else {
            const size_t i = rng() % model.size();
            CHECK(a.release(base + model[i].off));
            CHECK(!a.release(base + model[i].off));  // a second release is refused
            model.erase(model.begin() + (ptrdiff_t)i);
        }
        check_arena(a, model, size);
    }
    for (const Block &b : model) CHECK(a.release(base + b.off));
    CHECK(a.used() == 0 && a.free_ranges().size() == 1 && a.free_ranges().begin()->second == size);
}

// ---------------------------------------------------------------- admission
struct FakeQuery {
    int id;
    double arrive, cost;
    size_t need;
    double start = -1, done = -1;
    char *mem = nullptr;
};

static void test_admission(unsigned seed, int slots, int max_heavy)
{
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    const double heavy = 1e10;
    const size_t arena_bytes = (size_t)64 << 20;
    static char base_storage[1];
    Arena arena;
    arena.init(base_storage, arena_bytes);
    std::vector<FakeQuery> qs;
    double t = 0.0;
    for (int i = 0; i < 600; ++i) {
        t += -std::log(1.0 - U(rng)) * 0.004;  // Poisson arrivals
        FakeQuery q;
        q.id = i;
        q.arrive = t;
        const double r = U(rng);
        q.cost = r < 0.3 ? 1e10 + U(rng) * 6e11 : U(rng) * 9e9;  // heavy or light
        q.need = (size_t)(1 + (size_t)(U(rng) * (double)(arena_bytes / 3)));
        qs.push_back(q);
    }
    const double rate = 3.8e13;  // terms per second of the fake GPU
    std::deque<int> pending;
    std::vector<int> running;  // query ids
    size_t next = 0;
    double now = 0.0;
    int last_heavy_started = -1, last_light_started = -1;
    for (int iter = 0; iter < 100000 && (next < qs.size() || !pending.empty() || !running.empty()); ++iter) {
        // retire finished queries
        for (size_t k = 0; k < running.size();) {
            FakeQuery &q = qs[running[k]];
            if (q.done <= now) {
                CHECK(arena.release(q.mem));
                running.erase(running.begin() + (ptrdiff_t)k);
            } else {
                ++k;
            }
        }
        while (next < qs.size() && qs[next].arrive <= now) pending.push_back(qs[next++].id);
        // admit
        for (;;) {
            int heavy_running = 0;
            for (int id : running) heavy_running += qs[id].cost >= heavy ? 1 : 0;
            const bool heavy_full = heavy_running >= max_heavy;
            std::vector<sgwb::serve::PendingView> views;
            for (int id : pending) views.push_back({qs[id].cost, qs[id].need});
            const int idx = sgwb::serve::pick_admission(
                views, sgwb::serve::RunningView{slots - (int)running.size(), heavy_running}, heavy,
                [&](size_t i) { return arena.fits(views[i].need); }, max_heavy);
            if (idx == sgwb::serve::kAdmitNone) {
                // nothing admissible: a free slot, memory and no heavy in the way
                // would have admitted the head
                if ((int)running.size() < slots && !pending.empty()) {
                    FakeQuery &h = qs[pending.front()];
                    CHECK(!arena.fits(h.need) || (h.cost >= heavy && heavy_full));
                }
                break;
            }
            CHECK(idx >= 0 && idx < (int)pending.size());
            const int id = pending[(size_t)idx];
            FakeQuery &q = qs[id];
            // order: heavy after heavy, light after light
            if (q.cost >= heavy) {
                CHECK(!heavy_full);
                CHECK(id > last_heavy_started);
                last_heavy_started = id;
            } else {
                CHECK(id > last_light_started);
                last_light_started = id;
            }
            // everything before it in the queue is a heavy one waiting for the heavy slot
            // (or, once the first waiting heavy one is passed over, any later heavy one)
            bool heavy_blocked = false;
            for (int j = 0; j < idx; ++j) {
                const FakeQuery &w = qs[pending[(size_t)j]];
                CHECK(w.cost >= heavy);
                CHECK(heavy_full || heavy_blocked);
                heavy_blocked = true;
            }
            q.mem = arena.alloc(q.need);
            CHECK(q.mem != nullptr);
            q.start = now;
            q.done = now + q.cost / rate + 1e-4;
            pending.erase(pending.begin() + idx);
            running.push_back(id);
            CHECK((int)running.size() <= slots);
        }
        // advance the clock to the next event
        double nxt = 1e30;
        for (int id : running) nxt = std::min(nxt, qs[id].done);
        if (next < qs.size()) nxt = std::min(nxt, qs[next].arrive);
        if (nxt >= 1e30) break;
        now = std::max(now, nxt);
    }
    for (const FakeQuery &q : qs) CHECK(q.start >= q.arrive && q.done > q.start);  // all ran
    // a heavy query never waited for a light one that arrived after it to finish
    for (const FakeQuery &h : qs) {
        if (h.cost < heavy) continue;
        for (const FakeQuery &l : qs)
            if (l.cost < heavy && l.arrive > h.arrive && l.done <= h.start) CHECK(l.start < h.start);
    }
    CHECK(arena.used() == 0);
}

int main()
{
    for (unsigned s = 1; s <= 6; ++s) test_arena(s);
    for (unsigned s = 1; s <= 6; ++s)
        for (int slots : {1, 2, 4, 8})
            for (int max_heavy : {1, 2}) test_admission(s, slots, max_heavy);
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("serve policy: all checks passed\n");
    return 0;
}
