// Host test of the serving scheduler against a fake device: every wave the
// fake runs is checked for overlapping arena ranges, stale plan tables, the
// in-flight limit and the arena budget. Built with g++ (no HIP) by
// tests/test_serve_core.py.
#include <stdio.h>
#include <stdlib.h>

#include <atomic>
#include <chrono>
#include <map>
#include <mutex>
#include <random>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "../../paper_2012_08238_amd/csrc/serve_core.hpp"

using namespace sfft::serve;

static int g_fail = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            fprintf(stderr, "%s:%d: CHECK failed: %s\n", __FILE__, __LINE__, #c); \
            ++g_fail;                                                         \
        }                                                                     \
    } while (0)

struct Io {
    int tag = 0;       // 1: the fake fails the wave containing this request
    int expect_plan = 0;
};

using Clock = std::chrono::steady_clock;

// Fake device: a wave occupies its slot for base + per_item * n microseconds.
class FakeExec : public Executor<Io> {
public:
    FakeExec(int slots, size_t arena, std::map<uint32_t, size_t> tab, std::map<uint32_t, size_t> ws,
             int base_us, int per_item_us)
        : arena_(arena), tab_(tab), ws_(ws), base_(base_us), per_(per_item_us), slot_(slots) {}

    int upload(uint32_t plan, size_t off) override {
        std::lock_guard<std::mutex> lk(mu_);
        CHECK(off + tab_.at(plan) <= arena_);
        // the range must not overlap a range a running wave uses
        for (const auto& s : slot_)
            for (const auto& r : s.ranges) CHECK(off + tab_.at(plan) <= r.first || r.second <= off);
        // tables it overwrites are gone
        for (auto it = content_.begin(); it != content_.end();) {
            const size_t a = it->first, b = a + tab_.at(it->second);
            if (!(off + tab_.at(plan) <= a || b <= off)) it = content_.erase(it);
            else ++it;
        }
        content_[off] = plan;
        ++uploads;
        return 0;
    }

    int launch(int s, const std::vector<WaveItem<Io>>& items) override {
        std::lock_guard<std::mutex> lk(mu_);
        CHECK(!slot_[s].busy);
        std::vector<std::pair<size_t, size_t>> ranges;
        std::set<uint32_t> plans;
        bool fail = false;
        for (const auto& it : items) {
            CHECK((int)it.plan == it.io.expect_plan);
            auto c = content_.find(it.tab_off);
            CHECK(c != content_.end() && c->second == it.plan);   // tables present and current
            CHECK(it.ws_off + ws_.at(it.plan) <= arena_);
            ranges.emplace_back(it.ws_off, it.ws_off + ws_.at(it.plan));
            plans.insert(it.plan);
            if (it.io.tag == 1) fail = true;
        }
        for (uint32_t p : plans) {
            size_t off = 0;
            for (const auto& it : items)
                if (it.plan == p) off = it.tab_off;
            ranges.emplace_back(off, off + tab_.at(p));
        }
        // workspaces of this wave and of running waves never overlap each other or tables in use
        std::vector<std::pair<size_t, size_t>> all = ranges;
        size_t inflight = items.size();
        for (const auto& o : slot_)
            if (o.busy) {
                all.insert(all.end(), o.ranges.begin(), o.ranges.end());
                inflight += o.n;
            }
        for (size_t i = 0; i < items.size(); ++i)
            for (size_t j = 0; j < all.size(); ++j) {
                if (j == i) continue;
                const auto& a = all[i];
                const auto& b = all[j];
                // identical table ranges of one plan may be shared
                if (j >= items.size() && a == b) continue;
                CHECK(a.second <= b.first || b.second <= a.first);
            }
        size_t bytes = 0;
        {
            std::set<std::pair<size_t, size_t>> uniq(all.begin(), all.end());
            for (const auto& r : uniq) bytes += r.second - r.first;
        }
        CHECK(bytes <= arena_);
        // a workspace clobbers whatever tables lay in its range
        for (const auto& it : items) {
            const size_t a = it.ws_off, b = a + ws_.at(it.plan);
            for (auto c = content_.begin(); c != content_.end();) {
                const size_t x = c->first, y = x + tab_.at(c->second);
                if (!(b <= x || y <= a)) c = content_.erase(c);
                else ++c;
            }
        }
        if (inflight > max_inflight_seen) max_inflight_seen = inflight;
        if (items.size() > max_wave) max_wave = items.size();
        if (fail) return -3;
        slot_[s].busy = true;
        slot_[s].n = items.size();
        slot_[s].ranges = ranges;
        slot_[s].until = Clock::now() + std::chrono::microseconds(base_ + per_ * (int)items.size());
        ++waves;
        return 0;
    }

    int query(int s) override {
        std::lock_guard<std::mutex> lk(mu_);
        if (!slot_[s].busy) return 1;
        if (hold.load() || Clock::now() < slot_[s].until) return 0;
        slot_[s].busy = false;
        slot_[s].ranges.clear();
        slot_[s].n = 0;
        return 1;
    }

    std::atomic<size_t> uploads{0}, waves{0}, max_wave{0}, max_inflight_seen{0};
    std::atomic<bool> hold{false};   // while set, no wave completes

private:
    struct Slot {
        bool busy = false;
        size_t n = 0;
        std::vector<std::pair<size_t, size_t>> ranges;
        Clock::time_point until;
    };
    std::mutex mu_;
    size_t arena_;
    std::map<uint32_t, size_t> tab_, ws_;
    int base_, per_;
    std::vector<Slot> slot_;
    std::map<size_t, uint32_t> content_;  // arena offset -> plan whose tables are there
};

static void test_allocator() {
    std::mt19937_64 rng(7);
    const size_t unit = 256, cap = 64 * unit;
    RangeAllocator a(cap, unit);
    std::vector<bool> used(64, false);
    std::vector<std::pair<size_t, size_t>> live;
    for (int step = 0; step < 20000; ++step) {
        if (live.empty() || rng() % 2) {
            const size_t n = 1 + rng() % (6 * unit);
            size_t off = 0;
            const size_t k = (n + unit - 1) / unit;
            // first fit by brute force
            long want = -1;
            for (size_t i = 0; i + k <= 64 && want < 0; ++i) {
                bool ok = true;
                for (size_t j = 0; j < k; ++j) ok = ok && !used[i + j];
                if (ok) want = (long)i;
            }
            const bool got = a.alloc(n, &off);
            CHECK(got == (want >= 0));
            if (got) {
                CHECK(off == (size_t)want * unit);
                for (size_t j = 0; j < k; ++j) used[off / unit + j] = true;
                live.emplace_back(off, n);
            }
        } else {
            const size_t i = rng() % live.size();
            a.release(live[i].first, live[i].second);
            const size_t k = (live[i].second + unit - 1) / unit;
            for (size_t j = 0; j < k; ++j) used[live[i].first / unit + j] = false;
            live.erase(live.begin() + (long)i);
        }
        size_t u = 0;
        for (bool b : used) u += b;
        CHECK(a.in_use() == u * unit);
    }
    for (auto& l : live) a.release(l.first, l.second);
    CHECK(a.in_use() == 0 && a.free_ranges() == 1 && a.largest_free() == cap);
}

// Polls pred every 100 us for up to 20 s.
template <class F>
static bool wait_until(F pred) {
    for (int i = 0; i < 200000; ++i) {
        if (pred()) return true;
        std::this_thread::sleep_for(std::chrono::microseconds(100));
    }
    return false;
}

struct Env {
    std::map<uint32_t, size_t> tab, ws;
};

static void test_batching_and_overlap() {
    Env e;
    e.tab = {{1, 1000}, {2, 3000}};
    e.ws = {{1, 5000}, {2, 9000}};
    const size_t arena = 1 << 20;
    FakeExec ex(2, arena, e.tab, e.ws, 3000, 20);
    ServerCore<Io> core(&ex, arena, 64, 2, 64);
    core.add_plan(1, e.tab[1]);
    core.add_plan(2, e.tab[2]);
    std::vector<uint64_t> t;
    uint64_t k = 0;
    // waves stay in flight until released, so the later arrivals meet the first wave running
    // (no dependence on how fast the scheduler thread runs)
    ex.hold = true;
    CHECK(core.submit(1, e.ws[1], Io{0, 1}, &k) == kCoreOk);
    t.push_back(k);
    CHECK(wait_until([&] { return ex.waves.load() >= 1; }));   // first wave is running
    for (int i = 0; i < 40; ++i) {
        const uint32_t p = 1 + i % 2;
        CHECK(core.submit(p, e.ws[p], Io{0, (int)p}, &k) == kCoreOk);
        t.push_back(k);
    }
    CHECK(wait_until([&] { return ex.waves.load() >= 2; }));   // a second wave beside it
    ex.hold = false;
    for (uint64_t x : t) {
        double lat = -1;
        int st = 1;
        CHECK(core.wait(x, &lat, &st) == kCoreOk);
        CHECK(st == 0 && lat > 0);
    }
    const CoreStats s = core.stats();
    CHECK(s.completed == 41 && s.failed == 0 && s.submitted == 41);
    CHECK(s.waves < 10);                 // later arrivals were batched
    CHECK(s.max_busy_slots == 2);        // and ran beside the wave in flight
    CHECK(ex.max_wave >= 10);
    CHECK(s.misses == 2 && s.evictions == 0);   // each plan uploaded once, then resident
    CHECK(s.in_use == 1024 + 3072);      // the two resident tables, rounded to 256 B
    CHECK(s.p50 > 0 && s.p99 >= s.p50);
    double lat;
    int st;
    CHECK(core.poll(t[0], nullptr, &lat, &st) == kCoreNotFound);  // released by wait
}

static void test_budget_and_eviction() {
    Env e;
    e.tab = {{1, 4096}, {2, 4096}, {3, 4096}};
    e.ws = {{1, 8192}, {2, 8192}, {3, 8192}};
    // room for one table and two workspaces, or two tables and one workspace
    const size_t arena = 4096 + 2 * 8192;
    FakeExec ex(3, arena, e.tab, e.ws, 400, 10);
    ServerCore<Io> core(&ex, arena, 16, 3, 16);
    for (uint32_t p = 1; p <= 3; ++p) core.add_plan(p, e.tab[p]);
    std::vector<uint64_t> t;
    for (int i = 0; i < 60; ++i) {
        const uint32_t p = 1 + (i / 3) % 3;
        uint64_t k = 0;
        CHECK(core.submit(p, e.ws[p], Io{0, (int)p}, &k) == kCoreOk);
        t.push_back(k);
    }
    for (uint64_t x : t) {
        int st = 1;
        CHECK(core.wait(x, nullptr, &st) == kCoreOk && st == 0);
    }
    const CoreStats s = core.stats();
    CHECK(s.completed == 60);
    CHECK(s.peak <= arena);
    CHECK(s.evictions > 0);
    CHECK(ex.uploads == s.misses);
    // a request that can never fit is refused at once
    uint64_t k;
    CHECK(core.submit(1, arena, Io{0, 1}, &k) == kCoreNoMem);
    CHECK(core.submit(9, 16, Io{0, 9}, &k) == kCoreNotFound);
    CHECK(core.stats().rejected == 2);
}

static void test_inflight_limit_and_failure() {
    Env e;
    e.tab = {{1, 512}};
    e.ws = {{1, 1024}};
    const size_t arena = 1 << 16;
    FakeExec ex(4, arena, e.tab, e.ws, 1000, 10);
    ServerCore<Io> core(&ex, arena, 3, 4, 8);
    core.add_plan(1, e.tab[1]);
    std::vector<uint64_t> t;
    for (int i = 0; i < 30; ++i) {
        uint64_t k = 0;
        CHECK(core.submit(1, e.ws[1], Io{i == 17 ? 1 : 0, 1}, &k) == kCoreOk);
        t.push_back(k);
    }
    int failed = 0;
    for (size_t i = 0; i < t.size(); ++i) {
        int st = 0;
        CHECK(core.wait(t[i], nullptr, &st) == kCoreOk);
        if (st != 0) {
            ++failed;
            CHECK(st == -3);
        }
    }
    CHECK(ex.max_inflight_seen <= 3);
    CHECK(failed >= 1 && failed <= 3);   // only the wave holding request 17 fails
    const CoreStats s = core.stats();
    CHECK(s.failed == (uint64_t)failed && s.completed == 30 - (uint64_t)failed);
    CHECK(s.in_use == 512);   // only the resident table remains
}

static void test_concurrent_clients() {
    Env e;
    for (uint32_t p = 1; p <= 5; ++p) {
        e.tab[p] = 1000 * p;
        e.ws[p] = 3000 + 777 * p;
    }
    const size_t arena = 40000;
    FakeExec ex(3, arena, e.tab, e.ws, 200, 5);
    ServerCore<Io> core(&ex, arena, 12, 3, 6);
    for (uint32_t p = 1; p <= 5; ++p) core.add_plan(p, e.tab[p]);
    std::atomic<int> done{0}, bad{0};
    std::vector<std::thread> th;
    for (int c = 0; c < 4; ++c)
        th.emplace_back([&, c] {
            std::mt19937 rng(100 + c);
            std::vector<uint64_t> mine;
            for (int i = 0; i < 150; ++i) {
                const uint32_t p = 1 + rng() % 5;
                uint64_t k = 0;
                if (c == 3 && i % 3 == 0) {   // this client queues bursts of three with one call
                    const Io io[3] = {Io{0, (int)p}, Io{0, (int)p}, Io{0, (int)p}};
                    uint64_t ks[3];
                    if (core.submit_many(p, e.ws[p], io, 3, ks) != kCoreOk) ++bad;
                    mine.push_back(ks[0]);
                    mine.push_back(ks[1]);
                    k = ks[2];
                    i += 2;
                } else if (core.submit(p, e.ws[p], Io{0, (int)p}, &k) != kCoreOk) {
                    ++bad;
                }
                mine.push_back(k);
                if (rng() % 4 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 300));
                if (mine.size() > 5) {
                    int st = 1;
                    if (core.wait(mine.front(), nullptr, &st) != kCoreOk || st != 0) ++bad;
                    mine.erase(mine.begin());
                    ++done;
                }
            }
            for (uint64_t k : mine) {
                int st = 1;
                if (core.wait(k, nullptr, &st) != kCoreOk || st != 0) ++bad;
                ++done;
            }
        });
    for (auto& x : th) x.join();
    CHECK(bad == 0 && done == 600);
    const CoreStats s = core.stats();
    CHECK(s.completed == 600 && s.peak <= arena && ex.max_inflight_seen <= 12 && ex.max_wave <= 6);
}

static void test_drain_on_stop() {
    Env e;
    e.tab = {{1, 256}};
    e.ws = {{1, 256}};
    FakeExec ex(1, 1 << 14, e.tab, e.ws, 300, 1);
    auto* core = new ServerCore<Io>(&ex, 1 << 14, 4, 1, 2);
    core->add_plan(1, 256);
    std::vector<uint64_t> t(20);
    for (auto& k : t) CHECK(core->submit(1, 256, Io{0, 1}, &k) == kCoreOk);
    core->stop();   // returns once everything queued has run
    const CoreStats s = core->stats();
    CHECK(s.completed == 20);
    for (auto k : t) {
        int done = 0;
        CHECK(core->poll(k, &done, nullptr, nullptr) == kCoreOk && done == 1);
    }
    delete core;
}

static void test_submit_many() {
    Env e;
    e.tab = {{1, 512}};
    e.ws = {{1, 2048}};
    const size_t arena = 1 << 16;
    FakeExec ex(2, arena, e.tab, e.ws, 500, 1);
    ServerCore<Io> core(&ex, arena, 16, 2, 16);
    core.add_plan(1, 512);
    std::vector<Io> io(40, Io{0, 1});
    std::vector<uint64_t> t(40, 0);
    // all or none: an unknown plan or one that can never fit queues nothing
    CHECK(core.submit_many(7, 2048, io.data(), io.size(), t.data()) == kCoreNotFound);
    CHECK(core.submit_many(1, arena, io.data(), io.size(), t.data()) == kCoreNoMem);
    CHECK(core.stats().submitted == 0);
    CHECK(core.submit_many(1, 2048, io.data(), 0, t.data()) == kCoreOk);
    CHECK(core.submit_many(1, 2048, io.data(), io.size(), t.data()) == kCoreOk);
    for (size_t i = 1; i < t.size(); ++i) CHECK(t[i] == t[i - 1] + 1);   // tickets in submission order
    for (uint64_t x : t) {
        int st = 1;
        CHECK(core.wait(x, nullptr, &st) == kCoreOk && st == 0);
    }
    const CoreStats s = core.stats();
    CHECK(s.completed == 40 && s.submitted == 40 && s.rejected == 80);
    CHECK(ex.max_inflight_seen <= 16 && s.peak <= arena);
}

int main() {
    test_allocator();
    test_submit_many();
    test_batching_and_overlap();
    test_budget_and_eviction();
    test_inflight_limit_and_failure();
    test_concurrent_clients();
    test_drain_on_stop();
    if (g_fail) {
        fprintf(stderr, "%d checks failed\n", g_fail);
        return 1;
    }
    printf("serve_core_test: all checks passed\n");
    return 0;
}
