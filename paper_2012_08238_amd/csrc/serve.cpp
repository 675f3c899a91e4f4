// Serving loop on the device: the scheduler of serve_core.hpp driving an
// executor that runs every wave of admitted requests as the batched stage
// launches of steps.hpp on one of its streams. Plan tables and request
// workspaces live in one device arena of the server's memory budget.
#include <string.h>

#include <algorithm>
#include <atomic>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "common.hpp"
#include "host.hpp"
#include "internal.hpp"
#include "serve_core.hpp"
#include "steps.hpp"

using namespace sfft;

namespace {

constexpr int kMaxInflight = 1024;
constexpr int kMaxStreams = 16;

struct ServedPlan {
    Resolved R;
    std::vector<char> image;  // device table image (table_layout order), then the estimation-only loops' at tab_e
    size_t ws_bytes = 0;      // workspace, then the estimation-only loops' at ws_e
    size_t tab_e = 0, ws_e = 0;
};

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

class HipExecutor final : public serve::Executor<IoDesc> {
public:
    HipExecutor(int device, char* arena, int slots, int max_wave)
        : device_(device), arena_(arena), max_wave_(max_wave), slots_(slots) {}

    ~HipExecutor() override {
        for (Slot& s : slots_) {
            if (s.stream) (void)hipStreamSynchronize(s.stream);
            if (s.done) (void)hipEventDestroy(s.done);
            if (s.stream) (void)hipStreamDestroy(s.stream);
            if (s.h_stage) (void)hipHostFree(s.h_stage);
            if (s.d_stage) (void)hipFree(s.d_stage);
        }
    }

    sfft_status init() {
        // a request takes two launch entries when its plan has estimation-only loops
        const size_t me = 2 * (size_t)max_wave_;
        stage_bytes_ = align256(sizeof(SigDesc) * me) + align256(sizeof(IoDesc) * me) + max_prefix_entries(me) * 4;
        for (Slot& s : slots_) {
            if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess)
                return set_error(SFFT_E_DEVICE, "server stream setup");
            if (hipHostMalloc(&s.h_stage, stage_bytes_, hipHostMallocDefault) != hipSuccess ||
                hipMalloc(&s.d_stage, stage_bytes_) != hipSuccess)
                return set_error(SFFT_E_NOMEM, "server staging buffers");
        }
        return SFFT_OK;
    }

    void thread_init() override { (void)hipSetDevice(device_); }

    int upload(uint32_t plan, size_t off) override {
        const ServedPlan* p = get(plan);
        const hipError_t e = hipMemcpy(arena_ + off, p->image.data(), p->image.size(), hipMemcpyHostToDevice);
        return e == hipSuccess ? 0 : (int)SFFT_E_DEVICE;
    }

    int launch(int slot, const std::vector<serve::WaveItem<IoDesc>>& items) override {
        Slot& sl = slots_[slot];
        const size_t nreq = items.size();
        if (nreq == 0 || nreq > (size_t)max_wave_) return SFFT_E_INVALID;
        // launch entries: each request, followed by its plan's estimation-only loops (if any)
        size_t n = 0;
        for (size_t i = 0; i < nreq; ++i) n += get(items[i].plan)->R.est ? 2 : 1;
        std::vector<const Resolved*> sig(n);
        uint32_t xcd = 1;
        const size_t o_io = align256(sizeof(SigDesc) * n);
        const size_t o_pre = o_io + align256(sizeof(IoDesc) * n);
        SigDesc* hd = reinterpret_cast<SigDesc*>(sl.h_stage);
        IoDesc* hi = reinterpret_cast<IoDesc*>(sl.h_stage + o_io);
        for (size_t i = 0, k = 0; i < nreq; ++i) {
            const ServedPlan* p = get(items[i].plan);
            sig[k] = &p->R;
            xcd &= p->R.xcd_order;
            hd[k] = make_desc(p->R, arena_ + items[i].tab_off, arena_ + items[i].ws_off);
            hi[k] = items[i].io;
            if (p->R.est) {
                sig[k + 1] = p->R.est.get();
                hd[k + 1] = make_desc(*p->R.est, arena_ + items[i].tab_off + p->tab_e, arena_ + items[i].ws_off + p->ws_e);
                hi[k + 1] = items[i].io;
                link_est(&hd[k], reinterpret_cast<const SigDesc*>(sl.d_stage) + k + 1, p->R);
                ++k;
            }
            ++k;
        }
        // A lone request reads only its descriptors from the staging buffer (its I/O pointers
        // travel as kernel arguments) and needs no stage plan. Bytes the buffer already holds
        // (the slot's previous wave staged the same descriptors: same plan, same arena
        // placement) are not copied again: the copy is a device launch of its own on the
        // request's path.
        std::vector<Step> steps;
        std::vector<uint32_t> prefix;
        size_t need = sizeof(SigDesc) * n;
        if (nreq > 1) {
            plan_steps(sig, &steps, &prefix);
            need = o_pre + prefix.size() * 4;
            if (need > stage_bytes_) return SFFT_E_INVALID;
            memcpy(sl.h_stage + o_pre, prefix.data(), prefix.size() * 4);
        }
        hipError_t e = hipSuccess;
        if (!(need <= sl.held.size() && memcmp(sl.held.data(), sl.h_stage, need) == 0)) {
            e = hipMemcpyAsync(sl.d_stage, sl.h_stage, need, hipMemcpyHostToDevice, sl.stream);
            if (e == hipSuccess) sl.held.assign(sl.h_stage, sl.h_stage + need);
            else sl.held.clear();
        }
        if (e == hipSuccess && nreq == 1) {
            // a lone request takes the single-signal launch sequence (as sfft_execute_ex; its
            // residual is one launch instead of two)
            if (launch_single(*sig[0], reinterpret_cast<const SigDesc*>(sl.d_stage), items[0].io, sl.stream) != SFFT_OK)
                e = hipErrorLaunchFailure;
        } else if (e == hipSuccess) {
            e = issue_steps(steps, reinterpret_cast<const SigDesc*>(sl.d_stage),
                            reinterpret_cast<const IoDesc*>(sl.d_stage + o_io),
                            reinterpret_cast<const uint32_t*>(sl.d_stage + o_pre), (uint32_t)n, xcd, -1, sl.stream);
        }
        if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
        if (e != hipSuccess) {
            // the staging buffer is reused by the slot's next wave: let this one drain first
            sl.held.clear();
            (void)hipStreamSynchronize(sl.stream);
            return SFFT_E_DEVICE;
        }
        return 0;
    }

    int query(int slot) override {
        const hipError_t q = hipEventQuery(slots_[slot].done);
        if (q == hipSuccess) return 1;
        if (q == hipErrorNotReady) return 0;
        return SFFT_E_DEVICE;
    }

    uint32_t add(std::unique_ptr<ServedPlan> p) {
        std::lock_guard<std::mutex> lk(mu_);
        plans_.push_back(std::move(p));
        return (uint32_t)plans_.size() - 1;
    }
    const ServedPlan* get(uint32_t id) {
        std::lock_guard<std::mutex> lk(mu_);
        return plans_[id].get();
    }

private:
    struct Slot {
        hipStream_t stream = nullptr;
        hipEvent_t done = nullptr;
        char* h_stage = nullptr;  // pinned: descriptors, I/O pointers, prefixes of one wave
        char* d_stage = nullptr;
        std::vector<char> held;   // the leading bytes d_stage is known to hold
    };
    int device_;
    char* arena_;
    int max_wave_;
    size_t stage_bytes_ = 0;
    std::vector<Slot> slots_;
    std::mutex mu_;
    std::vector<std::unique_ptr<ServedPlan>> plans_;  // id = index; entries never move or die
};

std::string plan_key(const sfft_params& p) {
    std::string k;
    auto put = [&](const void* v, size_t n) { k.append(reinterpret_cast<const char*>(v), n); };
    put(&p.N, 8);
    put(&p.K, 4);
    put(&p.B, 4);
    put(&p.L, 4);
    put(&p.d, 4);
    put(&p.w, 8);
    put(&p.seed, 8);
    put(&p.vote_threshold, 4);
    put(&p.n_resid, 4);
    put(&p.gauss_c, 8);
    put(&p.flags, 4);
    put(&p.strip_cols, 4);
    put(&p.comb_b, 4);
    put(&p.comb_loops, 4);
    put(&p.comb_keep, 4);
    put(&p.est_loops, 4);
    put(&p.est_B, 4);
    put(&p.est_w, 8);
    const int32_t has = p.sigma != nullptr;
    put(&has, 4);
    if (p.sigma && p.tau && p.L > 0 && p.L <= kMaxL) {
        put(p.sigma, (size_t)p.L * 4);
        put(p.tau, (size_t)p.L * 4);
    }
    return k;
}

}  // namespace

struct sfft_server_s {
    int device = 0;
    char* arena = nullptr;
    size_t budget = 0;
    std::unique_ptr<HipExecutor> ex;
    std::unique_ptr<serve::ServerCore<IoDesc>> core;
    std::mutex cache_mu;
    std::unordered_map<std::string, uint32_t> cache;  // parameter set -> plan id
    std::atomic<uint64_t> invalid{0};
};

namespace {

void server_free(sfft_server_t s) {
    if (!s) return;
    if (s->core) s->core->stop();
    s->core.reset();
    s->ex.reset();
    if (s->arena) (void)hipFree(s->arena);
    delete s;
}

// Plan id of a parameter set, building and registering its tables on first use.
sfft_status served_plan(sfft_server_t s, const sfft_params& p, uint32_t* id, size_t* ws_bytes) {
    const std::string key = plan_key(p);
    std::lock_guard<std::mutex> lk(s->cache_mu);
    auto it = s->cache.find(key);
    if (it != s->cache.end()) {
        *id = it->second;
        *ws_bytes = s->ex->get(*id)->ws_bytes;
        return SFFT_OK;
    }
    auto sp = std::make_unique<ServedPlan>();
    std::string err;
    const sfft_status st = resolve_params(p, &sp->R, &err);
    if (st != SFFT_OK) return set_error(st, err);
    HostTables T;
    build_tables(sp->R, &T);
    sp->image = pack_tables(sp->R, T);
    sp->ws_bytes = workspace_layout(sp->R).total;
    if (sp->R.est) {
        HostTables Te;
        build_tables(*sp->R.est, &Te);
        const std::vector<char> he = pack_tables(*sp->R.est, Te);
        sp->tab_e = align256(sp->image.size());
        sp->image.resize(sp->tab_e, 0);
        sp->image.insert(sp->image.end(), he.begin(), he.end());
        sp->ws_e = align256(sp->ws_bytes);
        sp->ws_bytes = sp->ws_e + workspace_layout(*sp->R.est).total;
    }
    const size_t tab = sp->image.size(), ws = sp->ws_bytes;
    if (align256(tab) + align256(ws) > s->core->arena_capacity())
        return set_error(SFFT_E_NOMEM, "request needs " + std::to_string(align256(tab) + align256(ws)) +
                                           " bytes of device memory, more than the server budget");
    *id = s->ex->add(std::move(sp));
    s->core->add_plan(*id, tab);
    s->cache.emplace(key, *id);
    *ws_bytes = ws;
    return SFFT_OK;
}

sfft_status core_status(int rc) {
    switch (rc) {
        case serve::kCoreOk: return SFFT_OK;
        case serve::kCoreNoMem: return set_error(SFFT_E_NOMEM, "request can never fit the server budget");
        case serve::kCoreNotFound: return set_error(SFFT_E_NOTFOUND, "unknown ticket");
        default: return set_error(SFFT_E_INVALID, "server request refused");
    }
}

}  // namespace

extern "C" {

sfft_status sfft_server_create(sfft_server_t* out, size_t hbm_budget_bytes, int32_t max_inflight, int32_t n_streams) {
    if (!out) return set_error(SFFT_E_INVALID, "null output pointer");
    *out = nullptr;
    if (max_inflight < 1 || max_inflight > kMaxInflight)
        return set_error(SFFT_E_INVALID, "max_inflight must be in [1, 1024]");
    if (n_streams < 1 || n_streams > kMaxStreams) return set_error(SFFT_E_INVALID, "n_streams must be in [1, 16]");
    if (hbm_budget_bytes < (size_t(1) << 20)) return set_error(SFFT_E_INVALID, "hbm_budget_bytes below 1 MiB");
    auto* s = new (std::nothrow) sfft_server_s();
    if (!s) return set_error(SFFT_E_NOMEM, "host allocation");
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = init_kernel_attributes();
    if (e != hipSuccess) {
        server_free(s);
        return hip_fail(e, "server device setup");
    }
    s->budget = hbm_budget_bytes;
    if (hipMalloc(&s->arena, hbm_budget_bytes) != hipSuccess) {
        s->arena = nullptr;
        server_free(s);
        return set_error(SFFT_E_NOMEM, "server arena of hbm_budget_bytes");
    }
    s->ex = std::make_unique<HipExecutor>(s->device, s->arena, n_streams, max_inflight);
    const sfft_status st = s->ex->init();
    if (st != SFFT_OK) {
        server_free(s);
        return st;
    }
    // a wave takes at most max_inflight / n_streams requests, so that under a burst every stream
    // holds a wave and consecutive waves overlap (as steps in flight do) instead of one stream
    // running everything admitted
    const int32_t wave = std::max<int32_t>(1, (max_inflight + n_streams - 1) / n_streams);
    s->core = std::make_unique<serve::ServerCore<IoDesc>>(s->ex.get(), hbm_budget_bytes, max_inflight, n_streams,
                                                         wave);
    *out = s;
    return SFFT_OK;
}

sfft_status sfft_server_prepare(sfft_server_t s, const sfft_params* p) {
    if (!s || !p) return set_error(SFFT_E_INVALID, "null argument");
    uint32_t id;
    size_t ws;
    const sfft_status st = served_plan(s, *p, &id, &ws);
    if (st == SFFT_E_INVALID) s->invalid++;
    return st;
}

sfft_status sfft_server_submit(sfft_server_t s, const sfft_params* p, const void* x_dev, int64_t* out_idx,
                               void* out_val, double* out_resid, uint64_t* ticket) {
    if (!s || !p || !x_dev || !out_idx || !out_val || !ticket) {
        if (s) s->invalid++;
        return set_error(SFFT_E_INVALID, "null argument");
    }
    if ((reinterpret_cast<uintptr_t>(x_dev) & 15u) || (reinterpret_cast<uintptr_t>(out_idx) & 7u) ||
        (reinterpret_cast<uintptr_t>(out_val) & 7u) || (reinterpret_cast<uintptr_t>(out_resid) & 7u)) {
        s->invalid++;
        return set_error(SFFT_E_INVALID, "x_dev must be 16-byte and outputs 8-byte aligned");
    }
    uint32_t id;
    size_t ws;
    sfft_status st = served_plan(s, *p, &id, &ws);
    if (st != SFFT_OK) {
        s->invalid++;
        return st;
    }
    const IoDesc io{reinterpret_cast<const float2*>(x_dev), out_idx, reinterpret_cast<float2*>(out_val), out_resid};
    return core_status(s->core->submit(id, ws, io, ticket));
}

sfft_status sfft_server_submit_batch(sfft_server_t s, const sfft_params* p, int32_t n, const void* const* x_dev,
                                     int64_t* const* out_idx, void* const* out_val, double* const* out_resid,
                                     uint64_t* tickets) {
    if (!s || !p || n < 0 || (n > 0 && (!x_dev || !out_idx || !out_val || !tickets))) {
        if (s) s->invalid += n > 0 ? (uint64_t)n : 1u;
        return set_error(SFFT_E_INVALID, "null argument or n < 0");
    }
    std::vector<IoDesc> io((size_t)n);
    for (int32_t i = 0; i < n; ++i) {
        double* res = out_resid ? out_resid[i] : nullptr;
        if (!x_dev[i] || !out_idx[i] || !out_val[i] || (reinterpret_cast<uintptr_t>(x_dev[i]) & 15u) ||
            (reinterpret_cast<uintptr_t>(out_idx[i]) & 7u) || (reinterpret_cast<uintptr_t>(out_val[i]) & 7u) ||
            (reinterpret_cast<uintptr_t>(res) & 7u)) {
            s->invalid += (uint64_t)n;
            return set_error(SFFT_E_INVALID, "request " + std::to_string(i) +
                                                 ": null pointer, or x_dev not 16-byte / outputs not 8-byte aligned");
        }
        io[i] = IoDesc{reinterpret_cast<const float2*>(x_dev[i]), out_idx[i], reinterpret_cast<float2*>(out_val[i]),
                       res};
    }
    if (n == 0) return SFFT_OK;
    uint32_t id;
    size_t ws;
    const sfft_status st = served_plan(s, *p, &id, &ws);
    if (st != SFFT_OK) {
        s->invalid += (uint64_t)n;
        return st;
    }
    return core_status(s->core->submit_many(id, ws, io.data(), io.size(), tickets));
}

sfft_status sfft_server_poll(sfft_server_t s, uint64_t ticket, int32_t* done, double* latency_s, int32_t* req_status) {
    if (!s) return set_error(SFFT_E_INVALID, "null server");
    int d = 0, rs = 0;
    double lat = 0;
    const int rc = s->core->poll(ticket, &d, &lat, &rs);
    if (rc != serve::kCoreOk) return core_status(rc);
    if (done) *done = d;
    if (latency_s) *latency_s = lat;
    if (req_status) *req_status = rs;
    return SFFT_OK;
}

sfft_status sfft_server_wait(sfft_server_t s, uint64_t ticket, double* latency_s, int32_t* req_status) {
    if (!s) return set_error(SFFT_E_INVALID, "null server");
    int rs = 0;
    double lat = 0;
    const int rc = s->core->wait(ticket, &lat, &rs);
    if (rc != serve::kCoreOk) return core_status(rc);
    if (latency_s) *latency_s = lat;
    if (req_status) *req_status = rs;
    return SFFT_OK;
}

sfft_status sfft_server_stats_get(sfft_server_t s, sfft_server_stats* out) {
    if (!s || !out) return set_error(SFFT_E_INVALID, "null argument");
    const serve::CoreStats c = s->core->stats();
    memset(out, 0, sizeof(*out));
    out->submitted = c.submitted;
    out->completed = c.completed;
    out->rejected = c.rejected + s->invalid.load();
    out->failed = c.failed;
    out->batches = c.waves;
    out->max_batch = c.max_wave_seen;
    out->max_waves_in_flight = c.max_busy_slots;
    out->p50_latency_s = c.p50;
    out->p99_latency_s = c.p99;
    out->mean_latency_s = c.mean;
    out->hbm_in_use = c.in_use;
    out->hbm_peak = c.peak;
    out->hbm_budget = s->budget;
    out->plan_cache_hits = c.hits;
    out->plan_cache_misses = c.misses;
    out->plan_cache_evictions = c.evictions;
    return SFFT_OK;
}

sfft_status sfft_server_destroy(sfft_server_t s) {
    if (!s) return set_error(SFFT_E_INVALID, "null server");
    (void)hipSetDevice(s->device);
    server_free(s);
    return SFFT_OK;
}

}  // extern "C"
