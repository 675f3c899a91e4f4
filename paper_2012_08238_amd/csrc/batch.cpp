// Batches of uneven signals: every stage is launched once over all signals of
// the batch (workgroup -> signal through a per-launch prefix array), and the
// launch sequence is captured once into a HIP graph and replayed.
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "host.hpp"
#include "internal.hpp"
#include "kernels.hpp"
#include "steps.hpp"

using namespace sfft;

struct sfft_batch_s {
    int device = 0;
    int32_t n = 0;                 // signals (plans)
    int32_t ne = 0;                // launch entries: one per plan, two for a plan with estimation-only loops
    std::vector<int32_t> ent_plan; // entry -> signal
    std::vector<sfft_plan_t> plans;
    char* d_ws = nullptr;
    SigDesc* d_descs = nullptr;
    IoDesc* d_ios = nullptr;
    IoDesc* h_ios = nullptr;  // pinned staging of the per-run I/O pointers
    uint32_t* d_prefix = nullptr;
    std::vector<Step> steps;
    std::vector<IoDesc> last_io;
    bool io_valid = false;
    hipStream_t cap_stream = nullptr;
    // two graphs: [0] the bucketization launches, [1] every later stage, so a
    // caller can bracket the bucketization with its own events
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    hipEvent_t done = nullptr;
    hipStream_t last_stream = nullptr;
    bool launched = false;
    size_t ws_bytes = 0;
    uint32_t xcd_order = 1;
    // parallel branches: contiguous groups of signals whose stage sequences are
    // captured on separate streams of one graph, so one group's later stages
    // overlap another group's bucketization
    struct Branch {
        int32_t g0 = 0, n = 0;     // entry range
        std::vector<Step> steps;
    };
    std::vector<Branch> branches;
    std::vector<hipStream_t> bstream;
    std::vector<hipEvent_t> bjoin;
    hipEvent_t fork = nullptr;
    std::mutex mu;
};

namespace {

void batch_free(sfft_batch_t b) {
    if (!b) return;
    for (int i = 0; i < 2; ++i) {
        if (b->exec[i]) (void)hipGraphExecDestroy(b->exec[i]);
        if (b->graph[i]) (void)hipGraphDestroy(b->graph[i]);
    }
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    for (hipStream_t x : b->bstream)
        if (x) (void)hipStreamDestroy(x);
    for (hipEvent_t x : b->bjoin)
        if (x) (void)hipEventDestroy(x);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->done) (void)hipEventDestroy(b->done);
    if (b->d_ws) (void)hipFree(b->d_ws);
    if (b->d_descs) (void)hipFree(b->d_descs);
    if (b->d_ios) (void)hipFree(b->d_ios);
    if (b->d_prefix) (void)hipFree(b->d_prefix);
    if (b->h_ios) (void)hipHostFree(b->h_ios);
    delete b;
}

// part 0: bucketization steps, part 1: the others
sfft_status issue_part(sfft_batch_t b, hipStream_t s, int part) {
    const hipError_t e = issue_steps(b->steps, b->d_descs, b->d_ios, b->d_prefix, (uint32_t)b->ne, b->xcd_order, part, s);
    return e == hipSuccess ? SFFT_OK : hip_fail(e, "batched launch");
}

// Every branch on its own stream, forked from and joined back into `s`.
sfft_status issue_branches(sfft_batch_t b, hipStream_t s) {
    hipError_t e = hipEventRecord(b->fork, s);
    for (size_t g = 0; g < b->branches.size() && e == hipSuccess; ++g) {
        const auto& br = b->branches[g];
        e = hipStreamWaitEvent(b->bstream[g], b->fork, 0);
        if (e == hipSuccess)
            e = issue_steps(br.steps, b->d_descs + br.g0, b->d_ios + br.g0, b->d_prefix, (uint32_t)br.n, b->xcd_order,
                            -1, b->bstream[g]);
        if (e == hipSuccess) e = hipEventRecord(b->bjoin[g], b->bstream[g]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, b->bjoin[g], 0);
    }
    return e == hipSuccess ? SFFT_OK : hip_fail(e, "batched launch (branches)");
}

}  // namespace

extern "C" {

sfft_status sfft_batch_create(sfft_batch_t* out, const sfft_plan_t* plans, int32_t n) {
    return sfft_batch_create_ex(out, plans, n, 1);
}

sfft_status sfft_batch_create_ex(sfft_batch_t* out, const sfft_plan_t* plans, int32_t n, int32_t n_branches) {
    if (!out || !plans || n < 1) return set_error(SFFT_E_INVALID, "need an output pointer and n >= 1 plans");
    if (n_branches < 1 || n_branches > 8) return set_error(SFFT_E_INVALID, "n_branches must be in [1, 8]");
    *out = nullptr;
    for (int32_t i = 0; i < n; ++i)
        if (!plans[i]) return set_error(SFFT_E_INVALID, "null plan in batch");
    const int dev = plan_device(plans[0]);
    for (int32_t i = 1; i < n; ++i)
        if (plan_device(plans[i]) != dev) return set_error(SFFT_E_INVALID, "all plans of a batch must be on one device");
    auto* b = new (std::nothrow) sfft_batch_s();
    if (!b) return set_error(SFFT_E_NOMEM, "host allocation");
    b->device = dev;
    b->n = n;
    b->plans.assign(plans, plans + n);
    hipError_t e = hipSetDevice(dev);
    if (e != hipSuccess) {
        batch_free(b);
        return hip_fail(e, "hipSetDevice");
    }
    // launch entries: each plan, followed by its estimation-only loops (if any)
    std::vector<const Resolved*> ent;
    std::vector<int32_t> first(n + 1, 0);
    for (int32_t i = 0; i < n; ++i) {
        const Resolved& R = plan_resolved(plans[i]);
        first[i] = (int32_t)ent.size();
        ent.push_back(&R);
        b->ent_plan.push_back(i);
        if (R.est) {
            ent.push_back(R.est.get());
            b->ent_plan.push_back(i);
        }
    }
    first[n] = (int32_t)ent.size();
    const int32_t ne = (int32_t)ent.size();
    b->ne = ne;
    // one workspace per entry
    std::vector<size_t> ws_off(ne);
    size_t tot = 0;
    for (int32_t k = 0; k < ne; ++k) {
        ws_off[k] = tot;
        tot += (workspace_layout(*ent[k]).total + 255) & ~size_t(255);
    }
    b->ws_bytes = tot;
    if (hipMalloc(&b->d_ws, tot) != hipSuccess || hipMalloc(&b->d_descs, sizeof(SigDesc) * ne) != hipSuccess ||
        hipMalloc(&b->d_ios, sizeof(IoDesc) * ne) != hipSuccess ||
        hipHostMalloc(&b->h_ios, sizeof(IoDesc) * ne, hipHostMallocDefault) != hipSuccess) {
        batch_free(b);
        return set_error(SFFT_E_NOMEM, "batch allocation");
    }
    e = hipMemset(b->d_ws, 0, tot);
    if (e != hipSuccess) {
        batch_free(b);
        return hip_fail(e, "workspace clear");
    }
    std::vector<SigDesc> descs(ne);
    for (int32_t i = 0; i < n; ++i) {
        const int32_t k = first[i];
        char* tab = const_cast<char*>(plan_tables(plans[i]));
        descs[k] = make_desc(*ent[k], tab, b->d_ws + ws_off[k]);
        if (ent[k]->est) {
            descs[k + 1] = make_desc(*ent[k + 1], tab + plan_est_table_offset(plans[i]), b->d_ws + ws_off[k + 1]);
            link_est(&descs[k], b->d_descs + k + 1, *ent[k]);
        }
    }
    e = hipMemcpy(b->d_descs, descs.data(), sizeof(SigDesc) * ne, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        batch_free(b);
        return hip_fail(e, "descriptor upload");
    }
    // one launch per stage and variant, each with its own prefix over all entries
    std::vector<uint32_t> prefix;
    std::vector<const Resolved*> sig(n);
    for (int32_t i = 0; i < n; ++i) sig[i] = &plan_resolved(plans[i]);
    const int32_t nb = std::min(n_branches, n);
    if (nb == 1) {
        plan_steps(ent, &b->steps, &prefix);
    } else {
        // contiguous groups of about equal signal bytes, none empty
        std::vector<double> pre(n + 1, 0.0);
        for (int32_t i = 0; i < n; ++i) pre[i + 1] = pre[i] + (double)sig[i]->N;
        std::vector<int32_t> cut(nb + 1, 0);
        cut[nb] = n;
        for (int32_t g = 1; g < nb; ++g) {
            const double target = pre[n] * g / nb;
            int32_t c = cut[g - 1] + 1;
            while (c < n && pre[c] + 0.5 * (double)sig[c]->N <= target) ++c;
            cut[g] = std::min(c, n - (nb - g));
        }
        for (int32_t g = 0; g < nb; ++g) {
            const int32_t start = first[cut[g]], end = first[cut[g + 1]];   // signals -> entries
            sfft_batch_s::Branch br;
            br.g0 = start;
            br.n = end - start;
            std::vector<const Resolved*> part(ent.begin() + start, ent.begin() + end);
            plan_steps(part, &br.steps, &prefix);
            b->branches.push_back(std::move(br));
        }
    }
    b->xcd_order = 1;
    for (int32_t i = 0; i < n; ++i) b->xcd_order &= plan_resolved(plans[i]).xcd_order;
    if (hipMalloc(&b->d_prefix, prefix.size() * 4) != hipSuccess) {
        batch_free(b);
        return set_error(SFFT_E_NOMEM, "prefix allocation");
    }
    e = hipMemcpy(b->d_prefix, prefix.data(), prefix.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    if (e == hipSuccess && !b->branches.empty()) {
        e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
        b->bstream.assign(b->branches.size(), nullptr);
        b->bjoin.assign(b->branches.size(), nullptr);
        for (size_t g = 0; g < b->branches.size() && e == hipSuccess; ++g) {
            e = hipStreamCreateWithFlags(&b->bstream[g], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&b->bjoin[g], hipEventDisableTiming);
        }
    }
    if (e != hipSuccess) {
        batch_free(b);
        return hip_fail(e, "batch setup");
    }
    b->last_io.resize(ne);
    *out = b;
    return SFFT_OK;
}

static sfft_status batch_run(sfft_batch_t b, const void* const* x_dev, int64_t* const* out_idx,
                             void* const* out_val, double* const* out_resid, sfft_stream_t stream,
                             void* ev_fold_begin, void* ev_fold_end) {
    if (!b || !x_dev || !out_idx || !out_val) return set_error(SFFT_E_INVALID, "null argument");
    std::lock_guard<std::mutex> lk(b->mu);
    hipError_t e = hipSetDevice(b->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (b->launched && s != b->last_stream) {
        const hipError_t q = hipEventQuery(b->done);
        if (q == hipErrorNotReady) return set_error(SFFT_E_BUSY, "batch is executing on another stream");
        if (q != hipSuccess) return hip_fail(q, "hipEventQuery");
    }
    for (int32_t i = 0; i < b->n; ++i) {
        if (!x_dev[i] || !out_idx[i] || !out_val[i]) return set_error(SFFT_E_INVALID, "null signal or output pointer");
        if (reinterpret_cast<uintptr_t>(x_dev[i]) & 15u) return set_error(SFFT_E_INVALID, "x_dev must be 16-byte aligned");
    }
    // per entry (a plan's estimation-only loops read the same signal)
    std::vector<IoDesc> io(b->ne);
    for (int32_t k = 0; k < b->ne; ++k) {
        const int32_t i = b->ent_plan[k];
        io[k] = IoDesc{reinterpret_cast<const float2*>(x_dev[i]), out_idx[i], reinterpret_cast<float2*>(out_val[i]),
                       out_resid ? out_resid[i] : nullptr};
    }
    const bool same = b->io_valid && memcmp(io.data(), b->last_io.data(), sizeof(IoDesc) * b->ne) == 0;
    if (!same) {
        // the pinned staging buffer may still feed the previous run's copy
        if (b->launched) {
            e = hipEventSynchronize(b->done);
            if (e != hipSuccess) return hip_fail(e, "wait for previous batch run");
        }
        memcpy(b->h_ios, io.data(), sizeof(IoDesc) * b->ne);
        e = hipMemcpyAsync(b->d_ios, b->h_ios, sizeof(IoDesc) * b->ne, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "I/O descriptor upload");
        b->last_io = io;
        b->io_valid = true;
    }
    if (!b->branches.empty() && (ev_fold_begin || ev_fold_end))
        return set_error(SFFT_E_UNSUPPORTED, "bucketization events need a batch without branches");
    for (int part = 0; part < 2; ++part) {
        if (b->exec[part]) continue;
        if (!b->branches.empty() && part == 0) continue;   // one graph holds every branch
        if (b->branches.empty()) {
            // no graph for a part without launches (a batch of fused signals has no bucketization launch)
            bool any = false;
            for (const Step& st : b->steps) any = any || ((st.kind == kStepFold) == (part == 0));
            if (!any) continue;
        }
        e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "graph capture begin");
        const sfft_status st = b->branches.empty() ? issue_part(b, b->cap_stream, part) : issue_branches(b, b->cap_stream);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(b->cap_stream, &g);
        if (st != SFFT_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return hip_fail(e, "graph capture end");
        b->graph[part] = g;
        e = hipGraphInstantiate(&b->exec[part], g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            b->exec[part] = nullptr;
            return hip_fail(e, "graph instantiate");
        }
    }
    if (ev_fold_begin) {
        e = hipEventRecord(reinterpret_cast<hipEvent_t>(ev_fold_begin), s);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    }
    if (b->exec[0]) {
        e = hipGraphLaunch(b->exec[0], s);
        if (e != hipSuccess) return hip_fail(e, "graph launch");
    }
    if (ev_fold_end) {
        e = hipEventRecord(reinterpret_cast<hipEvent_t>(ev_fold_end), s);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    }
    if (b->exec[1]) {
        e = hipGraphLaunch(b->exec[1], s);
        if (e != hipSuccess) return hip_fail(e, "graph launch");
    }
    e = hipEventRecord(b->done, s);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    b->last_stream = s;
    b->launched = true;
    return SFFT_OK;
}

sfft_status sfft_batch_run(sfft_batch_t b, const void* const* x_dev, int64_t* const* out_idx, void* const* out_val,
                           double* const* out_resid, sfft_stream_t stream) {
    return batch_run(b, x_dev, out_idx, out_val, out_resid, stream, nullptr, nullptr);
}

sfft_status sfft_batch_run_timed(sfft_batch_t b, const void* const* x_dev, int64_t* const* out_idx,
                                 void* const* out_val, double* const* out_resid, sfft_stream_t stream,
                                 void* ev_fold_begin, void* ev_fold_end) {
    return batch_run(b, x_dev, out_idx, out_val, out_resid, stream, ev_fold_begin, ev_fold_end);
}

sfft_status sfft_batch_destroy(sfft_batch_t b) {
    if (!b) return set_error(SFFT_E_INVALID, "null batch");
    (void)hipSetDevice(b->device);
    if (b->launched) (void)hipEventSynchronize(b->done);
    batch_free(b);
    return SFFT_OK;
}

sfft_status sfft_execute_batch(const sfft_plan_t* plans, const void* const* x_dev, int64_t* const* out_idx,
                               void* const* out_val, double* const* out_resid, int32_t n, sfft_stream_t stream) {
    sfft_batch_t b = nullptr;
    sfft_status st = sfft_batch_create(&b, plans, n);
    if (st != SFFT_OK) return st;
    st = sfft_batch_run(b, x_dev, out_idx, out_val, out_resid, stream);
    sfft_batch_destroy(b);
    return st;
}

}  // extern "C"
