// C ABI of the gfx950 sparse FFT: plans, single execution, batches, traces.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "host.hpp"
#include "internal.hpp"
#include "kernels.hpp"

namespace sfft {

thread_local std::string g_last_error;

sfft_status set_error(sfft_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

sfft_status hip_fail(hipError_t e, const char* what) {
    return set_error(SFFT_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                       \
    do {                                          \
        hipError_t _e = (expr);                   \
        if (_e != hipSuccess) return hip_fail(_e, what); \
    } while (0)

hipError_t init_kernel_attributes() {
    static std::once_flag once;
    static hipError_t status = hipSuccess;
    std::call_once(once, [] { status = set_kernel_attributes_impl(); });
    return status;
}

// Fill a device descriptor with the plan tables at `tab` and the workspace at `ws`.
SigDesc make_desc(const Resolved& R, char* tab, char* ws) {
    const TabLayout t = table_layout(R);
    const WsLayout w = workspace_layout(R);
    SigDesc d{};
    d.sigma = reinterpret_cast<const uint32_t*>(tab + t.sigma);
    d.sigma_inv = reinterpret_cast<const uint32_t*>(tab + t.sigma_inv);
    d.tau = reinterpret_cast<const uint32_t*>(tab + t.tau);
    d.invG = reinterpret_cast<const float2*>(tab + t.invG);
    d.tw = reinterpret_cast<const float2*>(tab + t.tw);
    d.tpos = reinterpret_cast<const uint32_t*>(tab + t.tpos);
    d.rou = reinterpret_cast<const double2*>(tab + t.rou);
    d.comb_tau = reinterpret_cast<const uint32_t*>(tab + t.ctau);
    d.ctw = reinterpret_cast<const float2*>(tab + t.ctw);
    d.gw = reinterpret_cast<const float2*>(tab + t.gw);
    d.tb = R.tb;
    d.step = 6.283185307179586476925286766559 / (double)R.N;
    d.uhat = reinterpret_cast<float2*>(ws + w.uhat);
    d.jbits = reinterpret_cast<uint32_t*>(ws + w.jbits);
    d.jlist = reinterpret_cast<uint32_t*>(ws + w.jlist);
    d.cand = reinterpret_cast<uint32_t*>(ws + w.cand);
    d.est = reinterpret_cast<float2*>(ws + w.est);
    d.keys = reinterpret_cast<uint64_t*>(ws + w.keys);
    d.rpart = reinterpret_cast<double*>(ws + w.rpart);
    d.resid_own = reinterpret_cast<double*>(ws + w.resid_own);
    d.ctr = reinterpret_cast<uint32_t*>(ws + w.ctr);
    d.ubuf = reinterpret_cast<float2*>(ws + w.ubuf);
    d.gmax = reinterpret_cast<uint32_t*>(ws + w.gmax);
    d.cbits = reinterpret_cast<uint32_t*>(ws + w.cbits);
    d.rec_f = reinterpret_cast<uint32_t*>(ws + w.rec_f);
    d.rec_v = reinterpret_cast<float2*>(ws + w.rec_v);
    d.iterate = R.iterate;
    d.sub_rl = R.sub_rl;
    d.sub_rh = R.sub_rh;
    d.phase = R.phase;
    d.comb_loops = R.comb_loops;
    d.comb_log2b = R.comb_log2b;
    d.comb_keep = R.comb_keep;
    d.fft_mode = R.fft_mode;
    d.N = R.N;
    d.maskN = R.N - 1;
    d.log2N = R.log2N;
    d.B = R.B;
    d.log2B = R.log2B;
    d.M = R.M;
    d.log2M = R.log2M;
    d.L = R.L;
    d.w = R.w;
    d.Mw = R.Mw;
    d.Mw4 = R.Mw4;
    // s = w / (2 gauss_c): t^2 / 2s^2 = (t kappa)^2 ln 2 with kappa = 2 gauss_c / (w sqrt(2 ln 2))
    d.wkappa = (float)(2.0 * R.gauss_c / ((double)R.w * 1.1774100225154747));
    d.K = R.K;
    d.dK = R.dK;
    d.T = R.T;
    d.S = R.S;
    d.cap = R.cap;
    d.mode = R.mode;
    d.C = R.C;
    d.log2C = R.log2C;
    d.strips = R.B / R.C;
    d.vote_units = R.vote_units;
    d.vote_upl = R.vote_upl;
    d.vote_split = R.vote_split;
    d.vote_pairs = R.vote_pairs;
    d.vote_sub = R.vote_sub;
    memcpy(d.vote_pair, R.vote_pair, sizeof(d.vote_pair));
    d.resid_blocks = R.resid_blocks;
    d.resid_log2kl = R.resid_log2kl;
    d.est_units = R.est_units;
    d.lmax = R.lmax;
    d.combine = (R.flags & SFFT_FLAG_MEAN_ESTIMATE) ? 1u : 0u;
    d.eloops = nullptr;
    d.L_est = 0;
    return d;
}

void link_est(SigDesc* d, const SigDesc* d_est_dev, const Resolved& R) {
    d->eloops = d_est_dev;
    d->L_est = R.L_est();
}

// Bucketization and B-point FFT (+ selection) of one descriptor.
static sfft_status launch_buckets(const Resolved& R, const SigDesc* d_desc, const IoDesc& io, hipStream_t s) {
    Launch a{};
    a.descs = d_desc;
    a.nsig = 0;
    a.xcd_order = R.xcd_order;
    a.one_io = io;
    HIP_TRY(launch_fold(a, R.fold_variant, R.fold_units, R.strip_lds, s), "bucketization launch");
    a.xcd_order = 0;
    if (R.fft_mode) {
        HIP_TRY(launch_fft_large(a, R.log2B, 0, R.fft_p1_units, s), "fft pass 1 launch");
        HIP_TRY(launch_fft_large(a, R.log2B, 1, R.fft_p2_units, s), "fft pass 2 launch");
        HIP_TRY(launch_fft_large(a, R.log2B, 2, R.L, s), "selection launch");
    } else {
        HIP_TRY(launch_fft_select(a, R.log2B, R.L, s), "fft/select launch");
    }
    return SFFT_OK;
}

// Launch every stage for one signal (nsig == 0 form of Launch). d_desc[1] holds
// the estimation-only loops when the plan has them.
sfft_status launch_single(const Resolved& R, const SigDesc* d_desc, const IoDesc& io, hipStream_t s) {
    if (R.fused) {
        Launch a{};
        a.descs = d_desc;
        a.nsig = 0;
        a.xcd_order = 0;
        a.one_io = io;
        HIP_TRY(launch_fused(a, vote_key(R.L), 1, R.fused_lds, s), "fused launch");
        return SFFT_OK;
    }
    sfft_status st = launch_buckets(R, d_desc, io, s);
    if (st == SFFT_OK && R.est) st = launch_buckets(*R.est, d_desc + 1, io, s);
    if (st != SFFT_OK) return st;
    Launch a{};
    a.descs = d_desc;
    a.nsig = 0;
    a.xcd_order = 0;
    a.one_io = io;
    if (R.comb_loops) HIP_TRY(launch_comb(a, R.comb_log2b, R.comb_loops, s), "comb prefilter launch");
    if (R.phase)
        HIP_TRY(launch_decode(a, R.vote_units, 0, s), "phase decode launch");
    else
        HIP_TRY(launch_vote(a, vote_key(R.L), R.vote_units, R.vote_dyn_lds, R.vote_lds > 0, 0, s), "vote launch");
    // the estimates and the K largest: one launch when one workgroup covers the candidates
    auto tail = [&](uint32_t round) -> hipError_t {
        if (R.est_units == 1) return launch_tail_one(a, R.lmax, R.fin_lds, round, s);
        hipError_t e = launch_estimate(a, R.lmax, R.est_units, round, s);
        return e == hipSuccess ? launch_finalize(a, 1, R.fin_lds, round, s) : e;
    };
    HIP_TRY(tail(0), "estimate / top-K launch");
    if (R.iterate) {
        HIP_TRY(launch_subtract(a, R.L, R.sub_lds, s), "subtraction launch");
        HIP_TRY(launch_reselect(a, R.log2B, R.L, s), "reselection launch");
        if (R.phase)
            HIP_TRY(launch_decode(a, R.vote_units, 1, s), "second phase decode launch");
        else
            HIP_TRY(launch_vote(a, vote_key(R.L), R.vote_units, R.vote_dyn_lds, R.vote_lds > 0, 1, s), "second vote launch");
        HIP_TRY(tail(1), "second estimate / top-K launch");
    }
    if (R.S) HIP_TRY(launch_residual_one(a, R.resid_blocks, R.resid_lds, s), "residual launch");
    return SFFT_OK;
}

}  // namespace sfft

using namespace sfft;

// ------------------------------------------------------------------ plan object
struct sfft_plan_s {
    Resolved R;
    int device = 0;
    char* d_tab = nullptr;       // tables of the plan, then (at tab_e) of its estimation-only loops
    char* d_ws = nullptr;        // workspace, idem (at ws_e)
    size_t tab_e = 0, ws_e = 0;
    SigDesc* d_desc = nullptr;   // [2 nd]: nd = 1 + has estimation-only loops descriptors on the plan's
                                 // workspace, then nd on the device's scratch array (if it fits)
    int nd = 1;
    bool scratch_ok = false;     // the workspace fits the scratch array and its address is known
    std::string scratch_err;
    sfft_status scratch_st = SFFT_E_UNSUPPORTED;
    size_t tab_bytes = 0, ws_bytes = 0;
    hipEvent_t done = nullptr;
    hipStream_t last_stream = nullptr;
    bool launched = false;
    std::mutex mu;
};

namespace sfft {

sfft_status plan_create(const sfft_params& p, sfft_plan_t* out) {
    if (!out) return set_error(SFFT_E_INVALID, "null output pointer");
    *out = nullptr;
    Resolved R;
    std::string err;
    sfft_status st = resolve_params(p, &R, &err);
    if (st != SFFT_OK) return set_error(st, err);
    HostTables T;
    build_tables(R, &T);
    auto* pl = new (std::nothrow) sfft_plan_s();
    if (!pl) return set_error(SFFT_E_NOMEM, "host allocation");
    pl->R = std::move(R);
    const Resolved& Rr = pl->R;
    auto cleanup = [&](sfft_status s) {
        if (pl->d_tab) (void)hipFree(pl->d_tab);
        if (pl->d_ws) (void)hipFree(pl->d_ws);
        if (pl->d_desc) (void)hipFree(pl->d_desc);
        if (pl->done) (void)hipEventDestroy(pl->done);
        delete pl;
        return s;
    };
    hipError_t e = hipGetDevice(&pl->device);
    if (e != hipSuccess) return cleanup(hip_fail(e, "hipGetDevice"));
    e = init_kernel_attributes();
    if (e != hipSuccess) return cleanup(hip_fail(e, "kernel attributes"));
    std::vector<char> h = pack_tables(Rr, T);
    size_t ws_total = workspace_layout(Rr).total;
    const int nd = Rr.est ? 2 : 1;
    if (Rr.est) {
        // the estimation-only loops' tables and workspace follow, 256-byte aligned
        HostTables Te;
        build_tables(*Rr.est, &Te);
        const std::vector<char> he = pack_tables(*Rr.est, Te);
        pl->tab_e = (h.size() + 255) & ~size_t(255);
        h.resize(pl->tab_e, 0);
        h.insert(h.end(), he.begin(), he.end());
        pl->ws_e = (ws_total + 255) & ~size_t(255);
        ws_total = pl->ws_e + workspace_layout(*Rr.est).total;
    }
    pl->tab_bytes = h.size();
    pl->ws_bytes = ws_total;
    if (hipMalloc(&pl->d_tab, h.size()) != hipSuccess) return cleanup(set_error(SFFT_E_NOMEM, "device tables"));
    if (hipMalloc(&pl->d_ws, ws_total) != hipSuccess) return cleanup(set_error(SFFT_E_NOMEM, "device workspace"));
    if (hipMalloc(&pl->d_desc, sizeof(SigDesc) * 2 * nd) != hipSuccess)
        return cleanup(set_error(SFFT_E_NOMEM, "device descriptor"));
    pl->nd = nd;
    e = hipMemcpy(pl->d_tab, h.data(), h.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return cleanup(hip_fail(e, "table upload"));
    e = hipMemset(pl->d_ws, 0, ws_total);
    if (e != hipSuccess) return cleanup(hip_fail(e, "workspace clear"));
    SigDesc d[4];
    d[0] = make_desc(Rr, pl->d_tab, pl->d_ws);
    if (Rr.est) {
        d[1] = make_desc(*Rr.est, pl->d_tab + pl->tab_e, pl->d_ws + pl->ws_e);
        link_est(&d[0], pl->d_desc + 1, Rr);
    }
    // the same descriptors on this device's scratch array, for sfft_execute_noalloc
    char* sp = nullptr;
    const hipError_t se = scratch_address(pl->device, &sp);
    if (se != hipSuccess) {
        pl->scratch_err = std::string("scratch array address: ") + hipGetErrorString(se);
        pl->scratch_st = SFFT_E_DEVICE;
    } else if (ws_total > scratch_bytes()) {
        pl->scratch_err = "the plan's workspace (" + std::to_string(ws_total) + " bytes) exceeds the scratch array (" +
                          std::to_string(scratch_bytes()) + " bytes)";
    } else {
        pl->scratch_ok = true;
        d[nd] = make_desc(Rr, pl->d_tab, sp);
        if (Rr.est) {
            d[nd + 1] = make_desc(*Rr.est, pl->d_tab + pl->tab_e, sp + pl->ws_e);
            link_est(&d[nd], pl->d_desc + nd + 1, Rr);
        }
    }
    e = hipMemcpy(pl->d_desc, d, sizeof(SigDesc) * (pl->scratch_ok ? 2 * nd : nd), hipMemcpyHostToDevice);
    if (e != hipSuccess) return cleanup(hip_fail(e, "descriptor upload"));
    e = hipEventCreateWithFlags(&pl->done, hipEventDisableTiming);
    if (e != hipSuccess) return cleanup(hip_fail(e, "event"));
    *out = pl;
    return SFFT_OK;
}

const Resolved& plan_resolved(sfft_plan_t p) { return p->R; }
const char* plan_tables(sfft_plan_t p) { return p->d_tab; }
size_t plan_est_table_offset(sfft_plan_t p) { return p->tab_e; }
int plan_device(sfft_plan_t p) { return p->device; }
size_t plan_table_bytes(sfft_plan_t p) { return p->tab_bytes; }
size_t plan_ws_bytes(sfft_plan_t p) { return p->ws_bytes; }

}  // namespace sfft

namespace {

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

sfft_status check_busy(sfft_plan_t p, hipStream_t s) {
    if (p->launched && s != p->last_stream) {
        const hipError_t q = hipEventQuery(p->done);
        if (q == hipErrorNotReady) return set_error(SFFT_E_BUSY, "plan is executing on another stream");
        if (q != hipSuccess) return hip_fail(q, "hipEventQuery");
    }
    return SFFT_OK;
}

}  // namespace

namespace sfft {

sfft_status plan_execute(sfft_plan_t p, const void* x_dev, int64_t* out_idx, void* out_val, double* out_resid,
                         sfft_stream_t stream, bool scratch) {
    if (!p || !x_dev || !out_idx || !out_val) return set_error(SFFT_E_INVALID, "null argument");
    if (scratch && !p->scratch_ok) return set_error(p->scratch_st, p->scratch_err);
    if (!aligned16(x_dev)) return set_error(SFFT_E_INVALID, "x_dev must be 16-byte aligned");
    if ((reinterpret_cast<uintptr_t>(out_val) & 7u) || (reinterpret_cast<uintptr_t>(out_idx) & 7u) ||
        (reinterpret_cast<uintptr_t>(out_resid) & 7u))
        return set_error(SFFT_E_INVALID, "outputs must be 8-byte aligned");
    std::lock_guard<std::mutex> lk(p->mu);
    HIP_TRY(hipSetDevice(p->device), "hipSetDevice");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    sfft_status st = check_busy(p, s);
    if (st != SFFT_OK) return st;
    HIP_TRY(hipGetLastError(), "earlier device work");
    IoDesc io{reinterpret_cast<const float2*>(x_dev), out_idx, reinterpret_cast<float2*>(out_val), out_resid};
    st = launch_single(p->R, p->d_desc + (scratch ? p->nd : 0), io, s);
    if (st != SFFT_OK) return st;
    HIP_TRY(hipEventRecord(p->done, s), "hipEventRecord");
    p->last_stream = s;
    p->launched = true;
    return SFFT_OK;
}

}  // namespace sfft

extern "C" {

const char* sfft_version(void) { return "sfft-mi355x 0.1 (gfx950)"; }

const char* sfft_last_error(void) { return g_last_error.c_str(); }

const char* sfft_status_string(sfft_status s) {
    switch (s) {
        case SFFT_OK: return "ok";
        case SFFT_E_INVALID: return "invalid argument";
        case SFFT_E_NOMEM: return "out of memory";
        case SFFT_E_DEVICE: return "device error";
        case SFFT_E_UNSUPPORTED: return "unsupported";
        case SFFT_E_BUSY: return "busy";
        case SFFT_E_NOTFOUND: return "not found";
    }
    return "unknown status";
}

sfft_status sfft_params_init(sfft_params* p, int64_t N, int32_t K, int32_t B, int32_t L, int64_t w) {
    if (!p) return set_error(SFFT_E_INVALID, "null params");
    memset(p, 0, sizeof(*p));
    p->N = N;
    p->K = K;
    p->B = B;
    p->L = L;
    p->w = w;
    p->d = 2;
    return SFFT_OK;
}

sfft_status sfft_plan(sfft_plan_t* out, int64_t N, int32_t K, int32_t B, int32_t L, int64_t w) {
    sfft_params p;
    sfft_params_init(&p, N, K, B, L, w);
    return plan_create(p, out);
}

sfft_status sfft_plan_ex(sfft_plan_t* out, const sfft_params* p) {
    if (!p) return set_error(SFFT_E_INVALID, "null params");
    return plan_create(*p, out);
}

sfft_status sfft_destroy(sfft_plan_t p) {
    if (!p) return set_error(SFFT_E_INVALID, "null plan");
    (void)hipSetDevice(p->device);
    if (p->launched) (void)hipEventSynchronize(p->done);
    (void)hipFree(p->d_tab);
    (void)hipFree(p->d_ws);
    (void)hipFree(p->d_desc);
    (void)hipEventDestroy(p->done);
    delete p;
    return SFFT_OK;
}

static void copy_perms(const Resolved& R, uint32_t* sigma, uint32_t* sigma_inv, uint32_t* tau) {
    const uint32_t Le = R.L_est();
    if (sigma) memcpy(sigma, R.sigma.data(), R.L * 4);
    if (sigma_inv) memcpy(sigma_inv, R.sigma_inv.data(), R.L * 4);
    if (tau) memcpy(tau, R.tau.data(), R.L * 4);
    if (Le) {
        if (sigma) memcpy(sigma + R.L, R.est->sigma.data(), Le * 4);
        if (sigma_inv) memcpy(sigma_inv + R.L, R.est->sigma_inv.data(), Le * 4);
        if (tau) memcpy(tau + R.L, R.est->tau.data(), Le * 4);
    }
}

sfft_status sfft_plan_get_perms(sfft_plan_t p, uint32_t* sigma, uint32_t* sigma_inv, uint32_t* tau) {
    if (!p) return set_error(SFFT_E_INVALID, "null plan");
    copy_perms(p->R, sigma, sigma_inv, tau);
    return SFFT_OK;
}

static void fill_desc(const Resolved& R, size_t tab_bytes, size_t ws_bytes, sfft_plan_desc* out) {
    out->N = R.N;
    out->w = R.w;
    out->K = (int32_t)R.K;
    out->B = (int32_t)R.B;
    out->L = (int32_t)R.L;
    out->d = (int32_t)R.d;
    out->T = (int32_t)R.T;
    out->n_resid = (int32_t)R.S;
    out->fold_mode = (int32_t)R.mode;
    out->strip_cols = (int32_t)R.C;
    out->cand_cap = R.cap;
    out->table_bytes = tab_bytes;
    out->workspace_bytes = ws_bytes;
    out->sampled_fraction_expected = 1.0 - pow(1.0 - (double)R.w / (double)R.N, (double)R.L);
    out->sub_reach_lo = (int32_t)R.sub_rl;
    out->sub_reach_hi = (int32_t)R.sub_rh;
    out->sub_tail_bound = R.sub_bound;
    out->vote_pairs = (int32_t)R.vote_pairs;
    memcpy(out->vote_pair, R.vote_pair, sizeof(out->vote_pair));
}

sfft_status sfft_plan_describe(sfft_plan_t p, sfft_plan_desc* out) {
    if (!p || !out) return set_error(SFFT_E_INVALID, "null argument");
    fill_desc(p->R, p->tab_bytes, p->ws_bytes, out);
    return SFFT_OK;
}

sfft_status sfft_params_describe(const sfft_params* p, sfft_plan_desc* out) {
    if (!p || !out) return set_error(SFFT_E_INVALID, "null argument");
    Resolved R;
    std::string err;
    const sfft_status st = resolve_params(*p, &R, &err);
    if (st != SFFT_OK) return set_error(st, err);
    size_t tab = table_layout(R).total, ws = workspace_layout(R).total;
    if (R.est) {   // the estimation-only loops' tables and workspace follow, 256-byte aligned
        tab = ((tab + 255) & ~size_t(255)) + table_layout(*R.est).total;
        ws = ((ws + 255) & ~size_t(255)) + workspace_layout(*R.est).total;
    }
    fill_desc(R, tab, ws, out);
    return SFFT_OK;
}

sfft_status sfft_host_tables(const sfft_params* p, uint32_t* sigma, uint32_t* sigma_inv, uint32_t* tau,
                             uint32_t* tpos, double* window, double* gain) {
    if (!p) return set_error(SFFT_E_INVALID, "null params");
    Resolved R;
    std::string err;
    const sfft_status st = resolve_params(*p, &R, &err);
    if (st != SFFT_OK) return set_error(st, err);
    copy_perms(R, sigma, sigma_inv, tau);
    if (tpos && R.S) memcpy(tpos, R.tpos.data(), (size_t)R.S * 4);
    if (window || gain) {
        HostTables T;
        build_tables(R, &T);
        if (window) memcpy(window, T.window.data(), (size_t)R.w * 8);
        if (gain)
            for (uint32_t k = 0; k < R.M; ++k) {
                gain[2 * k] = T.gain[k].real();
                gain[2 * k + 1] = T.gain[k].imag();
            }
    }
    return SFFT_OK;
}


sfft_status sfft_execute_ex(sfft_plan_t p, const void* x_dev, int64_t* out_idx, void* out_val, double* out_resid,
                            sfft_stream_t stream) {
    return plan_execute(p, x_dev, out_idx, out_val, out_resid, stream, false);
}

sfft_status sfft_execute(sfft_plan_t p, const void* x_dev, int64_t* out_idx, void* out_val, sfft_stream_t stream) {
    return sfft_execute_ex(p, x_dev, out_idx, out_val, nullptr, stream);
}

sfft_status sfft_plan_read_trace(sfft_plan_t p, sfft_trace* t) {
    if (!p || !t) return set_error(SFFT_E_INVALID, "null argument");
    std::lock_guard<std::mutex> lk(p->mu);
    HIP_TRY(hipSetDevice(p->device), "hipSetDevice");
    if (p->launched) HIP_TRY(hipEventSynchronize(p->done), "wait for execution");
    const Resolved& R = p->R;
    const WsLayout w = workspace_layout(R);
    const size_t wpl = (R.B + 31) / 32;
    if (t->uhat) {
        HIP_TRY(hipMemcpy(t->uhat, p->d_ws + w.uhat, (size_t)R.L * R.B * 8, hipMemcpyDeviceToHost), "copy uhat");
        if (R.fft_mode) {
            // two-pass layout: bucket h's value is e^{+2 pi i (s tau h mod B)/B} V[s h mod B], s = sigma^{-1}
            std::vector<float> v(t->uhat, t->uhat + (size_t)2 * R.L * R.B);
            const uint32_t Bm = R.B - 1;
            for (uint32_t r = 0; r < R.L; ++r) {
                const uint32_t s = R.sigma_inv[r], tau = R.tau[r];
                for (uint32_t h = 0; h < R.B; ++h) {
                    const size_t m = (size_t)r * R.B + ((s * h) & Bm);
                    const double a = 6.283185307179586476925286766559 * (double)((s * tau * h) & Bm) / (double)R.B;
                    const double c = cos(a), sn = sin(a), x = v[2 * m], y = v[2 * m + 1];
                    t->uhat[2 * ((size_t)r * R.B + h)] = (float)(x * c - y * sn);
                    t->uhat[2 * ((size_t)r * R.B + h) + 1] = (float)(x * sn + y * c);
                }
            }
        }
    }
    if (t->jbits) HIP_TRY(hipMemcpy(t->jbits, p->d_ws + w.jbits, (size_t)R.L * wpl * 4, hipMemcpyDeviceToHost), "copy jbits");
    if (t->jlist) HIP_TRY(hipMemcpy(t->jlist, p->d_ws + w.jlist, (size_t)R.L * R.dK * 4, hipMemcpyDeviceToHost), "copy jlist");
    if (t->cbits && R.comb_loops)
        HIP_TRY(hipMemcpy(t->cbits, p->d_ws + w.cbits, (size_t)R.comb_loops * R.comb_words * 4, hipMemcpyDeviceToHost),
                "copy comb bitmaps");
    uint32_t ctr[4] = {0, 0, 0, 0};
    HIP_TRY(hipMemcpy(ctr, p->d_ws + w.ctr, 16, hipMemcpyDeviceToHost), "copy counters");
    const uint32_t n = std::min(ctr[0], R.cap);
    t->cand_count = n;
    t->rec_count = R.iterate ? std::min(ctr[2], R.K) : 0;
    if (R.iterate && t->rec_idx)
        HIP_TRY(hipMemcpy(t->rec_idx, p->d_ws + w.rec_f, (size_t)R.K * 4, hipMemcpyDeviceToHost), "copy first-round frequencies");
    if (R.iterate && t->rec_val)
        HIP_TRY(hipMemcpy(t->rec_val, p->d_ws + w.rec_v, (size_t)R.K * 8, hipMemcpyDeviceToHost), "copy first-round values");
    if (t->cand && n) HIP_TRY(hipMemcpy(t->cand, p->d_ws + w.cand, (size_t)n * 4, hipMemcpyDeviceToHost), "copy candidates");
    return SFFT_OK;
}

}  // extern "C"
