/*
 * sfft.h - C ABI of the MI355X (gfx950) flat-window voting sparse FFT.
 *
 * The library recovers the K largest Fourier coefficients of a length-N
 * complex64 signal x with the sFFT1.0 method of Table 1 of "Empirical
 * Evaluation of Typical Sparse Fast Fourier Transform Algorithms"
 * (arXiv 2012.08238): flat filter, probability-and-statistics (voting)
 * location, energy-concentration estimation, voting framework. Per random
 * bucketization r < L it permutes the time index (i -> sigma_r*i + tau_r mod N,
 * Eq.(6)-(7), spectrum identity Eq.(9)), windows w samples with the flat
 * filter (sinc Eq.(12) x Gaussian Eq.(13)), aliases them into B buckets
 * (Eq.(11)) and takes a B-point FFT; the d*K largest buckets vote for the
 * frequencies they hash, frequencies with at least T votes are estimated from
 * their buckets (median over the L bucketizations) and the K largest are
 * returned. An optional FP64 residual (formula method, Eq.(2)) checks the
 * result on S seeded time samples.
 *
 * Conventions
 *  - The forward DFT carries 1/N (Eq.(2)): a unit-magnitude tone in x returns
 *    a value of magnitude ~1.
 *  - N and B are powers of two, 16 <= N <= 2^30, N/B >= 2, 1 <= d*K <= B,
 *    1 <= L <= 32, w even with 2 <= w <= N, K <= 4096. Anything else returns
 *    SFFT_E_INVALID synchronously and changes nothing.
 *  - "Device" pointers are HIP device memory on the plan's device; "host"
 *    pointers are ordinary host memory. complex64 is two packed floats
 *    (re, im), complex128 two packed doubles.
 *  - Outputs: out_idx int64[K] ascending frequency indices, padded with -1;
 *    out_val complex64[K] matching values, padded with 0.
 *  - Every call that launches GPU work is asynchronous on the given stream
 *    (NULL = the default stream) and never synchronises the host; results are
 *    valid once that stream has reached the call.
 *  - No exception crosses the ABI. Errors return a negative sfft_status; the
 *    message of the last error on the calling thread is sfft_last_error().
 *    A HIP error observed by a call is reported as SFFT_E_DEVICE by that call.
 *  - The library is deterministic: the same plan and input give bitwise the
 *    same output, alone or inside a batch.
 */
#ifndef SFFT_MI355X_H
#define SFFT_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sfft_plan_s* sfft_plan_t;     /* owns device tables + one workspace */
typedef struct sfft_batch_s* sfft_batch_t;   /* owns per-signal workspaces + a HIP graph */
typedef struct sfft_server_s* sfft_server_t; /* owns queue, plan cache, streams */
typedef void* sfft_stream_t;                 /* a hipStream_t */

typedef enum {
    SFFT_OK = 0,
    SFFT_E_INVALID = -1,     /* bad argument or parameter set */
    SFFT_E_NOMEM = -2,       /* device or host allocation failed */
    SFFT_E_DEVICE = -3,      /* a HIP call failed (including sticky errors of earlier work) */
    SFFT_E_UNSUPPORTED = -4, /* valid request this library does not implement */
    SFFT_E_BUSY = -5,        /* plan still executing on another stream; or server full */
    SFFT_E_NOTFOUND = -6     /* unknown ticket */
} sfft_status;

/* Plan flags. */
#define SFFT_FLAG_NO_RESIDUAL 0x1u  /* skip the FP64 residual step */
#define SFFT_FLAG_FOLD_GATHER 0x2u  /* force the gather form of the bucketization */
#define SFFT_FLAG_FOLD_STRIP  0x4u  /* force the streamed column-strip form */
#define SFFT_FLAG_XCD_ORDER   0x8u  /* bucketization: give each XCD a contiguous range of column strips */
#define SFFT_FLAG_MEAN_ESTIMATE 0x10u /* combine the L loop estimates by their mean (the averaging of the
                                         energy-concentration method) instead of the coordinate-wise median */
#define SFFT_FLAG_ITERATE 0x20u       /* one round of the iterative framework (frameworks section): the K
                                         recovered coefficients (f, v) are subtracted from every loop's
                                         buckets, v e^{+2 pi i tau f/N} Gw(sigma f - h N/B) from each bucket h
                                         (Gw = sum_n g_n e^{+2 pi i n o/N}, Eq.(9)): from every bucket, or
                                         from the bucket of sigma f and the R on either side when a bound
                                         on |Gw| beyond them is <= 1e-6 of the centre gain (smallest R >= 1;
                                         sfft_plan_desc.sub_reach_*). A window whose response needs more
                                         than 129 buckets (or a gain table of more than 2^22 entries) gives
                                         SFFT_E_UNSUPPORTED;
                                         the residual buckets are selected and voted again (frequencies
                                         already recovered excluded), new candidates are estimated from the
                                         residual buckets, each recovered value is corrected by the combined
                                         residual estimate, and the K largest of both are returned.
                                         Requires B <= 16384 (else SFFT_E_UNSUPPORTED). */
#define SFFT_FLAG_PHASE_LOCATION 0x40u /* locate by phase encoding (the sFFT3.0 row of Table 1, phase
                                         encoding method) instead of voting: L is even and loops 2j, 2j+1
                                         form a pair with sigma_{2j+1} = sigma_{2j}, tau_{2j+1} = tau_{2j}+1
                                         (the odd loops' draws are replaced; explicit sigma/tau must already
                                         be paired). Each selected bucket h of loop 2j decodes
                                         f = floor(angle(u_{2j+1}[h] conj(u_{2j}[h])) N/(2 pi) + 1/2) mod N,
                                         kept when sigma_{2j} f hashes to h; a frequency decoded by at least T
                                         pairs (vote_threshold, default 1, at most L/2) is a candidate and is
                                         estimated from the loops of the pairs that decode it only. With
                                         SFFT_FLAG_ITERATE the recovered values are kept and the residual is
                                         decoded for new frequencies. Requires B <= 16384. */
#define SFFT_FLAG_FFT_TWO_PASS 0x80u  /* take the B-point FFT in two passes through the workspace (the
                                         form used for B > 16384) also for 4096 <= B <= 16384: small
                                         workgroups that can share a compute unit with other work instead
                                         of one workgroup holding the whole transform in LDS. Results equal
                                         the one-workgroup form to FP32 rounding. Not combinable with
                                         SFFT_FLAG_ITERATE or SFFT_FLAG_PHASE_LOCATION (SFFT_E_UNSUPPORTED);
                                         other B: SFFT_E_INVALID. */

#define SFFT_MAX_VOTE_PAIRS 32
#define SFFT_FLAG_VOTE_BY_LOOP 0x100u /* votes: enumerate the frequencies of the selected buckets of
                                         loops 0..L-T (by the pigeonhole principle every frequency with
                                         >= T votes is voted by one of them) and test each against the
                                         other loops. The candidate set is the same in either form. */
#define SFFT_FLAG_VOTE_BY_PAIR 0x200u /* votes: split the loops into T-1 groups of consecutive loops;
                                         any T loops hold two of one group, so every frequency with >= T
                                         votes is voted by both loops of a pair within a group. Each pair
                                         enumerates its first loop's selected buckets and tests its
                                         second loop; only those that pass are tested against the rest.
                                         Needs T >= 2 and at most 32 pairs (else SFFT_E_INVALID). Without
                                         either flag the plan takes the form with fewer expected tests. */
#define SFFT_FLAG_FUSED 0x400u        /* run the whole path of the signal (bucketization by gathering, FFT,
                                         selection, votes, estimates, the K largest, residual) in one
                                         workgroup of one launch, the stages separated by barriers instead
                                         of kernel boundaries; in a batch every such signal shares one
                                         launch of persistent workgroups (the batch section's one-launch
                                         form for small signals). Results are those of the per-stage path.
                                         Needs 32 <= B <= 4096, L <= 16, K <= 1024, and none of
                                         SFFT_FLAG_ITERATE, SFFT_FLAG_PHASE_LOCATION, SFFT_FLAG_FFT_TWO_PASS,
                                         SFFT_FLAG_FOLD_STRIP, the comb prefilter or estimation-only loops
                                         (else SFFT_E_UNSUPPORTED). */

/* Full parameter set. Fill with sfft_params_init() and then override fields. */
typedef struct {
    int64_t N;              /* signal length, power of two */
    int32_t K;              /* number of coefficients returned */
    int32_t B;              /* number of buckets per bucketization, power of two */
    int32_t L;              /* number of random bucketizations (loops) */
    int32_t d;              /* buckets kept per loop = d*K (the location method keeps 2K: d = 2) */
    int64_t w;              /* flat window length (time support), even */
    uint64_t seed;          /* SplitMix64 seed of sigma_r, tau_r and the residual samples */
    int32_t vote_threshold; /* T; 0 selects the strict majority floor(L/2)+1 */
    int32_t n_resid;        /* S residual time samples; 0 selects 4096. They come in runs of 8
                             * consecutive positions, one stream draw per run (its start rounded
                             * down to a multiple of 8); the first S positions in run order */
    double gauss_c;         /* window length / (2 * Gaussian std); 0 selects the Fig. 1 ratio 4.861870431316438 */
    uint32_t flags;         /* SFFT_FLAG_* */
    int32_t strip_cols;     /* tile width of the strip bucketization (power of two); 0 = automatic */
    const uint32_t* sigma;  /* optional host uint32[L]: explicit odd scalings (NULL = draw from seed) */
    const uint32_t* tau;    /* optional host uint32[L]: explicit shifts; required iff sigma is given */
    /* Comb prefilter (the spike-train bucketization of the sFFT2.0 row, Eq.(15)-(16)):
     * comb_loops in [0, 8] (0 = off) shifts tau_c drawn after the residual runs' draws,
     * each taking the comb_b samples x[tau_c + j N/comb_b]; the comb_keep (0 = d*K)
     * largest of their comb_b-point DFT mark residues mod comb_b, and only
     * frequencies whose residue is marked by some shift can be located.
     * comb_b: power of two in [2, min(N/2, 16384)]; comb_keep <= comb_b. */
    int32_t comb_b;
    int32_t comb_loops;
    int32_t comb_keep;
    /* Estimation-only loops (location and estimation loops separated): est_loops in
     * [0, 32 - L] more random bucketizations with est_B buckets (power of two,
     * K <= est_B <= 16384, N/est_B >= 2) and a flat window of est_w samples (0 = w est_B / B;
     * even, <= N). They are not selected or voted; every located frequency is estimated by
     * the median (or mean) over all L + est_loops loops. Their sigma, tau are the next
     * 2 est_loops draws of the stream, after the comb shifts. Not combinable with
     * SFFT_FLAG_ITERATE or SFFT_FLAG_PHASE_LOCATION (SFFT_E_UNSUPPORTED). */
    int32_t est_loops;
    int32_t est_B;
    int64_t est_w;
} sfft_params;

/* Resolved plan description (what the plan actually runs). */
typedef struct {
    int64_t N, w;
    int32_t K, B, L, d, T, n_resid;
    int32_t fold_mode;      /* 0 = gather, 1 = strip */
    int32_t strip_cols;
    int64_t cand_cap;       /* capacity of the candidate list: (L-T+1)*d*K*N/B (votes), (L/2)*d*K (phase) */
    size_t table_bytes;     /* resident device tables */
    size_t workspace_bytes; /* one execution's device workspace */
    double sampled_fraction_expected; /* 1-(1-w/N)^L (Table 2, sFFT1.0 sampling, log N -> L) */
    /* SFFT_FLAG_ITERATE: each recovered coefficient of bucket h0 is subtracted from the buckets
     * h0 - sub_reach_lo .. h0 + sub_reach_hi (all B of them when the two add up to B - 1), and
     * sub_tail_bound bounds the window response in every other bucket relative to the centre
     * gain (<= 1e-6; 0 when no bucket is left out). All three are 0 without the flag. */
    int32_t sub_reach_lo, sub_reach_hi;
    double sub_tail_bound;
    /* Vote enumeration: vote_pairs = 0 by loop (loops 0..L-T), else the number of loop pairs,
     * vote_pair[e] = first loop | second loop << 8, in the order in which a frequency voted
     * by several pairs is counted from the first (see SFFT_FLAG_VOTE_BY_PAIR). */
    int32_t vote_pairs;
    uint16_t vote_pair[SFFT_MAX_VOTE_PAIRS];
} sfft_plan_desc;

/* Host copies of one execution's intermediates (all pointers host, caller-owned,
 * any may be NULL to skip). Sizes in elements. */
typedef struct {
    float* uhat;            /* float[2*L*B]: bucket spectra after the B-point FFT, [loop][bucket] (re, im) */
    uint32_t* jbits;        /* uint32[L*B/32]: selected-bucket bitmaps, bit h of word h/32 of loop r */
    uint32_t* jlist;        /* uint32[L*d*K]: selected buckets per loop, ascending */
    uint32_t* cand;         /* uint32[cand_cap]: frequencies with >= T votes, unordered */
    int64_t cand_count;     /* out: number of valid entries written to cand */
    uint32_t* cbits;        /* uint32[comb_loops * max(1, comb_b/32)]: residues kept per comb loop */
    /* With SFFT_FLAG_ITERATE, uhat, jbits, jlist and cand above are those of the second round (residual
     * buckets, their selection, the new candidates) and the first round's outputs are: */
    uint32_t* rec_idx;      /* uint32[K]: first-round frequencies, ascending, 0xFFFFFFFF padded */
    float* rec_val;         /* float[2*K]: their values (re, im) */
    int64_t rec_count;      /* out: number of valid first-round entries (0 without SFFT_FLAG_ITERATE) */
} sfft_trace;

/* ---- parameters and plans --------------------------------------------------------- */

/* Fill *p with N, K, B, L, w and the defaults (d=2, seed=0, T=floor(L/2)+1,
 * S=4096, Fig. 1 Gaussian ratio, no flags). Host only; no device work. */
sfft_status sfft_params_init(sfft_params* p, int64_t N, int32_t K, int32_t B, int32_t L, int64_t w);

/* Build a plan on the current HIP device: validates, draws sigma_r (odd) and
 * tau_r from SplitMix64(seed) in the order sigma_0, tau_0, sigma_1, ...,
 * followed by one draw per run of 8 residual positions; inverts sigma_r mod N; builds the flat
 * window (Eq.(12) x Eq.(13), FP64), the gain table
 * Gtab[o] = sum_n g_n e^{+2 pi i n o/N}, o in [-N/2B, N/2B) (FP64; Eq.(14)),
 * FFT twiddles and FP64 residual phase tables; uploads them and allocates one
 * workspace. Synchronous (the only host->device crossing of the plan). */
sfft_status sfft_plan(sfft_plan_t* out, int64_t N, int32_t K, int32_t B, int32_t L, int64_t w);
sfft_status sfft_plan_ex(sfft_plan_t* out, const sfft_params* p);

/* Release a plan. Waits for the plan's in-flight work first. */
sfft_status sfft_destroy(sfft_plan_t p);

/* Host copies of sigma_r, sigma_r^{-1} mod N and tau_r (uint32[L + est_loops] each, the
 * estimation-only loops last; any may be NULL). */
sfft_status sfft_plan_get_perms(sfft_plan_t p, uint32_t* sigma, uint32_t* sigma_inv, uint32_t* tau);

/* Resolved description of the plan. */
sfft_status sfft_plan_describe(sfft_plan_t p, sfft_plan_desc* out);

/* Host only, no device: the description that sfft_plan_ex(p) would give (the same
 * validation and status; table and workspace sizes as that plan would allocate them). */
sfft_status sfft_params_describe(const sfft_params* p, sfft_plan_desc* out);

/* Host-only build of the plan's FP64 tables without any device (for checking
 * the host logic): sigma, sigma_inv, tau uint32[L + est_loops]; tpos uint32[S];
 * window double[w]; gain double[2*(N/B)] as (re, im) pairs for
 * o = -N/2B .. N/2B-1. Any pointer may be NULL. */
sfft_status sfft_host_tables(const sfft_params* p, uint32_t* sigma, uint32_t* sigma_inv,
                             uint32_t* tau, uint32_t* tpos, double* window, double* gain);

/* ---- execution -------------------------------------------------------------------- */

/* Run the whole path on x_dev (device complex64[N], read only during the call)
 * into out_idx (device int64[K]) and out_val (device complex64[K]).
 * Asynchronous on `stream`. Returns SFFT_E_BUSY if the plan's previous
 * execution was issued on a different stream and has not finished. */
sfft_status sfft_execute(sfft_plan_t p, const void* x_dev, int64_t* out_idx, void* out_val,
                         sfft_stream_t stream);

/* As sfft_execute, and also writes out_resid (device double[2], may be NULL):
 * [0] = mean_t |x_t - sum_k v_k e^{+2 pi i t f_k/N}|^2, [1] = mean_t |x_t|^2 over the
 * S residual samples, computed in FP64 (formula method). */
sfft_status sfft_execute_ex(sfft_plan_t p, const void* x_dev, int64_t* out_idx, void* out_val,
                            double* out_resid, sfft_stream_t stream);

/* For callers that cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): sfft_execute_ex with the same arguments and results,
 * bitwise, that calls no allocating routine. Its workspace is one 64 MiB array per GPU
 * (held until the process ends; its address is taken when the first plan is created on
 * that GPU) instead of the plan's own workspace. Every call on a GPU shares that array
 * and leaves its contents behind: calls that overlap on one GPU (any plans, any streams)
 * race, so the caller orders them on one stream or waits between them. A plan whose
 * workspace (sfft_plan_desc.workspace_bytes) exceeds 64 MiB returns SFFT_E_UNSUPPORTED;
 * SFFT_E_DEVICE if the array's address could not be taken. sfft_plan_read_trace keeps
 * reading the plan's own workspace (the last sfft_execute/_ex). */
sfft_status sfft_execute_noalloc(sfft_plan_t p, const void* x_dev, int64_t* out_idx, void* out_val,
                                 double* out_resid, sfft_stream_t stream);

/* Synchronously copy the intermediates of the plan's last execution to host
 * buffers (waits for that execution). For parity checking. */
sfft_status sfft_plan_read_trace(sfft_plan_t p, sfft_trace* t);

/* ---- batches (uneven sizes, one HIP graph) ------------------------------------------ */

/* A batch of n signals, signal i run with plans[i] (plans may repeat: each
 * signal gets its own workspace). The sequence of batched launches is captured
 * into one HIP graph on first run and replayed afterwards. The plans must
 * outlive the batch. */
sfft_status sfft_batch_create(sfft_batch_t* out, const sfft_plan_t* plans, int32_t n);

/* As sfft_batch_create, with the signals split into n_branches contiguous groups
 * of about equal bytes (n_branches in [1, 8]) whose stage sequences are captured
 * on parallel streams of one graph: one group's FFT, vote and estimation stages
 * overlap another group's bucketization. Results are unchanged (bitwise).
 * sfft_batch_run_timed needs n_branches = 1 (else SFFT_E_UNSUPPORTED). */
sfft_status sfft_batch_create_ex(sfft_batch_t* out, const sfft_plan_t* plans, int32_t n, int32_t n_branches);

/* Run the batch: x_dev[i] device complex64[N_i]; out_idx[i] device int64[K_i];
 * out_val[i] device complex64[K_i]; out_resid NULL or an array of n device
 * double[2] (entries may be NULL). Asynchronous on `stream`; a batch runs one
 * call at a time (SFFT_E_BUSY while its previous run is unfinished on another
 * stream). Each signal's result is bitwise the one sfft_execute gives alone. */
sfft_status sfft_batch_run(sfft_batch_t b, const void* const* x_dev, int64_t* const* out_idx,
                           void* const* out_val, double* const* out_resid, sfft_stream_t stream);
/* As sfft_batch_run, and also records the caller's HIP events (hipEvent_t, may
 * be NULL) on `stream` immediately before and after the batch's bucketization
 * launches, so that hipEventElapsedTime gives that stage's device time. */
sfft_status sfft_batch_run_timed(sfft_batch_t b, const void* const* x_dev, int64_t* const* out_idx,
                                 void* const* out_val, double* const* out_resid, sfft_stream_t stream,
                                 void* ev_fold_begin, void* ev_fold_end);
sfft_status sfft_batch_destroy(sfft_batch_t b);

/* One-shot convenience: create, run once, destroy (the graph is not kept). */
sfft_status sfft_execute_batch(const sfft_plan_t* plans, const void* const* x_dev,
                               int64_t* const* out_idx, void* const* out_val,
                               double* const* out_resid, int32_t n, sfft_stream_t stream);

/* ---- serving ---------------------------------------------------------------------- */

typedef struct {
    uint64_t submitted, completed, rejected, failed;
    uint64_t batches;           /* waves launched (one batched launch sequence each) */
    uint64_t max_batch;         /* largest wave so far */
    uint64_t max_waves_in_flight; /* most waves running at once (on different streams) */
    double p50_latency_s, p99_latency_s, mean_latency_s;  /* submission -> completion observed */
    size_t hbm_in_use, hbm_peak, hbm_budget; /* arena bytes held by workspaces + resident plan tables */
    uint64_t plan_cache_hits, plan_cache_misses, plan_cache_evictions; /* table residency per admission */
} sfft_server_stats;

/* Serving loop (continuous batching of sFFT requests of any N, K, B, L, w).
 * The server reserves one device arena of hbm_budget_bytes on the current
 * device; request workspaces and resident plan tables are placed in it. A
 * worker thread admits queued requests in submission order while the head
 * request's footprint (its workspace, plus its plan tables when they are not
 * resident) fits in the arena and fewer than max_inflight requests are
 * admitted or running; idle resident tables are evicted least recently used
 * first when space is short. Whenever one of the n_streams streams is free, the
 * admitted requests (at most ceil(max_inflight / n_streams)) leave as one wave: a
 * batched launch sequence (as sfft_batch_run; a lone request, the sequence of
 * sfft_execute_ex) on that stream. Requests that arrive while waves run are
 * batched into the next wave, and waves on different streams overlap on the
 * device. Each request's result is bitwise the one sfft_execute_ex gives for
 * its parameter set alone. Plans are cached by parameter set (host tables kept
 * for the server's lifetime). max_inflight in [1, 1024], n_streams in [1, 16],
 * hbm_budget_bytes >= 1 MiB. */
sfft_status sfft_server_create(sfft_server_t* out, size_t hbm_budget_bytes, int32_t max_inflight,
                               int32_t n_streams);

/* Build and cache the plan of a parameter set without queueing work (the first
 * request of a parameter set otherwise pays for its FP64 table build). Host
 * work only; the tables become resident with the first admitted request. */
sfft_status sfft_server_prepare(sfft_server_t s, const sfft_params* p);

/* Queue one request. x_dev, out_idx, out_val (and out_resid, may be NULL) as in
 * sfft_execute_ex; they must stay valid and x_dev unchanged until the ticket
 * completes. Returns SFFT_E_INVALID for a bad parameter set or pointer (only
 * this request is refused) and SFFT_E_NOMEM if the request alone can never fit
 * the budget. Thread safe. */
sfft_status sfft_server_submit(sfft_server_t s, const sfft_params* p, const void* x_dev,
                               int64_t* out_idx, void* out_val, double* out_resid, uint64_t* ticket);

/* Queue n requests of one parameter set at once (a burst: one admission pass and one
 * wake-up of the worker instead of n). Request i reads x_dev[i] and writes out_idx[i],
 * out_val[i] and out_resid[i] (out_resid may be NULL, or hold NULL entries) under the
 * rules of sfft_server_submit; tickets[i] receives its ticket, in submission order. All
 * or none: a bad pointer in any request gives SFFT_E_INVALID, a parameter set that can
 * never fit SFFT_E_NOMEM, and then no request is queued. n = 0 queues nothing. Thread
 * safe. */
sfft_status sfft_server_submit_batch(sfft_server_t s, const sfft_params* p, int32_t n, const void* const* x_dev,
                                     int64_t* const* out_idx, void* const* out_val, double* const* out_resid,
                                     uint64_t* tickets);

/* Non-blocking status of a ticket: *done = 1 once its outputs are complete on
 * the device; then *latency_s = completion - submission time and *req_status
 * the request's own status (SFFT_OK or SFFT_E_DEVICE). Unknown or released
 * tickets give SFFT_E_NOTFOUND. */
sfft_status sfft_server_poll(sfft_server_t s, uint64_t ticket, int32_t* done, double* latency_s,
                             int32_t* req_status);

/* Block until the ticket completes, report it as sfft_server_poll and release
 * it. One waiter per ticket. */
sfft_status sfft_server_wait(sfft_server_t s, uint64_t ticket, double* latency_s, int32_t* req_status);

sfft_status sfft_server_stats_get(sfft_server_t s, sfft_server_stats* out);

/* Run every queued request to completion, then release the arena, streams and plans. */
sfft_status sfft_server_destroy(sfft_server_t s);

/* ---- misc ------------------------------------------------------------------------- */

const char* sfft_status_string(sfft_status s);
const char* sfft_last_error(void);
const char* sfft_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SFFT_MI355X_H */
