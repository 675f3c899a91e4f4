// Host-side plan logic: validation, permutations, FP64 tables.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <thread>

#include "common.hpp"
#include "host.hpp"
#include "kernels.hpp"

namespace sfft {

namespace {
size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

constexpr double kSubTail = 1e-6;           // largest response left beyond the subtraction reach
constexpr uint32_t kSubMaxBuckets = 129;    // buckets a coefficient is removed from, at most
constexpr uint64_t kSubMaxGain = 1u << 22;  // entries of the subtraction gain table, at most

// Bounds on the flat window's response Gw(o) = sum_{n<w} g_n e^{+2 pi i n o/N}, from the
// window's definition: g_n = e^{-t^2/2s^2} sin(pi t/B)/(pi t), t = n - w/2, s = w/(2 c).
// The same formula over every integer t has, by Poisson summation, the response
// e^{+pi i w o/N} sum_k F(o/N - k) with F the continuous spectrum of the product: the
// boxcar of width 1/B convolved with the Gaussian's spectrum,
//   F(nu) = (erf(sqrt2 pi s (nu + 1/2B)) - erf(sqrt2 pi s (nu - 1/2B))) / 2 >= 0,
// largest at 0 and decreasing in |nu|. The samples cut off at t < -w/2 and t >= w/2 change
// the response by at most Tc = sum over those t of |g|, which is below
//   (4 / (pi w)) (e^{-c^2/2} + s sqrt(pi/2) erfc(c/sqrt2))
// (each one-sided sum of the decreasing e^{-t^2/2s^2}/(pi t), t >= w/2, is at most its first
// term plus the integral from w/2). So |Gw(0)| >= F(0) - Tc and, for |o| in
// [(R + 1/2) N/B, N/2], |Gw(o)| <= F((R + 1/2)/B) + 2 sum_{m>=0} F(1/2 + m) + Tc.
double window_F(double nu, double s, double B) {
    const double a = 1.4142135623730951 * 3.14159265358979323846 * s;
    nu = fabs(nu);
    const double lo = nu - 0.5 / B, hi = nu + 0.5 / B;
    if (lo > 0) return 0.5 * (erfc(a * lo) - erfc(a * hi));
    return 0.5 * (erf(a * hi) - erf(a * lo));
}

double window_cut(double w, double c) {
    const double s = w / (2.0 * c);
    return 4.0 / (3.14159265358979323846 * w) *
           (exp(-0.5 * c * c) + s * 1.2533141373155003 * erfc(c / 1.4142135623730951));
}

// Largest response beyond R buckets on either side, relative to the centre gain
// (a bound; +inf when the centre bound is not positive).
double response_tail(uint32_t R, const Resolved& P) {
    const double B = (double)P.B, s = (double)P.w / (2.0 * P.gauss_c);
    const double cut = window_cut((double)P.w, P.gauss_c);
    const double centre = window_F(0.0, s, B) - cut;
    if (!(centre > 0)) return INFINITY;
    double alias = 0.0;
    for (int m = 0; m < 64; ++m) alias += window_F(0.5 + m, s, B);
    return (window_F(((double)R + 0.5) / B, s, B) + 2.0 * alias + cut) / centre;
}
}  // namespace

// Reach of the subtraction round: the smallest R >= 1 whose tail bound is at most kSubTail
// (buckets h0 - R .. h0 + R), or every bucket (h0 - B/2 + 1 .. h0 + B/2) once 2R + 1 would
// exceed B. SFFT_E_UNSUPPORTED when that needs more than kSubMaxBuckets buckets or a gain
// table of more than kSubMaxGain entries.
static sfft_status subtraction_reach(Resolved* R, std::string* err) {
    for (uint32_t r = 1;; ++r) {
        if (2 * r + 1 > R->B) {   // every bucket: nothing is left out
            R->sub_rl = R->B / 2 - 1;
            R->sub_rh = R->B / 2;
            R->sub_bound = 0.0;
            break;
        }
        const double t = response_tail(r, *R);
        if (t <= kSubTail) {
            R->sub_rl = R->sub_rh = r;
            R->sub_bound = t;
            break;
        }
        if (2 * r + 1 > kSubMaxBuckets) break;
    }
    const uint64_t nb = (uint64_t)R->sub_rl + R->sub_rh + 1;
    if (R->sub_rh == 0 || nb > kSubMaxBuckets || nb * R->M > kSubMaxGain) {
        *err = "the subtraction round needs the window's response beyond 64 buckets (or a gain table of more "
               "than 2^22 entries) below 1e-6 of its centre: widen w or raise gauss_c";
        return SFFT_E_UNSUPPORTED;
    }
    return SFFT_OK;
}

sfft_status resolve_params(const sfft_params& p, Resolved* out, std::string* err) {
    Resolved R{};
    auto bad = [&](const char* m) {
        *err = m;
        return SFFT_E_INVALID;
    };
    if (!is_pow2((uint64_t)p.N) || p.N < 16 || p.N > (int64_t(1) << 30))
        return bad("N must be a power of two in [16, 2^30]");
    if (p.B < 2 || !is_pow2((uint64_t)p.B) || p.N / p.B < 2) return bad("B must be a power of two >= 2 with N/B >= 2");
    if (p.K < 1 || p.K > kMaxK) return bad("K must be in [1, 4096]");
    if (p.d < 1 || (int64_t)p.d * p.K > p.B) return bad("need 1 <= d*K <= B");
    if (p.L < 1 || p.L > kMaxL) return bad("L must be in [1, 32]");
    if (p.w < 2 || p.w > p.N || (p.w & 1)) return bad("w must be even and in [2, N]");
    const bool phase = (p.flags & SFFT_FLAG_PHASE_LOCATION) != 0;
    if (phase && (p.L & 1)) return bad("phase-encoding location needs an even L");
    const int32_t T = p.vote_threshold ? p.vote_threshold : (phase ? 1 : p.L / 2 + 1);
    if (T < 1 || T > (phase ? p.L / 2 : p.L)) return bad("vote threshold must be in [1, L] (phase location: [1, L/2])");
    if (p.n_resid < 0 || p.n_resid > (1 << 24)) return bad("n_resid must be in [0, 2^24]");
    if (p.gauss_c < 0 || !isfinite(p.gauss_c)) return bad("gauss_c must be >= 0 and finite");
    if ((p.sigma == nullptr) != (p.tau == nullptr)) return bad("sigma and tau must be given together");
    if ((p.flags & SFFT_FLAG_FOLD_GATHER) && (p.flags & SFFT_FLAG_FOLD_STRIP))
        return bad("FOLD_GATHER and FOLD_STRIP are exclusive");
    if (p.comb_loops < 0 || p.comb_loops > kMaxCombLoops) return bad("comb_loops must be in [0, 8]");
    if (p.comb_loops > 0) {
        if (p.comb_b < 2 || !is_pow2((uint64_t)p.comb_b) || (int64_t)p.comb_b > p.N / 2 || p.comb_b > kMaxCombB)
            return bad("comb_b must be a power of two in [2, min(N/2, 16384)]");
        const int64_t keep = p.comb_keep ? p.comb_keep : (int64_t)p.d * p.K;
        if (keep < 1 || keep > p.comb_b) return bad("comb_keep must be in [1, comb_b]");
    }
    if (p.B > kMaxB) {
        *err = "B > 2^18 is not supported by this library";
        return SFFT_E_UNSUPPORTED;
    }
    if ((p.flags & SFFT_FLAG_ITERATE) && p.B > kMaxFftLds) {
        *err = "the subtraction round needs B <= 16384";
        return SFFT_E_UNSUPPORTED;
    }
    if (phase && p.B > kMaxFftLds) {
        *err = "phase-encoding location needs B <= 16384";
        return SFFT_E_UNSUPPORTED;
    }
    if (p.flags & SFFT_FLAG_FFT_TWO_PASS) {
        if (p.B < 4096 || p.B > kMaxFftLds) return bad("FFT_TWO_PASS applies to 4096 <= B <= 16384");
        if (p.flags & (SFFT_FLAG_ITERATE | SFFT_FLAG_PHASE_LOCATION)) {
            *err = "the two-pass FFT combines with neither the subtraction round nor phase location";
            return SFFT_E_UNSUPPORTED;
        }
    }
    if (p.est_loops < 0 || p.est_loops > kMaxL - p.L) return bad("est_loops must be in [0, 32 - L]");
    if (p.est_loops > 0) {
        if (p.est_B < 2 || !is_pow2((uint64_t)p.est_B) || p.N / p.est_B < 2 || p.est_B < p.K)
            return bad("est_B must be a power of two with K <= est_B and N/est_B >= 2");
        const int64_t we = p.est_w ? p.est_w : p.w * (int64_t)p.est_B / p.B;
        if (we < 2 || we > p.N || (we & 1)) return bad("est_w must be even and in [2, N]");
        if (p.est_B > kMaxFftLds || (p.flags & (SFFT_FLAG_ITERATE | SFFT_FLAG_PHASE_LOCATION))) {
            *err = "estimation-only loops need est_B <= 16384 and neither the subtraction round nor phase location";
            return SFFT_E_UNSUPPORTED;
        }
    }
    R.N = (uint32_t)p.N;
    R.K = (uint32_t)p.K;
    R.B = (uint32_t)p.B;
    R.L = (uint32_t)p.L;
    R.d = (uint32_t)p.d;
    R.w = (uint32_t)p.w;
    R.T = (uint32_t)T;
    R.S = (p.flags & SFFT_FLAG_NO_RESIDUAL) ? 0u : (p.n_resid ? (uint32_t)p.n_resid : 4096u);
    R.seed = p.seed;
    R.gauss_c = p.gauss_c > 0 ? p.gauss_c : kDefaultGaussC;
    R.flags = p.flags;
    R.dK = R.d * R.K;
    R.M = R.N / R.B;
    R.Mw = (R.w + R.B - 1) / R.B;
    R.Mw4 = (R.Mw + 3u) & ~3u;
    R.log2N = ilog2(R.N);
    R.log2B = ilog2(R.B);
    R.log2M = ilog2(R.M);
    R.rsh = (R.log2N + 1) / 2;
    R.tb = std::min<uint32_t>(8u, R.log2N);
    uint32_t lm = 4;
    while (lm < R.L + (uint32_t)std::max<int32_t>(p.est_loops, 0)) lm <<= 1;   // every estimating loop
    R.lmax = lm;
    R.phase = phase ? 1u : 0u;
    // candidates: every enumerated frequency of loops 0..L-T (votes), one per
    // selected bucket of the first loop of each pair (phase decoding)
    const uint64_t cap = phase ? (uint64_t)(R.L / 2) * R.dK : (uint64_t)(R.L - R.T + 1) * R.dK * R.M;
    if (cap >= (1ull << 31)) {
        *err = "candidate capacity (L-T+1)*d*K*N/B exceeds 2^31";
        return SFFT_E_UNSUPPORTED;
    }
    R.cap = (uint32_t)cap;

    // random permutations: sigma_r odd, tau_r, then the residual positions
    R.sigma.resize(R.L);
    R.tau.resize(R.L);
    R.sigma_inv.resize(R.L);
    SplitMix64 rng(p.seed);
    for (uint32_t r = 0; r < R.L; ++r) {
        R.sigma[r] = (uint32_t)((rng.next() & (R.N - 1)) | 1u);
        R.tau[r] = (uint32_t)(rng.next() & (R.N - 1));
    }
    R.tpos.resize(R.S);
    for (uint32_t j = 0; j < R.S; j += kResRun) {   // runs of kResRun consecutive positions, one draw each
        const uint32_t s0 = (uint32_t)(rng.next() & (R.N - 1)) & ~(kResRun - 1u);
        for (uint32_t i = 0; i < kResRun && j + i < R.S; ++i) R.tpos[j + i] = s0 + i;
    }
    // comb prefilter shifts: the next draws of the same stream
    R.comb_loops = (uint32_t)p.comb_loops;
    R.comb_b = R.comb_loops ? (uint32_t)p.comb_b : 0u;
    R.comb_log2b = R.comb_loops ? ilog2(R.comb_b) : 0u;
    R.comb_keep = R.comb_loops ? (uint32_t)(p.comb_keep ? p.comb_keep : p.d * p.K) : 0u;
    R.comb_words = R.comb_loops ? std::max<uint32_t>(1u, R.comb_b / 32) : 0u;
    R.comb_tau.resize(R.comb_loops);
    for (uint32_t c = 0; c < R.comb_loops; ++c) R.comb_tau[c] = (uint32_t)(rng.next() & (R.N - 1));
    // estimation-only loops: the next draws, resolved as a plan of their own
    if (p.est_loops > 0) {
        std::vector<uint32_t> es(p.est_loops), et(p.est_loops);
        for (int32_t r = 0; r < p.est_loops; ++r) {
            es[r] = (uint32_t)((rng.next() & (R.N - 1)) | 1u);
            et[r] = (uint32_t)(rng.next() & (R.N - 1));
        }
        sfft_params pe = p;
        pe.B = p.est_B;
        pe.L = p.est_loops;
        pe.w = p.est_w ? p.est_w : p.w * (int64_t)p.est_B / p.B;
        pe.d = 1;
        pe.vote_threshold = p.est_loops;   // keeps the (unused) capacity bound at K N/est_B
        pe.n_resid = 0;
        pe.flags = SFFT_FLAG_NO_RESIDUAL | (p.flags & SFFT_FLAG_XCD_ORDER);
        pe.strip_cols = 0;
        pe.sigma = es.data();
        pe.tau = et.data();
        pe.comb_b = pe.comb_loops = pe.comb_keep = 0;
        pe.est_loops = 0;
        auto E = std::make_shared<Resolved>();
        const sfft_status st = resolve_params(pe, E.get(), err);
        if (st != SFFT_OK) return st;
        E->est_only = 1;
        E->cap = 0;   // no candidates of their own
        E->vote_units = 0;
        E->est_units = 0;
        R.est = std::move(E);
    }
    if (p.sigma) {
        for (uint32_t r = 0; r < R.L; ++r) {
            if (!(p.sigma[r] & 1u) || p.sigma[r] >= R.N || p.tau[r] >= R.N)
                return bad("explicit sigma must be odd and < N, tau < N");
            if (phase && (r & 1) && (p.sigma[r] != p.sigma[r - 1] || p.tau[r] != ((p.tau[r - 1] + 1u) & (R.N - 1))))
                return bad("phase location: explicit loops 2j+1 must repeat sigma_{2j} with tau_{2j}+1");
            R.sigma[r] = p.sigma[r];
            R.tau[r] = p.tau[r];
        }
    } else if (phase) {
        // pairs (2j, 2j+1): same scaling, shifts tau and tau+1 (the odd draws are replaced)
        for (uint32_t r = 1; r < R.L; r += 2) {
            R.sigma[r] = R.sigma[r - 1];
            R.tau[r] = (R.tau[r - 1] + 1u) & (R.N - 1);
        }
    }
    for (uint32_t r = 0; r < R.L; ++r)
        R.sigma_inv[r] = (uint32_t)(inverse_mod_2_64(R.sigma[r]) & (R.N - 1));

    // bucketization form: stream full-height column strips when the L windows
    // touch most of the signal's cache lines (L*w/N > 1/8), else gather.
    uint32_t C = 0;
    if (p.strip_cols) {
        if (!is_pow2((uint64_t)p.strip_cols) || p.strip_cols < 2 || (uint32_t)p.strip_cols > R.B)
            return bad("strip_cols must be a power of two in [2, B]");
        C = (uint32_t)p.strip_cols;
    } else {
        C = std::min<uint32_t>(R.B, std::max<uint32_t>(2u, kStripLdsBytes / (8u * R.M)));
        while (C > 32u && R.L * C > 4u * kFoldNT) C >>= 1;   // at most 4 (loop, column) items per thread
    }
    const bool strip_ok = C >= 2 && (uint64_t)R.M * C * 8ull <= 131072ull;
    if (p.flags & SFFT_FLAG_FOLD_STRIP) {
        if (!strip_ok) return bad("strip bucketization tile does not fit in LDS for this N/B");
        R.mode = 1;
    } else if (p.flags & SFFT_FLAG_FOLD_GATHER) {
        R.mode = 0;
    } else {
        R.mode = (strip_ok && 8ull * R.L * R.w > R.N) ? 1u : 0u;
    }
    R.C = C;
    R.log2C = ilog2(C);
    R.strip_lds = R.M * C * 8u;
    R.fold_units = R.mode ? R.B / C : (R.L * R.B + kFoldNT - 1) / kFoldNT;
    // vote workgroups: chunks of kVoteUnit candidates that never straddle two loops
    R.vote_upl = (R.dK * R.M + kVoteUnit - 1) / kVoteUnit;
    R.vote_units = phase ? (R.L / 2 * R.dK + kDecUnit - 1) / kDecUnit : (R.L - R.T + 1) * R.vote_upl;
    // two-phase vote tests where few buckets are selected (a random candidate rarely gets a
    // second vote among the first L - T + 2 loops) and the threshold is the default majority
    R.vote_split = (!phase && R.L >= 4 && R.L <= 16 && R.T == R.L / 2 + 1 && (uint64_t)R.dK * 32u <= R.B) ? 1u : 0u;
    // Enumeration by loop pairs: the L loops split into T-1 groups of consecutive loops (sizes
    // differ by at most one); any T loops hold two of one group (pigeonhole), so a frequency
    // with >= T votes is voted by both loops of some pair within a group. A pair enumerates
    // its first loop's selected buckets and tests its second loop; the few that pass take the
    // other loops' tests. Cost per enumerated frequency, in bitmap tests: by loop L-1 (or, in
    // two phases, the first phase's tests plus the rest for the share with a second vote), by
    // pair 1 + 25 (L-2) q with q = dK/B (the rest is gathered across the wave, 64 positions
    // per round, and tested one frequency per lane with a list reservation per round), each
    // plus 6 for the chunk's fixed work (slots, barriers, list reservation) over the chunk's
    // runs of kVoteUnit. The weights are fitted to vote timings at q = 1.2%, 3%, 9.8% and 12%:
    // pairs pay off where few buckets are selected.
    R.vote_pairs = 0;
    R.vote_sub = 1;
    memset(R.vote_pair, 0, sizeof(R.vote_pair));
    if (!phase && R.T >= 2) {
        const uint32_t g = R.T - 1, base = R.L / g, extra = R.L % g;
        uint32_t np = 0, first = 0;
        for (uint32_t i = 0; i < g; ++i) {
            const uint32_t size = base + (i < extra ? 1u : 0u);
            for (uint32_t a = first; a < first + size; ++a)
                for (uint32_t b = a + 1; b < first + size; ++b) {
                    if (np < SFFT_MAX_VOTE_PAIRS) R.vote_pair[np] = (uint16_t)(a | (b << 8));
                    ++np;
                }
            first += size;
        }
        const double q = (double)R.dK / (double)R.B;
        double by_loop = (double)(R.L - 1);
        if (R.vote_split) {
            const uint32_t P1 = R.L - R.T + 2;
            by_loop = (double)(P1 - 1) + 3.0 * (1.0 - pow(1.0 - q, (double)(P1 - 1))) * (double)(R.L - P1);
        }
        const double sub = R.log2M >= 4 ? (double)kVotePairSub : 1.0;
        const double cost_loop = (double)(R.L - R.T + 1) * (by_loop + 6.0);
        const double cost_pair = (double)np * (1.0 + 25.0 * q * (double)(R.L - 2) + 6.0 / sub);
        const bool fits = np >= 1 && np <= SFFT_MAX_VOTE_PAIRS;
        if (p.flags & SFFT_FLAG_VOTE_BY_PAIR) {
            if (!fits) return bad("vote by pairs needs T >= 2 and at most 32 loop pairs");
            R.vote_pairs = np;
        } else if (!(p.flags & SFFT_FLAG_VOTE_BY_LOOP) && fits && cost_pair < cost_loop) {
            R.vote_pairs = np;
        }
        if (!R.vote_pairs) memset(R.vote_pair, 0, sizeof(R.vote_pair));
    } else if (p.flags & SFFT_FLAG_VOTE_BY_PAIR) {
        return bad("vote by pairs needs T >= 2 and location by votes");
    }
    if ((p.flags & SFFT_FLAG_VOTE_BY_PAIR) && (p.flags & SFFT_FLAG_VOTE_BY_LOOP))
        return bad("SFFT_FLAG_VOTE_BY_PAIR and SFFT_FLAG_VOTE_BY_LOOP are exclusive");
    if (R.vote_pairs) {
        R.vote_sub = R.log2M >= 4 ? kVotePairSub : 1u;
        const uint32_t chunk = R.vote_sub * kVoteUnit;
        R.vote_upl = (R.dK * R.M + chunk - 1) / chunk;
        R.vote_units = R.vote_pairs * R.vote_upl;
    }
    const uint32_t wpl = (R.B + 31) / 32;
    const uint32_t vbytes = (R.L * wpl * 4u + 15u) & ~15u;
    R.vote_lds = vbytes <= 98304u ? vbytes : 0u;   // bitmaps staged in LDS up to 96 KB (B = 65536 at L <= 12)
    R.vote_dyn_lds = vote_slot_words(R.log2M, R.vote_sub) * 4u + R.vote_lds;
    // B-point FFT: in one workgroup's LDS up to kMaxFftLds, else two passes
    // (B = B1 * B2, tiles of 16 sequences per workgroup) and a selection workgroup per loop
    R.fft_mode = (R.B > (uint32_t)kMaxFftLds || (p.flags & SFFT_FLAG_FFT_TWO_PASS)) ? 1u : 0u;
    if (R.fft_mode) {
        const uint32_t lb1 = (R.log2B + 1) / 2, lb2 = R.log2B / 2;
        R.fft_p1_units = R.L * ((1u << lb2) / 16u);
        R.fft_p2_units = R.L * ((1u << lb1) / 16u);
    }
    // residual: a wave's lanes are (run, output subset) pairs, 2^resid_log2kl subsets per run:
    // 8 (16 from K = 512) for many outputs; below K = 64 about 16 outputs per lane, so that a
    // small plan's residual takes a few workgroups per signal instead of 16 (each workgroup
    // stages the outputs and their phase steps once)
    R.resid_log2kl = R.K >= 512 ? 4u : (R.K > 64 ? 3u : (ilog2(R.K) > 4u ? ilog2(R.K) - 4u : 0u));
    {
        const uint32_t runs = (R.S + kResRun - 1) / kResRun;
        const uint32_t runs_per_wg = (kResNT / 64u) * (64u >> R.resid_log2kl);
        R.resid_blocks = (runs + runs_per_wg - 1) / runs_per_wg;
    }
    uint32_t P = 1;
    while (P < R.K) P <<= 1;
    R.resid_lds = R.K * 16u + R.K * 8u + R.K * 4u;   // staged outputs: e^{+2 pi i f/N}, values, frequencies
    R.fin_lds = P * 8u + P * 4u;         // selected values, frequencies (sort size P)
    R.iterate = (p.flags & SFFT_FLAG_ITERATE) ? 1u : 0u;
    // estimation workgroups stride over the candidates, so their number only sets the
    // parallelism: about one candidate per thread for the expected count, at most 32.
    // Voting: K plus the false frequencies, N P(Binom(L, dK/B) >= T) (each loop selects a
    // bucket of a random frequency with probability dK/B); phase location: the capacity.
    double expect = (double)R.cap;
    if (!phase) {
        const double q = std::min(1.0, (double)R.dK / (double)R.B);
        double tail = 0.0, c = 1.0;   // c = binomial coefficient C(L, j)
        for (uint32_t j = 0; j <= R.L; ++j) {
            if (j >= R.T) tail += c * pow(q, (double)j) * pow(1.0 - q, (double)(R.L - j));
            c = c * (double)(R.L - j) / (double)(j + 1);
        }
        expect = std::min((double)R.cap, (double)R.K + (double)R.N * tail);
    }
    expect += (double)(R.K * R.iterate);
    R.est_units = (uint32_t)std::max(1.0, std::min(32.0, std::ceil(expect / (double)kFinNT)));
    // subtraction round: phased values [K], sort keys [P], offsets [K], run starts [B] (16 bit)
    R.sub_lds = R.iterate ? ((R.K * 8u + P * 4u + R.K * 4u + R.B * 2u + 15u) & ~15u) : 0u;
    if (R.iterate) {
        const sfft_status st = subtraction_reach(&R, err);
        if (st != SFFT_OK) return st;
    }
    R.xcd_order = (p.flags & SFFT_FLAG_XCD_ORDER) ? 1u : 0u;
    R.fold_variant = fold_variant(R.mode, R.strip_lds, R.L << R.log2C, R.Mw4 / 4);
    R.fused = 0;
    R.fused_lds = 0;
    if (p.flags & SFFT_FLAG_FUSED) {
        // one workgroup per signal: the transform in its LDS with B/16 <= 256, at most 4 selected
        // outputs per thread, one vote kernel instance per L, the bitmaps staged in LDS; the
        // buckets are gathered, and none of the extra rounds or loops
        const uint32_t extra = SFFT_FLAG_ITERATE | SFFT_FLAG_PHASE_LOCATION | SFFT_FLAG_FFT_TWO_PASS | SFFT_FLAG_FOLD_STRIP;
        if ((p.flags & extra) || R.comb_loops || R.est || R.log2B < kFusedLog2BMin || R.log2B > kFusedLog2BMax ||
            R.L > kFusedMaxL || R.K > kFusedMaxK || !R.vote_lds) {
            *err = "SFFT_FLAG_FUSED needs 32 <= B <= 4096, L <= 16, K <= 1024 and no subtraction round, phase "
                   "location, two-pass FFT, strip bucketization, comb prefilter or estimation-only loops";
            return SFFT_E_UNSUPPORTED;
        }
        R.fused = 1;
        R.mode = 0;
        R.fold_variant = fold_variant(0u, 0u, 0u, 0u);
        R.fused_lds = std::max({fused_fft_lds(R.log2B), R.vote_dyn_lds, R.fin_lds, R.S ? R.resid_lds : 0u});
    }
    *out = std::move(R);
    return SFFT_OK;
}

void build_tables(const Resolved& R, HostTables* t) {
    const double pi = 3.14159265358979323846;
    const uint32_t N = R.N, B = R.B, M = R.M, w = R.w;
    // flat window: Gaussian (Eq.(13)) times sinc (Eq.(12), read as
    // sin(pi t/B)/(pi t) with centre value 1/B), centred at n = w/2,
    // Gaussian std = w / (2 gauss_c)
    t->window.resize(w);
    const double s = (double)w / (2.0 * R.gauss_c);
    for (uint32_t n = 0; n < w; ++n) {
        const double tt = (double)n - (double)w / 2.0;
        const double gauss = exp(-0.5 * (tt / s) * (tt / s));
        const double sinc = (tt == 0.0) ? 1.0 / (double)B : sin(pi * tt / (double)B) / (pi * tt);
        t->window[n] = gauss * sinc;
    }
    // e^{+2 pi i m/N} = hi[m >> rsh] * lo[m & (2^rsh - 1)]
    const uint32_t nlo = 1u << R.rsh, nhi = N >> R.rsh;
    t->rt_lo.resize(2 * (size_t)nlo);
    t->rt_hi.resize(2 * (size_t)nhi);
    for (uint32_t m = 0; m < nlo; ++m) {
        const double a = 2.0 * pi * (double)m / (double)N;
        t->rt_lo[2 * m] = cos(a);
        t->rt_lo[2 * m + 1] = sin(a);
    }
    for (uint32_t m = 0; m < nhi; ++m) {
        const double a = 2.0 * pi * (double)((uint64_t)m << R.rsh) / (double)N;
        t->rt_hi[2 * m] = cos(a);
        t->rt_hi[2 * m + 1] = sin(a);
    }
    // roots of unity e^{2 pi i j / 2^tb} (device phases: table entry times a short series)
    t->rou.resize(2u << R.tb);
    for (uint32_t j = 0; j < (1u << R.tb); ++j) {
        const double a = 2.0 * pi * (double)j / (double)(1u << R.tb);
        t->rou[2 * j] = cos(a);
        t->rou[2 * j + 1] = sin(a);
    }
    // gain table Gtab[o] = sum_n g_n e^{+2 pi i (n o mod N)/N}, exact FP64 sum, at
    // o = -M/2 .. M/2-1; with the subtraction round at the offsets of every bucket in
    // its reach too, o = -(sub_rh M + M/2) .. (sub_rl M + M/2) - 1, of which the M
    // entries from sub_rh M on are Gtab
    const uint32_t G = R.iterate ? (R.sub_rl + R.sub_rh + 1) * M : M;
    const uint32_t gc = R.iterate ? R.sub_rh * M + M / 2 : M / 2;   // index of o = 0
    std::vector<std::complex<double>>& gout = R.iterate ? t->gain_wide : t->gain;
    gout.assign(G, std::complex<double>(0.0, 0.0));
    const uint32_t lomask = nlo - 1;
    auto work = [&](uint32_t k0, uint32_t k1) {
        for (uint32_t k = k0; k < k1; ++k) {
            const int64_t o = (int64_t)k - (int64_t)gc;
            const uint32_t step = (uint32_t)((o % (int64_t)N + (int64_t)N) % (int64_t)N);
            double re = 0.0, im = 0.0;
            uint32_t m = 0;  // n * o mod N, advanced by step
            for (uint32_t n = 0; n < w; ++n) {
                const double* hi = &t->rt_hi[2 * (size_t)(m >> R.rsh)];
                const double* lo = &t->rt_lo[2 * (size_t)(m & lomask)];
                const double c = hi[0] * lo[0] - hi[1] * lo[1];
                const double sn = hi[0] * lo[1] + hi[1] * lo[0];
                re += t->window[n] * c;
                im += t->window[n] * sn;
                m = (m + step) & (N - 1);
            }
            gout[k] = std::complex<double>(re, im);
        }
    };
    const uint64_t work_total = (uint64_t)G * w;
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (work_total < (1u << 20)) nth = 1;
    nth = std::min<unsigned>(nth, G);
    std::vector<std::thread> th;
    for (unsigned i = 0; i < nth; ++i) {
        const uint32_t k0 = (uint32_t)((uint64_t)G * i / nth), k1 = (uint32_t)((uint64_t)G * (i + 1) / nth);
        th.emplace_back(work, k0, k1);
    }
    for (auto& x : th) x.join();
    if (R.iterate) {
        const size_t g0 = (size_t)R.sub_rh * M;
        t->gain.assign(t->gain_wide.begin() + g0, t->gain_wide.begin() + g0 + M);
        t->gw.resize(2 * (size_t)G);
        for (uint32_t k = 0; k < G; ++k) {
            t->gw[2 * k] = (float)t->gain_wide[k].real();
            t->gw[2 * k + 1] = (float)t->gain_wide[k].imag();
        }
    }
    // device tables (the window taps themselves are computed by the bucketization kernels)
    t->invG.resize(2 * (size_t)M);
    for (uint32_t k = 0; k < M; ++k) {
        const std::complex<double> inv = 1.0 / t->gain[k];
        t->invG[2 * k] = (float)inv.real();
        t->invG[2 * k + 1] = (float)inv.imag();
    }
    t->tw.resize(2 * (size_t)B);
    for (uint32_t m = 0; m < B; ++m) {
        const double a = -2.0 * pi * (double)m / (double)B;
        t->tw[2 * m] = (float)cos(a);
        t->tw[2 * m + 1] = (float)sin(a);
    }
    t->ctw.resize(2 * (size_t)R.comb_b);
    for (uint32_t m = 0; m < R.comb_b; ++m) {
        const double a = -2.0 * pi * (double)m / (double)R.comb_b;
        t->ctw[2 * m] = (float)cos(a);
        t->ctw[2 * m + 1] = (float)sin(a);
    }
}

WsLayout workspace_layout(const Resolved& R) {
    WsLayout l{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + std::max<size_t>(bytes, 16));
        return o;
    };
    const size_t wpl = (R.B + 31) / 32;
    l.uhat = take((size_t)R.L * R.B * 8);
    l.jbits = take((size_t)R.L * wpl * 4);
    l.jlist = take((size_t)R.L * R.dK * 4);
    l.cand = take((size_t)R.cap * 4);
    const size_t nest = (size_t)R.cap + (R.iterate ? R.K : 0u);   // + the recovered coefficients
    l.est = take(nest * 8);
    l.keys = take(nest * 8);
    l.rpart = take((size_t)std::max<uint32_t>(R.resid_blocks, 1) * 16);
    l.resid_own = take(16);
    l.ctr = take(16);
    l.ubuf = take(R.fft_mode ? (size_t)R.L * R.B * 8 : 16);
    l.gmax = take(R.fft_mode ? (size_t)R.L * (R.B / 16) * 4 : 16);
    l.cbits = take((size_t)R.comb_loops * R.comb_words * 4);
    l.rec_f = take(R.iterate ? (size_t)R.K * 4 : 16);
    l.rec_v = take(R.iterate ? (size_t)R.K * 8 : 16);
    l.total = off;
    return l;
}

TabLayout table_layout(const Resolved& R) {
    TabLayout l{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + std::max<size_t>(bytes, 16));
        return o;
    };
    l.sigma = take((size_t)R.L * 4);
    l.sigma_inv = take((size_t)R.L * 4);
    l.tau = take((size_t)R.L * 4);
    l.tpos = take((size_t)R.S * 4);
    l.invG = take((size_t)R.M * 8);
    l.tw = take((size_t)R.B * 8);
    l.rou = take((size_t)16 << R.tb);
    l.ctau = take((size_t)R.comb_loops * 4);
    l.ctw = take((size_t)R.comb_b * 8);
    l.gw = take(R.iterate ? (size_t)(R.sub_rl + R.sub_rh + 1) * R.M * 8 : 16);
    l.total = off;
    return l;
}

}  // namespace sfft

namespace sfft {

std::vector<char> pack_tables(const Resolved& R, const HostTables& T) {
    const TabLayout tl = table_layout(R);
    std::vector<char> h(tl.total, 0);
    memcpy(&h[tl.sigma], R.sigma.data(), (size_t)R.L * 4);
    memcpy(&h[tl.sigma_inv], R.sigma_inv.data(), (size_t)R.L * 4);
    memcpy(&h[tl.tau], R.tau.data(), (size_t)R.L * 4);
    if (R.S) memcpy(&h[tl.tpos], R.tpos.data(), (size_t)R.S * 4);
    memcpy(&h[tl.invG], T.invG.data(), T.invG.size() * 4);
    memcpy(&h[tl.tw], T.tw.data(), T.tw.size() * 4);
    memcpy(&h[tl.rou], T.rou.data(), T.rou.size() * 8);
    if (R.comb_loops) {
        memcpy(&h[tl.ctau], R.comb_tau.data(), (size_t)R.comb_loops * 4);
        memcpy(&h[tl.ctw], T.ctw.data(), T.ctw.size() * 4);
    }
    if (R.iterate) memcpy(&h[tl.gw], T.gw.data(), T.gw.size() * 4);
    return h;
}

}  // namespace sfft
