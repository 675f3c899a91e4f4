// Host-side plan logic (pure C++, no device calls): parameter validation,
// random permutations, FP64 window / gain / twiddle / phase tables.
#pragma once

#include <stdint.h>

#include <complex>
#include <memory>
#include <string>
#include <vector>

#include "../../include/sfft.h"

namespace sfft {

// Every derived size of a validated parameter set.
struct Resolved {
    uint32_t N, K, B, L, d, w, T, S;
    uint32_t dK, M, Mw, Mw4, cap, lmax;
    uint32_t rsh;               // two-field split of the host gain-table phases
    uint32_t tb;                // device root-of-unity table bits, min(8, log2N)
    uint32_t log2N, log2B, log2M;
    uint32_t mode, C, log2C;    // bucketization form (0 gather, 1 strip) and strip width
    uint32_t fft_mode;          // 0 one-workgroup FFT (B <= 16384), 1 two-pass FFT
    uint32_t comb_b, comb_log2b, comb_loops, comb_keep, comb_words;  // comb prefilter
    uint32_t iterate, sub_lds;  // one subtraction round (iterative framework); its LDS bytes
    uint32_t sub_rl, sub_rh;    // subtraction reach: a coefficient is removed from buckets h0 - sub_rl .. h0 + sub_rh
    double sub_bound;           // bound on what it leaves beyond them, relative to the centre gain
    uint32_t phase;             // location by phase encoding over loop pairs
    uint32_t est_only;          // a plan's estimation-only loops (bucketization + FFT only)
    std::shared_ptr<const struct Resolved> est;  // the estimation-only loops of this plan, or null
    std::vector<uint32_t> comb_tau;
    uint32_t fft_p1_units, fft_p2_units;   // two-pass FFT workgroups per signal
    uint64_t seed;
    double gauss_c;
    uint32_t flags;
    std::vector<uint32_t> sigma, sigma_inv, tau, tpos;
    // units per stage
    uint32_t fold_units, vote_units, vote_upl, resid_blocks, vote_lds, strip_lds, resid_lds, fin_lds;
    uint32_t resid_log2kl;      // residual: lanes per run, log2
    uint32_t vote_split;        // votes in two phases (dK/B <= 1/32, T = L/2 + 1, 4 <= L <= 16)
    uint32_t vote_pairs;        // 0: votes enumerated by loop; else the number of loop pairs
    uint32_t vote_sub;          // kVoteUnit-candidate runs per vote chunk
    uint16_t vote_pair[SFFT_MAX_VOTE_PAIRS];   // pair e: first loop | second loop << 8
    uint32_t vote_dyn_lds;      // vote dynamic LDS: slot words + staged bitmaps (vote_lds, 0 = not staged)
    uint32_t est_units;
    uint32_t L_est() const { return est ? est->L : 0u; }
    uint32_t xcd_order;
    uint32_t fold_variant;      // bucketization kernel variant (kernels.hpp fold_variant)
    uint32_t fused, fused_lds;  // the whole path in one workgroup of one launch; its dynamic LDS bytes
};

struct HostTables {
    std::vector<double> window;                 // g_n, n < w
    std::vector<std::complex<double>> gain;     // Gtab[o], o = -M/2 .. M/2-1
    std::vector<std::complex<double>> gain_wide;  // [(sub_rl+sub_rh+1) M] gain at o = -(sub_rh M + M/2) ..
                                                  // (sub_rl M + M/2) - 1 (iteration only)
    std::vector<float> invG;                    // [M] (re, im) pairs of 1/Gtab
    std::vector<float> tw;                      // [B] (re, im) pairs of e^{-2 pi i m/B}
    std::vector<double> rt_hi, rt_lo;           // (re, im) pairs of e^{+2 pi i m/N}, two bit fields
    std::vector<double> rou;                    // (re, im) pairs of e^{2 pi i j / 2^tb}
    std::vector<float> ctw;                     // [comb_b] (re, im) pairs of e^{-2 pi i m/comb_b}
    std::vector<float> gw;                      // (re, im) pairs of gain_wide (iteration only)
};

constexpr double kDefaultGaussC = 4.861870431316438;  // 516 / (2 * 16 * sqrt(11)), Fig. 1 example

// Validate p and derive every size. On failure returns a status and sets *err.
sfft_status resolve_params(const sfft_params& p, Resolved* out, std::string* err);

// FP64 tables of a resolved plan (window, gain, and the float tables the GPU reads).
void build_tables(const Resolved& R, HostTables* t);

// SplitMix64 (Steele, Lea & Flood 2014): Weyl counter + xor-shift-multiply finaliser.
struct SplitMix64 {
    uint64_t state;
    explicit SplitMix64(uint64_t seed) : state(seed) {}
    uint64_t next() {
        state += 0x9E3779B97F4A7C15ull;
        uint64_t z = state;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
};

// Inverse of an odd a modulo 2^64 by Newton's iteration x <- x (2 - a x), which
// doubles the number of correct low bits each step (a*a == 1 mod 8 for odd a).
inline uint64_t inverse_mod_2_64(uint64_t a) {
    uint64_t x = a;
    for (int i = 0; i < 5; ++i) x *= 2ull - a * x;
    return x;
}

inline bool is_pow2(uint64_t v) { return v && !(v & (v - 1)); }
inline uint32_t ilog2(uint64_t v) {
    uint32_t r = 0;
    while ((1ull << r) < v) ++r;
    return r;
}

// Device workspace layout of one execution (byte offsets, 256-aligned).
struct WsLayout {
    size_t uhat, jbits, jlist, cand, est, keys, rpart, resid_own, ctr, ubuf, gmax, cbits, rec_f, rec_v, total;
};
WsLayout workspace_layout(const Resolved& R);

// Device table layout (byte offsets into one allocation).
struct TabLayout {
    size_t sigma, sigma_inv, tau, tpos, invG, tw, rou, ctau, ctw, gw, total;
};
TabLayout table_layout(const Resolved& R);

// The device table image of a plan (table_layout(R).total bytes), ready to upload.
std::vector<char> pack_tables(const Resolved& R, const HostTables& T);

}  // namespace sfft
