// Shared host/device definitions of the gfx950 sparse-FFT path.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sfft.h"

namespace sfft {

constexpr int kMaxL = 32;        // loops supported (bitmaps, median sorting network)
constexpr int kMaxK = 4096;      // outputs supported (final sort in LDS)
constexpr int kMaxFftLds = 16384;  // largest B transformed inside one workgroup's LDS
constexpr int kMaxB = 1 << 18;     // larger B: two-pass (four-step) FFT through the workspace
constexpr int kRouMax = 256;       // entries of the FP64 root-of-unity table
constexpr int kMaxCombLoops = 8;   // comb prefilter loops
constexpr int kMaxCombB = 16384;   // comb size (one workgroup's LDS FFT)

// Per-signal execution descriptor: plan tables (read only, shared by every
// execution of a plan) plus one workspace. Lives in device memory; kernels
// read it through uniform (scalar) loads.
struct SigDesc {
    // plan tables
    const uint32_t* sigma;      // [L] odd scalings
    const uint32_t* sigma_inv;  // [L] inverses mod N
    const uint32_t* tau;        // [L] shifts
    const float2* invG;         // [M] 1/Gtab[o], o = -M/2 .. M/2-1
    const float2* tw;           // [B] e^{-2 pi i m/B}
    const uint32_t* tpos;       // [S] residual sample positions
    const double2* rou;         // [2^tb] e^{2 pi i j / 2^tb}, FP64
    const uint32_t* comb_tau;   // [comb_loops] time shifts of the comb prefilter
    const float2* ctw;          // [Bc] e^{-2 pi i m/Bc}
    const float2* gw;           // [(sub_rl+sub_rh+1) M] gain at offsets o in [-c, (sub_rl+sub_rh+1) M - c),
                                // c = sub_rh M + M/2: gw[o + c] (iteration only)
    // workspace
    float2* uhat;               // [L][B] bucket values in column order (bucket of column col is
                                // sigma^{-1}(col - tau) mod B), then their B-point DFT in bucket order
    uint32_t* jbits;            // [L][B/32] selected buckets
    uint32_t* jlist;            // [L][dK] selected buckets, ascending
    uint32_t* cand;             // [cap] frequencies with >= T votes
    float2* est;                // [cap (+ K with iteration)] median estimates
    uint64_t* keys;             // [cap (+ K with iteration)] ordering keys of the estimates
    double* rpart;              // [2 * resid_blocks] residual partial sums
    double* resid_own;          // [2] residual when the caller gives no buffer
    uint32_t* ctr;              // [4] counters: 0 candidates, 2 first-round outputs, 3 residual workgroups
                                // done (single-signal residual); 0 and 3 cleared by the bucketization
    float2* ubuf;               // [L][B] two-pass FFT intermediate (B > kMaxFftLds only)
    uint32_t* cbits;            // [comb_loops][max(1, Bc/32)] residues kept by each comb loop
    uint32_t* gmax;             // [L][B/16] largest energy of each 16 consecutive DFT outputs (idem)
    uint32_t* rec_f;            // [K] first-round frequencies, ascending, 0xFFFFFFFF padded (iteration only)
    float2* rec_v;              // [K] first-round values
    // sizes
    uint32_t N, maskN, log2N;
    uint32_t B, log2B;
    uint32_t M, log2M;          // M = N/B (bucket width in bins = rows of the strip view)
    uint32_t L, w, Mw, Mw4;     // Mw = ceil(w/B) window taps per bucket, Mw4 = Mw rounded up to 4
    float wkappa;               // Gaussian factor of the window: e^{-t^2/2s^2} = 2^{-(t wkappa)^2}
    uint32_t K, dK, T, S, cap;
    uint32_t tb;                // root-of-unity table bits, min(8, log2N)
    double step;                // 2 pi / N
    uint32_t mode;              // 0 gather, 1 strip
    uint32_t fft_mode;          // 0: one-workgroup FFT, uhat in bucket order; 1: two-pass FFT of the
                                // column-order values, uhat[r][m] = V[m] with bucket h <-> m = sigma_r^{-1} h mod B
    uint32_t C, log2C, strips;  // strip bucketization tile: C columns x M rows
    uint32_t vote_units;        // vote workgroups
    uint32_t vote_upl;          // vote workgroups per enumerated loop (chunks of kVoteUnit candidates)
    uint32_t vote_split;        // 1: votes tested in two phases (few selected buckets, T = L/2 + 1)
    uint32_t vote_pairs;        // 0: enumeration by loop; else by these loop pairs (vote_pair)
    uint32_t vote_sub;          // kVoteUnit-candidate runs per vote chunk (by pair at N/B >= 16: kVotePairSub)
    uint16_t vote_pair[SFFT_MAX_VOTE_PAIRS];   // first loop | second loop << 8
    uint32_t resid_blocks;      // residual workgroups
    uint32_t resid_log2kl;      // residual: lanes per run (the outputs split 2^resid_log2kl ways)
    uint32_t est_units;         // estimation workgroups (striding over the candidates)
    uint32_t lmax;              // power of two >= L used by the median network
    uint32_t combine;           // 0: coordinate-wise median over the loops, 1: mean
    uint32_t comb_loops;        // comb prefilter loops (0 = off)
    uint32_t comb_log2b;        // log2 Bc
    uint32_t comb_keep;         // residues kept per comb loop
    uint32_t iterate;           // 1: one subtraction round after the first recovery
    uint32_t sub_rl, sub_rh;    // subtraction reach in buckets below / above a coefficient's own
    uint32_t phase;             // 1: location by phase encoding over loop pairs (2j, 2j+1)
    const SigDesc* eloops;      // estimation-only loops of the same signal (own B, window, tables), or null
    uint32_t L_est;             // their number
};

// Per-signal caller buffers of one execution.
struct IoDesc {
    const float2* x;            // [N]
    int64_t* out_idx;           // [K]
    float2* out_val;            // [K]
    double* out_resid;          // [2] or nullptr
};

// Kernel argument: either one signal (nsig == 0: desc = descs[0], io = one_io,
// unit = blockIdx.x) or a batch (unit -> signal through prefix[0..nsig]).
struct Launch {
    const SigDesc* descs;
    const IoDesc* ios;
    const uint32_t* prefix;     // [nsig+1] exclusive prefix of units per signal
    uint32_t nsig;
    uint32_t xcd_order;         // 1: consecutive units run on the same XCD (see xcd_unit)
    IoDesc one_io;
};

constexpr uint32_t kNumXcd = 8;  // MI355X: 8 accelerator complex dies, workgroups dealt round-robin

constexpr uint32_t kVoteNT = 256;
constexpr uint32_t kVotePerThread = 16;
constexpr uint32_t kVoteUnit = kVoteNT * kVotePerThread;  // candidates per vote workgroup
// Vote grid cap: at most this many workgroups (a few per compute unit of the 256), each
// looping over its share of the chunks, so that a vote launch does not take every compute
// unit's LDS and wave slots from the bucketization running beside it on another stream.
constexpr uint32_t kVoteMaxGrid = 4u * 256u;
// LDS words for the selected-bucket slots one vote workgroup enumerates (N/B = 2^log2M
// candidates per slot), a multiple of 4 so the staged bitmaps after them stay 16-byte aligned
constexpr uint32_t kVotePairSub = 4;   // by pair (N/B >= 16): kVoteUnit-candidate runs per chunk
// selected-bucket slot words of a chunk of sub * kVoteUnit candidates
__host__ __device__ constexpr uint32_t vote_slot_words(uint32_t log2M, uint32_t sub = 1u) {
    return (((sub * kVoteUnit) >> log2M) + 1u + 3u) & ~3u;
}
// Vote kernel instance of a plan with L location loops: L itself up to 16, else 32.
__host__ __device__ constexpr uint32_t vote_key(uint32_t L) { return L <= 16u ? L : 32u; }
constexpr uint32_t kVoteKeys = 17;   // distinct vote_key values
constexpr uint32_t kFoldNT = 256;
constexpr uint32_t kFftNT = 256;
constexpr uint32_t kFinNT = 256;   // estimation workgroups
constexpr uint32_t kSelNT = 1024;  // top-K selection workgroup (one per signal)
constexpr uint32_t kResNT = 256;
constexpr uint32_t kResRun = 8;        // residual positions per run (consecutive samples, one 64-byte line)
constexpr uint32_t kSubNT = 256;
constexpr uint32_t kDecPerThread = 4;                     // decoded buckets per thread
constexpr uint32_t kDecUnit = kVoteNT * kDecPerThread;    // decoded buckets per workgroup
constexpr uint32_t kStripLdsBytes = 65536;  // strip tile budget
// fused single-launch form (small plans, one workgroup per signal)
constexpr uint32_t kFusedNT = 256;          // threads of its workgroup
constexpr uint32_t kFusedMaxK = 1024;       // K it supports (selected entries: 4 per thread)
constexpr uint32_t kFusedLog2BMin = 5, kFusedLog2BMax = 12;   // B = 32 .. 4096
constexpr uint32_t kFusedMaxL = 16;
constexpr uint32_t kFusedMaxGrid = 2048;    // persistent workgroups of one launch (8 per compute unit)

}  // namespace sfft
