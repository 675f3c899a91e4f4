// Location by votes, estimation, the K largest and the FP64 residual: device bodies
// shared by the per-stage kernels and the fused single-signal kernel. A body runs on one
// workgroup for unit `unit` of signal `sig` of a launch.
#pragma once

#include "device.hpp"

namespace sfft {

// Whether f is among the n ascending entries of a (binary search in global memory).
__device__ __forceinline__ bool in_sorted(const uint32_t* a, uint32_t n, uint32_t f) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (gld(a + mid) < f) lo = mid + 1u; else hi = mid;
    }
    return lo < n && gld(a + lo) == f;
}

// Append each lane's candidates (bit qq of emask: fv[qq]) to the unordered
// candidate list with one reservation per wave that has any (no block barrier).
template <int P>
__device__ __forceinline__ void append_wave(const uint32_t (&fv)[P], uint32_t emask, uint32_t* ctr, uint32_t* cand,
                                            uint32_t cap) {
    if (__ballot(emask != 0u) == 0ull) return;   // wave-uniform
    const uint32_t cnt = (uint32_t)__popc(emask);
    const uint32_t incl = wave_incl_scan(cnt);
    const uint32_t total = __shfl(incl, 63, 64);
    uint32_t base = 0;
    if ((threadIdx.x & 63u) == 63u) base = atomicAdd(ctr, total);
    uint32_t pos = __shfl(base, 63, 64) + incl - cnt;
#pragma unroll
    for (int qq = 0; qq < P; ++qq) {
        if ((emask >> qq) & 1u) {
            if (pos < cap) gst(cand + pos, fv[qq]);
            ++pos;
        }
    }
}

// ---------------------------------------------------------------- votes
// A frequency with >= T votes out of L is voted by one of the loops 0..L-T
// (pigeonhole), so only the frequencies of those loops' selected buckets are
// enumerated: f = sigma_r0^{-1} p for the N/B permuted positions p of each
// selected bucket. Each frequency is counted from the first loop that voted
// for it (later loops skip it), so I' has no duplicates; votes are bitmap tests.
// In the subtraction round (round 1) the frequencies recovered by the first
// round are not candidates again.
//
// By loop pair (vote_pairs > 0): the loops split into T-1 groups of consecutive loops, so any
// T loops hold two of one group and every frequency with >= T votes is voted by both loops of
// some pair within a group. Pair (r0, r1) enumerates loop r0's selected buckets like a loop
// does, tests loop r1 first, and finishes only those r1 voted for; a frequency is counted from
// the first pair in list order whose two loops both voted for it. Same candidate set.
//
// Loop r hashes f = sigma_r0^{-1} p to bucket ((c_r p + N/2B) mod N) >> log2(N/B)
// with c_r = sigma_r sigma_r0^{-1} (mod N, a workgroup constant). A thread takes
// kVotePerThread consecutive positions p of one selected bucket (when N/B allows),
// so each loop's hash argument advances by the constant c_r per candidate (an add
// instead of a multiply) and the bucket is a bit-field of it. Instances: VL = L for
// L <= 16 (every test unconditional); VL = 32 covers 17..32 with the surplus tests
// masked. STAGED: the L selected-bucket bitmaps are copied to LDS first.

// Bit planes a count of at most n needs (at least one).
__host__ __device__ constexpr int vote_planes(int n) {
    int b = 1;
    while ((1 << b) <= n) ++b;
    return b;
}

// Vote counts of a thread's candidates, bit-sliced: bit qq of plane b is bit b of candidate
// qq's count, so one add of a loop's vote mask (bit qq: the loop voted for candidate qq)
// counts it for every candidate at once.
template <int NP>
struct VoteCount {
    uint32_t c[NP];
    __device__ __forceinline__ VoteCount() {
#pragma unroll
        for (int b = 0; b < NP; ++b) c[b] = 0u;
    }
    // x: the mask of the (k+1)-th loop added; a count of at most k+1 has no plane above
    // bit log2(k+1), so the carry stops there
    __device__ __forceinline__ void add(uint32_t x, int k) {
#pragma unroll
        for (int b = 0; b < NP; ++b) {
            if (((k + 1) >> b) == 0) break;
            const uint32_t t = c[b] & x;
            c[b] ^= x;
            x = t;
        }
    }
    // bit qq: candidate qq's count is at least t
    __device__ __forceinline__ uint32_t ge(uint32_t t) const {
        if (t >= (1u << NP)) return 0u;
        uint32_t gt = 0u, eq = 0xffffffffu;
#pragma unroll
        for (int b = NP - 1; b >= 0; --b) {
            if ((t >> b) & 1u) {
                eq &= c[b];
            } else {
                gt |= eq & c[b];
                eq &= ~c[b];
            }
        }
        return gt | eq;
    }
    // candidate qq's count
    __device__ __forceinline__ uint32_t of(uint32_t qq) const {
        uint32_t v = 0u;
#pragma unroll
        for (int b = 0; b < NP; ++b) v |= ((c[b] >> qq) & 1u) << b;
        return v;
    }
};

// One chunk of vote_sub x kVoteUnit candidates (unit `unit` of signal `sig`). sdyn: the
// chunk's selected-bucket slots (vote_slot_words(log2 N/B, vote_sub) words), then (staged) the L
// selected-bucket bitmaps, which (like the comb residues) are copied only when `restage`
// (the workgroup's previous chunk was another signal's).
template <int VL, bool STAGED>
__device__ __forceinline__ void vote_chunk(const Launch& a, uint32_t sig, uint32_t unit, uint32_t round, bool restage,
                                           uint32_t* sdyn, uint32_t* s_comb, uint32_t* s_pq) {
    constexpr bool kExact = VL <= 16;
    constexpr uint32_t kLog2PT = 4;
    static_assert((1u << kLog2PT) == kVotePerThread, "candidates per thread");
    const auto& d = desc_of(a, sig);
    const uint32_t wpl = (d.B + 31u) >> 5;
    const uint32_t L = kExact ? (uint32_t)VL : d.L;
    const uint32_t T = d.T, M = d.M, log2M = d.log2M, maskN = d.maskN, log2B = d.log2B, dK = d.dK;
    const uint32_t* jbits = d.jbits;
    // this workgroup: candidates [start, end) of enumerated loop r0, i.e. the
    // permuted positions of selected-bucket slots slot0 .. slot0 + nslots - 1. By loop the
    // units run over loops r0 = 0..L-T; by pair over the pairs e = (r0, r1), r0 < r1.
    const uint32_t upl = d.vote_upl;
    const uint32_t npair = d.vote_pairs;
    const uint32_t e = unit / upl;
    const uint32_t pr = npair ? (uint32_t)d.vote_pair[e] : 0u;
    const uint32_t r0 = npair ? (pr & 255u) : e;
    const uint32_t r1 = pr >> 8;
    const uint32_t per_loop = dK * M;
    const uint32_t sub = d.vote_sub;   // runs of kVoteUnit candidates in this chunk
    const uint32_t start = (unit - e * upl) * (sub * kVoteUnit);
    const uint32_t end = min(start + sub * kVoteUnit, per_loop);
    const uint32_t slot0 = start >> log2M;
    const uint32_t nslots = ((end - 1u) >> log2M) - slot0 + 1u;
    const uint32_t sinv0 = ((CU32)d.sigma_inv)[r0];
    uint32_t* s_slot = sdyn;
    uint32_t* sbits = sdyn + vote_slot_words(log2M, sub);
    const uint32_t* jl = d.jlist + (size_t)r0 * dK + slot0;
    for (uint32_t i = threadIdx.x; i < nslots; i += kVoteNT) s_slot[i] = gld(jl + i);
    // loop slots: slot 0 is r0 (it voted for every candidate it enumerates, so it is not
    // tested); by loop, slots 1..r0 the loops before it, then the loops after it in order;
    // by pair, slot 1 the pair's second loop r1, then the other loops in order
    uint32_t cr[VL], boff[VL], lp[VL];   // c_r, bitmap offset and loop of each slot: uniform
#pragma unroll
    for (int j = 0; j < VL; ++j) {
        uint32_t r;
        if (j == 0) {
            r = r0;
        } else if (npair) {
            if (j == 1) {
                r = r1;
            } else {
                r = (uint32_t)j - 2u;
                if (r >= r0) ++r;
                if (r >= r1) ++r;
            }
        } else {
            r = (uint32_t)j <= r0 ? (uint32_t)j - 1u : (uint32_t)j;
        }
        const uint32_t rr = kExact ? r : min(r, L - 1u);
        cr[j] = ((CU32)d.sigma)[rr] * sinv0;
        boff[j] = rr * wpl;
        lp[j] = rr;
    }
    const uint32_t ncomb = d.comb_loops, cmask = (1u << d.comb_log2b) - 1u;
    if (ncomb && restage) {
        const uint32_t cw = max(1u, (cmask + 1u) >> 5);
        for (uint32_t i = threadIdx.x; i < cw; i += kVoteNT) {
            uint32_t v = 0;
            for (uint32_t c = 0; c < ncomb; ++c) v |= gld(d.cbits + c * cw + i);
            s_comb[i] = v;
        }
    }
    if (STAGED && restage) {
        // 16-byte loads, four in flight per thread (the LDS copy is sized to whole 16-byte
        // units; the last unit may read up to 12 bytes past the bitmaps, inside the
        // workspace's 256-byte aligned region, into LDS words that are never tested)
        typedef uint32_t u4v __attribute__((ext_vector_type(4)));
        const uint32_t nw4 = (L * wpl + 3u) >> 2;
        const u4v* src = reinterpret_cast<const u4v*>(jbits);
        u4v* dst = reinterpret_cast<u4v*>(sbits);
        for (uint32_t i0 = threadIdx.x; i0 < nw4; i0 += 4 * kVoteNT) {
            u4v t[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) t[e] = gld(src + min(i0 + e * kVoteNT, nw4 - 1u));
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t i = i0 + e * kVoteNT;
                if (log2B < 5u) {   // one word per loop: its B bits repeated (see test_hi)
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        uint32_t v = t[e][c] & ((1u << d.B) - 1u);
                        for (uint32_t sb = d.B; sb < 32u; sb <<= 1) v |= v << sb;
                        t[e][c] = v;
                    }
                }
                if (i < nw4) dst[i] = t[e];
            }
        }
    }
    __syncthreads();
    // whether slot r's loop selected the bucket of hash argument qv, i.e. bits
    // [log2M, log2M + log2B) of qv: its bitmap word (bits above log2M + 5) and the bit in it
    const uint32_t wb_off = log2M + 5u, wb_w = (log2B > 5u ? log2B : 5u) - 5u, hb_w = log2B < 5u ? log2B : 5u;
    auto test1 = [&](int r, uint32_t qv) -> uint32_t {
        const uint32_t word = __builtin_amdgcn_ubfe(qv, wb_off, wb_w);
        const uint32_t hb = __builtin_amdgcn_ubfe(qv, log2M, hb_w);
        uint32_t wd;
        if constexpr (STAGED) wd = sbits[boff[r] + word];
        else wd = gld(jbits + boff[r] + word);
        return kExact || (uint32_t)r < L ? __builtin_amdgcn_ubfe(wd, hb, 1u) : 0u;
    };
    auto test = [&](int r, uint32_t qv) -> uint32_t { return test1(r, qv) << r; };
    // The same test from hi = bits [log2M, log2M + 32) of the hash argument (bucket at bit 0):
    // the bit-field extract takes the bit index from hi's low 5 bits. Below 32 buckets those
    // bits hold log2B bits of the bucket and higher bits of the argument, so the LDS copy
    // repeats each loop's B bits across its word; read from global memory the index is masked.
    auto test_hi = [&](int r, uint32_t hi) -> uint32_t {
        const uint32_t word = __builtin_amdgcn_ubfe(hi, 5u, wb_w);
        uint32_t wd, hb = hi;
        if constexpr (STAGED) {
            wd = sbits[boff[r] + word];
        } else {
            wd = gld(jbits + boff[r] + word);
            hb = __builtin_amdgcn_ubfe(hi, 0u, hb_w);
        }
        return kExact || (uint32_t)r < L ? __builtin_amdgcn_ubfe(wd, hb, 1u) : 0u;
    };
    uint32_t* ctr = d.ctr;
    uint32_t* cand = d.cand;
    const uint32_t cap = d.cap;
    const uint32_t half = M >> 1;
    const uint32_t before_r0 = ((1u << r0) - 1u) << 1;   // slots of the loops before r0
    // >= T votes, counted once: from the first loop that voted (loop r0, slot 0, always did)
    auto voted = [&](uint32_t votes) -> uint32_t {
        return ((votes & before_r0) == 0u && (uint32_t)__popc(votes) >= T) ? 1u : 0u;
    };
    // By pair, a position p whose frequency the pair's two loops voted for: the other loops'
    // tests; it passes with >= T votes, counted from the first pair whose loops both voted.
    const bool n24 = d.log2N <= 24u;   // hash arguments mod N from 24-bit products
    auto pair_passes = [&](uint32_t p) -> bool {
        uint32_t cnt = 2u, vset = (1u << r0) | (1u << r1);
        const uint32_t pm24 = p & maskN;
#pragma unroll
        for (int j = 2; j < VL; ++j) {
            const uint32_t qv = (n24 ? __umul24(cr[j] & maskN, pm24) : cr[j] * p) + half;
            const uint32_t b = test1(j, qv);
            cnt += b;
            vset |= b << lp[j];
        }
        if (cnt < T) return false;
        for (uint32_t e2 = 0; e2 < e; ++e2) {
            const uint32_t q2 = d.vote_pair[e2];
            const uint32_t pm = (1u << (q2 & 255u)) | (1u << (q2 >> 8));
            if ((vset & pm) == pm) return false;
        }
        return true;
    };
    uint32_t fv[kVotePerThread];
    uint32_t emask = 0;   // bit qq: candidate qq of this thread passes
    if (log2M >= kLog2PT) {
        // candidates ci0 .. ci0 + kVotePerThread - 1: consecutive positions of one bucket
        // (the chunk bounds are multiples of kVotePerThread here). Each tested slot r keeps
        // a mask m[r] (bit qq: its loop voted for candidate qq); the votes of the thread's
        // candidates are then counted bit-sliced over those masks.
        const uint32_t ci0 = start + (threadIdx.x << kLog2PT);
        uint32_t p0 = 0;
        if (npair) {   // block-uniform
            // Each of the chunk's runs of kVoteUnit candidates: the pair's second loop for this
            // thread's 16 (bit 16 s + qq of m1: run s, candidate qq). Then the positions it voted
            // for, compacted across the wave (an exclusive scan of the lanes' counts) and taken 64
            // at a time, one per lane: the other loops' tests, the comb residue, the recovered
            // set and the list.
            static_assert(kVotePairSub == 4, "the run's base position is picked from four");
            uint32_t p0s[kVotePairSub];
            uint64_t m1 = 0u;
            const uint32_t sh = 32u - log2M;
#pragma unroll
            for (uint32_t sr = 0; sr < kVotePairSub; ++sr) {
                p0s[sr] = 0u;
                const uint32_t cs = ci0 + sr * kVoteUnit;
                if (sr < sub && cs < end) {
                    const uint32_t h = s_slot[(cs >> log2M) - slot0];
                    p0s[sr] = (h << log2M) - half + (cs & (M - 1u));
                    uint64_t q1 = (uint64_t)(cr[1] * p0s[sr] + half) << sh;
                    const uint64_t c1q = (uint64_t)cr[1] << sh;
                    uint32_t mr = 0u;
#pragma unroll
                    for (uint32_t qq = 0; qq < kVotePerThread; ++qq) {
                        mr |= test_hi(1, (uint32_t)(q1 >> 32)) << qq;
                        q1 += c1q;
                    }
                    m1 |= (uint64_t)mr << (kVotePerThread * sr);
                }
            }
            uint32_t* wq = s_pq + (threadIdx.x & ~63u);
            const uint32_t lane = threadIdx.x & 63u;
            const uint32_t c = (uint32_t)__popcll(m1);
            const uint32_t incl = wave_incl_scan(c);
            const uint32_t total = __shfl(incl, 63, 64);
            const uint32_t base = incl - c;
            const uint32_t n1 = round ? min(gld(ctr + 2), d.K) : 0u;   // first-round frequencies
            uint64_t mm = m1;   // this lane's positions not yet queued; the next has wave index k
            uint32_t k = base;
            for (uint32_t done = 0; done < total; done += 64u) {   // wave-uniform
                while (mm && k < done + 64u) {
                    const uint32_t b = (uint32_t)__builtin_ctzll(mm);
                    mm &= mm - 1u;
                    const uint32_t sr = b >> kLog2PT;
                    const uint32_t pb = sr == 0u ? p0s[0] : (sr == 1u ? p0s[1] : (sr == 2u ? p0s[2] : p0s[3]));
                    wq[k - done] = pb + (b & (kVotePerThread - 1u));
                    ++k;
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                uint32_t fa[1] = {0u};
                bool pass = false;
                if (done + lane < total) {
                    const uint32_t p = wq[lane];
                    pass = pair_passes(p);
                    fa[0] = (sinv0 * p) & maskN;
                    if (pass && ncomb) {
                        const uint32_t res = fa[0] & cmask;
                        pass = (s_comb[res >> 5] >> (res & 31u)) & 1u;
                    }
                    if (pass && n1) pass = !in_sorted(d.rec_f, n1, fa[0]);
                }
                append_wave<1>(fa, pass ? 1u : 0u, ctr, cand, cap);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");   // this round's reads before the next writes
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
            return;
        }
        if (ci0 < end) {
            const uint32_t h = s_slot[(ci0 >> log2M) - slot0];
            p0 = (h << log2M) - half + (ci0 & (M - 1u));   // mod 2^32: N divides it
            constexpr uint32_t kAll = (1u << kVotePerThread) - 1u;   // the thread's candidates
            // a loop's hash argument times 2^(32 - log2M) in 64 bits, so that its high word
            // starts at the bucket; one 64-bit add per candidate
            const uint32_t sh = 32u - log2M;
            uint32_t m[VL];
            uint64_t q[VL], cq[VL];
#pragma unroll
            for (int r = 1; r < VL; ++r) {
                m[r] = 0u;
                q[r] = (uint64_t)(cr[r] * p0 + half) << sh;
                cq[r] = (uint64_t)cr[r] << sh;
            }
            bool split = false;
            if constexpr (kExact && VL >= 4) {
                split = d.vote_split != 0u;
                if (split) {
                    constexpr int P1 = VL - VL / 2 + 1;   // slots 0 .. P1-1: loops 0 .. P1-1
                    // Few selected buckets (dK/B small) and T = L/2 + 1: the first P1 = L - T + 2
                    // loops (r0 and every loop before it among them) are tested for all
                    // candidates; one with fewer than 2 votes there cannot reach T (the other
                    // L - P1 = T - 2 loops add at most T - 2), so only the rest test those loops.
#pragma unroll
                    for (uint32_t qq = 0; qq < kVotePerThread; ++qq) {
#pragma unroll
                        for (int r = 1; r < P1; ++r) {
                            m[r] |= test_hi(r, (uint32_t)(q[r] >> 32)) << qq;
                            q[r] += cq[r];
                        }
                    }
                    VoteCount<vote_planes(P1 - 1)> c1;
                    uint32_t any = 0u, excl = 0u;
#pragma unroll
                    for (int r = 1; r < P1; ++r) {
                        c1.add(m[r], r - 1);
                        any |= m[r];
                        if ((uint32_t)r <= r0) excl |= m[r];   // counted from a loop before r0
                    }
                    emask = c1.ge(T - 1u) & ~excl & kAll;
                    uint32_t smask = any & ~excl & ~emask;   // 2 .. T-1 votes so far
                    while (smask) {
                        const uint32_t qq = (uint32_t)__builtin_ctz(smask);
                        smask &= smask - 1u;
                        const uint32_t p = p0 + qq;
                        uint32_t v2 = c1.of(qq);
#pragma unroll
                        for (int r = P1; r < VL; ++r) v2 += test1(r, cr[r] * p + half);
                        if (v2 >= T - 1u) emask |= 1u << qq;
                    }
                }
            }
            if (!split) {
#pragma unroll
                for (uint32_t qq = 0; qq < kVotePerThread; ++qq) {
#pragma unroll
                    for (int r = 1; r < VL; ++r) {
                        m[r] |= test_hi(r, (uint32_t)(q[r] >> 32)) << qq;
                        q[r] += cq[r];
                    }
                }
                VoteCount<vote_planes(VL - 1)> c;
                uint32_t excl = 0u;
#pragma unroll
                for (int r = 1; r < VL; ++r) {
                    c.add(m[r], r - 1);
                    if ((uint32_t)r <= r0) excl |= m[r];
                }
                emask = c.ge(T - 1u) & ~excl & kAll;   // T = 1: every candidate
            }
        }
        // the frequencies, f = sigma_r0^{-1} p, only where some lane of the wave passes
        if (__ballot(emask != 0u) != 0ull) {
            uint32_t f = sinv0 * p0;
#pragma unroll
            for (uint32_t qq = 0; qq < kVotePerThread; ++qq) {
                fv[qq] = f & maskN;
                f += sinv0;
            }
        } else {
#pragma unroll
            for (uint32_t qq = 0; qq < kVotePerThread; ++qq) fv[qq] = 0u;
        }
    } else {
        // fewer positions per bucket than candidates per thread: each candidate on its own
#pragma unroll
        for (uint32_t qq = 0; qq < kVotePerThread; ++qq) {
            const uint32_t ci = start + qq * kVoteNT + threadIdx.x;   // candidate index within loop r0
            fv[qq] = 0u;
            if (ci < end) {
                const uint32_t h = s_slot[(ci >> log2M) - slot0];
                const uint32_t p = (h << log2M) - half + (ci & (M - 1u));
                fv[qq] = (sinv0 * p) & maskN;
                if (npair) {
                    if (test1(1, cr[1] * p + half) && pair_passes(p)) emask |= 1u << qq;
                } else {
                    uint32_t votes = 1u;
#pragma unroll
                    for (int r = 1; r < VL; ++r) votes |= test(r, cr[r] * p + half);
                    emask |= voted(votes) << qq;
                }
            }
        }
    }
    // the comb prefilter's residues and the first round's frequencies, on the passing ones only
    const uint32_t n1 = round ? min(gld(ctr + 2), d.K) : 0u;   // first-round frequencies (ascending)
    if (ncomb || n1) {
#pragma unroll
        for (uint32_t qq = 0; qq < kVotePerThread; ++qq) {
            if ((emask >> qq) & 1u) {
                const uint32_t f = fv[qq];
                bool keep = true;
                if (ncomb) {
                    const uint32_t res = f & cmask;
                    keep = (s_comb[res >> 5] >> (res & 31u)) & 1u;
                }
                if (keep && n1) keep = !in_sorted(d.rec_f, n1, f);
                if (!keep) emask &= ~(1u << qq);
            }
        }
    }
    append_wave<kVotePerThread>(fv, emask, ctr, cand, cap);
}

// Frequency decoded from bucket h of pair j (loops 2j and 2j+1, shifts tau and
// tau+1): the lone frequency of a single-ton bucket turns its value by
// e^{+2 pi i f/N} per sample of shift, so f = floor(t + 1/2) mod N with
// t = angle(u_{2j+1}[h] conj(u_{2j}[h])) N / (2 pi) (FP64 from the float buckets).
__device__ __forceinline__ uint32_t decode_bucket(const float2* uhat, uint32_t B, uint32_t j, uint32_t h,
                                                  uint32_t N) {
    const float2 a = gld(uhat + (size_t)(2u * j) * B + h);
    const float2 b = gld(uhat + (size_t)(2u * j + 1u) * B + h);
    const double re = (double)b.x * (double)a.x + (double)b.y * (double)a.y;
    const double im = (double)b.y * (double)a.x - (double)b.x * (double)a.y;
    const double t = atan2(im, re) * (double)N / 6.283185307179586;
    return (uint32_t)(int64_t)floor(t + 0.5) & (N - 1u);
}

// Whether pair j locates f: the bucket h of sigma_{2j} f is selected in loop 2j
// and decodes to f.
__device__ __forceinline__ bool pair_decodes(const __attribute__((address_space(4))) SigDesc& d, uint32_t sg,
                                             uint32_t j, uint32_t f) {
    const uint32_t B = d.B, M = d.M, wpl = (B + 31u) >> 5;
    const uint32_t h = ((((sg * f) & d.maskN) + (M >> 1)) >> d.log2M) & (B - 1u);
    if (!((gld(d.jbits + (size_t)(2u * j) * wpl + (h >> 5)) >> (h & 31u)) & 1u)) return false;
    return decode_bucket(d.uhat, B, j, h, d.N) == f;
}

// ---------------------------------------------------------------- estimation + output
template <int N>
__device__ __forceinline__ void sort_net(float* v) {
    // bitonic sorting network, ascending, fully unrolled over registers
#pragma unroll
    for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const int l = i ^ j;
                if (l > i) {
                    const bool up = (i & k) == 0;
                    const float lo = fminf(v[i], v[l]), hi = fmaxf(v[i], v[l]);
                    v[i] = up ? lo : hi;
                    v[l] = up ? hi : lo;
                }
            }
        }
    }
}

template <int LMAX>
__device__ __forceinline__ float median_of(float* v, uint32_t L) {
    sort_net<LMAX>(v);
    const uint32_t h = L >> 1;
    float a = 0.f, b = 0.f;
#pragma unroll
    for (int r = 0; r < LMAX; ++r) {
        if ((uint32_t)r == h) b = v[r];
        if ((uint32_t)r + 1u == h) a = v[r];
    }
    return (L & 1u) ? b : (a + b) * 0.5f;
}


constexpr double inv_fact(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return 1.0 / f;
}

// e^{+2 pi i m/N} in FP64 for an exact integer m in [0, N): the root of unity
// e^{2 pi i (m >> sh) / 2^tb} from the 2^tb-entry table `rou` (tb = log2 N - sh
// <= 8) times e^{i delta}, delta = (m mod 2^sh) 2 pi / N < 2 pi / 2^tb, whose cos
// and sin come from their Taylor series to delta^8 and delta^7 (truncation
// below 1e-20). `step` = 2 pi / N.
__device__ __forceinline__ double2 phase_of(const double2* rou, uint32_t m, uint32_t sh, double step) {
    const double2 T = rou[m >> sh];
    const double delta = (double)(m & ((1u << sh) - 1u)) * step;
    const double z = -delta * delta;
    const double s = fma(fma(fma(inv_fact(7), z, inv_fact(5)), z, inv_fact(3)), z, 1.0) * delta;
    const double c = fma(fma(fma(fma(inv_fact(8), z, inv_fact(6)), z, inv_fact(4)), z, inv_fact(2)), z, 1.0);
    return make_double2(T.x * c - T.y * s, T.x * s + T.y * c);
}

// Copy the 2^tb roots of unity (tb <= 8) to LDS.
template <int NT>
__device__ __forceinline__ void stage_rou(double2* dst, const double2* src, uint32_t tb) {
    for (uint32_t i = threadIdx.x; i < (1u << tb); i += NT) dst[i] = gld(src + i);
}


// For each f in I': e_r = uhat_r[h_r(f)] * e^{-2 pi i (tau_r f mod N)/N} / Gtab[o_r(f)]
// (the energy-concentration estimate of the one frequency assumed in the
// bucket), x'_f = median_r Re e_r + i median_r Im e_r (or the mean over r); the
// estimate and its ordering key (-|x'_f|^2, then f) go to est/keys. In round 1
// the new candidates are estimated from the residual buckets, and each first-
// round frequency (appended after them) gets v + its combined residual estimate.
// est_units workgroups per signal stride over the candidates.
template <int LMAX>
__device__ __forceinline__ void estimate_body(const Launch& a, uint32_t sig, uint32_t unit, uint32_t round) {
    __shared__ uint32_t s_sig[kMaxL], s_tau[kMaxL], s_sinv[kMaxL];
    __shared__ double2 s_rou[kRouMax];
    const auto& d = desc_of(a, sig);
    const uint32_t fftm = d.fft_mode;
    const uint32_t mean = d.combine;
    const uint32_t L = d.L, maskN = d.maskN, log2M = d.log2M, M = d.M, B = d.B, N = d.N;
    const uint32_t rsh = d.log2N - d.tb;
    const double step = d.step;
    // loops L .. L+Le-1: the estimation-only loops (own B, window gain, buckets; same N)
    const uint32_t Le = d.L_est, Lt = L + Le;
    const CDesc ed = Le ? (CDesc)d.eloops : (CDesc)a.descs + (a.nsig ? sig : 0u);
    const uint32_t Be = ed->B, Me = ed->M, log2Me = ed->log2M;
    // the candidate count, the loop tables, the roots of unity and this thread's first
    // candidate are loaded together: one round trip before the buckets' (the candidate
    // is read at an index clamped into the list and used only if it exists)
    const uint32_t c0 = gld(d.ctr), c2 = round ? gld(d.ctr + 2) : 0u;
    uint32_t tsig = 0, ttau = 0, tsinv = 0;
    if (threadIdx.x < Lt) {
        const bool xe = threadIdx.x >= L;
        const uint32_t q = xe ? threadIdx.x - L : threadIdx.x;
        tsig = gld((xe ? ed->sigma : d.sigma) + q);
        ttau = gld((xe ? ed->tau : d.tau) + q);
        tsinv = gld((xe ? ed->sigma_inv : d.sigma_inv) + q);
    }
    static_assert(kRouMax <= kFinNT, "one root of unity per thread");
    double2 trou = make_double2(0.0, 0.0);
    if (threadIdx.x < (1u << d.tb)) trou = gld(d.rou + threadIdx.x);
    const uint32_t* cand = d.cand;
    const uint32_t first = unit * kFinNT + threadIdx.x;
    const uint32_t fpre = gld(cand + min(first, d.cap - 1u));
    const uint32_t nc = min(c0, d.cap);
    const uint32_t n = nc + (round ? min(c2, d.K) : 0u);
    if (unit * kFinNT >= n) return;   // block-uniform: no candidate for this workgroup
    if (threadIdx.x < Lt) {
        s_sig[threadIdx.x] = tsig;
        s_tau[threadIdx.x] = ttau;
        s_sinv[threadIdx.x] = tsinv;
    }
    if (threadIdx.x < (1u << d.tb)) s_rou[threadIdx.x] = trou;
    __syncthreads();
    const float2* invG = d.invG;
    const float2* uhat = d.uhat;
    const float2* tw = d.tw;
    float2* est = d.est;
    uint64_t* keys = d.keys;
    const uint32_t stride = d.est_units * kFinNT;
    const uint32_t phase = d.phase;
    for (uint32_t i = unit * kFinNT + threadIdx.x; i < n; i += stride) {
        const bool rec = i >= nc;   // a first-round frequency (round 1)
        const uint32_t f = rec ? gld(d.rec_f + (i - nc)) : (i == first ? fpre : gld(cand + i));
        if (rec && phase) {
            // phase location keeps the recovered single-ton estimates
            const float2 v0 = gld(d.rec_v + (i - nc));
            const float mag = fmaf(v0.x, v0.x, v0.y * v0.y);
            gst(est + i, v0);
            gst(keys + i, ((uint64_t)(0xFFFFFFFFu - __float_as_uint(mag)) << 32) | (uint64_t)f);
            continue;
        }
        // loops that estimate f: all, or (phase location) those of the pairs that decode it
        uint32_t use = (Lt >= 32u) ? 0xFFFFFFFFu : ((1u << Lt) - 1u);
        if (phase) {
            use = 0;
            for (uint32_t j = 0; j < (L >> 1); ++j)
                if (pair_decodes(d, s_sig[2u * j], j, f)) use |= 3u << (2u * j);
        }
        const uint32_t m = (uint32_t)__popc(use);
        float re[LMAX], im[LMAX];
#pragma unroll
        for (int r = 0; r < LMAX; ++r) {
            re[r] = __builtin_inff();
            im[r] = __builtin_inff();
            if ((uint32_t)r < Lt && ((use >> r) & 1u)) {
                const bool xe = (uint32_t)r >= L;
                const uint32_t Bx = xe ? Be : B, Mx = xe ? Me : M, l2M = xe ? log2Me : log2M;
                const uint32_t p = (s_sig[r] * f) & maskN;
                const uint32_t h = ((p + (Mx >> 1)) >> l2M) & (Bx - 1u);
                const uint32_t o = (p - (h << l2M) + (N >> 1)) & maskN;   // o + N/2
                const uint32_t gi = o - (N >> 1) + (Mx >> 1);
                const float2 g = gld((xe ? ed->invG : invG) + gi);
                float2 uv;
                if (xe) {
                    uv = gld(ed->uhat + (size_t)(r - L) * Be + h);
                } else if (fftm) {
                    // two-pass FFT layout: X[h] = e^{+2 pi i (s tau h mod B)/B} V[s h mod B], s = sigma^{-1}
                    const uint32_t si = s_sinv[r];
                    const float2 t = gld(tw + ((si * s_tau[r] * h) & (B - 1u)));   // e^{-2 pi i ./B}
                    uv = cmul(gld(uhat + (size_t)r * B + ((si * h) & (B - 1u))), make_float2(t.x, -t.y));
                } else {
                    uv = gld(uhat + (size_t)r * B + h);
                }
                const uint32_t k = (s_tau[r] * f) & maskN;
                const double2 pk = phase_of(s_rou, k, rsh, step);   // e^{+2 pi i k/N}
                const float2 rot = make_float2((float)pk.x, -(float)pk.y);
                const float2 e = cmul(cmul(uv, rot), g);
                re[r] = e.x;
                im[r] = e.y;
            }
        }
        float mr, mi;
        if (mean) {
            // the average of the loop estimates, summed in loop order
            float sr = 0.f, si = 0.f;
#pragma unroll
            for (int r = 0; r < LMAX; ++r) {
                if ((uint32_t)r < Lt && ((use >> r) & 1u)) {
                    sr += re[r];
                    si += im[r];
                }
            }
            mr = sr / (float)m;
            mi = si / (float)m;
        } else {
            mr = median_of<LMAX>(re, m);
            mi = median_of<LMAX>(im, m);
        }
        if (rec) {
            const float2 v0 = gld(d.rec_v + (i - nc));
            mr = v0.x + mr;
            mi = v0.y + mi;
        }
        const float mag = fmaf(mr, mr, mi * mi);
        gst(est + i, make_float2(mr, mi));
        gst(keys + i, ((uint64_t)(0xFFFFFFFFu - __float_as_uint(mag)) << 32) | (uint64_t)f);
    }
}

// The K smallest keys of the estimates (the K largest |x'_f|^2, ties -> lower f),
// returned in ascending f and padded with (-1, 0). The K-th smallest key comes
// from a radix select over 8-bit digits from the top, which stops as soon as
// every key with the selected prefix is needed; up to kFinKPT keys per thread are
// held in registers across its passes. The selected entries are then ordered by f
// with a counting sort: the range [min f, max f] is cut into kSelNT bins, each
// entry goes to its bin's run, and its rank is the run's start plus the entries of
// the run below it (frequencies are distinct). One workgroup per signal. Dynamic
// LDS: P values and P frequencies (P = 2^ceil(log2 K)).
// With the subtraction round, round 0 keeps its K largest in the workspace
// (rec_f, rec_v, count in ctr[2]) instead of the outputs; round 1 writes the
// outputs.
// NT threads (a multiple of 64, at least 256); EPT = selected entries per thread, NT EPT >= K.
constexpr int kFinKPT = 4;                 // keys per thread held in registers
template <int NT, int EPT>
__device__ __forceinline__ void finalize_body(const Launch& a, uint32_t sig, uint32_t round) {
    extern __shared__ f4v lds_raw[];
    __shared__ uint32_t hist[256];
    __shared__ uint32_t bc[4];
    __shared__ uint32_t s_bin[NT], s_fill[NT], s_red[2 * (NT / 64)], s_scan[NT / 64];
    const auto& d = desc_of(a, sig);
    const IoDesc io = io_of(a, sig);
    uint32_t P = 1;
    while (P < d.K) P <<= 1;
    float2* s_v = reinterpret_cast<float2*>(lds_raw);
    uint32_t* s_f = reinterpret_cast<uint32_t*>(s_v + P);
    const float2* est = d.est;
    const uint64_t* keys = d.keys;
    const uint32_t K = d.K;
    // the candidate count and the first kFinKPT keys of each thread are loaded together
    // (keys read at indices clamped into the array; those at or beyond the count unused)
    const uint32_t c0 = gld(d.ctr), c2 = round ? gld(d.ctr + 2) : 0u;
    const uint32_t nkeys = d.cap + (d.iterate ? K : 0u);
    uint64_t kr[kFinKPT];
#pragma unroll
    for (int e = 0; e < kFinKPT; ++e) kr[e] = gld(keys + min(threadIdx.x + e * NT, nkeys - 1u));
    const uint32_t nc = min(c0, d.cap);
    const uint32_t n = nc + (round ? min(c2, K) : 0u);
    const bool inreg = n <= (uint32_t)kFinKPT * NT;   // block-uniform
    // fn(key, index) for every candidate key (registers or global memory)
    auto for_keys = [&](auto&& fn) {
        if (inreg) {
#pragma unroll
            for (int e = 0; e < kFinKPT; ++e) {
                const uint32_t i = threadIdx.x + e * NT;
                if (i < n) fn(kr[e], i);
            }
        } else {
            for (uint32_t i = threadIdx.x; i < n; i += NT) fn(gld(keys + i), i);
        }
    };
    uint64_t thr = ~0ull;
    if (n > K) {
        uint64_t prefix = 0, pmask = 0;
        uint32_t kk = K;
        const uint32_t lane = threadIdx.x & 63u;
        for (int pass = 0; pass < 8; ++pass) {
            const int shift = 56 - 8 * pass;
            for (int i = threadIdx.x; i < 256; i += NT) hist[i] = 0;
            __syncthreads();
            for_keys([&](uint64_t key, uint32_t) {
                if ((key & pmask) == prefix) atomicAdd(&hist[(uint32_t)(key >> shift) & 255u], 1u);
            });
            __syncthreads();
            if (threadIdx.x < 64) {
                const int lo = 4 * (int)lane;   // lane 0 owns the smallest digits
                const uint32_t h0 = hist[lo], h1 = hist[lo + 1], h2 = hist[lo + 2], h3 = hist[lo + 3];
                const uint32_t s = h0 + h1 + h2 + h3;
                const uint32_t incl = wave_incl_scan(s);
                const uint32_t excl = incl - s;
                if (excl < kk && kk <= incl) {
                    uint32_t acc = excl, dsel, rem, cnt;
                    if (acc + h0 >= kk) {
                        dsel = lo;
                        rem = kk - acc;
                        cnt = h0;
                    } else if (acc += h0, acc + h1 >= kk) {
                        dsel = lo + 1;
                        rem = kk - acc;
                        cnt = h1;
                    } else if (acc += h1, acc + h2 >= kk) {
                        dsel = lo + 2;
                        rem = kk - acc;
                        cnt = h2;
                    } else {
                        acc += h2;
                        dsel = lo + 3;
                        rem = kk - acc;
                        cnt = h3;
                    }
                    bc[0] = dsel;
                    bc[1] = rem;
                    bc[2] = cnt;
                }
            }
            __syncthreads();
            prefix |= (uint64_t)bc[0] << shift;
            pmask |= 255ull << shift;
            kk = bc[1];
            const bool all_needed = bc[2] == kk;   // every key with this prefix is among the K
            __syncthreads();
            if (all_needed) {
                prefix |= ~pmask;   // the largest key with the prefix
                break;
            }
        }
        thr = prefix;
    }
    if (threadIdx.x == 0) bc[2] = 0;
    __syncthreads();
    for_keys([&](uint64_t key, uint32_t i) {
        if (key <= thr) {
            const uint32_t pos = atomicAdd(&bc[2], 1u);
            if (pos < P) {
                s_f[pos] = (uint32_t)key;
                s_v[pos] = gld(est + i);
            }
        }
    });
    __syncthreads();
    const uint32_t cnt = min(bc[2], K);
    // this thread's entries (positions threadIdx.x + e NT) and the range of f
    uint32_t ef[EPT];
    float2 ev[EPT];
    uint32_t fmin = 0xFFFFFFFFu, fmax = 0u;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const uint32_t q = threadIdx.x + e * NT;
        ef[e] = 0u;
        ev[e] = make_float2(0.f, 0.f);
        if (q < cnt) {
            ef[e] = s_f[q];
            ev[e] = s_v[q];
            fmin = min(fmin, ef[e]);
            fmax = max(fmax, ef[e]);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        fmin = min(fmin, (uint32_t)__shfl_xor((int)fmin, off, 64));
        fmax = max(fmax, (uint32_t)__shfl_xor((int)fmax, off, 64));
    }
    const uint32_t wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63u) == 0u) {
        s_red[wid] = fmin;
        s_red[NT / 64 + wid] = fmax;
    }
    s_bin[threadIdx.x] = 0u;
    s_fill[threadIdx.x] = 0u;
    __syncthreads();
    fmin = s_red[0];
    fmax = s_red[NT / 64];
#pragma unroll
    for (int w = 1; w < (int)(NT / 64); ++w) {
        fmin = min(fmin, s_red[w]);
        fmax = max(fmax, s_red[NT / 64 + w]);
    }
    // bin width: ceil((fmax - fmin + 1) / NT) >= 1 (64-bit: the range can reach 2^32)
    const uint32_t width =
        cnt ? (uint32_t)(((uint64_t)fmax - fmin + (uint64_t)NT) / (uint64_t)NT) : 1u;
    uint32_t eb[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const uint32_t q = threadIdx.x + e * NT;
        eb[e] = 0u;
        if (q < cnt) {
            eb[e] = (ef[e] - fmin) / width;   // < NT
            atomicAdd(&s_bin[eb[e]], 1u);
        }
    }
    __syncthreads();
    uint32_t tot;
    const uint32_t start = block_excl_scan<NT>(s_bin[threadIdx.x], s_scan, tot);
    __syncthreads();
    s_bin[threadIdx.x] = start;   // run start of bin threadIdx.x
    __syncthreads();
    // every entry into its bin's run (any order within the run)
    uint32_t ep[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const uint32_t q = threadIdx.x + e * NT;
        ep[e] = 0u;
        if (q < cnt) {
            ep[e] = s_bin[eb[e]] + atomicAdd(&s_fill[eb[e]], 1u);
            s_f[ep[e]] = ef[e];
        }
    }
    __syncthreads();
    const bool keep = d.iterate && round == 0;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const uint32_t q = threadIdx.x + e * NT;
        if (q < cnt) {
            const uint32_t b = eb[e], r0 = s_bin[b], r1 = b + 1u < NT ? s_bin[b + 1u] : cnt;
            uint32_t rank = r0;
            for (uint32_t t = r0; t < r1; ++t) rank += s_f[t] < ef[e] ? 1u : 0u;
            if (keep) {
                gst(d.rec_f + rank, ef[e]);
                gst(d.rec_v + rank, ev[e]);
            } else {
                gst(io.out_idx + rank, (int64_t)ef[e]);
                gst(io.out_val + rank, ev[e]);
            }
        }
    }
    for (uint32_t k = cnt + threadIdx.x; k < K; k += NT) {
        if (keep) {
            gst(d.rec_f + k, 0xFFFFFFFFu);
            gst(d.rec_v + k, make_float2(0.f, 0.f));
        } else {
            gst(io.out_idx + k, (int64_t)-1);
            gst(io.out_val + k, make_float2(0.f, 0.f));
        }
    }
    if (keep && threadIdx.x == 0) gst(d.ctr + 2, cnt);
}

// ---------------------------------------------------------------- FP64 residual
// E_res = mean_t |x_t - sum_k v_k e^{+2 pi i (t f_k mod N)/N}|^2 and
// E_in = mean_t |x_t|^2 over the S residual positions, which come in runs of
// kResRun consecutive samples. Lane (run, kl) of a wave sums the model over the
// outputs k = kl, kl + KL, ... (KL = 2^resid_log2kl) for the kResRun samples of its
// run: the phase of the exact integer t0 f mod N at the run start t0 (phase_of, FP64),
// then one complex multiply by e^{+2 pi i f/N} per further sample. The KL lanes of a
// run are added by a fixed shuffle tree; the run's lane kl = 0 forms the two energy
// sums of its samples; lanes, then waves, are added in a fixed order, and each
// workgroup writes its two partial sums; residual_sum_kernel reduces them. Padding
// outputs (index -1) are staged as f = 0, v = 0 and add exact zeros. The per-sample
// factors e^{+2 pi i f/N} are evaluated once per workgroup into LDS.
// stage = false: the outputs and the roots of unity are still in LDS from the previous
// unit of the same signal run by this workgroup (block-uniform).
__device__ __forceinline__ void residual_body(const Launch& a, uint32_t sig, uint32_t unit, bool stage = true) {
    extern __shared__ f4v lds_raw[];
    constexpr uint32_t NW = kResNT / 64;
    __shared__ double2 s_red[NW];
    __shared__ double2 s_rou[kRouMax];
    const auto& d = desc_of(a, sig);
    const IoDesc io = io_of(a, sig);
    const uint32_t K = d.K, maskN = d.maskN, log2kl = d.resid_log2kl;
    const uint32_t rsh = d.log2N - d.tb;
    const double step = d.step;
    double2* s_st = reinterpret_cast<double2*>(lds_raw);
    float2* s_v = reinterpret_cast<float2*>(s_st + K);
    uint32_t* s_f = reinterpret_cast<uint32_t*>(s_v + K);
    if (stage) {
        stage_rou<kResNT>(s_rou, d.rou, d.tb);
        for (uint32_t k = threadIdx.x; k < K; k += kResNT) {
            const int64_t f = gld(io.out_idx + k);
            const bool pad = f < 0;
            s_f[k] = pad ? 0u : (uint32_t)f;
            s_v[k] = pad ? make_float2(0.f, 0.f) : gld(io.out_val + k);
        }
        __syncthreads();
        for (uint32_t k = threadIdx.x; k < K; k += kResNT) s_st[k] = phase_of(s_rou, s_f[k], rsh, step);
        __syncthreads();
    }
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    const uint32_t KL = 1u << log2kl, kl = lane & (KL - 1u);
    const uint32_t run = (unit * NW + wv) * (64u >> log2kl) + (lane >> log2kl);
    const uint32_t j0 = run * kResRun;
    const bool valid = j0 < d.S;
    const uint32_t t0 = valid ? gld(d.tpos + j0) : 0u;
    double mr[kResRun], mi[kResRun];
#pragma unroll
    for (uint32_t i = 0; i < kResRun; ++i) mr[i] = mi[i] = 0.0;
    for (uint32_t k = kl; k < K; k += KL) {
        const uint32_t f = s_f[k];
        const double vr = (double)s_v[k].x, vi = (double)s_v[k].y;
        double2 p = phase_of(s_rou, (t0 * f) & maskN, rsh, step);   // e^{+2 pi i t0 f/N}
        const double2 st = s_st[k];                                // e^{+2 pi i f/N}
#pragma unroll
        for (uint32_t i = 0; i < kResRun; ++i) {
            mr[i] = fma(vr, p.x, fma(-vi, p.y, mr[i]));
            mi[i] = fma(vr, p.y, fma(vi, p.x, mi[i]));
            if (i + 1 < kResRun) {
                const double px = p.x * st.x - p.y * st.y;
                p.y = p.x * st.y + p.y * st.x;
                p.x = px;
            }
        }
    }
    for (uint32_t off = KL >> 1; off > 0; off >>= 1) {
#pragma unroll
        for (uint32_t i = 0; i < kResRun; ++i) {
            mr[i] += __shfl_xor(mr[i], (int)off, 64);
            mi[i] += __shfl_xor(mi[i], (int)off, 64);
        }
    }
    double ea = 0.0, eb = 0.0;
    if (valid && kl == 0) {
        const uint32_t cnt = min(kResRun, d.S - j0);
        const f4v* xs = reinterpret_cast<const f4v*>(io.x + t0);   // t0 is a multiple of kResRun: 64-byte aligned
        f4v xv[kResRun / 2];
#pragma unroll
        for (uint32_t q = 0; q < kResRun / 2; ++q) xv[q] = gld(xs + q);
#pragma unroll
        for (uint32_t i = 0; i < kResRun; ++i) {
            if (i < cnt) {
                const double xr = xv[i >> 1][(i & 1u) * 2u], xi = xv[i >> 1][(i & 1u) * 2u + 1u];
                const double er = xr - mr[i], ei = xi - mi[i];
                ea += er * er + ei * ei;
                eb += xr * xr + xi * xi;
            }
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        ea += __shfl_down(ea, off, 64);
        eb += __shfl_down(eb, off, 64);
    }
    if (lane == 0) s_red[wv] = make_double2(ea, eb);
    __syncthreads();
    if (threadIdx.x == 0) {
        double ta = 0.0, tb = 0.0;
#pragma unroll
        for (uint32_t w = 0; w < NW; ++w) {
            ta += s_red[w].x;
            tb += s_red[w].y;
        }
        gst(d.rpart + 2 * unit, ta);
        gst(d.rpart + 2 * unit + 1, tb);
    }
}

// The residual's per-workgroup partial sums reduced in a fixed order (per
// thread, a shuffle tree, then the waves in order) into the two outputs. One
// workgroup per signal, after every residual workgroup of the signal has written its partials.
__device__ __forceinline__ void residual_sum_body(const Launch& a, uint32_t sig) {
    constexpr uint32_t NW = kResNT / 64;
    __shared__ double2 s_red[NW];
    const auto& d = desc_of(a, sig);
    const IoDesc io = io_of(a, sig);
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    const double* rp = d.rpart;
    double A = 0.0, Bs = 0.0;   // thread i: partials i, i + 256, ... in order
    for (uint32_t u = threadIdx.x; u < d.resid_blocks; u += kResNT) {
        A += gld(rp + 2 * u);
        Bs += gld(rp + 2 * u + 1);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        A += __shfl_down(A, off, 64);
        Bs += __shfl_down(Bs, off, 64);
    }
    if (lane == 0) s_red[wv] = make_double2(A, Bs);
    __syncthreads();
    if (threadIdx.x == 0) {
        double tA = 0.0, tB = 0.0;
#pragma unroll
        for (uint32_t w = 0; w < NW; ++w) {
            tA += s_red[w].x;
            tB += s_red[w].y;
        }
        double* out = io.out_resid ? io.out_resid : d.resid_own;
        gst(out + 0, tA / (double)d.S);
        gst(out + 1, tB / (double)d.S);
    }
}

}  // namespace sfft
