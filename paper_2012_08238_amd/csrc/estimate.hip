// Location by votes, energy-concentration estimation with the median over
// loops, the K largest in ascending order, and the FP64 residual (formula
// method, Eq.(2)).
#include "estimate_dev.hpp"

namespace sfft {

// The grid may be smaller than the launch's `units` chunks (it is capped so that the vote
// leaves room on every compute unit for other streams' work); each workgroup then takes
// a contiguous share of the chunks, mostly of one signal, whose tables it copies once.
template <int VL, bool STAGED>
// Staged instances are held to 80 VGPRs (six waves per SIMD): four vote waves per SIMD then
// leave room for a bucketization wave of another stream beside them.
__global__ __launch_bounds__(kVoteNT, STAGED ? 6 : 1) void vote_kernel(Launch a, uint32_t round, uint32_t units) {
    extern __shared__ uint32_t sdyn[];
    __shared__ uint32_t s_comb[kMaxCombB / 32];       // residues kept by the comb prefilter (union)
    __shared__ uint32_t s_pq[kVoteNT];                // by pair: each wave's queue of positions to finish
    const uint32_t b0 = (uint32_t)(((uint64_t)blockIdx.x * units) / gridDim.x);
    const uint32_t b1 = (uint32_t)(((uint64_t)(blockIdx.x + 1u) * units) / gridDim.x);
    uint32_t prev = 0xffffffffu;
    for (uint32_t blk = b0; blk < b1; ++blk) {
        uint32_t sig, unit;
        resolve_blk(a, blk, sig, unit);
        if (blk != b0) __syncthreads();   // the previous chunk's LDS reads are done
        vote_chunk<VL, STAGED>(a, sig, unit, round, sig != prev, sdyn, s_comb, s_pq);
        prev = sig;
    }
}

// ---------------------------------------------------------------- phase-encoding location
// Phase-encoding location (sFFT3.0 row of Table 1): every selected bucket of the
// first loop of every pair decodes one frequency; it is a candidate when its
// bucket hash matches (single-ton check), at least T pairs decode it, it is
// counted from the first pair that does (no duplicates), the comb prefilter (if
// any) keeps its residue, and (round 1) it was not recovered before. One thread
// per (pair, selected bucket), kDecPerThread per thread; one list reservation
// per wave.
__global__ __launch_bounds__(kVoteNT) void decode_kernel(Launch a, uint32_t round) {
    __shared__ uint32_t s_comb[kMaxCombB / 32];
    __shared__ uint32_t s_sig[kMaxL / 2];
    uint32_t sig, unit;
    resolve(a, sig, unit);
    const auto& d = desc_of(a, sig);
    const uint32_t np = d.L >> 1, dK = d.dK, B = d.B, M = d.M, log2M = d.log2M, maskN = d.maskN;
    if (threadIdx.x < np) s_sig[threadIdx.x] = gld(d.sigma + 2u * threadIdx.x);
    const uint32_t ncomb = d.comb_loops, cmask = (1u << d.comb_log2b) - 1u;
    if (ncomb) {
        const uint32_t cw = max(1u, (cmask + 1u) >> 5);
        for (uint32_t i = threadIdx.x; i < cw; i += kVoteNT) {
            uint32_t v = 0;
            for (uint32_t c = 0; c < ncomb; ++c) v |= gld(d.cbits + c * cw + i);
            s_comb[i] = v;
        }
    }
    __syncthreads();
    uint32_t* ctr = d.ctr;
    const uint32_t cap = d.cap, T = d.T, total_in = np * dK;
    const uint32_t n1 = round ? min(gld(ctr + 2), d.K) : 0u;
    uint32_t fv[kDecPerThread];
    uint32_t emask = 0;
#pragma unroll
    for (uint32_t qq = 0; qq < kDecPerThread; ++qq) {
        const uint32_t idx = unit * kDecUnit + qq * kVoteNT + threadIdx.x;
        bool emit = false;
        uint32_t f = 0;
        if (idx < total_in) {
            const uint32_t j = idx / dK;
            const uint32_t h = gld(d.jlist + (size_t)(2u * j) * dK + (idx - j * dK));
            f = decode_bucket(d.uhat, B, j, h, d.N);
            emit = ((((s_sig[j] * f) & maskN) + (M >> 1)) >> log2M & (B - 1u)) == h;
            if (emit) {
                uint32_t cnt = 1;
                for (uint32_t jj = 0; jj < np; ++jj) {
                    if (jj == j) continue;
                    if (pair_decodes(d, s_sig[jj], jj, f)) {
                        if (jj < j) {   // counted from an earlier pair
                            emit = false;
                            break;
                        }
                        ++cnt;
                    }
                }
                emit = emit && cnt >= T;
            }
            if (emit && ncomb) {
                const uint32_t res = f & cmask;
                emit = (s_comb[res >> 5] >> (res & 31u)) & 1u;
            }
            if (emit && n1) emit = !in_sorted(d.rec_f, n1, f);
        }
        fv[qq] = f;
        emask |= (emit ? 1u : 0u) << qq;
    }
    append_wave<kDecPerThread>(fv, emask, ctr, d.cand, cap);
}

// ---------------------------------------------------------------- estimation + output
template <int LMAX>
__global__ __launch_bounds__(kFinNT) void estimate_kernel(Launch a, uint32_t round) {
    uint32_t sig, unit;
    resolve(a, sig, unit);
    estimate_body<LMAX>(a, sig, unit, round);
}

// one workgroup of kSelNT threads per signal
__global__ __launch_bounds__(kSelNT) void finalize_kernel(Launch a, uint32_t round) {
    uint32_t sig, unit;
    resolve(a, sig, unit);
    finalize_body<kSelNT, kMaxK / kSelNT>(a, sig, round);
}

// One signal whose candidates one estimation workgroup covers (est_units = 1): the estimates
// and then, after a barrier (this workgroup wrote them), the K largest, in one launch. The
// top-K runs on the estimation workgroup's 256 threads (16 selected entries each, K <= 4096)
// and gives the same outputs as finalize_kernel (they are unique: the K largest in f order).
template <int LMAX>
__global__ __launch_bounds__(kFinNT) void tail_one_kernel(Launch a, uint32_t round) {
    uint32_t sig, unit;
    resolve(a, sig, unit);
    estimate_body<LMAX>(a, sig, 0u, round);
    __syncthreads();
    finalize_body<kFinNT, kMaxK / kFinNT>(a, sig, round);
}

// ---------------------------------------------------------------- subtraction round
// Iterative framework (frameworks section), subtraction step for loop r: a
// recovered coefficient (f, v) with p = sigma_r f mod N in bucket h0 at offset
// o = p - h0 N/B contributes v e^{+2 pi i (tau_r f mod N)/N} Gw(o - j N/B) to bucket
// h0 + j (Eq.(9) with the flat window's gain). It is removed from the buckets
// j = -sub_rl .. sub_rh, the plan's reach: every bucket, or as many as leave less
// than 1e-6 of the centre gain in the others. Each touched bucket is rewritten by one
// thread that subtracts its contributions in a fixed order (coefficients sorted
// by (h0, index)), so the result is independent of scheduling. Unit 0 also
// clears the candidate counter for the second vote. One workgroup per
// (signal, loop). Dynamic LDS: phased values [K], sort keys [P], offsets [K],
// first sorted position of each bucket's run [B] (16 bit).
__global__ __launch_bounds__(kSubNT) void subtract_kernel(Launch a) {
    extern __shared__ f4v lds_raw[];
    __shared__ double2 s_rou[kRouMax];
    uint32_t sig, r;
    resolve(a, sig, r);
    const auto& d = desc_of(a, sig);
    const uint32_t K = d.K, B = d.B, M = d.M, log2M = d.log2M, maskN = d.maskN, N = d.N;
    uint32_t P = 1;
    while (P < K) P <<= 1;
    float2* s_vph = reinterpret_cast<float2*>(lds_raw);
    uint32_t* s_key = reinterpret_cast<uint32_t*>(s_vph + K);
    int32_t* s_off = reinterpret_cast<int32_t*>(s_key + P);
    uint16_t* s_first = reinterpret_cast<uint16_t*>(s_off + K);
    const uint32_t n1 = min(gld(d.ctr + 2), K);
    if (r == 0 && threadIdx.x == 0) gst(d.ctr, 0u);
    if (n1 == 0) return;   // block-uniform: nothing was recovered
    uint32_t Q = 1;        // sort size: power of two >= n1
    while (Q < n1) Q <<= 1;
    const uint32_t sg = gld(d.sigma + r), tu = gld(d.tau + r);
    const uint32_t rsh = d.log2N - d.tb;
    stage_rou<kSubNT>(s_rou, d.rou, d.tb);
    for (uint32_t b = threadIdx.x; b < B; b += kSubNT) s_first[b] = 0xFFFFu;
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < Q; k += kSubNT) {
        uint32_t key = 0xFFFFFFFFu;
        if (k < n1) {
            const uint32_t f = gld(d.rec_f + k);
            const float2 v = gld(d.rec_v + k);
            const uint32_t p = (sg * f) & maskN;
            const uint32_t h0 = ((p + (M >> 1)) >> log2M) & (B - 1u);
            s_off[k] = (int32_t)((p - (h0 << log2M) + (N >> 1)) & maskN) - (int32_t)(N >> 1);
            const double2 ph = phase_of(s_rou, (tu * f) & maskN, rsh, d.step);   // e^{+2 pi i tau f/N}
            s_vph[k] = make_float2((float)((double)v.x * ph.x - (double)v.y * ph.y),
                                   (float)((double)v.x * ph.y + (double)v.y * ph.x));
            key = (h0 << 12) | k;   // h0 < 2^14, k < 2^12
        }
        s_key[k] = key;
    }
    __syncthreads();
    for (uint32_t kk = 2; kk <= Q; kk <<= 1) {
        for (uint32_t j = kk >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < Q; i += kSubNT) {
                const uint32_t l = i ^ j;
                if (l > i) {
                    const uint32_t x = s_key[i], y = s_key[l];
                    if ((x > y) == ((i & kk) == 0)) {
                        s_key[i] = y;
                        s_key[l] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t i = threadIdx.x; i < n1; i += kSubNT) {
        const uint32_t h = s_key[i] >> 12;
        if (i == 0 || (s_key[i - 1] >> 12) != h) s_first[h] = (uint16_t)i;
    }
    __syncthreads();
    float2* u = d.uhat + (size_t)r * B;
    const float2* gw = d.gw;
    const int32_t rl = (int32_t)d.sub_rl, rh = (int32_t)d.sub_rh;
    const int32_t c0 = rh * (int32_t)M + (int32_t)(M >> 1);   // gw index of offset 0
    for (uint32_t b = threadIdx.x; b < B; b += kSubNT) {
        // the coefficients of bucket hh = b - j reach bucket b, j = -rl .. rh, in that order
        bool any = false;
        for (int32_t j = -rl; j <= rh; ++j) any |= s_first[(b - (uint32_t)j) & (B - 1u)] != 0xFFFFu;
        if (!any) continue;
        float2 acc = gld(u + b);
        for (int32_t j = -rl; j <= rh; ++j) {
            const uint32_t hh = (b - (uint32_t)j) & (B - 1u);
            const int32_t sh = c0 - j * (int32_t)M;   // gw index = o - j M + c0
            for (uint32_t i = s_first[hh]; i < n1 && (s_key[i] >> 12) == hh; ++i) {
                const uint32_t k = s_key[i] & 4095u;
                const float2 c = cmul(s_vph[k], gld(gw + (s_off[k] + sh)));
                acc.x -= c.x;
                acc.y -= c.y;
            }
        }
        gst(u + b, acc);
    }
}

// ---------------------------------------------------------------- FP64 residual
__global__ __launch_bounds__(kResNT) void residual_kernel(Launch a) {
    uint32_t sig, unit;
    resolve(a, sig, unit);
    residual_body(a, sig, unit);
}

// launched after residual_kernel: the launch boundary makes the partials visible
__global__ __launch_bounds__(kResNT) void residual_sum_kernel(Launch a) {
    uint32_t sig, unit;
    resolve(a, sig, unit);
    residual_sum_body(a, sig);
}

// Single-signal form of the residual in one launch: residual_kernel's workgroups, and the one
// that finishes last (counted in ctr[3], which the bucketization cleared) reduces the partial
// sums as residual_sum_kernel does, in the same fixed order. The partials cross workgroups on
// different dies: each workgroup's partials are written back to memory (device-scope release)
// before it is counted, and the last one drops stale cached copies (device-scope acquire)
// before it reads them. Batches keep the two launches: there the step is bound by the
// bucketization, and a device-scope release per workgroup would write back each die's L2
// beside it.
__global__ __launch_bounds__(kResNT) void residual_one_kernel(Launch a) {
    __shared__ uint32_t s_last;
    uint32_t sig, unit;
    resolve(a, sig, unit);
    residual_body(a, sig, unit);
    const auto& d = desc_of(a, sig);
    if (threadIdx.x == 0) {   // the thread that wrote this workgroup's partials
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        s_last = atomicAdd(d.ctr + 3, 1u) == d.resid_blocks - 1u ? 1u : 0u;
    }
    __syncthreads();
    if (s_last) {   // block-uniform
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        residual_sum_body(a, sig);
    }
}

// ---------------------------------------------------------------- launchers
template <int VL>
hipError_t launch_vote_vl(const Launch& a, uint32_t units, uint32_t lds_bytes, uint32_t staged, uint32_t round,
                          hipStream_t s) {
    const uint32_t grid = min(units, kVoteMaxGrid);
    if (staged) hipLaunchKernelGGL((vote_kernel<VL, true>), dim3(grid), dim3(kVoteNT), lds_bytes, s, a, round, units);
    else hipLaunchKernelGGL((vote_kernel<VL, false>), dim3(grid), dim3(kVoteNT), lds_bytes, s, a, round, units);
    return hipGetLastError();
}

template <int... VLs>
struct VoteTable {
    static hipError_t launch(uint32_t key, const Launch& a, uint32_t units, uint32_t lds_bytes, uint32_t staged,
                             uint32_t round, hipStream_t s) {
        hipError_t e = hipErrorInvalidValue;
        ((key == (uint32_t)VLs ? (e = launch_vote_vl<VLs>(a, units, lds_bytes, staged, round, s), 0) : 0), ...);
        return e;
    }
    static hipError_t set_lds(uint32_t bytes) {
        hipError_t e = hipSuccess;
        ((e = e == hipSuccess ? hipFuncSetAttribute(reinterpret_cast<const void*>(&vote_kernel<VLs, true>),
                                                    hipFuncAttributeMaxDynamicSharedMemorySize, bytes)
                              : e),
         ...);
        ((e = e == hipSuccess ? hipFuncSetAttribute(reinterpret_cast<const void*>(&vote_kernel<VLs, false>),
                                                    hipFuncAttributeMaxDynamicSharedMemorySize, bytes)
                              : e),
         ...);
        return e;
    }
};
// one instance per vote_key value
typedef VoteTable<1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 32> Votes;

hipError_t launch_vote(const Launch& a, uint32_t key, uint32_t units, uint32_t lds_bytes, uint32_t staged,
                       uint32_t round, hipStream_t s) {
    return Votes::launch(key, a, units, lds_bytes, staged, round, s);
}

hipError_t launch_decode(const Launch& a, uint32_t units, uint32_t round, hipStream_t s) {
    hipLaunchKernelGGL(decode_kernel, dim3(units), dim3(kVoteNT), 0, s, a, round);
    return hipGetLastError();
}

hipError_t launch_estimate(const Launch& a, uint32_t lmax, uint32_t units, uint32_t round, hipStream_t s) {
    switch (lmax) {
        case 4: hipLaunchKernelGGL(estimate_kernel<4>, dim3(units), dim3(kFinNT), 0, s, a, round); break;
        case 8: hipLaunchKernelGGL(estimate_kernel<8>, dim3(units), dim3(kFinNT), 0, s, a, round); break;
        case 16: hipLaunchKernelGGL(estimate_kernel<16>, dim3(units), dim3(kFinNT), 0, s, a, round); break;
        case 32: hipLaunchKernelGGL(estimate_kernel<32>, dim3(units), dim3(kFinNT), 0, s, a, round); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_finalize(const Launch& a, uint32_t units, uint32_t lds, uint32_t round, hipStream_t s) {
    hipLaunchKernelGGL(finalize_kernel, dim3(units), dim3(kSelNT), lds, s, a, round);
    return hipGetLastError();
}

hipError_t launch_tail_one(const Launch& a, uint32_t lmax, uint32_t lds, uint32_t round, hipStream_t s) {
    switch (lmax) {
        case 4: hipLaunchKernelGGL(tail_one_kernel<4>, dim3(1), dim3(kFinNT), lds, s, a, round); break;
        case 8: hipLaunchKernelGGL(tail_one_kernel<8>, dim3(1), dim3(kFinNT), lds, s, a, round); break;
        case 16: hipLaunchKernelGGL(tail_one_kernel<16>, dim3(1), dim3(kFinNT), lds, s, a, round); break;
        case 32: hipLaunchKernelGGL(tail_one_kernel<32>, dim3(1), dim3(kFinNT), lds, s, a, round); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_subtract(const Launch& a, uint32_t units, uint32_t lds, hipStream_t s) {
    hipLaunchKernelGGL(subtract_kernel, dim3(units), dim3(kSubNT), lds, s, a);
    return hipGetLastError();
}

// largest subtraction LDS: K = 4096 (P = 4096), B = 16384
constexpr int kSubLdsMax = kMaxK * 8 + kMaxK * 4 + kMaxK * 4 + kMaxFftLds * 2;

// largest vote dynamic LDS: the slots at N/B = 2 plus 96 KB of staged bitmaps
constexpr int kVoteLdsMax = (int)vote_slot_words(1) * 4 + 98304;

hipError_t set_estimate_attributes() {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&subtract_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kSubLdsMax);
    if (e == hipSuccess) e = Votes::set_lds(kVoteLdsMax);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&residual_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                                kMaxK * 28);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&residual_one_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kMaxK * 28);
    return e;
}

hipError_t launch_residual(const Launch& a, uint32_t units, uint32_t lds, hipStream_t s) {
    hipLaunchKernelGGL(residual_kernel, dim3(units), dim3(kResNT), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_residual_one(const Launch& a, uint32_t units, uint32_t lds, hipStream_t s) {
    hipLaunchKernelGGL(residual_one_kernel, dim3(units), dim3(kResNT), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_residual_sum(const Launch& a, uint32_t units, hipStream_t s) {
    hipLaunchKernelGGL(residual_sum_kernel, dim3(units), dim3(kResNT), 0, s, a);
    return hipGetLastError();
}

}  // namespace sfft
