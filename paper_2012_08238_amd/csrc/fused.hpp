// The whole path of a small plan in one launch: one workgroup carries a signal
// through bucketization, B-point FFT and selection (loop by loop, the buckets
// gathered straight into LDS), the vote, the estimates, the K largest and the FP64
// residual, with workgroup barriers between the stages instead of kernel
// boundaries. The workgroups persist, each taking the signals blockIdx.x,
// blockIdx.x + gridDim.x, ... of the launch, so a batch of small signals costs one
// launch instead of one per stage. Every stage runs the same device code as the
// per-stage kernels (same taps, transform, tests and sums in the same order).
#pragma once

#include "estimate_dev.hpp"
#include "fft_dev.hpp"
#include "fold_dev.hpp"

namespace sfft {

namespace fused_detail {

// Between two stages of one signal: the workgroup barrier (with its workgroup-scope
// release and acquire) makes every thread's global writes of the stage visible to the
// whole workgroup, whose waves share one compute unit's caches, and orders the LDS
// reuse. No device-scope fence is needed: no other workgroup reads what this one
// writes (on MI355X a device-scope fence would also write back and invalidate the
// die's L2, which every other workgroup on that die then pays for).
__device__ __forceinline__ void stage_sync() { __syncthreads(); }

// Bucketization, transform and selection of every loop: loop r's B buckets are
// gathered into the transform's LDS in bucket order (the values the per-stage
// kernels pass through the workspace in column order), then transformed, stored
// to uhat[r] and selected.
template <int LOG2B>
__device__ __forceinline__ void fused_loops(const __attribute__((address_space(4))) SigDesc& d, const float2* x,
                                            void* lds) {
    using Cfg = FftCfg<LOG2B, (int)kFusedNT>;
    static_assert(Cfg::B / 16 <= (int)kFusedNT, "the transform's passes need B/16 <= threads");
    const FftLds<Cfg> sm(lds);
    const uint32_t L = d.L;
    for (uint32_t r = 0; r < L; ++r) {
        if (r) __syncthreads();   // the previous loop's selection is done with the LDS
        const float2 twv = fft_twiddle_load<Cfg>(d);   // in flight with the gathers
        const uint32_t s = gld(d.sigma + r), tu = gld(d.tau + r);
        for (uint32_t b = threadIdx.x; b < (uint32_t)Cfg::B; b += kFusedNT)
            sm.data[padi((int)b)] = gather_bucket(d, x, s, tu, b);
        fft_twiddle_store(sm, twv);
        fft_select_staged<Cfg>(d, r, sm);
    }
}

}  // namespace fused_detail

// VL = vote_key(L) (L <= 16, so VL = L); estimates over LMAX = 4, 8 or 16 >= L. The
// compiler gives each instance 256 VGPRs and about 185 AGPRs: one wave per SIMD, one
// workgroup per compute unit (a cap at 128 registers per lane for more workgroups spilled
// to scratch).
template <int VL>
__global__ __launch_bounds__(kFusedNT) void fused_kernel(Launch a, uint32_t units) {
    constexpr int LMAX = VL <= 4 ? 4 : (VL <= 8 ? 8 : 16);
    extern __shared__ f4v lds_raw[];
    __shared__ uint32_t s_comb[1];          // no comb prefilter in this form
    __shared__ uint32_t s_pq[kVoteNT];      // vote by pair: each wave's queue
    uint32_t* sdyn = reinterpret_cast<uint32_t*>(lds_raw);
    for (uint32_t blk = blockIdx.x; blk < units; blk += gridDim.x) {
        uint32_t sig, unit;
        resolve_blk(a, blk, sig, unit);
        const auto& d = desc_of(a, sig);
        const float2* x = io_of(a, sig).x;
        if (blk != blockIdx.x) fused_detail::stage_sync();   // the previous signal is done with the LDS
        if (threadIdx.x == 0) gst(d.ctr + 0, 0u);
        switch (d.log2B) {
            case 5: fused_detail::fused_loops<5>(d, x, lds_raw); break;
            case 6: fused_detail::fused_loops<6>(d, x, lds_raw); break;
            case 7: fused_detail::fused_loops<7>(d, x, lds_raw); break;
            case 8: fused_detail::fused_loops<8>(d, x, lds_raw); break;
            case 9: fused_detail::fused_loops<9>(d, x, lds_raw); break;
            case 10: fused_detail::fused_loops<10>(d, x, lds_raw); break;
            case 11: fused_detail::fused_loops<11>(d, x, lds_raw); break;
            case 12: fused_detail::fused_loops<12>(d, x, lds_raw); break;
            default: break;   // refused when the plan is made
        }
        fused_detail::stage_sync();
        for (uint32_t u = 0; u < d.vote_units; ++u) {
            if (u) __syncthreads();   // the previous chunk's LDS reads are done
            vote_chunk<VL, true>(a, sig, u, 0u, u == 0u, sdyn, s_comb, s_pq);
        }
        fused_detail::stage_sync();
        for (uint32_t u = 0; u < d.est_units; ++u) {
            if (u) __syncthreads();
            estimate_body<LMAX>(a, sig, u, 0u);
        }
        fused_detail::stage_sync();
        finalize_body<kFusedNT, kFusedMaxK / kFusedNT>(a, sig, 0u);
        if (d.S) {
            fused_detail::stage_sync();
            for (uint32_t u = 0; u < d.resid_blocks; ++u) {
                if (u) __syncthreads();   // the previous unit's partial sums are read
                residual_body(a, sig, u, u == 0u);   // the outputs are staged once
            }
            fused_detail::stage_sync();
            residual_sum_body(a, sig);
        }
    }
}

template <int VL>
hipError_t launch_fused_vl(const Launch& a, uint32_t units, uint32_t lds_bytes, hipStream_t s) {
    const uint32_t grid = units < kFusedMaxGrid ? units : kFusedMaxGrid;
    hipLaunchKernelGGL((fused_kernel<VL>), dim3(grid), dim3(kFusedNT), lds_bytes, s, a, units);
    return hipGetLastError();
}

template <int... VLs>
struct FusedTable {
    static hipError_t launch(uint32_t key, const Launch& a, uint32_t units, uint32_t lds_bytes, hipStream_t s) {
        hipError_t e = hipErrorInvalidValue;
        ((key == (uint32_t)VLs ? (e = launch_fused_vl<VLs>(a, units, lds_bytes, s), 0) : 0), ...);
        return e;
    }
};

// the instances of L = 9..16 (fused_hi.hip; a translation unit of their own, so the two halves compile in parallel)
hipError_t launch_fused_hi(const Launch& a, uint32_t key, uint32_t units, uint32_t lds_bytes, hipStream_t s);

}  // namespace sfft
