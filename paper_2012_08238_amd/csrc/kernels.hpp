// Launchers of the gfx950 kernels (defined in fold.hip, fft.hip and estimate.hip).
#pragma once

#include "common.hpp"

namespace sfft {

// Bucketization kernel variant of a plan: 0 = gather; otherwise the strip form
// with its tile size, items per thread and window-tap vectors encoded
// (fold_variant). Every signal of one launch must share the variant.
uint32_t fold_variant(uint32_t mode, uint32_t strip_lds, uint32_t items, uint32_t g4);
constexpr uint32_t kFoldVariant512 = 1u << 20;   // variant bit: the 512-thread full-tile instance
constexpr uint32_t kFoldVariantFull = 1u << 21;  // variant bit: the tile is exactly the threads' loads
// lds_bytes = strip tile bytes (strip variants)
hipError_t launch_fold(const Launch& a, uint32_t variant, uint32_t units, uint32_t lds_bytes, hipStream_t s);
// one workgroup per (signal, loop); every signal of the launch has B = 2^log2B <= 16384
hipError_t launch_fft_select(const Launch& a, uint32_t log2B, uint32_t units, hipStream_t s);
// comb prefilter: one workgroup per (signal, comb loop); every signal of the launch has Bc = 2^log2b <= 16384
hipError_t launch_comb(const Launch& a, uint32_t log2b, uint32_t units, hipStream_t s);
// B = 2^log2B > 16384: pass 0 = first FFT pass (units = L * B2/16 per signal),
// 1 = second pass (L * B1/16), 2 = selection (L); every signal of the launch has this B
hipError_t launch_fft_large(const Launch& a, uint32_t log2B, uint32_t pass, uint32_t units, hipStream_t s);
// lds_bytes = Resolved::vote_dyn_lds (max over the launch): the slot words, then (staged: the
// bitmaps are copied to LDS) L * ceil(B/32) * 4 bytes; key = vote_key(L), the same for every
// signal of the launch; round 1: the vote of the subtraction round (the first round's
// frequencies are excluded)
hipError_t launch_vote(const Launch& a, uint32_t key, uint32_t units, uint32_t lds_bytes, uint32_t staged,
                       uint32_t round, hipStream_t s);
// phase-encoding location: kDecUnit selected buckets per workgroup; round 1 excludes the first round's
// frequencies
hipError_t launch_decode(const Launch& a, uint32_t units, uint32_t round, hipStream_t s);
// estimates of the candidates: est_units workgroups per signal; lmax in {4, 8, 16, 32} >= L of
// every signal of the launch; round 1 adds the first round's coefficients to the candidates
hipError_t launch_estimate(const Launch& a, uint32_t lmax, uint32_t units, uint32_t round, hipStream_t s);
// the K largest estimates: one workgroup per signal; lds_bytes = Resolved::fin_lds (max over the launch);
// round 0 of an iterating signal keeps them in the workspace, otherwise they go to the outputs
hipError_t launch_finalize(const Launch& a, uint32_t units, uint32_t lds_bytes, uint32_t round, hipStream_t s);
// one signal (nsig == 0) with est_units = 1: the estimates and the K largest in one launch of one
// workgroup; lds_bytes = Resolved::fin_lds
hipError_t launch_tail_one(const Launch& a, uint32_t lmax, uint32_t lds_bytes, uint32_t round, hipStream_t s);
// subtraction round: one workgroup per (signal, loop); lds_bytes = Resolved::sub_lds (max over the launch)
hipError_t launch_subtract(const Launch& a, uint32_t units, uint32_t lds_bytes, hipStream_t s);
// selection of the residual buckets: one workgroup per (signal, loop); every signal has B = 2^log2B <= 16384
hipError_t launch_reselect(const Launch& a, uint32_t log2B, uint32_t units, hipStream_t s);
hipError_t launch_residual(const Launch& a, uint32_t units, uint32_t lds_bytes, hipStream_t s);
// one signal (nsig == 0): the residual and the sum of its partials in one launch (ctr[3] counts
// the finished workgroups; the bucketization clears it)
hipError_t launch_residual_one(const Launch& a, uint32_t units, uint32_t lds_bytes, hipStream_t s);
// the residual's partial sums into the outputs: one workgroup per signal, after launch_residual
hipError_t launch_residual_sum(const Launch& a, uint32_t units, hipStream_t s);
// fused single-launch form: one persistent workgroup takes whole signals (units = signals of the
// launch, each of one unit); key = vote_key(L) <= 16, the same for every signal; lds_bytes =
// Resolved::fused_lds (max over the launch)
hipError_t launch_fused(const Launch& a, uint32_t key, uint32_t units, uint32_t lds_bytes, hipStream_t s);
// LDS bytes of the fused form's transform and selection at B = 2^log2B (0 outside its range)
uint32_t fused_fft_lds(uint32_t log2B);
// raises the dynamic-LDS limit of the kernels that use more than 64 KB
hipError_t set_kernel_attributes_impl();
hipError_t set_fold_attributes();
hipError_t set_fft_attributes();
hipError_t set_estimate_attributes();

}  // namespace sfft
