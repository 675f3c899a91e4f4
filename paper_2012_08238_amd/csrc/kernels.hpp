// Launchers of the gfx950 kernels (defined in kernels.hip).
#pragma once

#include "common.hpp"

namespace sfft {

// mode 1 = strip (lds_bytes = tile bytes), mode 0 = gather
hipError_t launch_fold(const Launch& a, uint32_t mode, uint32_t units, uint32_t lds_bytes, hipStream_t s);
// one workgroup per (signal, loop); every signal of the launch has B = 2^log2B <= 16384
hipError_t launch_fft_select(const Launch& a, uint32_t log2B, uint32_t units, hipStream_t s);
// lds_bytes = L * ceil(B/32) * 4 when the selected-bucket bitmaps are staged in LDS, else 0
hipError_t launch_vote(const Launch& a, uint32_t units, uint32_t lds_bytes, hipStream_t s);
// one workgroup per signal; lmax in {4, 8, 16, 32} >= L of every signal of the launch
hipError_t launch_finalize(const Launch& a, uint32_t lmax, uint32_t units, hipStream_t s);
hipError_t launch_residual(const Launch& a, uint32_t units, hipStream_t s);
// raises the dynamic-LDS limit of the kernels that use more than 64 KB
hipError_t set_kernel_attributes_impl();

}  // namespace sfft
