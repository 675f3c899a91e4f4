// Internal helpers shared by the C ABI translation units.
#pragma once

#include <string>

#include "common.hpp"
#include "host.hpp"

namespace sfft {

sfft_status set_error(sfft_status s, const std::string& msg);
sfft_status hip_fail(hipError_t e, const char* what);

// Sets the maximum dynamic LDS of the kernels that need more than 64 KB.
// Called once per process before the first launch (and before any capture).
hipError_t init_kernel_attributes();

SigDesc make_desc(const Resolved& R, char* tab, char* ws);
// Point a plan's descriptor at the device descriptor of its estimation-only loops.
void link_est(SigDesc* d, const SigDesc* d_est_dev, const Resolved& R);
size_t plan_est_table_offset(sfft_plan_t p);
sfft_status launch_single(const Resolved& R, const SigDesc* d_desc, const IoDesc& io, hipStream_t s);

sfft_status plan_create(const sfft_params& p, sfft_plan_t* out);
const Resolved& plan_resolved(sfft_plan_t p);
const char* plan_tables(sfft_plan_t p);
int plan_device(sfft_plan_t p);
size_t plan_table_bytes(sfft_plan_t p);
size_t plan_ws_bytes(sfft_plan_t p);
// Asynchronous execution of a plan; scratch = true runs on the per-device scratch array
// (sfft_execute_noalloc) instead of the plan's workspace.
sfft_status plan_execute(sfft_plan_t p, const void* x_dev, int64_t* out_idx, void* out_val, double* out_resid,
                         sfft_stream_t stream, bool scratch);
// Per-device scratch array of sfft_execute_noalloc: its size, and its device address on
// `device` (which must be current; looked up once per device, then cached).
size_t scratch_bytes();
hipError_t scratch_address(int device, char** out);

}  // namespace sfft
