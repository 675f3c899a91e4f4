// The fused single-launch form: launchers of the instances L = 9..16.
#include "fused.hpp"

namespace sfft {

hipError_t launch_fused_hi(const Launch& a, uint32_t key, uint32_t units, uint32_t lds_bytes, hipStream_t s) {
    return FusedTable<9, 10, 11, 12, 13, 14, 15, 16>::launch(key, a, units, lds_bytes, s);
}

}  // namespace sfft
