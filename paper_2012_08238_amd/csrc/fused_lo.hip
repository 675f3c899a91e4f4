// The fused single-launch form: launchers of the instances L = 1..8 and the entry point.
#include "fused.hpp"

namespace sfft {

uint32_t fused_fft_lds(uint32_t log2B) {
    switch (log2B) {
        case 5: return (uint32_t)FftCfg<5, (int)kFusedNT>::lds_bytes();
        case 6: return (uint32_t)FftCfg<6, (int)kFusedNT>::lds_bytes();
        case 7: return (uint32_t)FftCfg<7, (int)kFusedNT>::lds_bytes();
        case 8: return (uint32_t)FftCfg<8, (int)kFusedNT>::lds_bytes();
        case 9: return (uint32_t)FftCfg<9, (int)kFusedNT>::lds_bytes();
        case 10: return (uint32_t)FftCfg<10, (int)kFusedNT>::lds_bytes();
        case 11: return (uint32_t)FftCfg<11, (int)kFusedNT>::lds_bytes();
        case 12: return (uint32_t)FftCfg<12, (int)kFusedNT>::lds_bytes();
        default: return 0u;
    }
}

hipError_t launch_fused(const Launch& a, uint32_t key, uint32_t units, uint32_t lds_bytes, hipStream_t s) {
    if (key > 8u) return launch_fused_hi(a, key, units, lds_bytes, s);
    return FusedTable<1, 2, 3, 4, 5, 6, 7, 8>::launch(key, a, units, lds_bytes, s);
}

}  // namespace sfft
