// Window taps of the flat window and the gather form of one bucket: device helpers
// shared by the bucketization kernels and the fused single-signal kernel.
#pragma once

#include "device.hpp"

namespace sfft {

// Window taps g_n, n = b + m B, of the flat window (sinc of Eq.(12) times the Gaussian of
// Eq.(13), centred at w/2, std s = w / (2 gauss_c)), computed in FP32 from the definition
// instead of read from a table: with t = n - w/2, g_n = e^{-t^2/2s^2} sin(pi t/B) / (pi t)
// (1/B at t = 0). Since sin(pi (t + B)/B) = -sin(pi t/B), one sinpi per bucket serves all
// its taps: sin(pi t/B) = (-1)^m sin(pi r0/B), r0 = (b - w/2) mod 2B (an exact argument);
// the Gaussian is 2^{-(t kappa)^2}. Every bucketization form computes its taps here, so
// the forms stay bitwise identical. (Relative error about 1e-6 against the FP64 window.)
struct WinTaps {
    int32_t t0;       // b - w/2
    float s0pi;       // sin(pi r0/B) / pi
    float kappa, invB;
    uint32_t log2B;
    __device__ __forceinline__ float operator()(uint32_t m) const {
        const int32_t t = t0 + (int32_t)(m << log2B);
        const float tf = (float)t;
        const float q = tf * kappa;
        const float e = exp2f(-(q * q));
        const float sg = (m & 1u) ? -s0pi : s0pi;
        const float g = e * (sg * __builtin_amdgcn_rcpf(tf));
        return t == 0 ? invB : g;
    }
};

__device__ __forceinline__ WinTaps win_taps(uint32_t b, uint32_t w, uint32_t log2B, float kappa) {
    const uint32_t B = 1u << log2B;
    const uint32_t r0 = (b - (w >> 1)) & (2u * B - 1u);
    WinTaps t;
    t.t0 = (int32_t)b - (int32_t)(w >> 1);
    t.invB = 1.0f / (float)B;
    t.s0pi = sinpif((float)r0 * t.invB) * 0.318309886183790672f;
    t.kappa = kappa;
    t.log2B = log2B;
    return t;
}

// Bucket b of a loop with scaling s and shift tu, gathered from the signal x: the sum
// over taps i = b + m B < w (m < Mw) of g_i x[(s i + tu) mod N], in tap order, four
// loads in flight. Every form of the bucketization sums the same taps in this order.
template <class Desc>
__device__ __forceinline__ float2 gather_bucket(const Desc& d, const float2* x, uint32_t s, uint32_t tu, uint32_t b) {
    const uint32_t log2B = d.log2B;
    const uint32_t Mw = d.Mw, Mw4 = d.Mw4, w = d.w, maskN = d.maskN;
    const WinTaps wt = win_taps(b, w, log2B, d.wkappa);
    float2 acc = make_float2(0.f, 0.f);
    for (uint32_t m4 = 0; m4 < Mw4; m4 += 4) {
        const f4v g = f4v{wt(m4), wt(m4 + 1u), wt(m4 + 2u), wt(m4 + 3u)};
        float2 xv[4];
        bool ok[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint32_t m = m4 + e;
            const uint32_t i = b + (m << log2B);
            ok[e] = m < Mw && i < w;
            xv[e] = gld(x + ((s * i + tu) & maskN));   // always in bounds; unused when !ok
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (ok[e]) {
                acc.x = fmaf(g[e], xv[e].x, acc.x);
                acc.y = fmaf(g[e], xv[e].y, acc.y);
            }
        }
    }
    return acc;
}

}  // namespace sfft
