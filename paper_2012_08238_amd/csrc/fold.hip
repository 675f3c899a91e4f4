// Bucketization kernels (Eq.(6)-(7), (11)-(13)): window the permuted signal and
// alias it into B buckets, per loop, stored in column order.
#include "fold_dev.hpp"

namespace sfft {

// ---------------------------------------------------------------- bucketization
// Every bucketization kernel raises its waves' issue priority: it streams the signals
// from HBM, and when later stages of other batches run beside it on the same compute
// units (other streams) the SIMD arbiter then issues its loads first, which keeps HBM busy.
__device__ __forceinline__ void fold_priority() { __builtin_amdgcn_s_setprio(3); }

// Strip form. View x as an (N/B) x B row-major matrix: time sample a = row*B + col.
// For loop r the window index of sample a is i = sigma^{-1}(a - tau) mod N and its
// bucket is i mod B, which depends on col only (B | N). Each workgroup streams a
// full-height strip of C columns into LDS (all PER 16-byte loads of a thread in
// flight at once) and then, for every (loop, column), sums the taps i = b + m*B
// that land in the column: they sit at rows (q + sigma*m) mod (N/B) of it.
template <int PER>
__global__ __launch_bounds__(kFoldNT) void fold_strip_kernel(Launch a) {
    fold_priority();
    extern __shared__ f4v lds4[];
    uint32_t sig, unit;
    resolve(a, sig, unit);
    const auto& d = desc_of(a, sig);
    const float2* x = io_of(a, sig).x;
    if (unit == 0 && threadIdx.x == 0) {
        gst(d.ctr + 0, 0u);
        gst(d.ctr + 3, 0u);   // residual workgroups done (single-signal residual)
    }
    const uint32_t log2C = d.log2C, C = 1u << log2C, R = d.M, B = d.B, log2B = d.log2B;
    const uint32_t col0 = unit << log2C;
    const uint32_t log2h = log2C - 1;  // 16-byte loads per row = C/2
    const uint32_t total = R << log2h;
    const f4v* xs = reinterpret_cast<const f4v*>(x);
    f4v v[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const uint32_t k = threadIdx.x + j * kFoldNT;
        if (k < total) {
            const uint32_t row = k >> log2h, c = k & ((1u << log2h) - 1u);
            v[j] = gld_nt(xs + ((((size_t)row << log2B) + col0) >> 1) + c);
        }
    }
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const uint32_t k = threadIdx.x + j * kFoldNT;
        if (k < total) lds4[k] = v[j];
    }
    __syncthreads();
    const float2* tile = reinterpret_cast<const float2*>(lds4);
    const uint32_t items = d.L << log2C;
    const uint32_t Mw = d.Mw, Mw4 = d.Mw4, w = d.w, maskN = d.maskN;
    const float kappa = d.wkappa;
    const uint32_t* sigma = d.sigma;
    const uint32_t* sigma_inv = d.sigma_inv;
    const uint32_t* tau = d.tau;
    float2* uhat = d.uhat;
    for (uint32_t it = threadIdx.x; it < items; it += kFoldNT) {
        const uint32_t r = it >> log2C, c = it & (C - 1u);
        const uint32_t s = gld(sigma + r), si = gld(sigma_inv + r), tu = gld(tau + r);
        const uint32_t b = (si * (col0 + c - tu)) & (B - 1u);
        const uint32_t q = ((s * b + tu) & maskN) >> log2B;
        const WinTaps wt = win_taps(b, w, log2B, kappa);
        float2 acc = make_float2(0.f, 0.f);
        for (uint32_t m4 = 0; m4 < Mw4; m4 += 4) {
            const f4v g = f4v{wt(m4), wt(m4 + 1u), wt(m4 + 2u), wt(m4 + 3u)};
            float2 xv[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t row = (q + s * (m4 + e)) & (R - 1u);
                xv[e] = tile[(row << log2C) + c];
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t m = m4 + e;
                if (m < Mw && b + (m << log2B) < w) {
                    acc.x = fmaf(g[e], xv[e].x, acc.x);
                    acc.y = fmaf(g[e], xv[e].y, acc.y);
                }
            }
        }
        gst(uhat + (size_t)r * B + col0 + c, acc);   // column order (see fft_select_kernel)
    }
}

// Strip form for the common shapes: each of the NT threads owns at most IPT (loop,
// column) items of G4*4 window taps. All tile loads are issued first (branch-free:
// out-of-tile slots reload the last element); while they are in flight the
// thread computes its items' buckets and window taps. The tile
// then passes through LDS in H row bands (LDS = tile/H, so more workgroups fit
// per CU); each band delivers the taps whose rows it holds, and the taps are
// summed in tap order at the end: same taps, same order as the other forms.
template <int PER, int IPT, int G4, int H, int NT = (int)kFoldNT, bool FULL = false>
__global__ __launch_bounds__(NT) void fold_strip_pf_kernel(Launch a) {
    fold_priority();
    extern __shared__ f4v lds4[];
    uint32_t sig, unit;
    resolve(a, sig, unit);
    const auto& d = desc_of(a, sig);
    const float2* x = io_of(a, sig).x;
    if (unit == 0 && threadIdx.x == 0) {
        gst(d.ctr + 0, 0u);
        gst(d.ctr + 3, 0u);   // residual workgroups done (single-signal residual)
    }
    const uint32_t log2C = d.log2C, C = 1u << log2C, R = d.M, B = d.B, log2B = d.log2B;
    const uint32_t col0 = unit << log2C;
    const uint32_t log2h = log2C - 1;
    const uint32_t total = R << log2h;
    const f4v* xs = reinterpret_cast<const f4v*>(x);
    f4v v[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const uint32_t k = min(threadIdx.x + j * NT, total - 1u);
        const uint32_t row = k >> log2h, c = k & ((1u << log2h) - 1u);
        v[j] = gld_nt(xs + ((((size_t)row << log2B) + col0) >> 1) + c);
    }
    const uint32_t items = d.L << log2C;
    const uint32_t Mw = d.Mw, w = d.w, maskN = d.maskN;
    const float kappa = d.wkappa;
    uint32_t ri[IPT], ci[IPT], si_[IPT], bi[IPT], qi[IPT], sv[IPT], tv[IPT];
    f4v gi[IPT][G4];
#pragma unroll
    for (int e = 0; e < IPT; ++e) {
        const uint32_t it = threadIdx.x + e * NT;
        ri[e] = it >> log2C;
        ci[e] = it & (C - 1u);
        si_[e] = sv[e] = tv[e] = 0u;
    }
    // sigma_r, sigma_r^{-1}, tau_r through the scalar cache in a uniform loop
    // over the loops: a vector load here would complete only after the tile's
    // loads (vector loads retire in issue order) and serialise the taps behind it
    const uint32_t L = d.L;
    for (uint32_t r = 0; r < L; ++r) {
        const uint32_t s = ((CU32)d.sigma)[r], sinv = ((CU32)d.sigma_inv)[r], tu = ((CU32)d.tau)[r];
#pragma unroll
        for (int e = 0; e < IPT; ++e) {
            if (ri[e] == r) {
                si_[e] = s;
                sv[e] = sinv;
                tv[e] = tu;
            }
        }
    }
#pragma unroll
    for (int e = 0; e < IPT; ++e) {
        const uint32_t it = threadIdx.x + e * NT;
        if (it < items) {
            const uint32_t b = (sv[e] * (col0 + ci[e] - tv[e])) & (B - 1u);
            bi[e] = b;
            qi[e] = ((si_[e] * b + tv[e]) & maskN) >> log2B;
            const WinTaps wt = win_taps(b, w, log2B, kappa);
#pragma unroll
            for (int k = 0; k < G4; ++k)
                gi[e][k] = f4v{wt(4u * k), wt(4u * k + 1u), wt(4u * k + 2u), wt(4u * k + 3u)};
        }
    }
    constexpr int TAPS = G4 * 4;
    float2 xv[IPT][TAPS];
    const uint32_t log2band = __builtin_ctz(total) - __builtin_ctz((uint32_t)H);  // float4 per band
    const uint32_t log2rb = __builtin_ctz(R) - __builtin_ctz((uint32_t)H);       // rows per band
    const float2* tile = reinterpret_cast<const float2*>(lds4);
#pragma unroll
    for (int h = 0; h < H; ++h) {
        if (h > 0) __syncthreads();   // the previous band has been read
        if constexpr (FULL) {
            // the tile is exactly PER loads per thread: band h is loads h PER/H .. (h+1) PER/H - 1,
            // known at compile time, so each load's registers are free once its band is stored
#pragma unroll
            for (int j = h * (PER / H); j < (h + 1) * (PER / H); ++j)
                lds4[threadIdx.x + (uint32_t)j * NT - ((uint32_t)h << log2band)] = v[j];
        } else {
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                const uint32_t k = threadIdx.x + j * NT;
                if (k < total && (k >> log2band) == (uint32_t)h) lds4[k - ((uint32_t)h << log2band)] = v[j];
            }
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < IPT; ++e) {
            const uint32_t it = threadIdx.x + e * NT;
            if (it < items) {
#pragma unroll
                for (int m = 0; m < TAPS; ++m) {
                    const uint32_t row = (qi[e] + si_[e] * (uint32_t)m) & (R - 1u);
                    if ((uint32_t)m < Mw && (row >> log2rb) == (uint32_t)h)
                        xv[e][m] = tile[((row & ((1u << log2rb) - 1u)) << log2C) + ci[e]];
                }
            }
        }
    }
#pragma unroll
    for (int e = 0; e < IPT; ++e) {
        const uint32_t it = threadIdx.x + e * NT;
        if (it < items) {
            const uint32_t b = bi[e];
            float2 acc = make_float2(0.f, 0.f);
#pragma unroll
            for (int m = 0; m < TAPS; ++m) {
                if ((uint32_t)m < Mw && b + ((uint32_t)m << log2B) < w) {
                    const float g = gi[e][m >> 2][m & 3];
                    acc.x = fmaf(g, xv[e][m].x, acc.x);
                    acc.y = fmaf(g, xv[e][m].y, acc.y);
                }
            }
            gst(d.uhat + (size_t)ri[e] * B + col0 + ci[e], acc);   // column order
        }
    }
}

// Gather form: one thread per (loop, bucket) reads its permuted samples
// directly (four loads in flight). Same taps in the same order as the strip
// form, so both give bitwise-identical buckets.
__global__ __launch_bounds__(kFoldNT) void fold_gather_kernel(Launch a) {
    fold_priority();
    uint32_t sig, unit;
    resolve(a, sig, unit);
    const auto& d = desc_of(a, sig);
    const float2* x = io_of(a, sig).x;
    if (unit == 0 && threadIdx.x == 0) {
        gst(d.ctr + 0, 0u);
        gst(d.ctr + 3, 0u);   // residual workgroups done (single-signal residual)
    }
    const uint32_t log2B = d.log2B, B = d.B;
    const uint32_t it = unit * kFoldNT + threadIdx.x;
    if (it >= (d.L << log2B)) return;
    // thread (loop r, column col) computes the bucket b whose samples all sit in
    // that column, so that the result is stored in column order like the strip form
    const uint32_t r = it >> log2B, col = it & (B - 1u);
    const uint32_t s = gld(d.sigma + r), tu = gld(d.tau + r);
    const uint32_t b = (gld(d.sigma_inv + r) * (col - tu)) & (B - 1u);
    const float2 acc = gather_bucket(d, x, s, tu, b);
    gst(d.uhat + it, acc);   // = uhat[r * B + col]
}

// ---------------------------------------------------------------- launchers
template <int PER>
static hipError_t set_strip_attr() {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&fold_strip_kernel<PER>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, 131072);
}

template <int IPT, int G4>
static hipError_t set_pf512_attr() {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&fold_strip_pf_kernel<16, IPT, G4, 2, 512, true>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
}

hipError_t set_fold_attributes() {
    hipError_t e;
    if ((e = set_strip_attr<16>()) != hipSuccess) return e;
    if ((e = set_strip_attr<32>()) != hipSuccess) return e;
    if ((e = set_pf512_attr<1, 1>()) != hipSuccess) return e;
    if ((e = set_pf512_attr<1, 2>()) != hipSuccess) return e;
    if ((e = set_pf512_attr<2, 1>()) != hipSuccess) return e;
    return set_pf512_attr<2, 2>();
}

uint32_t strip_per_thread(uint32_t lds_bytes) {
    const uint32_t f4 = (lds_bytes + 15) / 16;
    uint32_t per = 1;
    while (per * kFoldNT < f4) per <<= 1;
    return per;
}

uint32_t fold_variant(uint32_t mode, uint32_t strip_lds, uint32_t items, uint32_t g4) {
    if (mode == 0) return 0;
    const uint32_t per = strip_per_thread(strip_lds);
    uint32_t lp = 0;
    while ((1u << lp) < per) ++lp;
    const uint32_t ipt = (items + kFoldNT - 1) / kFoldNT;
    // a tile of exactly `per` loads per thread lets the kernel store each band from loads
    // known at compile time (their registers free once stored: 140 -> 96 VGPRs at 16 loads)
    const uint32_t full = strip_lds == per * kFoldNT * 16u ? kFoldVariantFull : 0u;
    if (per >= 4 && ipt >= 1 && ipt <= 2 && g4 >= 1 && g4 <= 2) return (1u << 16) | full | (lp << 8) | (ipt << 4) | g4;
    // up to four items per thread with a 32 KB tile (measured faster for N/B = 64; with a
    // 64 KB tile the plain strip kernel is as fast)
    if (per == 8 && ipt <= 4 && g4 >= 1 && g4 <= 2) return (1u << 16) | full | (lp << 8) | (4u << 4) | g4;
    // a full 128 KB tile (e.g. 64 columns of 256 rows): 512 threads of 16 loads, two 64 KB
    // bands, at most two items per thread
    if (per == 32 && strip_lds == 32u * kFoldNT * 16u && items <= 1024u && g4 >= 1 && g4 <= 2)
        return (1u << 16) | kFoldVariant512 | (4u << 8) | (((items + 511u) / 512u) << 4) | g4;
    return (1u << 16) | (lp << 8);
}

// row bands of the prefetching strip kernel: LDS holds at most 32 KB of the tile
constexpr uint32_t strip_bands(uint32_t per) { return per >= 16 ? per / 8 : 1; }

#define SFFT_PF(PER, IPT, G4)                                                                              \
    case (PER << 8) | (IPT << 4) | G4:                                                                     \
        if (full)                                                                                          \
            hipLaunchKernelGGL((fold_strip_pf_kernel<PER, IPT, G4, strip_bands(PER), (int)kFoldNT, true>), \
                               dim3(units), dim3(kFoldNT), lds_bytes / strip_bands(PER), s, a);            \
        else                                                                                               \
            hipLaunchKernelGGL((fold_strip_pf_kernel<PER, IPT, G4, strip_bands(PER)>), dim3(units),        \
                               dim3(kFoldNT), lds_bytes / strip_bands(PER), s, a);                         \
        break;

hipError_t launch_fold(const Launch& a, uint32_t variant, uint32_t units, uint32_t lds_bytes, hipStream_t s) {
    if (variant & kFoldVariant512) {
        // full 128 KB tile, 512 threads, two bands
        switch (variant & 0xFFu) {
            case 0x11:
                hipLaunchKernelGGL((fold_strip_pf_kernel<16, 1, 1, 2, 512, true>), dim3(units), dim3(512), lds_bytes / 2, s, a);
                break;
            case 0x12:
                hipLaunchKernelGGL((fold_strip_pf_kernel<16, 1, 2, 2, 512, true>), dim3(units), dim3(512), lds_bytes / 2, s, a);
                break;
            case 0x21:
                hipLaunchKernelGGL((fold_strip_pf_kernel<16, 2, 1, 2, 512, true>), dim3(units), dim3(512), lds_bytes / 2, s, a);
                break;
            case 0x22:
                hipLaunchKernelGGL((fold_strip_pf_kernel<16, 2, 2, 2, 512, true>), dim3(units), dim3(512), lds_bytes / 2, s, a);
                break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (variant == 0) {
        hipLaunchKernelGGL(fold_gather_kernel, dim3(units), dim3(kFoldNT), 0, s, a);
        return hipGetLastError();
    }
    const uint32_t per = 1u << ((variant >> 8) & 15u);
    const uint32_t ipt = (variant >> 4) & 15u, g4 = variant & 15u;
    const bool full = (variant & kFoldVariantFull) != 0;
    if (ipt == 0) {
        switch (per) {
            case 1: hipLaunchKernelGGL(fold_strip_kernel<1>, dim3(units), dim3(kFoldNT), lds_bytes, s, a); break;
            case 2: hipLaunchKernelGGL(fold_strip_kernel<2>, dim3(units), dim3(kFoldNT), lds_bytes, s, a); break;
            case 4: hipLaunchKernelGGL(fold_strip_kernel<4>, dim3(units), dim3(kFoldNT), lds_bytes, s, a); break;
            case 8: hipLaunchKernelGGL(fold_strip_kernel<8>, dim3(units), dim3(kFoldNT), lds_bytes, s, a); break;
            case 16: hipLaunchKernelGGL(fold_strip_kernel<16>, dim3(units), dim3(kFoldNT), lds_bytes, s, a); break;
            case 32: hipLaunchKernelGGL(fold_strip_kernel<32>, dim3(units), dim3(kFoldNT), lds_bytes, s, a); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch ((per << 8) | (ipt << 4) | g4) {
        SFFT_PF(4, 1, 1) SFFT_PF(4, 1, 2) SFFT_PF(4, 2, 1) SFFT_PF(4, 2, 2)
        SFFT_PF(8, 1, 1) SFFT_PF(8, 1, 2) SFFT_PF(8, 2, 1) SFFT_PF(8, 2, 2)
        SFFT_PF(16, 1, 1) SFFT_PF(16, 1, 2) SFFT_PF(16, 2, 1) SFFT_PF(16, 2, 2)
        SFFT_PF(32, 1, 1) SFFT_PF(32, 1, 2) SFFT_PF(32, 2, 1) SFFT_PF(32, 2, 2)
        SFFT_PF(8, 4, 1) SFFT_PF(8, 4, 2)
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
#undef SFFT_PF

}  // namespace sfft
