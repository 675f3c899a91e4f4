// Device-side helpers shared by the gfx950 kernels: typed global loads and
// stores, descriptor access through the constant address space, the launch
// unit -> (signal, unit) mapping, complex multiply, energy keys and scans.
//
// Index arithmetic is exact: every product sigma*i, tau*f, t*f is a wrapping
// 32-bit multiply masked by N-1, exact because N divides 2^32.
//
// Memory access: descriptors are read through the constant address space
// (scalar loads); data through explicit global-address-space loads and stores,
// streamed signal reads carry the non-temporal hint.
#pragma once

#include "common.hpp"
#include "kernels.hpp"

namespace sfft {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(4))) SigDesc* CDesc;
typedef const __attribute__((address_space(4))) IoDesc* CIo;
typedef const __attribute__((address_space(4))) uint32_t* CU32;

template <typename T>
__device__ __forceinline__ T gld(const T* p) {
    return *(const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ T gld_nt(const T* p) {
    return __builtin_nontemporal_load((const __attribute__((address_space(1))) T*)p);
}
template <typename T>
__device__ __forceinline__ void gst(T* p, const T& v) {
    *(__attribute__((address_space(1))) T*)p = v;
}
// two-component HIP vector types go through the native vector types
typedef float f2n __attribute__((ext_vector_type(2)));
typedef double d2n __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 gld(const float2* p) {
    const f2n t = *(const __attribute__((address_space(1))) f2n*)p;
    return make_float2(t.x, t.y);
}
__device__ __forceinline__ double2 gld(const double2* p) {
    const d2n t = *(const __attribute__((address_space(1))) d2n*)p;
    return make_double2(t.x, t.y);
}
__device__ __forceinline__ void gst(float2* p, const float2& v) {
    f2n t;
    t.x = v.x;
    t.y = v.y;
    *(__attribute__((address_space(1))) f2n*)p = t;
}

// ---------------------------------------------------------------- helpers
// Workgroups are dealt to the XCDs round-robin (workgroup b runs on XCD b mod 8).
// Renumber them so that XCD x runs the contiguous unit range starting at
// x*base + min(x, rem): each XCD then works on neighbouring units (adjacent
// column strips of the same rows) at the same time. A bijection on [0, grid).
__device__ __forceinline__ uint32_t xcd_unit(uint32_t blk, uint32_t grid) {
    const uint32_t x = blk % kNumXcd, i = blk / kNumXcd;
    const uint32_t base = grid / kNumXcd, rem = grid % kNumXcd;
    return x * base + min(x, rem) + i;
}

// (signal, unit) of launch-wide unit blk
__device__ __forceinline__ void resolve_blk(const Launch& a, uint32_t blk, uint32_t& sig, uint32_t& unit) {
    if (a.nsig == 0) {
        sig = 0;
        unit = blk;
        return;
    }
    const CU32 pre = (CU32)a.prefix;
    uint32_t lo = 0, hi = a.nsig;  // largest s with prefix[s] <= blk
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (pre[mid] <= blk) lo = mid; else hi = mid;
    }
    sig = lo;
    unit = blk - pre[lo];
}

__device__ __forceinline__ void resolve(const Launch& a, uint32_t& sig, uint32_t& unit) {
    resolve_blk(a, a.xcd_order ? xcd_unit(blockIdx.x, gridDim.x) : blockIdx.x, sig, unit);
}

__device__ __forceinline__ const __attribute__((address_space(4))) SigDesc& desc_of(const Launch& a, uint32_t sig) {
    return *((CDesc)a.descs + sig);
}

__device__ __forceinline__ IoDesc io_of(const Launch& a, uint32_t sig) {
    if (a.nsig == 0) return a.one_io;
    const __attribute__((address_space(4))) IoDesc& io = *((CIo)a.ios + sig);
    IoDesc r;
    r.x = io.x;
    r.out_idx = io.out_idx;
    r.out_val = io.out_val;
    r.out_resid = io.out_resid;
    return r;
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// |v|^2 as the bit pattern of a non-negative float (monotone as unsigned): the
// ordering key of bucket energies, computed the same way wherever it is needed
__device__ __forceinline__ uint32_t energy_key(float2 v) { return __float_as_uint(fmaf(v.x, v.x, v.y * v.y)); }

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const uint32_t lane = threadIdx.x & 63u;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = __shfl_up(v, off, 64);
        if (lane >= (uint32_t)off) v += t;
    }
    return v;
}

// Exclusive scan over the block (NT threads, NT/64 waves); `sh` holds NT/64 words.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* sh, uint32_t& total) {
    const uint32_t lane = threadIdx.x & 63u, wid = threadIdx.x >> 6;
    const uint32_t incl = wave_incl_scan(v);
    if (lane == 63u) sh[wid] = incl;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
        const uint32_t s = sh[w];
        if ((uint32_t)w < wid) off += s;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return off + incl - v;
}

}  // namespace sfft
