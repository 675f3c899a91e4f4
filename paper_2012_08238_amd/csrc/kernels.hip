// gfx950 kernels of the flat-window voting sparse FFT.
//
// Stage map (one launch per stage; a batch launches each stage once over all
// of its signals):
//   fold_strip / fold_gather  bucketization: window the permuted signal and
//                             alias it into B buckets (Eq.(6)-(7), (11)-(13))
//   fft_select<log2B>         B-point DFT of each loop's buckets in LDS and the
//                             d*K largest buckets (location by voting)
//   vote                      frequencies hashed by >= T selected buckets
//   finalize<LMAX>            energy-concentration estimates, median over
//                             loops, K largest, ascending order
//   residual                  FP64 residual on S samples (formula method, Eq.(2))
//
// Index arithmetic is exact: every product sigma*i, tau*f, t*f is a wrapping
// 32-bit multiply masked by N-1, exact because N divides 2^32.
//
// Memory access: descriptors are read through the constant address space
// (scalar loads); data through explicit global-address-space loads and stores,
// streamed signal reads carry the non-temporal hint.

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

__device__ __forceinline__ void resolve(const Launch& a, uint32_t& sig, uint32_t& unit) {
    const uint32_t blk = a.xcd_order ? xcd_unit(blockIdx.x, gridDim.x) : blockIdx.x;
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

// ---------------------------------------------------------------- bucketization
// Strip form. View x as an (N/B) x B row-major matrix: time sample a = row*B + col.
// For loop r the window index of sample a is i = sigma^{-1}(a - tau) mod N and its
// bucket is i mod B, which depends on col only (B | N). Each workgroup streams a
// full-height strip of C columns into LDS (all PER 16-byte loads of a thread in
// flight at once) and then, for every (loop, column), sums the taps i = b + m*B
// that land in the column: they sit at rows (q + sigma*m) mod (N/B) of it.
template <int PER>
__global__ __launch_bounds__(kFoldNT) void fold_strip_kernel(Launch a) {
    extern __shared__ f4v lds4[];
    uint32_t sig, unit;
    resolve(a, sig, unit);
    const auto& d = desc_of(a, sig);
    const float2* x = io_of(a, sig).x;
    if (unit == 0 && threadIdx.x == 0) {
        gst(d.ctr + 0, 0u);
        gst(d.ctr + 1, 0u);
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
    const uint32_t* sigma = d.sigma;
    const uint32_t* sigma_inv = d.sigma_inv;
    const uint32_t* tau = d.tau;
    const f4v* gT = reinterpret_cast<const f4v*>(d.gT);
    float2* uhat = d.uhat;
    for (uint32_t it = threadIdx.x; it < items; it += kFoldNT) {
        const uint32_t r = it >> log2C, c = it & (C - 1u);
        const uint32_t s = gld(sigma + r), si = gld(sigma_inv + r), tu = gld(tau + r);
        const uint32_t b = (si * (col0 + c - tu)) & (B - 1u);
        const uint32_t q = ((s * b + tu) & maskN) >> log2B;
        const f4v* gp = gT + (size_t)b * (Mw4 >> 2);
        float2 acc = make_float2(0.f, 0.f);
        for (uint32_t m4 = 0; m4 < Mw4; m4 += 4) {
            const f4v g = gld(gp + (m4 >> 2));
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

// Strip form for the common shapes: each thread owns at most IPT (loop, column)
// items of G4*4 window taps. All tile loads are issued first (branch-free:
// out-of-tile slots reload the last element); while they are in flight the
// thread computes its items' buckets and fetches their window taps. The tile
// then passes through LDS in H row bands (LDS = tile/H, so more workgroups fit
// per CU); each band delivers the taps whose rows it holds, and the taps are
// summed in tap order at the end: same taps, same order as the other forms.
template <int PER, int IPT, int G4, int H>
__global__ __launch_bounds__(kFoldNT) void fold_strip_pf_kernel(Launch a) {
    extern __shared__ f4v lds4[];
    uint32_t sig, unit;
    resolve(a, sig, unit);
    const auto& d = desc_of(a, sig);
    const float2* x = io_of(a, sig).x;
    if (unit == 0 && threadIdx.x == 0) {
        gst(d.ctr + 0, 0u);
        gst(d.ctr + 1, 0u);
    }
    const uint32_t log2C = d.log2C, C = 1u << log2C, R = d.M, B = d.B, log2B = d.log2B;
    const uint32_t col0 = unit << log2C;
    const uint32_t log2h = log2C - 1;
    const uint32_t total = R << log2h;
    const f4v* xs = reinterpret_cast<const f4v*>(x);
    f4v v[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const uint32_t k = min(threadIdx.x + j * kFoldNT, total - 1u);
        const uint32_t row = k >> log2h, c = k & ((1u << log2h) - 1u);
        v[j] = gld_nt(xs + ((((size_t)row << log2B) + col0) >> 1) + c);
    }
    const uint32_t items = d.L << log2C;
    const uint32_t Mw = d.Mw, w = d.w, maskN = d.maskN;
    const f4v* gT = reinterpret_cast<const f4v*>(d.gT);
    uint32_t ri[IPT], ci[IPT], si_[IPT], bi[IPT], qi[IPT], sv[IPT], tv[IPT];
    f4v gi[IPT][G4];
#pragma unroll
    for (int e = 0; e < IPT; ++e) {
        const uint32_t it = threadIdx.x + e * kFoldNT;
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
        const uint32_t it = threadIdx.x + e * kFoldNT;
        if (it < items) {
            const uint32_t b = (sv[e] * (col0 + ci[e] - tv[e])) & (B - 1u);
            bi[e] = b;
            qi[e] = ((si_[e] * b + tv[e]) & maskN) >> log2B;
#pragma unroll
            for (int k = 0; k < G4; ++k) gi[e][k] = gld(gT + (size_t)b * G4 + k);
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
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const uint32_t k = threadIdx.x + j * kFoldNT;
            if (k < total && (k >> log2band) == (uint32_t)h) lds4[k - ((uint32_t)h << log2band)] = v[j];
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < IPT; ++e) {
            const uint32_t it = threadIdx.x + e * kFoldNT;
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
        const uint32_t it = threadIdx.x + e * kFoldNT;
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
    uint32_t sig, unit;
    resolve(a, sig, unit);
    const auto& d = desc_of(a, sig);
    const float2* x = io_of(a, sig).x;
    if (unit == 0 && threadIdx.x == 0) {
        gst(d.ctr + 0, 0u);
        gst(d.ctr + 1, 0u);
    }
    const uint32_t log2B = d.log2B, B = d.B;
    const uint32_t it = unit * kFoldNT + threadIdx.x;
    if (it >= (d.L << log2B)) return;
    // thread (loop r, column col) computes the bucket b whose samples all sit in
    // that column, so that the result is stored in column order like the strip form
    const uint32_t r = it >> log2B, col = it & (B - 1u);
    const uint32_t s = gld(d.sigma + r), tu = gld(d.tau + r);
    const uint32_t b = (gld(d.sigma_inv + r) * (col - tu)) & (B - 1u);
    const uint32_t Mw = d.Mw, Mw4 = d.Mw4, w = d.w, maskN = d.maskN;
    const f4v* gp = reinterpret_cast<const f4v*>(d.gT) + (size_t)b * (Mw4 >> 2);
    float2 acc = make_float2(0.f, 0.f);
    for (uint32_t m4 = 0; m4 < Mw4; m4 += 4) {
        const f4v g = gld(gp + (m4 >> 2));
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
    gst(d.uhat + it, acc);   // = uhat[r * B + col]
}

// ---------------------------------------------------------------- B-point FFT
// In-register DFTs of size 2, 4, 8, 16 (forward, e^{-2 pi i jk/R}), natural
// order in and out, by radix-2 decimation in time.
__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }  // a * (-i)

template <int R>
struct SmallDft;

template <>
struct SmallDft<2> {
    __device__ __forceinline__ static void run(float2* v) {
        const float2 a = v[0], b = v[1];
        v[0] = make_float2(a.x + b.x, a.y + b.y);
        v[1] = make_float2(a.x - b.x, a.y - b.y);
    }
};

template <>
struct SmallDft<4> {
    __device__ __forceinline__ static void run(float2* v) {
        const float2 a0 = make_float2(v[0].x + v[2].x, v[0].y + v[2].y);
        const float2 a1 = make_float2(v[0].x - v[2].x, v[0].y - v[2].y);
        const float2 a2 = make_float2(v[1].x + v[3].x, v[1].y + v[3].y);
        const float2 a3 = mul_mi(make_float2(v[1].x - v[3].x, v[1].y - v[3].y));
        v[0] = make_float2(a0.x + a2.x, a0.y + a2.y);
        v[2] = make_float2(a0.x - a2.x, a0.y - a2.y);
        v[1] = make_float2(a1.x + a3.x, a1.y + a3.y);
        v[3] = make_float2(a1.x - a3.x, a1.y - a3.y);
    }
};

// cos / sin of 2 pi k / 16 for k = 0..7
__device__ constexpr float kC16[8] = {1.0f, 0.92387953251128676f, 0.70710678118654752f, 0.38268343236508977f,
                                      0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128676f};
__device__ constexpr float kS16[8] = {0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128676f,
                                      1.0f, 0.92387953251128676f, 0.70710678118654752f, 0.38268343236508977f};

template <int R>
struct SmallDft {
    // split into even / odd halves, combine with W_R^k = e^{-2 pi i k / R}
    __device__ __forceinline__ static void run(float2* v) {
        float2 e[R / 2], o[R / 2];
#pragma unroll
        for (int k = 0; k < R / 2; ++k) {
            e[k] = v[2 * k];
            o[k] = v[2 * k + 1];
        }
        SmallDft<R / 2>::run(e);
        SmallDft<R / 2>::run(o);
#pragma unroll
        for (int k = 0; k < R / 2; ++k) {
            const int t = k * (16 / R);
            const float2 w = make_float2(kC16[t], -kS16[t]);
            const float2 ow = (k == 0) ? o[k] : cmul(o[k], w);
            v[k] = make_float2(e[k].x + ow.x, e[k].y + ow.y);
            v[k + R / 2] = make_float2(e[k].x - ow.x, e[k].y - ow.y);
        }
    }
};

template <int LOG2B>
struct FftCfg {
    static constexpr int B = 1 << LOG2B;
    static constexpr int NT = B / 16 < 64 ? 64 : (B / 16 > 1024 ? 1024 : B / 16);
    static constexpr int LOG2TL = (LOG2B + 1) / 2;   // twiddle table split: m = hi * TL + lo
    static constexpr int TL = 1 << LOG2TL;
    static constexpr int TH = B >> LOG2TL;
    static constexpr int PADN = B + (B >> 4) + 1;    // one pad element per 16 (bank spread)
    static constexpr int CH = B >= NT ? B / NT : 1;  // energies held per thread
    static constexpr int NW = B >= 32 ? B / 32 : 1;  // bitmap words
    // candidate capacity of the prefiltered selection: (energy, bucket) pairs
    // placed in the data region after the bitmap words, a multiple of NT
    static constexpr int SELCAP_RAW = (PADN * 2 - NW - 64) / 2;
    static constexpr int SELCAP = (SELCAP_RAW > 4096 ? 4096 : SELCAP_RAW) / NT * NT;
    static constexpr size_t lds_bytes() {
        return (size_t)(PADN + TL + TH) * sizeof(float2) + (256 + 16 + 4) * sizeof(uint32_t);
    }
};

__device__ __forceinline__ int padi(int i) { return i + (i >> 4); }

// One Stockham autosort pass of radix R over the B values in LDS; Ns is the
// product of the radices of the passes before. Butterfly j reads
// lds[j + r*B/R], is twisted by W_{Ns R}^{r (j mod Ns)}, transformed, and
// written to lds[(j - j mod Ns) R + j mod Ns + r Ns]. Twiddles W_B^m come from
// two LDS tables: W_B^m = hi[m / TL] * lo[m mod TL].
template <int LOG2B, int LOG2R, int LOG2NS>
__device__ __forceinline__ void stockham_pass(float2* lds, const float2* tlo, const float2* thi) {
    using Cfg = FftCfg<LOG2B>;
    constexpr int B = Cfg::B, NT = Cfg::NT, R = 1 << LOG2R, Ns = 1 << LOG2NS;
    constexpr int NBF = B / R;
    constexpr int NPER = NBF >= NT ? NBF / NT : 1;
    constexpr int TSHIFT = LOG2B - LOG2NS - LOG2R;
    float2 v[NPER][R];
#pragma unroll
    for (int q = 0; q < NPER; ++q) {
        const int j = (int)threadIdx.x + q * NT;
        if (j < NBF) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = lds[padi(j + r * NBF)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NPER; ++q) {
        const int j = (int)threadIdx.x + q * NT;
        if (j < NBF) {
            const int k = j & (Ns - 1);
            if (Ns > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    const int m = (r * k) << TSHIFT;
                    const float2 w = cmul(thi[m >> Cfg::LOG2TL], tlo[m & (Cfg::TL - 1)]);
                    v[q][r] = cmul(v[q][r], w);
                }
            }
            SmallDft<R>::run(v[q]);
            const int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) lds[padi(base + r * Ns)] = v[q][r];
        }
    }
    __syncthreads();
}

template <int LOG2B, int LOG2NS>
__device__ __forceinline__ void fft_passes(float2* lds, const float2* tlo, const float2* thi) {
    constexpr int REM = LOG2B - LOG2NS;
    if constexpr (REM >= 4) {
        stockham_pass<LOG2B, 4, LOG2NS>(lds, tlo, thi);
        fft_passes<LOG2B, LOG2NS + 4>(lds, tlo, thi);
    } else if constexpr (REM > 0) {
        stockham_pass<LOG2B, REM, LOG2NS>(lds, tlo, thi);
    }
}

// k-th largest (1-based; k <= number of valid keys) of the keys held by the
// block, KPT per thread: radix select on 8-bit digits from the top through an
// LDS histogram. The first digit (shared by most keys) is counted with one
// atomic per distinct digit per wave. Returns the value and how many keys equal
// to it are among the k largest.
template <int NT, int KPT>
__device__ __forceinline__ void block_kth_largest(const uint32_t* key, const bool* kv, uint32_t k, uint32_t* hist,
                                                  uint32_t* bcast, uint32_t& theta, uint32_t& rank) {
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t prefix = 0, pmask = 0, kk = k;
#pragma unroll
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 24 - 8 * pass;
        for (int i = threadIdx.x; i < 256; i += NT) hist[i] = 0;
        __syncthreads();
#pragma unroll
        for (int c = 0; c < KPT; ++c) {
            const bool act = kv[c] && ((key[c] & pmask) == prefix);
            const uint32_t dg = (key[c] >> shift) & 255u;
            if (pass == 0) {
                uint64_t pend = __ballot(act);
                while (pend) {
                    const int leader = __ffsll((unsigned long long)pend) - 1;
                    const uint32_t dl = __shfl(dg, leader, 64);
                    const uint64_t same = __ballot(act && dg == dl) & pend;
                    if ((int)lane == leader) atomicAdd(&hist[dl], (uint32_t)__popcll(same));
                    pend &= ~same;
                }
            } else if (act) {
                atomicAdd(&hist[dg], 1u);
            }
        }
        __syncthreads();
        if (threadIdx.x < 64) {
            const int top = 255 - 4 * (int)lane;   // lane 0 owns the largest digits
            const uint32_t h0 = hist[top], h1 = hist[top - 1], h2 = hist[top - 2], h3 = hist[top - 3];
            const uint32_t s = h0 + h1 + h2 + h3;
            const uint32_t incl = wave_incl_scan(s);
            const uint32_t excl = incl - s;
            if (excl < kk && kk <= incl) {
                uint32_t acc = excl, dsel, rem;
                if (acc + h0 >= kk) {
                    dsel = top;
                    rem = kk - acc;
                } else if (acc += h0, acc + h1 >= kk) {
                    dsel = top - 1;
                    rem = kk - acc;
                } else if (acc += h1, acc + h2 >= kk) {
                    dsel = top - 2;
                    rem = kk - acc;
                } else {
                    acc += h2;
                    dsel = top - 3;
                    rem = kk - acc;
                }
                bcast[0] = dsel;
                bcast[1] = rem;
            }
        }
        __syncthreads();
        prefix |= bcast[0] << shift;
        pmask |= 255u << shift;
        kk = bcast[1];
        __syncthreads();
    }
    theta = prefix;
    rank = kk;
}

// Mask of this thread's keys (KPT per thread, block order = thread-major) among
// the k largest: every key above theta and the first `rank` keys equal to it.
template <int NT, int KPT>
__device__ __forceinline__ uint64_t select_mask(const uint32_t* key, const bool* kv, uint32_t theta, uint32_t rank,
                                                uint32_t* scan) {
    uint32_t eq = 0;
#pragma unroll
    for (int c = 0; c < KPT; ++c) eq += (kv[c] && key[c] == theta) ? 1u : 0u;
    uint32_t tot;
    uint32_t eqrank = block_excl_scan<NT>(eq, scan, tot);
    uint64_t selm = 0;
#pragma unroll
    for (int c = 0; c < KPT; ++c) {
        bool sel = false;
        if (kv[c]) {
            if (key[c] > theta) {
                sel = true;
            } else if (key[c] == theta) {
                sel = eqrank < rank;
                ++eqrank;
            }
        }
        if (sel) selm |= 1ull << c;
    }
    return selm;
}

// Write the selected buckets: the bitmap (built in LDS) and the ascending list.
template <int NT, int KPT, typename IdxF>
__device__ __forceinline__ void emit_selection(uint64_t selm, IdxF idx_of, uint32_t* bits, int nw, uint32_t* scan,
                                               uint32_t* jl, uint32_t* jb, uint32_t dK) {
    for (int i = threadIdx.x; i < nw; i += NT) bits[i] = 0;
    __syncthreads();
    uint32_t tot;
    uint32_t pos = block_excl_scan<NT>((uint32_t)__popcll(selm), scan, tot);
#pragma unroll
    for (int c = 0; c < KPT; ++c) {
        if ((selm >> c) & 1ull) {
            const uint32_t h = idx_of(c);
            atomicOr(&bits[h >> 5], 1u << (h & 31));
            if (pos < dK) gst(jl + pos, h);
            ++pos;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nw; i += NT) gst(jb + i, bits[i]);
}

// Selection of the dK largest |uhat|^2 (ties -> lower bucket): radix select on
// the IEEE bit patterns of the non-negative energies (monotone as unsigned),
// four 8-bit digits from the top. Digit counts go to an LDS histogram; the
// first digit (sign + high exponent bits, shared by most buckets) is counted
// with one atomic per distinct digit per wave.
template <int LOG2B>
__global__ __launch_bounds__(FftCfg<LOG2B>::NT) void fft_select_kernel(Launch a) {
    using Cfg = FftCfg<LOG2B>;
    constexpr int B = Cfg::B, NT = Cfg::NT, CH = Cfg::CH, NW = Cfg::NW;
    extern __shared__ f4v lds_raw[];
    float2* data = reinterpret_cast<float2*>(lds_raw);
    float2* tlo = data + Cfg::PADN;
    float2* thi = tlo + Cfg::TL;
    uint32_t* hist = reinterpret_cast<uint32_t*>(thi + Cfg::TH);
    uint32_t* scan = hist + 256;   // NT/64 <= 16 words
    uint32_t* bcast = scan + 16;   // [0] digit, [1] remaining rank
    uint32_t* bits = reinterpret_cast<uint32_t*>(data);  // reuses the data region at the end

    uint32_t sig, r;
    resolve(a, sig, r);
    const auto& d = desc_of(a, sig);
    float2* u = d.uhat + (size_t)r * B;
    const float2* tw = d.tw;
    {
        // the bucketization stored loop r's values in column order: column col
        // holds bucket b = sigma_r^{-1} (col - tau_r) mod B; place them by bucket
        const uint32_t sinv = d.sigma_inv[r], tu = d.tau[r];
        constexpr int LPT = (B + NT - 1) / NT;
        float2 tmp[LPT];
#pragma unroll
        for (int q = 0; q < LPT; ++q) {
            const int col = min((int)threadIdx.x + q * NT, B - 1);
            tmp[q] = gld(u + col);
        }
#pragma unroll
        for (int q = 0; q < LPT; ++q) {
            const uint32_t col = threadIdx.x + q * NT;
            if (col < (uint32_t)B) data[padi((int)((sinv * (col - tu)) & (uint32_t)(B - 1)))] = tmp[q];
        }
    }
    for (int j = threadIdx.x; j < Cfg::TL; j += NT) tlo[j] = gld(tw + j);
    for (int j = threadIdx.x; j < Cfg::TH; j += NT) thi[j] = gld(tw + (j << Cfg::LOG2TL));
    __syncthreads();
    fft_passes<LOG2B, 0>(data, tlo, thi);
    for (int h = threadIdx.x; h < B; h += NT) gst(u + h, data[padi(h)]);

    const bool valid = (int)threadIdx.x * CH < B;
    uint32_t key[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        key[c] = 0;
        if (valid) {
            const float2 v = data[padi(threadIdx.x * CH + c)];
            key[c] = energy_key(v);
        }
    }
    const uint32_t dK = d.dK;
    uint32_t* jl = d.jlist + (size_t)r * dK;
    uint32_t* jb = d.jbits + (size_t)r * NW;
    bool kv[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) kv[c] = valid;
    bool done = false;
    if constexpr (CH >= 4 && Cfg::SELCAP >= NT) {
        if (dK <= (uint32_t)NT) {
            // Every one of the dK largest energies is >= theta0, the dK-th largest of
            // the per-thread maxima (at least dK threads hold a value >= theta0), so
            // only the keys >= theta0 can be selected. Collect them (in bucket
            // order) and select exactly among those when they are few.
            uint32_t tmax[1] = {0};
            const bool tv[1] = {valid};
#pragma unroll
            for (int c = 0; c < CH; ++c) tmax[0] = max(tmax[0], key[c]);
            uint32_t theta0, rank0;
            block_kth_largest<NT, 1>(tmax, tv, dK, hist, bcast, theta0, rank0);
            uint32_t cnt = 0;
#pragma unroll
            for (int c = 0; c < CH; ++c) cnt += (valid && key[c] >= theta0) ? 1u : 0u;
            uint32_t total;
            uint32_t base = block_excl_scan<NT>(cnt, scan, total);
            if (total <= (uint32_t)Cfg::SELCAP) {   // block-uniform
                uint32_t* ckey = bits + Cfg::NW + 64;
                uint32_t* cidx = ckey + Cfg::SELCAP;
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    if (valid && key[c] >= theta0) {
                        ckey[base] = key[c];
                        cidx[base] = threadIdx.x * CH + c;
                        ++base;
                    }
                }
                __syncthreads();
                constexpr int CPT = Cfg::SELCAP / NT;
                uint32_t ck[CPT];
                bool cv[CPT];
#pragma unroll
                for (int q = 0; q < CPT; ++q) {
                    const uint32_t i = threadIdx.x * CPT + q;
                    cv[q] = i < total;
                    ck[q] = cv[q] ? ckey[i] : 0u;
                }
                uint32_t theta, rank;
                block_kth_largest<NT, CPT>(ck, cv, dK, hist, bcast, theta, rank);
                const uint64_t selm = select_mask<NT, CPT>(ck, cv, theta, rank, scan);
                emit_selection<NT, CPT>(selm, [&](int q) { return cidx[threadIdx.x * CPT + q]; }, bits, NW, scan,
                                        jl, jb, dK);
                done = true;
            }
        }
    }
    if (!done) {   // block-uniform
        uint32_t theta, rank;
        block_kth_largest<NT, CH>(key, kv, dK, hist, bcast, theta, rank);
        const uint64_t selm = select_mask<NT, CH>(key, kv, theta, rank, scan);
        emit_selection<NT, CH>(selm, [&](int c) { return (uint32_t)(threadIdx.x * CH + c); }, bits, NW, scan, jl, jb,
                               dK);
    }
}


// ---------------------------------------------------------------- two-pass FFT (B > 16384)
// The bucketization leaves the bucket values in column order, v[col] = u[b] with
// col = sigma b + tau mod B. Instead of moving them into bucket order first, the
// DFT V of v is taken as it stands: with s = sigma^{-1} mod B,
//   X[h] = sum_b u[b] e^{-2 pi i bh/B} = e^{+2 pi i (s tau h mod B)/B} V[s h mod B],
// so bucket h's DFT value is V at m = s h mod B times a unit phase, and the
// energies |X[h]|^2 are those of V at m (h = sigma m mod B). V is computed in four
// steps over the B1 x B2 row-major view (col = B2 j1 + j2, B = B1 B2): DFTs of
// length B1 down the columns, the twist W_B^{j2 k1}, DFTs of length B2 along the
// rows, V[k1 + B1 k2] = sum_j2 W_B2^{j2 k2} W_B^{j2 k1} sum_j1 W_B1^{j1 k1} v[B2 j1 + j2].
// Each workgroup transforms 16 sequences, so every global access moves 16
// consecutive values. The second pass also records the largest energy of every
// 16 consecutive V entries, which lets the selection visit few of them.
template <int LB>
struct LargeCfg {
    static constexpr int B = 1 << LB;
    static constexpr int LB1 = (LB + 1) / 2, LB2 = LB / 2;
    static constexpr int B1 = 1 << LB1, B2 = 1 << LB2;
    static constexpr int NT = 256;       // FFT pass workgroups: 16 sequences each
    static constexpr int G = B / 16;     // groups of 16 consecutive V entries
    static constexpr int SNT = 1024;     // selection workgroup
    static constexpr int NW = B / 32;    // bitmap words
    static constexpr int SELCAP = 8192;  // candidates of the prefiltered selection held in LDS
};

// NSEQ DFTs of length 2^LP at once in LDS (sequence q at q*SP, element j at
// padi(j)): Stockham autosort passes as stockham_pass, twiddles tp[m] = W_P^m.
template <int LP, int NSEQ, int NT>
struct SeqFft {
    static constexpr int P = 1 << LP;
    static constexpr int SP = P + (P >> 4) + 1;
    static constexpr size_t lds_bytes() { return (size_t)(NSEQ * SP + P) * sizeof(float2); }

    template <int LOG2R, int LOG2NS>
    __device__ __forceinline__ static void pass(float2* lds, const float2* tp) {
        constexpr int R = 1 << LOG2R, Ns = 1 << LOG2NS, NBF = P / R, TOT = NSEQ * NBF;
        constexpr int NPER = (TOT + NT - 1) / NT;
        constexpr int TSHIFT = LP - LOG2NS - LOG2R;
        float2 v[NPER][R];
#pragma unroll
        for (int q = 0; q < NPER; ++q) {
            const int idx = (int)threadIdx.x + q * NT;
            if (idx < TOT) {
                const float2* base = lds + (idx / NBF) * SP;
                const int j = idx % NBF;
#pragma unroll
                for (int r = 0; r < R; ++r) v[q][r] = base[padi(j + r * NBF)];
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NPER; ++q) {
            const int idx = (int)threadIdx.x + q * NT;
            if (idx < TOT) {
                const int j = idx % NBF, k = j & (Ns - 1);
                if (Ns > 1) {
#pragma unroll
                    for (int r = 1; r < R; ++r) v[q][r] = cmul(v[q][r], tp[(r * k) << TSHIFT]);
                }
                SmallDft<R>::run(v[q]);
                float2* base = lds + (idx / NBF) * SP;
                const int o = (j - k) * R + k;
#pragma unroll
                for (int r = 0; r < R; ++r) base[padi(o + r * Ns)] = v[q][r];
            }
        }
        __syncthreads();
    }

    template <int LOG2NS = 0>
    __device__ __forceinline__ static void run(float2* lds, const float2* tp) {
        constexpr int REM = LP - LOG2NS;
        if constexpr (REM >= 4) {
            pass<4, LOG2NS>(lds, tp);
            run<LOG2NS + 4>(lds, tp);
        } else if constexpr (REM > 0) {
            pass<REM, LOG2NS>(lds, tp);
        }
    }
};

// First pass: 16 columns j2 of the B1 x B2 view per workgroup -> ubuf, row-major
// [k1][j2], twisted. Units per signal: L * B2/16.
template <int LB>
__global__ __launch_bounds__(256) void fft_large_p1_kernel(Launch a) {
    using C = LargeCfg<LB>;
    using F = SeqFft<C::LB1, 16, C::NT>;
    extern __shared__ f4v lds_raw[];
    float2* data = reinterpret_cast<float2*>(lds_raw);
    float2* tp = data + 16 * F::SP;
    uint32_t sig, unit;
    resolve(a, sig, unit);
    const auto& d = desc_of(a, sig);
    constexpr uint32_t tiles = C::B2 / 16;
    const uint32_t r = unit / tiles, j20 = (unit % tiles) * 16u;
    const float2* v = d.uhat + (size_t)r * C::B;
    float2* y = d.ubuf + (size_t)r * C::B;
    const float2* tw = d.tw;
    constexpr int NE = 16 * C::B1 / C::NT;   // values per thread
    constexpr int CHK = 8;
    static_assert(NE % CHK == 0, "load chunks");
#pragma unroll
    for (int q0 = 0; q0 < NE; q0 += CHK) {
        float2 t[CHK];
#pragma unroll
        for (int u = 0; u < CHK; ++u) {
            const int e = (int)threadIdx.x + (q0 + u) * C::NT;
            t[u] = gld(v + (size_t)(e >> 4) * C::B2 + j20 + (e & 15));
        }
#pragma unroll
        for (int u = 0; u < CHK; ++u) {
            const int e = (int)threadIdx.x + (q0 + u) * C::NT;
            data[(e & 15) * F::SP + padi(e >> 4)] = t[u];
        }
    }
    for (int m = threadIdx.x; m < C::B1; m += C::NT) tp[m] = gld(tw + ((size_t)m << (LB - C::LB1)));
    __syncthreads();
    F::run(data, tp);
#pragma unroll 4
    for (int q = 0; q < NE; ++q) {
        const int e = (int)threadIdx.x + q * C::NT;
        const uint32_t k1 = (uint32_t)e >> 4, j2 = j20 + (uint32_t)(e & 15);
        const float2 t = gld(tw + ((j2 * k1) & (uint32_t)(C::B - 1)));   // W_B^{j2 k1}
        gst(y + (size_t)k1 * C::B2 + j2, cmul(data[(e & 15) * F::SP + padi((int)k1)], t));
    }
}

// Second pass: 16 rows k1 per workgroup -> V[k1 + B1 k2] into uhat, and the
// largest energy of each 16 consecutive V entries into gmax. Units: L * B1/16.
template <int LB>
__global__ __launch_bounds__(256) void fft_large_p2_kernel(Launch a) {
    using C = LargeCfg<LB>;
    using F = SeqFft<C::LB2, 16, C::NT>;
    extern __shared__ f4v lds_raw[];
    float2* data = reinterpret_cast<float2*>(lds_raw);
    float2* tp = data + 16 * F::SP;
    uint32_t sig, unit;
    resolve(a, sig, unit);
    const auto& d = desc_of(a, sig);
    constexpr uint32_t tiles = C::B1 / 16;
    const uint32_t r = unit / tiles, k10 = (unit % tiles) * 16u;
    const float2* y = d.ubuf + (size_t)r * C::B;
    float2* V = d.uhat + (size_t)r * C::B;
    uint32_t* gm = d.gmax + (size_t)r * C::G;
    constexpr int NE = 16 * C::B2 / C::NT;
    constexpr int CHK = 8;
    static_assert(NE % CHK == 0, "load chunks");
#pragma unroll
    for (int q0 = 0; q0 < NE; q0 += CHK) {
        float2 t[CHK];
#pragma unroll
        for (int u = 0; u < CHK; ++u) {
            const int e = (int)threadIdx.x + (q0 + u) * C::NT;
            t[u] = gld(y + (size_t)(k10 + (uint32_t)(e >> C::LB2)) * C::B2 + (e & (C::B2 - 1)));
        }
#pragma unroll
        for (int u = 0; u < CHK; ++u) {
            const int e = (int)threadIdx.x + (q0 + u) * C::NT;
            data[(e >> C::LB2) * F::SP + padi(e & (C::B2 - 1))] = t[u];
        }
    }
    for (int m = threadIdx.x; m < C::B2; m += C::NT) tp[m] = gld(d.tw + ((size_t)m << (LB - C::LB2)));
    __syncthreads();
    F::run(data, tp);
#pragma unroll 4
    for (int q = 0; q < NE; ++q) {
        const int e = (int)threadIdx.x + q * C::NT;
        const int c = e & 15, k2 = e >> 4;
        const float2 val = data[c * F::SP + padi(k2)];
        const uint32_t m0 = k10 + (uint32_t)C::B1 * (uint32_t)k2;   // multiple of 16
        gst(V + m0 + c, val);
        uint32_t mx = energy_key(val);
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, off, 64));
        if (c == 0) gst(gm + (m0 >> 4), mx);
    }
}

// k-th largest (1-based, k <= number of valid keys) of n keys produced by
// keyf(i, key) -> valid, streamed 4 times (8-bit digits from the top, LDS
// histogram). Returns the value and how many keys equal to it are among the k largest.
template <int NT, class KeyF>
__device__ __forceinline__ void stream_kth_largest(uint32_t n, uint32_t k, KeyF keyf, uint32_t* hist, uint32_t* bc,
                                                   uint32_t& theta, uint32_t& rank) {
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t prefix = 0, pmask = 0, kk = k;
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 24 - 8 * pass;
        for (uint32_t i = threadIdx.x; i < 256; i += NT) hist[i] = 0;
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < n; i += NT) {
            uint32_t key;
            if (keyf(i, key) && (key & pmask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (threadIdx.x < 64) {
            const int hi = 255 - 4 * (int)lane;   // lane 0 owns the largest digits
            const uint32_t h0 = hist[hi], h1 = hist[hi - 1], h2 = hist[hi - 2], h3 = hist[hi - 3];
            const uint32_t sum = h0 + h1 + h2 + h3;
            const uint32_t incl = wave_incl_scan(sum);
            const uint32_t excl = incl - sum;
            if (excl < kk && kk <= incl) {
                uint32_t acc = excl, dsel, rem;
                if (acc + h0 >= kk) {
                    dsel = hi;
                    rem = kk - acc;
                } else if (acc += h0, acc + h1 >= kk) {
                    dsel = hi - 1;
                    rem = kk - acc;
                } else if (acc += h1, acc + h2 >= kk) {
                    dsel = hi - 2;
                    rem = kk - acc;
                } else {
                    acc += h2;
                    dsel = hi - 3;
                    rem = kk - acc;
                }
                bc[0] = dsel;
                bc[1] = rem;
            }
        }
        __syncthreads();
        prefix |= bc[0] << shift;
        pmask |= 255u << shift;
        kk = bc[1];
        __syncthreads();
    }
    theta = prefix;
    rank = kk;
}

// Selection of the dK largest bucket energies (ties -> lower bucket) from V in m
// order; bucket h = sigma m mod B. Fast path: theta0 = the dK-th largest group
// maximum bounds the dK-th largest energy from below (at least dK groups hold an
// energy >= theta0), so only entries >= theta0 of groups whose maximum reaches
// theta0 are collected and selected exactly in LDS. When the bound admits too
// many entries (flat spectra) every entry is streamed instead. One workgroup per
// (signal, loop). Dynamic LDS: bitmap words + SELCAP (energy, bucket) pairs.
template <int LB>
__global__ __launch_bounds__(1024) void select_large_kernel(Launch a) {
    using C = LargeCfg<LB>;
    constexpr int NT = C::SNT, G = C::G, NW = C::NW, CAP = C::SELCAP;
    constexpr uint32_t Bm = (uint32_t)C::B - 1u;
    extern __shared__ uint32_t lds_words[];
    uint32_t* bits = lds_words;
    uint32_t* ckey = bits + NW;
    uint32_t* cidx = ckey + CAP;
    __shared__ uint32_t hist[256];
    __shared__ uint32_t bc[4];
    __shared__ uint32_t scan[NT / 64];
    __shared__ uint32_t s_cnt, s_eq;
    uint32_t sig, unit;
    resolve(a, sig, unit);
    const auto& d = desc_of(a, sig);
    const uint32_t r = unit, dK = d.dK;
    const uint32_t sg = ((CU32)d.sigma)[r];
    const float2* V = d.uhat + (size_t)r * C::B;
    const uint32_t* gm = d.gmax + (size_t)r * G;
    for (uint32_t i = threadIdx.x; i < (uint32_t)NW; i += NT) bits[i] = 0;
    if (threadIdx.x == 0) {
        s_cnt = 0;
        s_eq = 0;
    }
    __syncthreads();
    bool fast = dK <= (uint32_t)G;   // block-uniform
    uint32_t n = 0;
    if (fast) {
        uint32_t theta0, rank0;
        stream_kth_largest<NT>((uint32_t)G, dK, [&](uint32_t i, uint32_t& k) { k = gld(gm + i); return true; }, hist,
                               bc, theta0, rank0);
        for (uint32_t g = threadIdx.x; g < (uint32_t)G; g += NT) {
            if (gld(gm + g) < theta0) continue;
            const f4v* p = reinterpret_cast<const f4v*>(V + (size_t)g * 16u);
            f4v t[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) t[c] = gld(p + c);
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const f4v& q = t[c >> 1];
                const float2 val = (c & 1) ? make_float2(q[2], q[3]) : make_float2(q[0], q[1]);
                const uint32_t k = energy_key(val);
                if (k >= theta0) {
                    const uint32_t pos = atomicAdd(&s_cnt, 1u);
                    if (pos < (uint32_t)CAP) {
                        ckey[pos] = k;
                        cidx[pos] = (sg * (g * 16u + (uint32_t)c)) & Bm;
                    }
                }
            }
        }
        __syncthreads();
        n = s_cnt;
        fast = n <= (uint32_t)CAP;
    }
    // energy and bucket of entry i of the working set (candidates, or all of V)
    auto entry = [&](uint32_t i, uint32_t& k, uint32_t& h) {
        if (fast) {
            k = ckey[i];
            h = cidx[i];
        } else {
            k = energy_key(gld(V + i));
            h = (sg * i) & Bm;
        }
    };
    const uint32_t total = fast ? n : (uint32_t)C::B;
    uint32_t theta, rank;
    stream_kth_largest<NT>(total, dK, [&](uint32_t i, uint32_t& k) { uint32_t h; entry(i, k, h); return true; }, hist,
                           bc, theta, rank);
    // entries equal to theta: take the `rank` of lowest bucket
    uint32_t eq = 0;
    for (uint32_t i = threadIdx.x; i < total; i += NT) {
        uint32_t k, h;
        entry(i, k, h);
        eq += k == theta;
    }
    if (eq) atomicAdd(&s_eq, eq);
    __syncthreads();
    uint32_t hcut = (uint32_t)C::B;   // ties with bucket < hcut are selected
    if (s_eq > rank) {
        uint32_t th, rk;
        stream_kth_largest<NT>(total, rank, [&](uint32_t i, uint32_t& k) {
            uint32_t e, h;
            entry(i, e, h);
            k = Bm - h;
            return e == theta;
        }, hist, bc, th, rk);
        hcut = (uint32_t)C::B - th;
    }
    for (uint32_t i = threadIdx.x; i < total; i += NT) {
        uint32_t k, h;
        entry(i, k, h);
        if (k > theta || (k == theta && h < hcut)) atomicOr(&bits[h >> 5], 1u << (h & 31u));
    }
    __syncthreads();
    // bitmap out; buckets in ascending order into jlist
    constexpr int WPT = NW / NT;
    static_assert(WPT >= 1 && NW % NT == 0, "bitmap words per thread");
    uint32_t* jb = d.jbits + (size_t)r * NW;
    uint32_t* jl = d.jlist + (size_t)r * dK;
    uint32_t wv[WPT], cnt = 0;
#pragma unroll
    for (int q = 0; q < WPT; ++q) {
        wv[q] = bits[threadIdx.x * WPT + q];
        cnt += (uint32_t)__popc(wv[q]);
    }
#pragma unroll
    for (int q = 0; q < WPT; ++q) gst(jb + threadIdx.x * WPT + q, wv[q]);
    uint32_t tot;
    uint32_t pos = block_excl_scan<NT>(cnt, scan, tot);
#pragma unroll
    for (int q = 0; q < WPT; ++q) {
        uint32_t w = wv[q];
        while (w) {
            const uint32_t b = (uint32_t)__ffs((int)w) - 1u;
            w &= w - 1u;
            if (pos < dK) gst(jl + pos, (threadIdx.x * WPT + q) * 32u + b);
            ++pos;
        }
    }
}

// ---------------------------------------------------------------- votes
// A frequency with >= T votes out of L is voted by one of the loops 0..L-T
// (pigeonhole), so only the frequencies of those loops' selected buckets are
// enumerated: f = sigma_r0^{-1} p for the N/B permuted positions p of each
// selected bucket. Each frequency is counted from the first loop that voted
// for it (later loops skip it), so I' has no duplicates; votes are bitmap tests.
template <int LMAX>
__global__ __launch_bounds__(kVoteNT) void vote_kernel(Launch a, uint32_t staged) {
    extern __shared__ uint32_t sbits[];
    __shared__ uint32_t s_slot[kVoteUnit / 2 + 1];   // selected buckets of this chunk (N/B >= 2)
    uint32_t sig, unit;
    resolve(a, sig, unit);
    const auto& d = desc_of(a, sig);
    const uint32_t wpl = (d.B + 31u) >> 5;
    const uint32_t L = d.L, T = d.T, M = d.M, log2M = d.log2M, maskN = d.maskN, B = d.B, dK = d.dK;
    const uint32_t* jbits = d.jbits;
    // this workgroup: candidates [start, end) of enumerated loop r0, i.e. the
    // permuted positions of selected-bucket slots slot0 .. slot0 + nslots - 1
    const uint32_t upl = d.vote_upl;
    const uint32_t r0 = unit / upl;
    const uint32_t per_loop = dK * M;
    const uint32_t start = (unit - r0 * upl) * kVoteUnit;
    const uint32_t end = min(start + kVoteUnit, per_loop);
    const uint32_t slot0 = start >> log2M;
    const uint32_t nslots = ((end - 1u) >> log2M) - slot0 + 1u;
    const uint32_t sinv0 = d.sigma_inv[r0];
    const uint32_t* jl = d.jlist + (size_t)r0 * dK + slot0;
    for (uint32_t i = threadIdx.x; i < nslots; i += kVoteNT) s_slot[i] = gld(jl + i);
    uint32_t sg[LMAX];   // sigma_r, uniform: scalar loads
#pragma unroll
    for (int r = 0; r < LMAX; ++r) sg[r] = (uint32_t)r < L ? ((CU32)d.sigma)[r] : 0u;
    const uint32_t* bits = jbits;
    if (staged) {
        // 16-byte loads, four in flight per thread (the LDS copy is sized to whole 16-byte units)
        typedef uint32_t u4v __attribute__((ext_vector_type(4)));
        const uint32_t nw4 = (L * wpl + 3u) >> 2;
        const u4v* src = reinterpret_cast<const u4v*>(jbits);
        u4v* dst = reinterpret_cast<u4v*>(sbits);
        for (uint32_t i0 = threadIdx.x; i0 < nw4; i0 += 4 * kVoteNT) {
            u4v t[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) t[e] = gld(src + min(i0 + e * kVoteNT, nw4 - 1u));
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t i = i0 + e * kVoteNT;
                if (i < nw4) dst[i] = t[e];
            }
        }
        bits = sbits;
    }
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t* ctr = d.ctr;
    uint32_t* cand = d.cand;
    const uint32_t cap = d.cap;
    for (uint32_t qq = 0; qq < kVotePerThread; ++qq) {
        const uint32_t ci = start + qq * kVoteNT + threadIdx.x;   // candidate index within loop r0
        bool emit = false;
        uint32_t f = 0;
        if (ci < end) {
            const uint32_t h = s_slot[(ci >> log2M) - slot0];
            const uint32_t p = ((h << log2M) - (M >> 1) + (ci & (M - 1u))) & maskN;
            f = (sinv0 * p) & maskN;
            // all L bitmap tests issued together (no serial chain); bit r of `votes`
            // is set when loop r selected the bucket of f (loop r0 always did)
            uint32_t votes = 0;
#pragma unroll
            for (int r = 0; r < LMAX; ++r) {
                if ((uint32_t)r < L) {
                    const uint32_t pr = (sg[r] * f) & maskN;
                    const uint32_t hr = ((pr + (M >> 1)) >> log2M) & (B - 1u);
                    votes |= ((bits[(uint32_t)r * wpl + (hr >> 5)] >> (hr & 31u)) & 1u) << r;
                }
            }
            // counted once: from the first loop that voted for f
            emit = (votes & ((1u << r0) - 1u)) == 0u && (uint32_t)__popc(votes) >= T;
        }
        const uint64_t m = __ballot(emit);
        if (m) {
            const int leader = __ffsll((unsigned long long)m) - 1;
            uint32_t base = 0;
            if ((int)lane == leader) base = atomicAdd(ctr, (uint32_t)__popcll(m));
            base = __shfl(base, leader, 64);
            if (emit) {
                const uint32_t pos = base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
                if (pos < cap) gst(cand + pos, f);
            }
        }
    }
}

// ---------------------------------------------------------------- estimation + output
template <int N>
__device__ __forceinline__ void sort_net(float* v) {
    // bitonic sorting network, ascending, fully unrolled over registers
#pragma unroll
    for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const int l = i ^ j;
                if (l > i) {
                    const bool up = (i & k) == 0;
                    const float lo = fminf(v[i], v[l]), hi = fmaxf(v[i], v[l]);
                    v[i] = up ? lo : hi;
                    v[l] = up ? hi : lo;
                }
            }
        }
    }
}

template <int LMAX>
__device__ __forceinline__ float median_of(float* v, uint32_t L) {
    sort_net<LMAX>(v);
    const uint32_t h = L >> 1;
    float a = 0.f, b = 0.f;
#pragma unroll
    for (int r = 0; r < LMAX; ++r) {
        if ((uint32_t)r == h) b = v[r];
        if ((uint32_t)r + 1u == h) a = v[r];
    }
    return (L & 1u) ? b : (a + b) * 0.5f;
}


constexpr double inv_fact(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return 1.0 / f;
}

// e^{+2 pi i m/N} in FP64 for an exact integer m in [0, N): the root of unity
// e^{2 pi i (m >> sh) / 2^tb} from the 2^tb-entry table `rou` (tb = log2 N - sh
// <= 8) times e^{i delta}, delta = (m mod 2^sh) 2 pi / N < 2 pi / 2^tb, whose cos
// and sin come from their Taylor series to delta^8 and delta^7 (truncation
// below 1e-20). `step` = 2 pi / N.
__device__ __forceinline__ double2 phase_of(const double2* rou, uint32_t m, uint32_t sh, double step) {
    const double2 T = rou[m >> sh];
    const double delta = (double)(m & ((1u << sh) - 1u)) * step;
    const double z = -delta * delta;
    const double s = fma(fma(fma(inv_fact(7), z, inv_fact(5)), z, inv_fact(3)), z, 1.0) * delta;
    const double c = fma(fma(fma(fma(inv_fact(8), z, inv_fact(6)), z, inv_fact(4)), z, inv_fact(2)), z, 1.0);
    return make_double2(T.x * c - T.y * s, T.x * s + T.y * c);
}

// Copy the 2^tb roots of unity (tb <= 8) to LDS.
template <int NT>
__device__ __forceinline__ void stage_rou(double2* dst, const double2* src, uint32_t tb) {
    for (uint32_t i = threadIdx.x; i < (1u << tb); i += NT) dst[i] = gld(src + i);
}


// For each f in I': e_r = uhat_r[h_r(f)] * e^{-2 pi i (tau_r f mod N)/N} / Gtab[o_r(f)]
// (the energy-concentration estimate of the one frequency assumed in the
// bucket), x'_f = median_r Re e_r + i median_r Im e_r; then the K largest |x'_f|^2
// (ties -> lower f), returned in ascending f. One workgroup per signal.
// Dynamic LDS: P values and P frequencies (P = 2^ceil(log2 K)).
template <int LMAX>
__global__ __launch_bounds__(kFinNT) void finalize_kernel(Launch a) {
    extern __shared__ f4v lds_raw[];
    __shared__ uint32_t hist[256];
    __shared__ uint32_t bc[4];
    __shared__ uint32_t s_sig[kMaxL], s_tau[kMaxL], s_sinv[kMaxL];
    __shared__ double2 s_rou[kRouMax];
    uint32_t sig, unit;
    resolve(a, sig, unit);
    const auto& d = desc_of(a, sig);
    const IoDesc io = io_of(a, sig);
    const uint32_t fftm = d.fft_mode;
    const uint32_t L = d.L, maskN = d.maskN, log2M = d.log2M, M = d.M, B = d.B, N = d.N;
    const uint32_t rsh = d.log2N - d.tb;
    const double step = d.step;
    uint32_t P = 1;
    while (P < d.K) P <<= 1;
    float2* s_v = reinterpret_cast<float2*>(lds_raw);
    uint32_t* s_f = reinterpret_cast<uint32_t*>(s_v + P);
    if (threadIdx.x == 0) bc[3] = min(gld(d.ctr), d.cap);
    if (threadIdx.x < L) {
        s_sig[threadIdx.x] = gld(d.sigma + threadIdx.x);
        s_tau[threadIdx.x] = gld(d.tau + threadIdx.x);
        s_sinv[threadIdx.x] = gld(d.sigma_inv + threadIdx.x);
    }
    stage_rou<kFinNT>(s_rou, d.rou, d.tb);
    __syncthreads();
    const uint32_t n = bc[3];   // block-uniform by construction
    const uint32_t* cand = d.cand;
    const float2* invG = d.invG;
    const float2* uhat = d.uhat;
    const float2* tw = d.tw;
    float2* est = d.est;
    uint64_t* keys = d.keys;
    for (uint32_t i = threadIdx.x; i < n; i += kFinNT) {
        const uint32_t f = gld(cand + i);
        float re[LMAX], im[LMAX];
#pragma unroll
        for (int r = 0; r < LMAX; ++r) {
            re[r] = __builtin_inff();
            im[r] = __builtin_inff();
            if ((uint32_t)r < L) {
                const uint32_t p = (s_sig[r] * f) & maskN;
                const uint32_t h = ((p + (M >> 1)) >> log2M) & (B - 1u);
                const uint32_t o = (p - (h << log2M) + (N >> 1)) & maskN;   // o + N/2
                const uint32_t gi = o - (N >> 1) + (M >> 1);
                const float2 g = gld(invG + gi);
                float2 uv;
                if (fftm) {
                    // two-pass FFT layout: X[h] = e^{+2 pi i (s tau h mod B)/B} V[s h mod B], s = sigma^{-1}
                    const uint32_t si = s_sinv[r];
                    const float2 t = gld(tw + ((si * s_tau[r] * h) & (B - 1u)));   // e^{-2 pi i ./B}
                    uv = cmul(gld(uhat + (size_t)r * B + ((si * h) & (B - 1u))), make_float2(t.x, -t.y));
                } else {
                    uv = gld(uhat + (size_t)r * B + h);
                }
                const uint32_t k = (s_tau[r] * f) & maskN;
                const double2 pk = phase_of(s_rou, k, rsh, step);   // e^{+2 pi i k/N}
                const float2 rot = make_float2((float)pk.x, -(float)pk.y);
                const float2 e = cmul(cmul(uv, rot), g);
                re[r] = e.x;
                im[r] = e.y;
            }
        }
        const float mr = median_of<LMAX>(re, L);
        const float mi = median_of<LMAX>(im, L);
        const float mag = fmaf(mr, mr, mi * mi);
        gst(est + i, make_float2(mr, mi));
        gst(keys + i, ((uint64_t)(0xFFFFFFFFu - __float_as_uint(mag)) << 32) | (uint64_t)f);
    }
    __syncthreads();
    const uint32_t K = d.K;
    uint64_t thr = ~0ull;
    if (n > K) {
        // K-th smallest key (keys are unique: the low word is f)
        uint64_t prefix = 0, pmask = 0;
        uint32_t kk = K;
        const uint32_t lane = threadIdx.x & 63u;
        for (int pass = 0; pass < 8; ++pass) {
            const int shift = 56 - 8 * pass;
            for (int i = threadIdx.x; i < 256; i += kFinNT) hist[i] = 0;
            __syncthreads();
            for (uint32_t i = threadIdx.x; i < n; i += kFinNT) {
                const uint64_t key = gld(keys + i);
                if ((key & pmask) == prefix) atomicAdd(&hist[(uint32_t)(key >> shift) & 255u], 1u);
            }
            __syncthreads();
            if (threadIdx.x < 64) {
                const int lo = 4 * (int)lane;   // lane 0 owns the smallest digits
                const uint32_t h0 = hist[lo], h1 = hist[lo + 1], h2 = hist[lo + 2], h3 = hist[lo + 3];
                const uint32_t s = h0 + h1 + h2 + h3;
                const uint32_t incl = wave_incl_scan(s);
                const uint32_t excl = incl - s;
                if (excl < kk && kk <= incl) {
                    uint32_t acc = excl, dsel, rem;
                    if (acc + h0 >= kk) {
                        dsel = lo;
                        rem = kk - acc;
                    } else if (acc += h0, acc + h1 >= kk) {
                        dsel = lo + 1;
                        rem = kk - acc;
                    } else if (acc += h1, acc + h2 >= kk) {
                        dsel = lo + 2;
                        rem = kk - acc;
                    } else {
                        acc += h2;
                        dsel = lo + 3;
                        rem = kk - acc;
                    }
                    bc[0] = dsel;
                    bc[1] = rem;
                }
            }
            __syncthreads();
            prefix |= (uint64_t)bc[0] << shift;
            pmask |= 255ull << shift;
            kk = bc[1];
            __syncthreads();
        }
        thr = prefix;
    }
    if (threadIdx.x == 0) bc[2] = 0;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n; i += kFinNT) {
        const uint64_t key = gld(keys + i);
        if (key <= thr) {
            const uint32_t pos = atomicAdd(&bc[2], 1u);
            if (pos < P) {
                s_f[pos] = (uint32_t)key;
                s_v[pos] = gld(est + i);
            }
        }
    }
    __syncthreads();
    const uint32_t cnt = min(bc[2], K);
    uint32_t Q = 1;   // sort size: power of two >= cnt (<= P)
    while (Q < cnt) Q <<= 1;
    for (uint32_t i = cnt + threadIdx.x; i < Q; i += kFinNT) {
        s_f[i] = 0xFFFFFFFFu;
        s_v[i] = make_float2(0.f, 0.f);
    }
    __syncthreads();
    for (uint32_t k = 2; k <= Q; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < Q; i += kFinNT) {
                const uint32_t l = i ^ j;
                if (l > i) {
                    const bool up = (i & k) == 0;
                    const uint32_t fi = s_f[i], fl = s_f[l];
                    if ((fi > fl) == up) {
                        s_f[i] = fl;
                        s_f[l] = fi;
                        const float2 t = s_v[i];
                        s_v[i] = s_v[l];
                        s_v[l] = t;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t k = threadIdx.x; k < K; k += kFinNT) {
        if (k < cnt) {
            gst(io.out_idx + k, (int64_t)s_f[k]);
            gst(io.out_val + k, s_v[k]);
        } else {
            gst(io.out_idx + k, (int64_t)-1);
            gst(io.out_val + k, make_float2(0.f, 0.f));
        }
    }
}

// ---------------------------------------------------------------- FP64 residual
// E_res = mean_t |x_t - sum_k v_k e^{+2 pi i (t f_k mod N)/N}|^2 and
// E_in = mean_t |x_t|^2 over the S residual samples. The outputs are staged in
// LDS (dynamic: K values, K frequencies); the phase of the exact integer
// t f mod N is evaluated in FP64 (phase_of). Partial sums are reduced in a
// fixed order by the last workgroup to finish.
__global__ __launch_bounds__(kResNT) void residual_kernel(Launch a) {
    extern __shared__ f4v lds_raw[];
    __shared__ double sh[2][kResNT / 64];
    __shared__ uint32_t is_last;
    __shared__ double2 s_rou[kRouMax];
    uint32_t sig, unit;
    resolve(a, sig, unit);
    const auto& d = desc_of(a, sig);
    const IoDesc io = io_of(a, sig);
    const uint32_t K = d.K, maskN = d.maskN;
    const uint32_t rsh = d.log2N - d.tb;
    const double step = d.step;
    float2* s_v = reinterpret_cast<float2*>(lds_raw);
    uint32_t* s_f = reinterpret_cast<uint32_t*>(s_v + K);
    stage_rou<kResNT>(s_rou, d.rou, d.tb);
    for (uint32_t k = threadIdx.x; k < K; k += kResNT) {
        const int64_t f = gld(io.out_idx + k);
        s_f[k] = f < 0 ? 0xFFFFFFFFu : (uint32_t)f;
        s_v[k] = gld(io.out_val + k);
    }
    __syncthreads();
    const uint32_t j = unit * kResNT + threadIdx.x;
    double ea = 0.0, eb = 0.0;
    if (j < d.S) {
        const uint32_t t = gld(d.tpos + j);
        const float2 xv = gld(io.x + t);
        const double xr = xv.x, xi = xv.y;
        double mr = 0.0, mi = 0.0;
        for (uint32_t k = 0; k < K; ++k) {
            const uint32_t f = s_f[k];
            if (f == 0xFFFFFFFFu) continue;   // padding (uniform across the block)
            const double2 p = phase_of(s_rou, (t * f) & maskN, rsh, step);
            const float2 v = s_v[k];
            mr += (double)v.x * p.x - (double)v.y * p.y;
            mi += (double)v.x * p.y + (double)v.y * p.x;
        }
        const double er = xr - mr, ei = xi - mi;
        ea = er * er + ei * ei;
        eb = xr * xr + xi * xi;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        ea += __shfl_down(ea, off, 64);
        eb += __shfl_down(eb, off, 64);
    }
    const uint32_t lane = threadIdx.x & 63u, wid = threadIdx.x >> 6;
    if (lane == 0) {
        sh[0][wid] = ea;
        sh[1][wid] = eb;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double A = 0.0, Bs = 0.0;
#pragma unroll
        for (int w = 0; w < kResNT / 64; ++w) {
            A += sh[0][w];
            Bs += sh[1][w];
        }
        gst(d.rpart + 2 * unit, A);
        gst(d.rpart + 2 * unit + 1, Bs);
        __threadfence();
        const uint32_t prev = atomicAdd(d.ctr + 1, 1u);
        is_last = (prev + 1u == d.resid_blocks) ? 1u : 0u;
    }
    __syncthreads();
    if (is_last && threadIdx.x == 0) {
        __threadfence();
        const volatile double* rp = d.rpart;
        double A = 0.0, Bs = 0.0;
        for (uint32_t u = 0; u < d.resid_blocks; ++u) {
            A += rp[2 * u];
            Bs += rp[2 * u + 1];
        }
        double* out = io.out_resid ? io.out_resid : d.resid_own;
        gst(out + 0, A / (double)d.S);
        gst(out + 1, Bs / (double)d.S);
    }
}

// ---------------------------------------------------------------- launchers
template <int LOG2B>
static hipError_t launch_fft_t(const Launch& a, uint32_t units, hipStream_t s) {
    using Cfg = FftCfg<LOG2B>;
    hipLaunchKernelGGL(fft_select_kernel<LOG2B>, dim3(units), dim3(Cfg::NT), Cfg::lds_bytes(), s, a);
    return hipGetLastError();
}

template <int LOG2B>
static hipError_t set_fft_attr() {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&fft_select_kernel<LOG2B>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)FftCfg<LOG2B>::lds_bytes());
}

template <int PER>
static hipError_t set_strip_attr() {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&fold_strip_kernel<PER>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, 131072);
}

template <int LB>
constexpr size_t large_lds(uint32_t pass) {
    using C = LargeCfg<LB>;
    return pass == 0   ? SeqFft<C::LB1, 16, C::NT>::lds_bytes()
           : pass == 1 ? SeqFft<C::LB2, 16, C::NT>::lds_bytes()
                       : (size_t)(C::NW + 2 * C::SELCAP) * sizeof(uint32_t);
}

template <int LB>
hipError_t set_large_attr() {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&fft_large_p1_kernel<LB>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)large_lds<LB>(0));
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&fft_large_p2_kernel<LB>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)large_lds<LB>(1));
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&select_large_kernel<LB>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)large_lds<LB>(2));
    return e;
}

template <int LB>
hipError_t launch_large_t(const Launch& a, uint32_t pass, uint32_t units, hipStream_t s) {
    switch (pass) {
        case 0: hipLaunchKernelGGL(fft_large_p1_kernel<LB>, dim3(units), dim3(256), large_lds<LB>(0), s, a); break;
        case 1: hipLaunchKernelGGL(fft_large_p2_kernel<LB>, dim3(units), dim3(256), large_lds<LB>(1), s, a); break;
        case 2: hipLaunchKernelGGL(select_large_kernel<LB>, dim3(units), dim3(1024), large_lds<LB>(2), s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fft_large(const Launch& a, uint32_t log2B, uint32_t pass, uint32_t units, hipStream_t s) {
    switch (log2B) {
        case 15: return launch_large_t<15>(a, pass, units, s);
        case 16: return launch_large_t<16>(a, pass, units, s);
        case 17: return launch_large_t<17>(a, pass, units, s);
        case 18: return launch_large_t<18>(a, pass, units, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t set_kernel_attributes_impl() {
    hipError_t e;
    if ((e = set_large_attr<15>()) != hipSuccess) return e;
    if ((e = set_large_attr<16>()) != hipSuccess) return e;
    if ((e = set_large_attr<17>()) != hipSuccess) return e;
    if ((e = set_large_attr<18>()) != hipSuccess) return e;
    if ((e = set_strip_attr<16>()) != hipSuccess) return e;
    if ((e = set_strip_attr<32>()) != hipSuccess) return e;
    if ((e = set_fft_attr<13>()) != hipSuccess) return e;
    if ((e = set_fft_attr<14>()) != hipSuccess) return e;
    return hipSuccess;
}

hipError_t launch_fft_select(const Launch& a, uint32_t log2B, uint32_t units, hipStream_t s) {
    switch (log2B) {
        case 1: return launch_fft_t<1>(a, units, s);
        case 2: return launch_fft_t<2>(a, units, s);
        case 3: return launch_fft_t<3>(a, units, s);
        case 4: return launch_fft_t<4>(a, units, s);
        case 5: return launch_fft_t<5>(a, units, s);
        case 6: return launch_fft_t<6>(a, units, s);
        case 7: return launch_fft_t<7>(a, units, s);
        case 8: return launch_fft_t<8>(a, units, s);
        case 9: return launch_fft_t<9>(a, units, s);
        case 10: return launch_fft_t<10>(a, units, s);
        case 11: return launch_fft_t<11>(a, units, s);
        case 12: return launch_fft_t<12>(a, units, s);
        case 13: return launch_fft_t<13>(a, units, s);
        case 14: return launch_fft_t<14>(a, units, s);
        default: return hipErrorInvalidValue;
    }
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
    if (per >= 4 && ipt >= 1 && ipt <= 2 && g4 >= 1 && g4 <= 2) return (1u << 16) | (lp << 8) | (ipt << 4) | g4;
    return (1u << 16) | (lp << 8);
}

// row bands of the prefetching strip kernel: LDS holds at most 32 KB of the tile
constexpr uint32_t strip_bands(uint32_t per) { return per >= 16 ? per / 8 : 1; }

#define SFFT_PF(PER, IPT, G4)                                                                              \
    case (PER << 8) | (IPT << 4) | G4:                                                                     \
        hipLaunchKernelGGL((fold_strip_pf_kernel<PER, IPT, G4, strip_bands(PER)>), dim3(units), dim3(kFoldNT), \
                           lds_bytes / strip_bands(PER), s, a);                                            \
        break;

hipError_t launch_fold(const Launch& a, uint32_t variant, uint32_t units, uint32_t lds_bytes, hipStream_t s) {
    if (variant == 0) {
        hipLaunchKernelGGL(fold_gather_kernel, dim3(units), dim3(kFoldNT), 0, s, a);
        return hipGetLastError();
    }
    const uint32_t per = 1u << ((variant >> 8) & 255u);
    const uint32_t ipt = (variant >> 4) & 15u, g4 = variant & 15u;
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
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
#undef SFFT_PF

hipError_t launch_vote(const Launch& a, uint32_t lmax, uint32_t units, uint32_t lds_bytes, hipStream_t s) {
    const uint32_t staged = lds_bytes ? 1u : 0u;
    switch (lmax) {
        case 4: hipLaunchKernelGGL(vote_kernel<4>, dim3(units), dim3(kVoteNT), lds_bytes, s, a, staged); break;
        case 8: hipLaunchKernelGGL(vote_kernel<8>, dim3(units), dim3(kVoteNT), lds_bytes, s, a, staged); break;
        case 16: hipLaunchKernelGGL(vote_kernel<16>, dim3(units), dim3(kVoteNT), lds_bytes, s, a, staged); break;
        case 32: hipLaunchKernelGGL(vote_kernel<32>, dim3(units), dim3(kVoteNT), lds_bytes, s, a, staged); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_finalize(const Launch& a, uint32_t lmax, uint32_t units, uint32_t lds, hipStream_t s) {
    switch (lmax) {
        case 4: hipLaunchKernelGGL(finalize_kernel<4>, dim3(units), dim3(kFinNT), lds, s, a); break;
        case 8: hipLaunchKernelGGL(finalize_kernel<8>, dim3(units), dim3(kFinNT), lds, s, a); break;
        case 16: hipLaunchKernelGGL(finalize_kernel<16>, dim3(units), dim3(kFinNT), lds, s, a); break;
        case 32: hipLaunchKernelGGL(finalize_kernel<32>, dim3(units), dim3(kFinNT), lds, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_residual(const Launch& a, uint32_t units, uint32_t lds, hipStream_t s) {
    hipLaunchKernelGGL(residual_kernel, dim3(units), dim3(kResNT), lds, s, a);
    return hipGetLastError();
}

}  // namespace sfft
