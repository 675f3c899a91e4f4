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
__device__ __forceinline__ void resolve(const Launch& a, uint32_t& sig, uint32_t& unit) {
    const uint32_t blk = blockIdx.x;
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
        gst(uhat + (size_t)r * B + b, acc);
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
    const uint32_t log2B = d.log2B;
    const uint32_t it = unit * kFoldNT + threadIdx.x;
    if (it >= (d.L << log2B)) return;
    const uint32_t r = it >> log2B, b = it & (d.B - 1u);
    const uint32_t s = gld(d.sigma + r), tu = gld(d.tau + r);
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
            xv[e] = ok[e] ? gld(x + ((s * i + tu) & maskN)) : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (ok[e]) {
                acc.x = fmaf(g[e], xv[e].x, acc.x);
                acc.y = fmaf(g[e], xv[e].y, acc.y);
            }
        }
    }
    gst(d.uhat + it, acc);
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
    for (int h = threadIdx.x; h < B; h += NT) data[padi(h)] = gld(u + h);
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
            key[c] = __float_as_uint(fmaf(v.x, v.x, v.y * v.y));
        }
    }
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t prefix = 0, pmask = 0, kk = d.dK;
#pragma unroll
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 24 - 8 * pass;
        for (int i = threadIdx.x; i < 256; i += NT) hist[i] = 0;
        __syncthreads();
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const bool act = valid && ((key[c] & pmask) == prefix);
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
    // prefix = energy bits of the dK-th largest; take every key above it and the
    // kk lowest-index keys equal to it.
    uint32_t eq = 0;
#pragma unroll
    for (int c = 0; c < CH; ++c) eq += (valid && key[c] == prefix) ? 1u : 0u;
    uint32_t tot;
    uint32_t eqrank = block_excl_scan<NT>(eq, scan, tot);
    uint64_t selm = 0;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        bool sel = false;
        if (valid) {
            if (key[c] > prefix) {
                sel = true;
            } else if (key[c] == prefix) {
                sel = eqrank < kk;
                ++eqrank;
            }
        }
        if (sel) selm |= 1ull << c;
    }
    for (int i = threadIdx.x; i < NW; i += NT) bits[i] = 0;
    __syncthreads();
    const uint32_t nsel = (uint32_t)__popcll(selm);
    uint32_t pos = block_excl_scan<NT>(nsel, scan, tot);
    uint32_t* jl = d.jlist + (size_t)r * d.dK;
    const uint32_t dK = d.dK;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        if ((selm >> c) & 1ull) {
            const uint32_t h = threadIdx.x * CH + c;
            atomicOr(&bits[h >> 5], 1u << (h & 31));
            if (pos < dK) gst(jl + pos, h);
            ++pos;
        }
    }
    __syncthreads();
    uint32_t* jb = d.jbits + (size_t)r * NW;
    for (int i = threadIdx.x; i < NW; i += NT) gst(jb + i, bits[i]);
}

// ---------------------------------------------------------------- votes
// A frequency with >= T votes out of L is voted by one of the loops 0..L-T
// (pigeonhole), so only the frequencies of those loops' selected buckets are
// enumerated: f = sigma_r0^{-1} p for the N/B permuted positions p of each
// selected bucket. Each frequency is counted from the first loop that voted
// for it (later loops skip it), so I' has no duplicates; votes are bitmap tests.
__global__ __launch_bounds__(kVoteNT) void vote_kernel(Launch a, uint32_t staged) {
    extern __shared__ uint32_t sbits[];
    __shared__ uint32_t s_sig[kMaxL];
    uint32_t sig, unit;
    resolve(a, sig, unit);
    const auto& d = desc_of(a, sig);
    const uint32_t wpl = (d.B + 31u) >> 5;
    const uint32_t L = d.L, T = d.T, M = d.M, log2M = d.log2M, maskN = d.maskN, B = d.B, dK = d.dK;
    const uint32_t* jbits = d.jbits;
    const uint32_t* jlist = d.jlist;
    const uint32_t* sigma_inv = d.sigma_inv;
    if (threadIdx.x < L) s_sig[threadIdx.x] = gld(d.sigma + threadIdx.x);
    const uint32_t* bits = jbits;
    if (staged) {
        const uint32_t nw = L * wpl;
        for (uint32_t i = threadIdx.x; i < nw; i += kVoteNT) sbits[i] = gld(jbits + i);
        bits = sbits;
    }
    __syncthreads();
    const uint32_t per_loop = dK * M;
    const uint32_t total = (L - T + 1u) * per_loop;
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t* ctr = d.ctr;
    uint32_t* cand = d.cand;
    const uint32_t cap = d.cap;
    for (uint32_t qq = 0; qq < kVotePerThread; ++qq) {
        const uint32_t c = unit * kVoteUnit + qq * kVoteNT + threadIdx.x;
        bool emit = false;
        uint32_t f = 0;
        if (c < total) {
            const uint32_t r0 = c / per_loop;
            const uint32_t rem = c - r0 * per_loop;
            const uint32_t h = gld(jlist + r0 * dK + (rem >> log2M));
            const uint32_t p = ((h << log2M) - (M >> 1) + (rem & (M - 1u))) & maskN;
            f = (gld(sigma_inv + r0) * p) & maskN;
            uint32_t cnt = 1;
            bool dup = false;
            for (uint32_t r = 0; r < L; ++r) {
                if (r == r0) continue;
                const uint32_t pr = (s_sig[r] * f) & maskN;
                const uint32_t hr = ((pr + (M >> 1)) >> log2M) & (B - 1u);
                const uint32_t bit = (bits[r * wpl + (hr >> 5)] >> (hr & 31u)) & 1u;
                if (r < r0) {
                    if (bit) {
                        dup = true;
                        break;
                    }
                } else {
                    cnt += bit;
                    if (cnt + (L - 1u - r) < T) break;
                }
            }
            emit = !dup && cnt >= T;
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

// For each f in I': e_r = uhat_r[h_r(f)] * e^{-2 pi i (tau_r f mod N)/N} / Gtab[o_r(f)]
// (the energy-concentration estimate of the one frequency assumed in the
// bucket), x'_f = median_r Re e_r + i median_r Im e_r; then the K largest |x'_f|^2
// (ties -> lower f), returned in ascending f. One workgroup per signal.
template <int LMAX>
__global__ __launch_bounds__(kFinNT) void finalize_kernel(Launch a) {
    __shared__ uint32_t s_f[kMaxK];
    __shared__ float2 s_v[kMaxK];
    __shared__ uint32_t hist[256];
    __shared__ uint32_t bc[4];
    __shared__ uint32_t s_sig[kMaxL], s_tau[kMaxL];
    uint32_t sig, unit;
    resolve(a, sig, unit);
    const auto& d = desc_of(a, sig);
    const IoDesc io = io_of(a, sig);
    const uint32_t L = d.L, maskN = d.maskN, log2M = d.log2M, M = d.M, B = d.B, N = d.N;
    if (threadIdx.x == 0) bc[3] = min(gld(d.ctr), d.cap);
    if (threadIdx.x < L) {
        s_sig[threadIdx.x] = gld(d.sigma + threadIdx.x);
        s_tau[threadIdx.x] = gld(d.tau + threadIdx.x);
    }
    __syncthreads();
    const uint32_t n = bc[3];   // block-uniform by construction
    const uint32_t* cand = d.cand;
    const float2* invG = d.invG;
    const float2* uhat = d.uhat;
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
                const float2 uv = gld(uhat + (size_t)r * B + h);
                const uint32_t k = (s_tau[r] * f) & maskN;
                double sd, cd;
                sincospi((double)k * (2.0 / (double)N), &sd, &cd);
                const float2 ph = make_float2((float)cd, -(float)sd);
                const float2 e = cmul(cmul(uv, ph), g);
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
            if (pos < kMaxK) {
                s_f[pos] = (uint32_t)key;
                s_v[pos] = gld(est + i);
            }
        }
    }
    __syncthreads();
    const uint32_t cnt = min(bc[2], min(K, (uint32_t)kMaxK));
    uint32_t P = 1;
    while (P < cnt) P <<= 1;
    for (uint32_t i = cnt + threadIdx.x; i < P; i += kFinNT) {
        s_f[i] = 0xFFFFFFFFu;
        s_v[i] = make_float2(0.f, 0.f);
    }
    __syncthreads();
    for (uint32_t k = 2; k <= P; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < P; i += kFinNT) {
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
// LDS; the phase comes from two FP64 tables split on the bits of the exact
// integer t f mod N. Partial sums are reduced in a fixed order by the last
// workgroup to finish.
__global__ __launch_bounds__(kResNT) void residual_kernel(Launch a) {
    __shared__ uint32_t s_f[kMaxK];
    __shared__ float2 s_v[kMaxK];
    __shared__ double sh[2][kResNT / 64];
    __shared__ uint32_t is_last;
    uint32_t sig, unit;
    resolve(a, sig, unit);
    const auto& d = desc_of(a, sig);
    const IoDesc io = io_of(a, sig);
    const uint32_t K = d.K, maskN = d.maskN, rsh = d.rsh;
    for (uint32_t k = threadIdx.x; k < K; k += kResNT) {
        const int64_t f = gld(io.out_idx + k);
        s_f[k] = f < 0 ? 0xFFFFFFFFu : (uint32_t)f;
        s_v[k] = gld(io.out_val + k);
    }
    __syncthreads();
    const uint32_t j = unit * kResNT + threadIdx.x;
    const double2* rt_hi = d.rt_hi;
    const double2* rt_lo = d.rt_lo;
    double ea = 0.0, eb = 0.0;
    if (j < d.S) {
        const uint32_t t = gld(d.tpos + j);
        const float2 xv = gld(io.x + t);
        const double xr = xv.x, xi = xv.y;
        double mr = 0.0, mi = 0.0;
        const uint32_t lomask = (1u << rsh) - 1u;
        for (uint32_t k0 = 0; k0 < K; k0 += 4) {
            double2 hi[4], lo[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t k = k0 + e;
                const uint32_t f = k < K ? s_f[k] : 0xFFFFFFFFu;
                const uint32_t m = (t * f) & maskN;
                hi[e] = make_double2(0.0, 0.0);
                lo[e] = make_double2(0.0, 0.0);
                if (f != 0xFFFFFFFFu) {
                    hi[e] = gld(rt_hi + (m >> rsh));
                    lo[e] = gld(rt_lo + (m & lomask));
                }
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t k = k0 + e;
                if (k < K && s_f[k] != 0xFFFFFFFFu) {
                    const float2 v = s_v[k];
                    const double pr = hi[e].x * lo[e].x - hi[e].y * lo[e].y;
                    const double pi = hi[e].x * lo[e].y + hi[e].y * lo[e].x;
                    mr += (double)v.x * pr - (double)v.y * pi;
                    mi += (double)v.x * pi + (double)v.y * pr;
                }
            }
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

hipError_t set_kernel_attributes_impl() {
    hipError_t e;
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

hipError_t launch_fold(const Launch& a, uint32_t mode, uint32_t units, uint32_t lds_bytes, hipStream_t s) {
    if (mode == 1) {
        switch (strip_per_thread(lds_bytes)) {
            case 1: hipLaunchKernelGGL(fold_strip_kernel<1>, dim3(units), dim3(kFoldNT), lds_bytes, s, a); break;
            case 2: hipLaunchKernelGGL(fold_strip_kernel<2>, dim3(units), dim3(kFoldNT), lds_bytes, s, a); break;
            case 4: hipLaunchKernelGGL(fold_strip_kernel<4>, dim3(units), dim3(kFoldNT), lds_bytes, s, a); break;
            case 8: hipLaunchKernelGGL(fold_strip_kernel<8>, dim3(units), dim3(kFoldNT), lds_bytes, s, a); break;
            case 16: hipLaunchKernelGGL(fold_strip_kernel<16>, dim3(units), dim3(kFoldNT), lds_bytes, s, a); break;
            case 32: hipLaunchKernelGGL(fold_strip_kernel<32>, dim3(units), dim3(kFoldNT), lds_bytes, s, a); break;
            default: return hipErrorInvalidValue;
        }
    } else {
        hipLaunchKernelGGL(fold_gather_kernel, dim3(units), dim3(kFoldNT), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_vote(const Launch& a, uint32_t units, uint32_t lds_bytes, hipStream_t s) {
    const uint32_t staged = lds_bytes ? 1u : 0u;
    hipLaunchKernelGGL(vote_kernel, dim3(units), dim3(kVoteNT), lds_bytes, s, a, staged);
    return hipGetLastError();
}

hipError_t launch_finalize(const Launch& a, uint32_t lmax, uint32_t units, hipStream_t s) {
    switch (lmax) {
        case 4: hipLaunchKernelGGL(finalize_kernel<4>, dim3(units), dim3(kFinNT), 0, s, a); break;
        case 8: hipLaunchKernelGGL(finalize_kernel<8>, dim3(units), dim3(kFinNT), 0, s, a); break;
        case 16: hipLaunchKernelGGL(finalize_kernel<16>, dim3(units), dim3(kFinNT), 0, s, a); break;
        case 32: hipLaunchKernelGGL(finalize_kernel<32>, dim3(units), dim3(kFinNT), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_residual(const Launch& a, uint32_t units, hipStream_t s) {
    hipLaunchKernelGGL(residual_kernel, dim3(units), dim3(kResNT), 0, s, a);
    return hipGetLastError();
}

}  // namespace sfft
