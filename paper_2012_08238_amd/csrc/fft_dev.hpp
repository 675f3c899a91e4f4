// B-point FFT in one workgroup's LDS (Stockham radix-16/8/4/2 passes) and the
// selection of the largest bucket energies: device helpers shared by the FFT kernels
// and the fused single-signal kernel.
#pragma once

#include "device.hpp"

namespace sfft {

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
            // W = -i (t = 4) is a swap and a sign: no multiplications by zero
            const float2 ow = (k == 0) ? o[k] : (t == 4 ? mul_mi(o[k]) : cmul(o[k], w));
            v[k] = make_float2(e[k].x + ow.x, e[k].y + ow.y);
            v[k + R / 2] = make_float2(e[k].x - ow.x, e[k].y - ow.y);
        }
    }
};

// Sizes of the B = 2^LOG2B point transform and selection in one workgroup of NT threads:
// B/16 clamped to [64, 1024] by default, or NTO (a multiple of 64, at least that default
// for the passes to cover every butterfly) when the caller's workgroup has another width.
template <int LOG2B, int NTO = 0>
struct FftCfg {
    static constexpr int LOG2 = LOG2B;
    static constexpr int B = 1 << LOG2B;
    static constexpr int NT = NTO ? NTO : (B / 16 < 64 ? 64 : (B / 16 > 1024 ? 1024 : B / 16));
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
template <class Cfg, int LOG2R, int LOG2NS>
__device__ __forceinline__ void stockham_pass(float2* lds, const float2* tlo, const float2* thi) {
    constexpr int LOG2B = Cfg::LOG2;
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
                // W^{r m1} for r = 1..R-1: W^{m1} from the two tables, the other powers by
                // squarings and products (at most log2 R + 2 roundings deep) instead of two
                // table reads each
                const int m1 = k << TSHIFT;
                float2 w[R];
                w[1] = cmul(thi[m1 >> Cfg::LOG2TL], tlo[m1 & (Cfg::TL - 1)]);
#pragma unroll
                for (int r = 2; r < R; ++r) w[r] = (r & 1) ? cmul(w[r - 1], w[1]) : cmul(w[r / 2], w[r / 2]);
#pragma unroll
                for (int r = 1; r < R; ++r) v[q][r] = cmul(v[q][r], w[r]);
            }
            SmallDft<R>::run(v[q]);
            const int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) lds[padi(base + r * Ns)] = v[q][r];
        }
    }
    __syncthreads();
}

template <class Cfg, int LOG2NS>
__device__ __forceinline__ void fft_passes(float2* lds, const float2* tlo, const float2* thi) {
    constexpr int REM = Cfg::LOG2 - LOG2NS;
    if constexpr (REM >= 4) {
        stockham_pass<Cfg, 4, LOG2NS>(lds, tlo, thi);
        fft_passes<Cfg, LOG2NS + 4>(lds, tlo, thi);
    } else if constexpr (REM > 0) {
        stockham_pass<Cfg, REM, LOG2NS>(lds, tlo, thi);
    }
}

// k-th largest (1-based; k <= number of valid keys) of the keys held by the
// block, KPT per thread: radix select on 8-bit digits from the top through an
// LDS histogram. The first digit (shared by most keys) is counted with one
// atomic per distinct digit per wave. Returns the value and how many keys equal
// to it are among the k largest.
// With PASSES < 4 only the top 8 PASSES bits are decided: theta is then the k-th
// largest key with its lower bits cleared, a lower bound of it.
template <int NT, int KPT, int PASSES = 4>
__device__ __forceinline__ void block_kth_largest(const uint32_t* key, const bool* kv, uint32_t k, uint32_t* hist,
                                                  uint32_t* bcast, uint32_t& theta, uint32_t& rank) {
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t prefix = 0, pmask = 0, kk = k;
#pragma unroll
    for (int pass = 0; pass < PASSES; ++pass) {
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

// The dK largest |data[h]|^2 of the B values in LDS (ties -> lower h): bitmap
// jb[B/32] and, when jl is not null, the ascending list jl[dK]. LDS scratch as
// laid out by fft_select_kernel; the data region is reused for the bitmap.
template <class Cfg>
__device__ __forceinline__ void select_top(const float2* data, uint32_t dK, uint32_t* hist, uint32_t* scan,
                                           uint32_t* bcast, uint32_t* bits, uint32_t* jl, uint32_t* jb) {
    constexpr int LOG2B = Cfg::LOG2;
    constexpr int B = Cfg::B, NT = Cfg::NT, CH = Cfg::CH, NW = Cfg::NW;
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
    const uint32_t nl = jl ? dK : 0u;   // list entries written (none without a list)
    bool kv[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) kv[c] = valid;
    bool done = false;
    if constexpr (CH >= 4 && NT == 1024 && 2 * Cfg::PADN >= Cfg::NW + 64 + 4096 + 2 * (1024 + 32)) {
        if (dK <= (uint32_t)NT) {   // block-uniform
            // The candidates are the keys of the histogram bins (the top 12 bits of the
            // energy: exponent and three mantissa bits) from the top down to the bin that
            // holds the dK-th largest; when they are at most 1024, each one's rank among
            // them (larger energy first, then lower bucket) is counted directly and the
            // dK of rank below dK are selected. Otherwise the general path below.
            constexpr int NBIN = 4096;
            uint32_t* hb = bits + Cfg::NW + 64;   // histogram [NBIN]
            // candidates [1024 + padding]: (energy key << log2 B) | (B - 1 - bucket), so that
            // a larger value is a larger energy, or an equal one in a lower bucket
            uint64_t* ccomp = reinterpret_cast<uint64_t*>(hb + NBIN);
            __syncthreads();   // every thread has read its values from the data region reused below
#pragma unroll
            for (int q = 0; q < NBIN / NT; ++q) hb[threadIdx.x + q * NT] = 0u;
            if (threadIdx.x == 0) bcast[2] = 0u;
            __syncthreads();
#pragma unroll
            for (int c = 0; c < CH; ++c) atomicAdd(&hb[key[c] >> 20], 1u);
            __syncthreads();
            // thread t owns bins NBIN-1-4t .. NBIN-4-4t (largest first)
            uint32_t hc[NBIN / NT], hs = 0;
#pragma unroll
            for (int q = 0; q < NBIN / NT; ++q) {
                hc[q] = hb[NBIN - 1 - (int)threadIdx.x * (NBIN / NT) - q];
                hs += hc[q];
            }
            uint32_t tot;
            uint32_t above = block_excl_scan<NT>(hs, scan, tot);   // keys in the bins above this thread's
            if (above < dK && dK <= above + hs) {
#pragma unroll
                for (int q = 0; q < NBIN / NT; ++q) {
                    if (above < dK && dK <= above + hc[q]) {
                        bcast[0] = (uint32_t)(NBIN - 1 - (int)threadIdx.x * (NBIN / NT) - q) << 20;   // lower edge
                        bcast[1] = above + hc[q];                                                   // candidates
                    }
                    above += hc[q];
                }
            }
            __syncthreads();
            const uint32_t t0 = bcast[0], ncand = bcast[1];
            if (ncand <= 1024u) {   // block-uniform
                // collect the candidates (any order: the ranks below do not depend on it)
                uint32_t cnt = 0;
#pragma unroll
                for (int c = 0; c < CH; ++c) cnt += key[c] >= t0 ? 1u : 0u;
                const uint32_t incl = wave_incl_scan(cnt);
                uint32_t wbase = 0;
                if ((threadIdx.x & 63u) == 63u && incl) wbase = atomicAdd(&bcast[2], incl);
                uint32_t pos = __shfl(wbase, 63, 64) + incl - cnt;
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    if (key[c] >= t0) {
                        const uint32_t h = threadIdx.x * CH + c;
                        ccomp[pos] = ((uint64_t)key[c] << LOG2B) | (uint64_t)(B - 1 - h);
                        ++pos;
                    }
                }
                // PS threads (consecutive lanes) share a candidate when there are few; each reads
                // every PS-th group of 8 candidates, the list padded with zeros (never larger)
                const int PS = ncand <= 256u ? 4 : (ncand <= 512u ? 2 : 1);   // block-uniform
                const uint32_t npad = (ncand + 8u * PS - 1u) / (8u * PS) * (8u * PS);
                if (threadIdx.x < npad - ncand) ccomp[ncand + threadIdx.x] = 0ull;
                for (int i = threadIdx.x; i < NW; i += NT) bits[i] = 0u;
                __syncthreads();
                // rank of candidate j: the candidates with a larger value
                const uint32_t j = threadIdx.x / PS, part = threadIdx.x % PS;
                uint32_t rank = 0;
                uint64_t cj = 0;
                if (j < ncand) {
                    cj = ccomp[j];
                    typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));
                    const u64x2* c2 = reinterpret_cast<const u64x2*>(ccomp);
                    for (uint32_t g = part; g < npad / 8u; g += PS) {
                        u64x2 v[4];
#pragma unroll
                        for (int e = 0; e < 4; ++e) v[e] = c2[g * 4u + e];
#pragma unroll
                        for (int e = 0; e < 4; ++e) rank += (v[e].x > cj ? 1u : 0u) + (v[e].y > cj ? 1u : 0u);
                    }
                }
                if (PS >= 2) rank += __shfl_xor(rank, 1, 64);
                if (PS >= 4) rank += __shfl_xor(rank, 2, 64);
                if (j < ncand && part == 0 && rank < dK) {
                    const uint32_t hj = (uint32_t)(B - 1) - (uint32_t)(cj & (uint64_t)(B - 1));
                    atomicOr(&bits[hj >> 5], 1u << (hj & 31));
                }
                __syncthreads();
                // the bitmap, and the list in ascending bucket order
                constexpr int WPT = NW >= NT ? NW / NT : 1;
                uint32_t wv[WPT], c2 = 0;
#pragma unroll
                for (int q = 0; q < WPT; ++q) {
                    const uint32_t wi = threadIdx.x * WPT + q;
                    wv[q] = wi < (uint32_t)NW ? bits[wi] : 0u;
                    c2 += (uint32_t)__popc(wv[q]);
                    if (wi < (uint32_t)NW) gst(jb + wi, wv[q]);
                }
                uint32_t t2;
                uint32_t p2 = block_excl_scan<NT>(c2, scan, t2);
#pragma unroll
                for (int q = 0; q < WPT; ++q) {
                    uint32_t w = wv[q];
                    while (w) {
                        const uint32_t b = (uint32_t)__ffs((int)w) - 1u;
                        w &= w - 1u;
                        if (p2 < nl) gst(jl + p2, (threadIdx.x * WPT + q) * 32u + b);
                        ++p2;
                    }
                }
                done = true;
            }
        }
    }
    if constexpr (CH >= 4 && Cfg::SELCAP >= NT) {
        if (!done && dK <= (uint32_t)NT) {
            // Every one of the dK largest energies is >= theta0, the dK-th largest of
            // the per-thread maxima (at least dK threads hold a value >= theta0), so
            // only the keys >= theta0 can be selected. Collect them (in bucket
            // order) and select exactly among those when they are few.
            uint32_t tmax[1] = {0};
            const bool tv[1] = {valid};
#pragma unroll
            for (int c = 0; c < CH; ++c) tmax[0] = max(tmax[0], key[c]);
            uint32_t theta0, rank0;
            // (its top 16 bits suffice: any lower bound of it keeps every selected key)
            block_kth_largest<NT, 1, 2>(tmax, tv, dK, hist, bcast, theta0, rank0);
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
                                        jl, jb, nl);
                done = true;
            }
        }
    }
    if (!done) {   // block-uniform
        uint32_t theta, rank;
        block_kth_largest<NT, CH>(key, kv, dK, hist, bcast, theta, rank);
        const uint64_t selm = select_mask<NT, CH>(key, kv, theta, rank, scan);
        emit_selection<NT, CH>(selm, [&](int c) { return (uint32_t)(threadIdx.x * CH + c); }, bits, NW, scan, jl, jb,
                               nl);
    }
}

// LDS of the one-workgroup transform: the B values (padded), the two twiddle tables,
// the selection's histogram [256], scan words [16] and broadcast words [4]; the
// selection's bitmap reuses the data region.
template <class Cfg>
struct FftLds {
    float2* data;
    float2* tlo;
    float2* thi;
    uint32_t* hist;
    uint32_t* scan;    // NT/64 <= 16 words
    uint32_t* bcast;   // [0] digit, [1] remaining rank
    uint32_t* bits;
    __device__ __forceinline__ explicit FftLds(void* base) {
        data = reinterpret_cast<float2*>(base);
        tlo = data + Cfg::PADN;
        thi = tlo + Cfg::TL;
        hist = reinterpret_cast<uint32_t*>(thi + Cfg::TH);
        scan = hist + 256;
        bcast = scan + 16;
        bits = reinterpret_cast<uint32_t*>(data);
    }
};

// One twiddle table entry per thread (threads TL .. TL+TH-1 the hi table), loaded into a
// register so that the load can be in flight with the bucket values' loads.
template <class Cfg, class Desc>
__device__ __forceinline__ float2 fft_twiddle_load(const Desc& d) {
    static_assert(Cfg::TL + Cfg::TH <= Cfg::NT, "one twiddle entry per thread");
    const int j = (int)threadIdx.x;
    float2 t = make_float2(0.f, 0.f);
    if (j < Cfg::TL) t = gld(d.tw + j);
    else if (j < Cfg::TL + Cfg::TH) t = gld(d.tw + ((j - Cfg::TL) << Cfg::LOG2TL));
    return t;
}

template <class Cfg>
__device__ __forceinline__ void fft_twiddle_store(const FftLds<Cfg>& sm, float2 t) {
    const int j = (int)threadIdx.x;
    if (j < Cfg::TL) sm.tlo[j] = t;
    else if (j < Cfg::TL + Cfg::TH) sm.thi[j - Cfg::TL] = t;
}

// Loop r's B bucket values and the twiddle tables, placed in sm by the caller (not yet
// synchronised): their forward B-point DFT goes to uhat[r] (bucket order), and the dK
// largest energies to the loop's bitmap and ascending list.
template <class Cfg, class Desc>
__device__ __forceinline__ void fft_select_staged(const Desc& d, uint32_t r, const FftLds<Cfg>& sm) {
    constexpr int B = Cfg::B, NT = Cfg::NT, NW = Cfg::NW;
    float2* u = d.uhat + (size_t)r * B;
    __syncthreads();
    fft_passes<Cfg, 0>(sm.data, sm.tlo, sm.thi);
    for (int h = threadIdx.x; h < B; h += NT) gst(u + h, sm.data[padi(h)]);
    select_top<Cfg>(sm.data, d.dK, sm.hist, sm.scan, sm.bcast, sm.bits, d.jlist + (size_t)r * d.dK,
                    d.jbits + (size_t)r * NW);
}

}  // namespace sfft
