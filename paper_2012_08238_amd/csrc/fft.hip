// B-point DFT of each loop's bucket values and the selection of the d*K
// largest buckets: one workgroup per loop in LDS up to B = 16384, two passes
// through the workspace and a selection workgroup beyond.
#include "fft_dev.hpp"

namespace sfft {

// Selection of the dK largest |uhat|^2 (ties -> lower bucket): radix select on
// the IEEE bit patterns of the non-negative energies (monotone as unsigned),
// four 8-bit digits from the top. Digit counts go to an LDS histogram; the
// first digit (sign + high exponent bits, shared by most buckets) is counted
// with one atomic per distinct digit per wave.
template <int LOG2B>
__global__ __launch_bounds__(FftCfg<LOG2B>::NT) void fft_select_kernel(Launch a) {
    using Cfg = FftCfg<LOG2B>;
    constexpr int B = Cfg::B, NT = Cfg::NT;
    extern __shared__ f4v lds_raw[];
    const FftLds<Cfg> sm(lds_raw);
    uint32_t sig, r;
    resolve(a, sig, r);
    const auto& d = desc_of(a, sig);
    {
        // the bucketization stored loop r's values in column order: column col
        // holds bucket b = sigma_r^{-1} (col - tau_r) mod B; place them by bucket.
        // The twiddle entries are loaded first, so their loads are in flight with these.
        const float2 twv = fft_twiddle_load<Cfg>(d);
        const float2* u = d.uhat + (size_t)r * B;
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
            if (col < (uint32_t)B) sm.data[padi((int)((sinv * (col - tu)) & (uint32_t)(B - 1)))] = tmp[q];
        }
        fft_twiddle_store(sm, twv);
    }
    fft_select_staged<Cfg>(d, r, sm);
}

// Selection of the residual buckets of the subtraction round: loop r's B bucket
// values (bucket order, as fft_select_kernel left them, then corrected by the
// subtraction) are staged in LDS and the dK largest energies selected as in the
// first round. Same LDS layout as fft_select_kernel.
template <int LOG2B>
__global__ __launch_bounds__(FftCfg<LOG2B>::NT) void reselect_kernel(Launch a) {
    using Cfg = FftCfg<LOG2B>;
    constexpr int B = Cfg::B, NT = Cfg::NT, NW = Cfg::NW;
    extern __shared__ f4v lds_raw[];
    float2* data = reinterpret_cast<float2*>(lds_raw);
    uint32_t* hist = reinterpret_cast<uint32_t*>(data + Cfg::PADN + Cfg::TL + Cfg::TH);
    uint32_t* scan = hist + 256;
    uint32_t* bcast = scan + 16;
    uint32_t* bits = reinterpret_cast<uint32_t*>(data);
    uint32_t sig, r;
    resolve(a, sig, r);
    const auto& d = desc_of(a, sig);
    const float2* u = d.uhat + (size_t)r * B;
    for (int h = threadIdx.x; h < B; h += NT) data[padi(h)] = gld(u + h);
    __syncthreads();
    select_top<Cfg>(data, d.dK, hist, scan, bcast, bits, d.jlist + (size_t)r * d.dK, d.jbits + (size_t)r * NW);
}

// ---------------------------------------------------------------- comb prefilter
// Spike-train bucketization of the sFFT2.0 row (Eq.(15)-(16)): comb loop c takes
// the Bc samples x[tau_c + j N/Bc]; their Bc-point DFT holds in bucket i the
// coefficients at f = i (mod Bc), so the comb_keep largest buckets mark the
// residues that may hold large coefficients (bitmap row c, ties -> lower
// residue). One workgroup per (signal, comb loop); same LDS layout as
// fft_select_kernel.
template <int LOG2B>
__global__ __launch_bounds__(FftCfg<LOG2B>::NT) void comb_kernel(Launch a) {
    using Cfg = FftCfg<LOG2B>;
    constexpr int B = Cfg::B, NT = Cfg::NT, NW = Cfg::NW;
    extern __shared__ f4v lds_raw[];
    float2* data = reinterpret_cast<float2*>(lds_raw);
    float2* tlo = data + Cfg::PADN;
    float2* thi = tlo + Cfg::TL;
    uint32_t* hist = reinterpret_cast<uint32_t*>(thi + Cfg::TH);
    uint32_t* scan = hist + 256;
    uint32_t* bcast = scan + 16;
    uint32_t* bits = reinterpret_cast<uint32_t*>(data);
    uint32_t sig, c;
    resolve(a, sig, c);
    const auto& d = desc_of(a, sig);
    const float2* x = io_of(a, sig).x;
    const uint32_t tc = ((CU32)d.comb_tau)[c], sh = d.log2N - (uint32_t)LOG2B, maskN = d.maskN;
    constexpr int LPT = (B + NT - 1) / NT;
    float2 tmp[LPT];
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
        const uint32_t j = min((uint32_t)threadIdx.x + (uint32_t)(q * NT), (uint32_t)B - 1u);
        tmp[q] = gld(x + ((tc + (j << sh)) & maskN));
    }
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
        const int j = (int)threadIdx.x + q * NT;
        if (j < B) data[padi(j)] = tmp[q];
    }
    const float2* tw = d.ctw;
    for (int j = threadIdx.x; j < Cfg::TL; j += NT) tlo[j] = gld(tw + j);
    for (int j = threadIdx.x; j < Cfg::TH; j += NT) thi[j] = gld(tw + (j << Cfg::LOG2TL));
    __syncthreads();
    fft_passes<Cfg, 0>(data, tlo, thi);
    select_top<Cfg>(data, d.comb_keep, hist, scan, bcast, bits, nullptr, d.cbits + (size_t)c * NW);
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
// [k1][j2], twisted. The twist W_B^m (m = j2 k1 mod B) is the product of two LDS table
// entries, W_B^{m mod B1} W_B^{B1 (m div B1)}, instead of a gather from the B-entry table
// per value (a 64-lane store instruction touched 64 table lines). Units per signal:
// L * B2/16.
template <int LB>
__global__ __launch_bounds__(256) void fft_large_p1_kernel(Launch a) {
    using C = LargeCfg<LB>;
    using F = SeqFft<C::LB1, 16, C::NT>;
    extern __shared__ f4v lds_raw[];
    float2* data = reinterpret_cast<float2*>(lds_raw);
    float2* tp = data + 16 * F::SP;
    float2* tlo = tp + F::P;      // W_B^i, i < B1
    float2* thi = tlo + C::B1;    // W_B^{B1 i}, i < B2
    uint32_t sig, unit;
    resolve(a, sig, unit);
    const auto& d = desc_of(a, sig);
    constexpr uint32_t tiles = C::B2 / 16;
    const uint32_t r = unit / tiles, j20 = (unit % tiles) * 16u;
    const float2* v = d.uhat + (size_t)r * C::B;
    float2* y = d.ubuf + (size_t)r * C::B;
    const float2* tw = d.tw;
    constexpr int NE = 16 * C::B1 / C::NT;   // values per thread
    constexpr int CHK = NE < 8 ? NE : 8;
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
    for (int m = threadIdx.x; m < C::B1; m += C::NT) tlo[m] = gld(tw + m);
    for (int m = threadIdx.x; m < C::B2; m += C::NT) thi[m] = gld(tw + ((size_t)m << C::LB1));
    __syncthreads();
    F::run(data, tp);
#pragma unroll 4
    for (int q = 0; q < NE; ++q) {
        const int e = (int)threadIdx.x + q * C::NT;
        const uint32_t k1 = (uint32_t)e >> 4, j2 = j20 + (uint32_t)(e & 15);
        const uint32_t m = (j2 * k1) & (uint32_t)(C::B - 1);
        const float2 t = cmul(thi[m >> C::LB1], tlo[m & (uint32_t)(C::B1 - 1)]);   // W_B^{j2 k1}
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
    constexpr int CHK = NE < 8 ? NE : 8;
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
    // WPT words per thread (B < 32 NT: the first NW threads hold one word each)
    constexpr int WPT = NW >= NT ? NW / NT : 1;
    static_assert(NW % WPT == 0 && (NW >= NT ? NW % NT == 0 : true), "bitmap words per thread");
    uint32_t* jb = d.jbits + (size_t)r * NW;
    uint32_t* jl = d.jlist + (size_t)r * dK;
    uint32_t wv[WPT], cnt = 0;
#pragma unroll
    for (int q = 0; q < WPT; ++q) {
        const uint32_t wi = threadIdx.x * WPT + q;
        wv[q] = wi < (uint32_t)NW ? bits[wi] : 0u;
        cnt += (uint32_t)__popc(wv[q]);
    }
#pragma unroll
    for (int q = 0; q < WPT; ++q) {
        const uint32_t wi = threadIdx.x * WPT + q;
        if (wi < (uint32_t)NW) gst(jb + wi, wv[q]);
    }
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

// ---------------------------------------------------------------- launchers
template <int LOG2B>
static hipError_t launch_fft_t(const Launch& a, uint32_t units, hipStream_t s) {
    using Cfg = FftCfg<LOG2B>;
    hipLaunchKernelGGL(fft_select_kernel<LOG2B>, dim3(units), dim3(Cfg::NT), Cfg::lds_bytes(), s, a);
    return hipGetLastError();
}

template <int LOG2B>
static hipError_t set_fft_attr() {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&fft_select_kernel<LOG2B>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)FftCfg<LOG2B>::lds_bytes());
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&comb_kernel<LOG2B>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)FftCfg<LOG2B>::lds_bytes());
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&reselect_kernel<LOG2B>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)FftCfg<LOG2B>::lds_bytes());
    return e;
}

template <int LOG2B>
static hipError_t launch_reselect_t(const Launch& a, uint32_t units, hipStream_t s) {
    using Cfg = FftCfg<LOG2B>;
    hipLaunchKernelGGL(reselect_kernel<LOG2B>, dim3(units), dim3(Cfg::NT), Cfg::lds_bytes(), s, a);
    return hipGetLastError();
}

hipError_t launch_reselect(const Launch& a, uint32_t log2B, uint32_t units, hipStream_t s) {
    switch (log2B) {
        case 1: return launch_reselect_t<1>(a, units, s);
        case 2: return launch_reselect_t<2>(a, units, s);
        case 3: return launch_reselect_t<3>(a, units, s);
        case 4: return launch_reselect_t<4>(a, units, s);
        case 5: return launch_reselect_t<5>(a, units, s);
        case 6: return launch_reselect_t<6>(a, units, s);
        case 7: return launch_reselect_t<7>(a, units, s);
        case 8: return launch_reselect_t<8>(a, units, s);
        case 9: return launch_reselect_t<9>(a, units, s);
        case 10: return launch_reselect_t<10>(a, units, s);
        case 11: return launch_reselect_t<11>(a, units, s);
        case 12: return launch_reselect_t<12>(a, units, s);
        case 13: return launch_reselect_t<13>(a, units, s);
        case 14: return launch_reselect_t<14>(a, units, s);
        default: return hipErrorInvalidValue;
    }
}

template <int LOG2B>
static hipError_t launch_comb_t(const Launch& a, uint32_t units, hipStream_t s) {
    using Cfg = FftCfg<LOG2B>;
    hipLaunchKernelGGL(comb_kernel<LOG2B>, dim3(units), dim3(Cfg::NT), Cfg::lds_bytes(), s, a);
    return hipGetLastError();
}

hipError_t launch_comb(const Launch& a, uint32_t log2b, uint32_t units, hipStream_t s) {
    switch (log2b) {
        case 1: return launch_comb_t<1>(a, units, s);
        case 2: return launch_comb_t<2>(a, units, s);
        case 3: return launch_comb_t<3>(a, units, s);
        case 4: return launch_comb_t<4>(a, units, s);
        case 5: return launch_comb_t<5>(a, units, s);
        case 6: return launch_comb_t<6>(a, units, s);
        case 7: return launch_comb_t<7>(a, units, s);
        case 8: return launch_comb_t<8>(a, units, s);
        case 9: return launch_comb_t<9>(a, units, s);
        case 10: return launch_comb_t<10>(a, units, s);
        case 11: return launch_comb_t<11>(a, units, s);
        case 12: return launch_comb_t<12>(a, units, s);
        case 13: return launch_comb_t<13>(a, units, s);
        case 14: return launch_comb_t<14>(a, units, s);
        default: return hipErrorInvalidValue;
    }
}

template <int LB>
constexpr size_t large_lds(uint32_t pass) {
    using C = LargeCfg<LB>;
    return pass == 0   ? SeqFft<C::LB1, 16, C::NT>::lds_bytes() + (size_t)(C::B1 + C::B2) * sizeof(float2)
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
        case 12: return launch_large_t<12>(a, pass, units, s);
        case 13: return launch_large_t<13>(a, pass, units, s);
        case 14: return launch_large_t<14>(a, pass, units, s);
        case 15: return launch_large_t<15>(a, pass, units, s);
        case 16: return launch_large_t<16>(a, pass, units, s);
        case 17: return launch_large_t<17>(a, pass, units, s);
        case 18: return launch_large_t<18>(a, pass, units, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t set_fft_attributes() {
    hipError_t e;
    if ((e = set_large_attr<12>()) != hipSuccess) return e;
    if ((e = set_large_attr<13>()) != hipSuccess) return e;
    if ((e = set_large_attr<14>()) != hipSuccess) return e;
    if ((e = set_large_attr<15>()) != hipSuccess) return e;
    if ((e = set_large_attr<16>()) != hipSuccess) return e;
    if ((e = set_large_attr<17>()) != hipSuccess) return e;
    if ((e = set_large_attr<18>()) != hipSuccess) return e;
    if ((e = set_fft_attr<13>()) != hipSuccess) return e;
    if ((e = set_fft_attr<14>()) != hipSuccess) return e;
    return hipSuccess;
}

hipError_t set_kernel_attributes_impl() {
    hipError_t e = set_fft_attributes();
    if (e == hipSuccess) e = set_fold_attributes();
    if (e == hipSuccess) e = set_estimate_attributes();
    return e;
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

}  // namespace sfft
