"""Plain FP64 CPU oracle of the flat-window voting sparse FFT (the sFFT1.0 row of
Table 1: flat filter, statistics location, energy estimation, voting framework).

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this package.
It shares no code, tables or constants with the HIP library and imports nothing
from it; the product path never calls it.

Everything is computed in float64 / exact Python or int64 integers, step by step
in the order the paper gives them, with no blocking or fusion:

  permutation (time scaling Eq.(7) + time shift Eq.(6), permuted-spectrum
  identity Eq.(9)) -> flat window (sinc Eq.(12) x Gaussian Eq.(13)) ->
  aliasing into B buckets (Eq.(11)) -> B-point DFT of the buckets -> keep the
  2K largest buckets and vote ("probability and statistics" location method)
  -> energy-concentration estimate per located frequency, combined over the
  random bucketizations by a coordinate-wise median -> K largest -> formula
  method (Eq.(2)) for the residual energy check.

Where the paper is silent or garbled the readings used here are the ones listed
in the design notes (window width from the Fig. 1 example, round-half-up
bucket hash, strict-majority vote threshold, median combiner, ...); each is
restated at the function that uses it.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Ratio between the flat window length and the Gaussian standard deviation,
# fixed by the Fig. 1 example of the flat-filter section: N=2048, B=16,
# Gaussian std = B*sqrt(log2 N) = 53.066 and window support 516, so
# std = support / (2 * C_G).
C_G = 516.0 / (2.0 * 16.0 * math.sqrt(11.0))

_MASK64 = (1 << 64) - 1


# ---------------------------------------------------------------------------
# Random draws: SplitMix64 (Steele, Lea & Flood, OOPSLA 2014), written from its
# published definition: a Weyl counter with increment 0x9E3779B97F4A7C15 and a
# two-multiply xor-shift finaliser.
# ---------------------------------------------------------------------------
def splitmix64(seed: int, n: int) -> list[int]:
    """First ``n`` outputs of SplitMix64 seeded with ``seed`` (as Python ints)."""
    state = seed & _MASK64
    out = []
    for _ in range(n):
        state = (state + 0x9E3779B97F4A7C15) & _MASK64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        out.append(z ^ (z >> 31))
    return out


RESID_RUN = 8   # residual-check positions come in runs of this many consecutive samples


def resid_draws(n_resid: int) -> int:
    """Stream outputs the residual positions take: one per run."""
    return -(-n_resid // RESID_RUN)


def draw_permutations(N: int, L: int, seed: int, n_resid: int = 0):
    """Random scaling sigma (odd, so invertible mod N = 2^m) and shift tau per
    bucketization, drawn in the order sigma_0, tau_0, sigma_1, tau_1, ...;
    then the ``n_resid`` residual-check time positions from the same stream, in
    runs: draw j gives the run start s_j = (draw & (N-1)) rounded down to a
    multiple of RESID_RUN, and the positions are s_j, s_j + 1, ..., the first
    n_resid of them in run order.

    The voting framework uses random frequency scaling per bucketization
    (voting-framework section); the random shift makes the phase of Eq.(9)
    random as well. The paper fixes no positions for the formula-method check
    (Eq.(2)); runs of consecutive samples are one valid choice.
    """
    nr = resid_draws(n_resid)
    draws = splitmix64(seed, 2 * L + nr)
    sigma = np.array([(draws[2 * r] & (N - 1)) | 1 for r in range(L)], dtype=np.int64)
    tau = np.array([draws[2 * r + 1] & (N - 1) for r in range(L)], dtype=np.int64)
    starts = [(draws[2 * L + j] & (N - 1)) & ~(RESID_RUN - 1) for j in range(nr)]
    tpos = np.array([starts[j // RESID_RUN] + j % RESID_RUN for j in range(n_resid)], dtype=np.int64)
    return sigma, tau, tpos


def draw_comb_shifts(N: int, L: int, seed: int, n_resid: int, n_comb: int) -> np.ndarray:
    """Time shifts of the comb (spike-train) prefilter loops: the next ``n_comb``
    outputs of the same SplitMix64 stream, after the 2L permutation draws and
    the residual positions' draws."""
    base = 2 * L + resid_draws(n_resid)
    draws = splitmix64(seed, base + n_comb)
    return np.array([draws[base + c] & (N - 1) for c in range(n_comb)], dtype=np.int64)


def draw_est_permutations(N: int, L: int, seed: int, n_resid: int, n_comb: int, L_est: int):
    """Scalings and shifts of the estimation-only loops: the next 2 L_est outputs
    of the same SplitMix64 stream (sigma, tau alternating), after the permutation
    draws, the residual positions and the comb shifts."""
    base = 2 * L + resid_draws(n_resid) + n_comb
    draws = splitmix64(seed, base + 2 * L_est)
    sigma = np.array([(draws[base + 2 * r] & (N - 1)) | 1 for r in range(L_est)], dtype=np.int64)
    tau = np.array([draws[base + 2 * r + 1] & (N - 1) for r in range(L_est)], dtype=np.int64)
    return sigma, tau


def modinv(sigma: int, N: int) -> int:
    """sigma^{-1} mod N (sigma odd, N a power of two)."""
    return pow(int(sigma), -1, int(N))


# ---------------------------------------------------------------------------
# Notation section: DFT with 1/N on the forward transform (Eq.(1)-(2)).
# ---------------------------------------------------------------------------
def dft_bruteforce(x: np.ndarray) -> np.ndarray:
    """O(N^2) evaluation of Eq.(2): xhat_i = (1/N) sum_j x_j w^{ij}, w = e^{-2 pi i/N}."""
    x = np.asarray(x, dtype=np.complex128)
    N = x.shape[0]
    jk = np.outer(np.arange(N), np.arange(N)) % N  # exact integer exponent
    F = np.exp(-2j * np.pi * jk / N) / N
    return F @ x


def dft(x: np.ndarray) -> np.ndarray:
    """Eq.(2) through a library FFT: numpy's forward FFT divided by N."""
    x = np.asarray(x, dtype=np.complex128)
    return np.fft.fft(x) / x.shape[0]


# ---------------------------------------------------------------------------
# Signal operations (Eq.(6)-(8)) as explicit matrices, for small N.
# ---------------------------------------------------------------------------
def shift_matrix(N: int, tau: int) -> np.ndarray:
    """S_tau of Eq.(6): entry 1 where j - tau == k (mod N)."""
    S = np.zeros((N, N))
    for j in range(N):
        S[j, (j - tau) % N] = 1.0
    return S


def scaling_matrix(N: int, sigma: int) -> np.ndarray:
    """P_sigma of Eq.(7): entry 1 where sigma*j == k (mod N)."""
    P = np.zeros((N, N))
    for j in range(N):
        P[j, (sigma * j) % N] = 1.0
    return P


def freqshift_matrix(N: int, b: int) -> np.ndarray:
    """V_b of Eq.(8): diagonal w^{b j}."""
    j = np.arange(N)
    return np.diag(np.exp(-2j * np.pi * ((b * j) % N) / N))


def permute(x: np.ndarray, sigma: int, tau: int) -> np.ndarray:
    """x'_i = x_{(sigma*i + tau) mod N}: scaling then shifting of the time index.
    (Eq.(9) family with no frequency offset; tau here equals -sigma*tau_paper.)"""
    N = x.shape[0]
    i = np.arange(N, dtype=np.int64)
    return x[(sigma * i + tau) % N]


# ---------------------------------------------------------------------------
# Flat filter (flat-filter section, Eq.(12)-(13)).
# ---------------------------------------------------------------------------
def flat_window(w: int, B: int, c_g: float = C_G) -> np.ndarray:
    """g_n for n in [0, w): Gaussian (Eq.(13)) times sinc (Eq.(12)), both centred
    at n = w/2.

    Eq.(12) is printed with its argument garbled; its centre value 1/B fixes the
    reading sinc_B(t) = sin(pi t / B) / (pi t), sinc_B(0) = 1/B (a boxcar of
    width N/B bins in frequency). The Gaussian std is tied to the window length
    by the Fig. 1 example: s = w / (2 c_g).
    """
    n = np.arange(w, dtype=np.float64)
    t = n - w / 2.0
    s = w / (2.0 * c_g)
    gauss = np.exp(-0.5 * (t / s) ** 2)
    sinc = np.empty(w)
    nz = t != 0
    sinc[nz] = np.sin(np.pi * t[nz] / B) / (np.pi * t[nz])
    sinc[~nz] = 1.0 / B
    return gauss * sinc


def gain_table(g: np.ndarray, N: int, B: int) -> np.ndarray:
    """Gtab[o] = sum_n g_n e^{+2 pi i n o / N} for o in [-N/2B, N/2B), as an array
    indexed by o + N/2B; exact FP64 sum with the exponent reduced mod N in integers.

    This is N * ghat_{-o}: the weight with which a frequency sitting o bins away
    from its bucket centre lands in that bucket (convolution theorem Eq.(4),
    composition of a bucket Eq.(14))."""
    M = N // B
    w = g.shape[0]
    out = np.empty(M, dtype=np.complex128)
    n = np.arange(w, dtype=np.int64)
    for k, o in enumerate(range(-M // 2, M // 2)):
        m = (n * o) % N
        out[k] = np.sum(g * np.exp(2j * np.pi * m / N))
    return out


def gain_full(g: np.ndarray, N: int) -> np.ndarray:
    """The flat window's complete response Gw(o) = sum_n g_n e^{+2 pi i n o / N} at
    every offset o, as an array indexed by o mod N: N times the library inverse FFT
    of the window zero-padded to length N. Gtab (gain_table) is its restriction
    to |o| <= N/2B."""
    w = g.shape[0]
    padded = np.zeros(N, dtype=np.complex128)
    padded[:w] = g
    return np.fft.ifft(padded) * N


# ---------------------------------------------------------------------------
# Bucket hash (flat-filter example: bucket = round(f / (N/B)), 64/128 -> 1).
# ---------------------------------------------------------------------------
def bucket_of(p, N: int, B: int):
    """Bucket of permuted frequency p: round-half-up of p/(N/B), taken mod B
    (the top half-bucket wraps to bucket 0)."""
    M = N // B
    return ((np.asarray(p, dtype=np.int64) + M // 2) // M) % B


def offset_in_bucket(p, N: int, B: int):
    """Signed distance o = p - h*(N/B) of permuted frequency p from the centre
    of its bucket h, wrapped into [-N/2B, N/2B)."""
    M = N // B
    p = np.asarray(p, dtype=np.int64)
    h = bucket_of(p, N, B)
    return ((p - h * M + N // 2) % N) - N // 2


# ---------------------------------------------------------------------------
# Stage 1: bucketization through the flat filter.
# ---------------------------------------------------------------------------
def bucketize(x: np.ndarray, g: np.ndarray, sigma: int, tau: int, B: int) -> np.ndarray:
    """One random bucketization.

    y_i = g_i x_{(sigma i + tau) mod N} for i < w (window applied to the
    permuted signal); u_b = sum over i == b (mod B) of y_i (aliasing, Eq.(11));
    uhat = B-point DFT of u without the 1/N factor, so that for an isolated
    frequency f, uhat[h] = Gtab[o] * xhat_f * e^{+2 pi i tau f / N}."""
    N = x.shape[0]
    w = g.shape[0]
    i = np.arange(w, dtype=np.int64)
    y = g * x[(sigma * i + tau) % N]
    u = np.zeros(B, dtype=np.complex128)
    np.add.at(u, i % B, y)
    return np.fft.fft(u)


def select_buckets(uhat: np.ndarray, dK: int):
    """Indices of the dK largest |uhat|^2 (ties -> lower bucket index), sorted,
    and the relative gap between the dK-th and (dK+1)-th energies."""
    E = uhat.real ** 2 + uhat.imag ** 2
    B = E.shape[0]
    order = np.lexsort((np.arange(B), -E))
    J = np.sort(order[:dK])
    if dK < B:
        e_in, e_out = E[order[dK - 1]], E[order[dK]]
        margin = (e_in - e_out) / e_in if e_in > 0 else 0.0
    else:
        margin = math.inf
    return J, float(margin)


# ---------------------------------------------------------------------------
# Spike-train (comb) bucketization: the sFFT2.0 prefilter (Table 1, spike train
# + flat filters). Eq.(15) reads garbled: its example (N=2048, B=128, buckets =
# residues mod 128) needs the spikes every N/B samples, i.e. B samples at stride
# N/B; with that reading Eq.(16) holds exactly.
# ---------------------------------------------------------------------------
def comb_buckets(x: np.ndarray, Bc: int, tau: int) -> np.ndarray:
    """Bc-point DFT of the Bc samples x[tau + j N/Bc]: bucket i holds
    Bc * sum over f = i (mod Bc) of xhat_f e^{+2 pi i tau f / N} (Eq.(16))."""
    N = x.shape[0]
    j = np.arange(Bc, dtype=np.int64)
    return np.fft.fft(x[(tau + j * (N // Bc)) % N])


def comb_mask(x: np.ndarray, Bc: int, taus, keep: int):
    """Residues mod Bc that may hold large coefficients: the union over the comb
    shifts of the ``keep`` largest |comb bucket|^2 (ties -> lower residue).
    Returns the mask and the selection margin of each shift."""
    mask = np.zeros(Bc, dtype=bool)
    margins = []
    for t in taus:
        J, m = select_buckets(comb_buckets(x, Bc, int(t)), keep)
        mask[J] = True
        margins.append(m)
    return mask, margins


# ---------------------------------------------------------------------------
# Stage 2a: location by probability and statistics (voting).
# ---------------------------------------------------------------------------
def vote_counts(J_list, sigma, N: int, B: int) -> np.ndarray:
    """c_f = number of bucketizations r whose selected set J_r holds the bucket
    of sigma_r f, for every frequency f in [0, N)."""
    f = np.arange(N, dtype=np.int64)
    c = np.zeros(N, dtype=np.int64)
    for r, J in enumerate(J_list):
        chosen = np.zeros(B, dtype=bool)
        chosen[np.asarray(J, dtype=np.int64)] = True
        c += chosen[bucket_of((int(sigma[r]) * f) % N, N, B)]
    return c


# ---------------------------------------------------------------------------
# Stage 2a': location by phase encoding (the sFFT3.0 row of Table 1; phase
# encoding method of the location section). Loops come in pairs 2j, 2j+1 with
# the same scaling and shifts tau and tau+1. Here a shift advances the time
# index (y_i = x[sigma i + tau]), so one more sample multiplies a lone
# frequency's bucket value by e^{+2 pi i f/N} and f = angle * N / (2 pi); the
# paper writes the same relation with the opposite sign because its shift
# operator delays and its root of unity is e^{-2 pi i/N}.
# ---------------------------------------------------------------------------
def pair_permutations(sigma, tau, N: int):
    """Loop 2j+1 takes loop 2j's scaling and the next shift: sigma_{2j+1} =
    sigma_{2j}, tau_{2j+1} = tau_{2j} + 1 mod N (the draws of the odd loops are
    replaced)."""
    sigma = np.array(sigma, dtype=np.int64, copy=True)
    tau = np.array(tau, dtype=np.int64, copy=True)
    sigma[1::2] = sigma[0::2]
    tau[1::2] = (tau[0::2] + 1) % N
    return sigma, tau


def decode_phase(u0, u1, N: int):
    """Frequency of a single-ton bucket from its values at shifts tau and tau+1:
    t = angle(u1 conj(u0)) N / (2 pi) (the angle of u1/u0 in (-pi, pi]) and
    f = floor(t + 1/2) mod N. Returns (f, t)."""
    theta = np.angle(np.asarray(u1) * np.conj(np.asarray(u0)))
    t = theta * N / (2.0 * math.pi)
    f = np.floor(t + 0.5).astype(np.int64) % N
    return f, t


def phase_locate(uhat_list, J_list, sigma, N: int, B: int, T: int = 1):
    """Candidates of the phase-encoding location: in pair j every selected
    bucket h of loop 2j decodes a frequency f from loops 2j and 2j+1; it counts
    for f when sigma_{2j} f hashes back to h (a single-ton bucket passes this
    check, a multi-ton one in general does not). Frequencies counted by at
    least T pairs are returned (mask over [0, N)), with every decode as
    (pair, bucket, t, f, passed)."""
    count = np.zeros(N, dtype=np.int64)
    decodes = []
    for j in range(len(uhat_list) // 2):
        h = np.asarray(J_list[2 * j], dtype=np.int64)
        f, t = decode_phase(uhat_list[2 * j][h], uhat_list[2 * j + 1][h], N)
        ok = bucket_of((int(sigma[2 * j]) * f) % N, N, B) == h
        np.add.at(count, f[ok], 1)
        decodes.append((j, h, t, f, ok))
    return count >= T, decodes


def decoding_loops(I, uhat_list, J_list, sigma, N: int, B: int) -> np.ndarray:
    """use[r, k]: loop r belongs to a pair that decodes frequency I[k] (the
    bucket of sigma f is selected in the pair's first loop and decodes to f).
    Phase-encoding location estimates each frequency from these loops only:
    there its bucket is a single-ton."""
    I = np.asarray(I, dtype=np.int64)
    L = len(uhat_list)
    use = np.zeros((L, I.shape[0]), dtype=bool)
    for j in range(L // 2):
        h = bucket_of((int(sigma[2 * j]) * I) % N, N, B)
        chosen = np.zeros(B, dtype=bool)
        chosen[np.asarray(J_list[2 * j], dtype=np.int64)] = True
        f, _ = decode_phase(uhat_list[2 * j][h], uhat_list[2 * j + 1][h], N)
        ok = chosen[h] & (f == I)
        use[2 * j] = ok
        use[2 * j + 1] = ok
    return use


def combine_masked(e: np.ndarray, use: np.ndarray, how: str) -> np.ndarray:
    """Median (or mean) over r of e[r, k] restricted to use[r, k] (at least one)."""
    out = np.empty(e.shape[1], dtype=np.complex128)
    for k in range(e.shape[1]):
        sub = e[use[:, k], k]
        out[k] = median_combine(sub[:, None])[0] if how == "median" else sub.mean()
    return out


# ---------------------------------------------------------------------------
# Stage 2b: estimation by energy concentration, median over bucketizations.
# ---------------------------------------------------------------------------
def loop_estimates(I, uhat_list, sigma, tau, G, N: int, B: int) -> np.ndarray:
    """e[r, k] = uhat_r[h] * e^{-2 pi i (tau_r f mod N)/N} / Gtab[o] for f = I[k]:
    the bucket value divided by the filter gain at the frequency's offset, with
    the shift phase of Eq.(9) removed."""
    M = N // B
    I = np.asarray(I, dtype=np.int64)
    L = len(uhat_list)
    e = np.empty((L, I.shape[0]), dtype=np.complex128)
    for r in range(L):
        p = (int(sigma[r]) * I) % N
        h = bucket_of(p, N, B)
        o = offset_in_bucket(p, N, B)
        phase = np.exp(-2j * np.pi * ((int(tau[r]) * I) % N) / N)
        e[r] = uhat_list[r][h] * phase / G[o + M // 2]
    return e


# ---------------------------------------------------------------------------
# Iterative framework: subtract the recovered coefficients before recovering
# again (frameworks section, iterative framework).
# ---------------------------------------------------------------------------
def subtract_recovered(uhat_r: np.ndarray, f_list, v_list, sigma_r: int, tau_r: int, Gfull: np.ndarray,
                       N: int, B: int) -> np.ndarray:
    """Loop r's bucket values with the recovered coefficients removed. A lone
    coefficient v at frequency f puts v e^{+2 pi i tau f/N} Gw(sigma f - h N/B) into
    every bucket h (Eq.(9) for the permuted spectrum, the window's response
    Gw = gain_full for the filter); that whole contribution is subtracted from
    all B buckets, for each recovered (f, v)."""
    M = N // B
    u = np.array(uhat_r, dtype=np.complex128, copy=True)
    centre = np.arange(B, dtype=np.int64) * M
    for f, v in zip(np.asarray(f_list, dtype=np.int64), np.asarray(v_list, dtype=np.complex128)):
        p = (int(sigma_r) * int(f)) % N
        ph = np.exp(2j * np.pi * ((int(tau_r) * int(f)) % N) / N)
        u -= v * ph * Gfull[(p - centre) % N]
    return u


def median_combine(e: np.ndarray) -> np.ndarray:
    """Coordinate-wise median over bucketizations (mean of the two middle values
    when the count is even)."""
    return np.median(e.real, axis=0) + 1j * np.median(e.imag, axis=0)


def mean_combine(e: np.ndarray) -> np.ndarray:
    """Average of the estimates over bucketizations (the averaging the
    energy-concentration method describes)."""
    return e.mean(axis=0)


def finalize(I, v, K: int):
    """K candidates of largest |v|^2 (ties -> lower frequency), ascending by
    frequency, padded with (-1, 0) when fewer than K candidates exist.
    Also returns the relative gap between the K-th and (K+1)-th |v|^2."""
    I = np.asarray(I, dtype=np.int64)
    mag = v.real ** 2 + v.imag ** 2
    order = np.lexsort((I, -mag))
    top = order[:K]
    sel = np.argsort(I[top], kind="stable")
    idx = np.full(K, -1, dtype=np.int64)
    val = np.zeros(K, dtype=np.complex128)
    n = top.shape[0]
    idx[:n] = I[top][sel]
    val[:n] = v[top][sel]
    if I.shape[0] > K:
        a, b = mag[order[K - 1]], mag[order[K]]
        margin = (a - b) / a if a > 0 else 0.0
    else:
        margin = math.inf
    return idx, val, float(margin)


# ---------------------------------------------------------------------------
# Formula method (Eq.(2) inverted for the K known frequencies): residual energy.
# ---------------------------------------------------------------------------
def residual_energy(x: np.ndarray, idx, val, tpos):
    """(E_res, E_in) over time positions tpos:
    E_res = mean_t |x_t - sum_k v_k e^{+2 pi i (t f_k mod N)/N}|^2,
    E_in = mean_t |x_t|^2. Padding entries (idx < 0) are ignored."""
    x = np.asarray(x, dtype=np.complex128)
    N = x.shape[0]
    idx = np.asarray(idx, dtype=np.int64)
    val = np.asarray(val, dtype=np.complex128)
    keep = idx >= 0
    f, v = idx[keep], val[keep]
    t = np.asarray(tpos, dtype=np.int64)
    xt = x[t]
    if f.shape[0]:
        m = np.outer(t, f) % N
        model = (np.exp(2j * np.pi * m / N) * v[None, :]).sum(axis=1)
    else:
        model = np.zeros_like(xt)
    d = xt - model
    e_res = float(np.mean(d.real ** 2 + d.imag ** 2))
    e_in = float(np.mean(xt.real ** 2 + xt.imag ** 2))
    return e_res, e_in


# ---------------------------------------------------------------------------
# The whole path.
# ---------------------------------------------------------------------------
@dataclass
class OracleResult:
    idx: np.ndarray                  # int64[K], ascending, -1 padded
    val: np.ndarray                  # complex128[K], 0 padded
    e_res: float = 0.0
    e_in: float = 0.0
    trace: dict = field(default_factory=dict)


def check_params(N, K, B, L, w, d=2):
    def pow2(v):
        return v > 0 and (v & (v - 1)) == 0
    if not (pow2(N) and 16 <= N <= (1 << 30)):
        raise ValueError("N must be a power of two in [16, 2^30]")
    if not (pow2(B) and 2 <= B and N // B >= 2):
        raise ValueError("B must be a power of two with N/B >= 2")
    if not (K >= 1 and 1 <= d * K <= B):
        raise ValueError("need 1 <= d*K <= B")
    if not (1 <= L <= 32):
        raise ValueError("L must be in [1, 32]")
    if not (2 <= w <= N and w % 2 == 0):
        raise ValueError("w must be even and in [2, N]")


def sfft(x, K: int, B: int, L: int, w: int, seed: int = 0, d: int = 2,
         T: int | None = None, c_g: float = C_G, sigma=None, tau=None,
         n_resid: int = 4096, tpos=None, combine: str = "median",
         comb_b: int = 0, comb_loops: int = 0, comb_keep: int = 0, iterate: bool = False,
         location: str = "vote", est_loops: int = 0, est_B: int = 0, est_w: int = 0) -> OracleResult:
    """Flat-window voting sFFT of signal x (length N = 2^m), FP64 throughout.
    combine: "median" (coordinate-wise, default) or "mean" of the loop estimates.
    comb_loops > 0 adds the comb prefilter: a frequency is a candidate only if
    its residue mod comb_b is among the comb_keep (default d*K) largest comb
    buckets of some comb shift.
    iterate=True adds one round of the iterative framework: the K recovered
    coefficients are subtracted from every loop's buckets, the residual buckets
    are selected and voted again (frequencies already recovered excluded),
    new candidates are estimated from the residual, the recovered ones are
    corrected by the median residual estimate, and the K largest are returned.
    location="phase" locates by phase encoding instead of voting: L is even,
    loops 2j and 2j+1 share a scaling with shifts tau and tau+1, each selected
    bucket of loop 2j decodes one frequency, and T (default 1) is the number of
    pairs that must decode it; a located frequency is estimated from the loops
    of the pairs that decoded it, and with iterate=True the recovered values
    are kept while the residual is decoded for new frequencies.
    est_loops > 0 adds loops that only estimate (location and estimation loops
    separated): est_loops more random bucketizations with est_B buckets and a
    flat window of est_w samples (default w est_B / B); every located frequency
    is estimated by the median (or mean) over all L + est_loops loops."""
    x = np.asarray(x, dtype=np.complex128)
    N = x.shape[0]
    check_params(N, K, B, L, w, d)
    phase = location == "phase"
    if location not in ("vote", "phase"):
        raise ValueError("location must be 'vote' or 'phase'")
    if phase and L % 2:
        raise ValueError("phase-encoding location needs an even number of loops")
    if T is None:
        T = 1 if phase else L // 2 + 1       # one decoding pair / strict majority of the L votes
    if sigma is None:
        sigma, tau, tp = draw_permutations(N, L, seed, n_resid)
        if tpos is None:
            tpos = tp
    sigma = np.asarray(sigma, dtype=np.int64)
    tau = np.asarray(tau, dtype=np.int64)
    if phase:
        sigma, tau = pair_permutations(sigma, tau, N)
    if tpos is None:
        tpos = np.zeros(0, dtype=np.int64)
    sigma_inv = np.array([modinv(s, N) for s in sigma], dtype=np.int64)

    g = flat_window(w, B, c_g)
    G = gain_table(g, N, B)
    uhat = [bucketize(x, g, int(sigma[r]), int(tau[r]), B) for r in range(L)]
    sel = [select_buckets(u, d * K) for u in uhat]
    J = [s[0] for s in sel]
    decodes = None
    if phase:
        voted, decodes = phase_locate(uhat, J, sigma, N, B, T)
        counts = None
    else:
        counts = vote_counts(J, sigma, N, B)
        voted = counts >= T
    cmask, cmargins, ctaus = None, [], np.zeros(0, dtype=np.int64)
    if comb_loops:
        ctaus = draw_comb_shifts(N, L, seed, n_resid, comb_loops)
        cmask, cmargins = comb_mask(x, comb_b, ctaus, comb_keep or d * K)
        voted &= cmask[np.arange(N, dtype=np.int64) % comb_b]
    I = np.nonzero(voted)[0].astype(np.int64)
    e = loop_estimates(I, uhat, sigma, tau, G, N, B)
    est = {}
    if est_loops:
        if phase or iterate:
            raise ValueError("estimation-only loops combine with voting location and one round only")
        Bx = est_B
        wx = est_w or w * Bx // B
        check_params(N, K, Bx, est_loops, wx, 1)
        sx, tx = draw_est_permutations(N, L, seed, n_resid, comb_loops, est_loops)
        gx = flat_window(wx, Bx, c_g)
        Gx = gain_table(gx, N, Bx)
        ux = [bucketize(x, gx, int(sx[r]), int(tx[r]), Bx) for r in range(est_loops)]
        e = np.vstack([e, loop_estimates(I, ux, sx, tx, Gx, N, Bx)])
        est = dict(est_sigma=sx, est_tau=tx, est_uhat=ux)
    comb = {"median": median_combine, "mean": mean_combine}[combine]
    use = None
    if phase:
        use = decoding_loops(I, uhat, J, sigma, N, B)
        v = combine_masked(e, use, combine)
    else:
        v = comb(e) if I.shape[0] else np.zeros(0, dtype=np.complex128)
    idx, val, fmargin = finalize(I, v, K)
    it = {}
    if iterate:
        keep1 = idx >= 0
        K1, V1 = idx[keep1], val[keep1]
        Gf = gain_full(g, N)
        ures = [subtract_recovered(uhat[r], K1, V1, int(sigma[r]), int(tau[r]), Gf, N, B) for r in range(L)]
        sel2 = [select_buckets(u, d * K) for u in ures]
        J2 = [s[0] for s in sel2]
        decodes2 = None
        if phase:
            voted2, decodes2 = phase_locate(ures, J2, sigma, N, B, T)
        else:
            voted2 = vote_counts(J2, sigma, N, B) >= T
        if cmask is not None:
            voted2 &= cmask[np.arange(N, dtype=np.int64) % comb_b]
        voted2[K1] = False
        I2 = np.nonzero(voted2)[0].astype(np.int64)
        e2 = loop_estimates(I2, ures, sigma, tau, G, N, B)
        eK = loop_estimates(K1, ures, sigma, tau, G, N, B)
        use2 = None
        if phase:
            # new frequencies from the pairs that decode them in the residual; the
            # recovered values (single-ton estimates) are kept
            use2 = decoding_loops(I2, ures, J2, sigma, N, B)
            v2 = combine_masked(e2, use2, combine)
            vK = V1
        else:
            v2 = comb(e2) if I2.shape[0] else np.zeros(0, dtype=np.complex128)
            vK = V1 + (comb(eK) if K1.shape[0] else 0)
        Iall, vall = np.concatenate([I2, K1]), np.concatenate([v2, vK])
        it = dict(idx1=idx, val1=val, final_margin1=fmargin, ures=ures, J2=J2,
                  select_margin2=[s[1] for s in sel2], I2=I2, e2=e2, eK=eK, decodes2=decodes2,
                  I_all2=Iall, v_all2=vall, use2=use2)
        idx, val, fmargin = finalize(Iall, vall, K)
    e_res, e_in = residual_energy(x, idx, val, tpos) if len(tpos) else (0.0, 0.0)
    trace = dict(sigma=sigma, tau=tau, sigma_inv=sigma_inv, g=g, G=G, uhat=uhat,
                 J=J, select_margin=[s[1] for s in sel], counts=counts, I=I,
                 e=e, v=v, final_margin=fmargin, T=T, tpos=np.asarray(tpos), decodes=decodes, use=use,
                 comb_mask=cmask, comb_margin=cmargins, comb_tau=ctaus, **it, **est)
    return OracleResult(idx=idx, val=val, e_res=e_res, e_in=e_in, trace=trace)


# ---------------------------------------------------------------------------
# Error metrics of the experimental platform (L0 / L1 / L2 against the best
# K-term approximation) and the approximation factor of Eq.(5).
# ---------------------------------------------------------------------------
def best_k_term(xhat: np.ndarray, K: int):
    """Support and values of the K largest |xhat| (ties -> lower index)."""
    mag = np.abs(xhat)
    order = np.lexsort((np.arange(xhat.shape[0]), -mag))[:K]
    order = np.sort(order)
    return order.astype(np.int64), xhat[order]


def recovery_errors(xhat: np.ndarray, idx, val, K: int) -> dict:
    """L0 = best-support frequencies missed; L1 = (1/K) sum of |error| over the
    union of supports; L2 = l2 error over that union; C = the Eq.(5) ratio
    ||xhat - x'||_2 / ||xhat - yhat||_2 (inf when the best K-term error is 0)."""
    idx = np.asarray(idx, dtype=np.int64)
    val = np.asarray(val, dtype=np.complex128)
    keep = idx >= 0
    idx, val = idx[keep], val[keep]
    bsup, bval = best_k_term(xhat, K)
    rec = dict(zip(idx.tolist(), val.tolist()))
    best = dict(zip(bsup.tolist(), bval.tolist()))
    union = sorted(set(rec) | set(best))
    diffs = np.array([rec.get(f, 0.0) - best.get(f, 0.0) for f in union], dtype=np.complex128)
    L0 = len(set(best) - set(rec))
    L1 = float(np.sum(np.abs(diffs)) / K)
    L2 = float(np.sqrt(np.sum(np.abs(diffs) ** 2)))
    xp = np.zeros_like(xhat)
    xp[idx] = val
    num = float(np.linalg.norm(xhat - xp))
    yp = np.zeros_like(xhat)
    yp[bsup] = bval
    den = float(np.linalg.norm(xhat - yp))
    C = num / den if den > 0 else (0.0 if num == 0 else math.inf)
    return dict(L0=L0, L1=L1, L2=L2, C=C)


def sampled_fraction(N: int, w: int, sigma, tau) -> float:
    """Fraction of the N time samples read by the L bucketizations."""
    hit = np.zeros(N, dtype=bool)
    i = np.arange(w, dtype=np.int64)
    for s, t in zip(sigma, tau):
        hit[(int(s) * i + int(t)) % N] = True
    return float(hit.mean())
