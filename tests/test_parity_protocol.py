"""CPU checks of the parity comparator (tests/parity.py) that the GPU tests use.

A stand-in for a GPU run is made from the oracle's own trace, rounded to the
precision the GPU returns (complex64 bucket spectra and values). The comparator
must accept it and report what it compared; it must reject planted mistakes (a
certain tone swapped out, a value off by 1e-3, a firm bucket dropped, a spurious
candidate); and at a real near-tie (the C1 signal of seed 101, whose 10th and 11th
largest estimates are true unit tones 4e-9 apart) it must accept either choice
and count it.
"""
import copy

import numpy as np
import pytest

import oracle.sfft_oracle as O
from paper_2012_08238_amd.signals import make_signal
from parity import compare, compare_iterate


def _bits(jl, B):
    words = np.zeros((B + 31) // 32, np.uint32)
    for h in jl:
        words[h >> 5] |= np.uint32(1) << np.uint32(h & 31)
    return words


def _as_gpu(r, K, B, L, rnd=True):
    """A GPU-shaped result made from the oracle result r (first round of the trace)."""
    tr = r.trace
    c64 = (lambda a: np.asarray(a).astype(np.complex64).astype(np.complex128)) if rnd else np.asarray
    uh = np.array([c64(u) for u in tr["uhat"]])
    jl = np.array([np.sort(j) for j in tr["J"]], dtype=np.uint32)
    return dict(idx=r.idx.copy(), val=c64(r.val),
                trace=dict(uhat=uh, jlist=jl, jbits=np.array([_bits(j, B) for j in jl]),
                           cand=np.asarray(tr["I"], dtype=np.uint32)),
                perms=(tr["sigma"].astype(np.uint32), tr["sigma_inv"].astype(np.uint32),
                       tr["tau"].astype(np.uint32)))


@pytest.fixture(scope="module")
def c1():
    out = {}
    for seed in (0, 1):
        sig = make_signal(1 << 14, 10, None, seed=100 + seed)
        out[seed] = O.sfft(sig.x.astype(np.complex64).astype(np.complex128), 10, 128, 5, 512, seed=seed,
                           n_resid=0)
    return out


def test_accepts_the_oracle_and_counts(c1):
    p = compare(_as_gpu(c1[0], 10, 128, 5), c1[0], 10, 128, 5)
    assert (p.certain, p.band, p.values, p.loops, p.loops_tied) == (10, 0, 10, 5, 0)
    assert p.cand_equal and p.support_equal and not p.ambiguous


def test_near_tie_either_choice(c1):
    r = c1[1]
    assert r.trace["final_margin"] < 1e-6
    g = _as_gpu(r, 10, 128, 5)
    p = compare(g, r, 10, 128, 5)
    assert p.certain == 1 and p.band == 9 and p.values == 10
    # the other tone of the tie: (K+1)-th in place of the K-th
    v, I = r.trace["v"], r.trace["I"]
    mag = np.abs(v) ** 2
    order = np.lexsort((I, -mag))
    kth, nxt = int(I[order[9]]), int(I[order[10]])
    idx = np.sort(np.array([f for f in r.idx if f != kth] + [nxt]))
    pos = {int(f): k for k, f in enumerate(I)}
    g2 = copy.deepcopy(g)
    g2["idx"] = idx
    g2["val"] = np.array([v[pos[int(f)]] for f in idx]).astype(np.complex64).astype(np.complex128)
    p2 = compare(g2, r, 10, 128, 5)
    assert p2.certain == 1 and p2.band == 9 and not p2.support_equal


def test_rejects_swapped_certain_tone(c1):
    r = c1[0]
    g = _as_gpu(r, 10, 128, 5)
    v, I = r.trace["v"], r.trace["I"]
    out = int(I[np.lexsort((I, -np.abs(v) ** 2))[10]])
    g["idx"] = np.sort(np.concatenate([r.idx[1:], [out]]))
    pos = {int(f): k for k, f in enumerate(I)}
    g["val"] = np.array([v[pos[int(f)]] for f in g["idx"]])
    with pytest.raises(AssertionError):
        compare(g, r, 10, 128, 5)


def test_rejects_value_error(c1):
    g = _as_gpu(c1[0], 10, 128, 5)
    g["val"][3] *= 1 + 1e-3
    with pytest.raises(AssertionError, match="value"):
        compare(g, c1[0], 10, 128, 5)


def test_rejects_dropped_firm_bucket(c1):
    r = c1[0]
    g = _as_gpu(r, 10, 128, 5)
    E = np.abs(r.trace["uhat"][2]) ** 2
    top = int(np.argmax(E))
    others = [h for h in range(128) if h not in set(g["trace"]["jlist"][2].tolist())]
    jl = np.sort(np.array([h for h in g["trace"]["jlist"][2] if h != top] + [others[0]], np.uint32))
    g["trace"]["jlist"][2] = jl
    g["trace"]["jbits"][2] = _bits(jl, 128)
    with pytest.raises(AssertionError, match="firmly"):
        compare(g, r, 10, 128, 5)


def test_rejects_spurious_candidate(c1):
    r = c1[0]
    g = _as_gpu(r, 10, 128, 5)
    extra = next(f for f in range(1 << 14) if f not in set(r.trace["I"].tolist()))
    g["trace"]["cand"] = np.append(g["trace"]["cand"], np.uint32(extra))
    with pytest.raises(AssertionError, match="vote for"):
        compare(g, r, 10, 128, 5)


def test_rejects_uhat_error(c1):
    g = _as_gpu(c1[0], 10, 128, 5)
    g["trace"]["uhat"][1][7] += 1e-3 * np.max(np.abs(g["trace"]["uhat"][1]))
    with pytest.raises(AssertionError, match="spectra"):
        compare(g, c1[0], 10, 128, 5)


def test_iterate_accepts_the_oracle_and_rejects_wrong_subtraction():
    N, K, B, L, w = 1 << 14, 10, 128, 5, 256     # w = 2B: the response spans several buckets
    sig = make_signal(N, K, 20.0, seed=5)
    x = sig.x.astype(np.complex64).astype(np.complex128)
    r = O.sfft(x, K, B, L, w, seed=3, n_resid=0, iterate=True)
    tr = r.trace
    plain = _as_gpu(O.sfft(x, K, B, L, w, seed=3, n_resid=0), K, B, L)
    c64 = lambda a: np.asarray(a).astype(np.complex64).astype(np.complex128)  # noqa: E731
    n1 = int(np.sum(tr["idx1"] >= 0))
    jl2 = np.array([np.sort(j) for j in tr["J2"]], dtype=np.uint32)
    g = dict(idx=r.idx.copy(), val=c64(r.val), perms=plain["perms"],
             trace=dict(uhat=np.array([c64(u) for u in tr["ures"]]), jlist=jl2,
                        jbits=np.array([_bits(j, B) for j in jl2]), cand=np.asarray(tr["I2"], np.uint32),
                        rec_idx=tr["idx1"][:n1], rec_val=c64(tr["val1"][:n1])))
    first, second = compare_iterate(g, plain, r, K, B, L)
    assert second is not None and second.values >= 1 and first.values == n1
    # the residual buckets of a neighbours-only subtraction differ beyond the tolerance
    M = N // B
    Gf = O.gain_full(tr["g"], N)
    bad = copy.deepcopy(g)
    for rr in range(L):
        u = np.array(tr["uhat"][rr], dtype=np.complex128)
        for f, v in zip(tr["idx1"][:n1], tr["val1"][:n1]):
            p = (int(tr["sigma"][rr]) * int(f)) % N
            h0 = int(O.bucket_of(p, N, B))
            ph = np.exp(2j * np.pi * ((int(tr["tau"][rr]) * int(f)) % N) / N)
            for j in (-1, 0, 1):
                h = (h0 + j) % B
                u[h] -= v * ph * Gf[(p - h * M) % N]
        bad["trace"]["uhat"][rr] = c64(u)
    with pytest.raises(AssertionError, match="residual buckets"):
        compare_iterate(bad, plain, r, K, B, L)
