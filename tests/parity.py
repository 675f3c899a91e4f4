"""Parity protocol of the HIP path against the FP64 oracle (test infrastructure).

Every decision the two sides take is compared exactly where the oracle's
decision is not a near-tie at the precision the GPU works in. Where it is one,
the GPU's choice must be one that the tie allows, and the case is counted, never
dropped:

- Bucket spectra agree within UHAT_TOL of the loop's largest bucket. The measured
  difference delta_r of loop r bounds how far each GPU energy |u|^2 can lie from
  the oracle's.
- Selected buckets. Buckets whose oracle energy clears the d*K-boundary by more
  than that bound are "firm": a firm bucket must be selected, and a firmly excluded
  one must not be. The rest of the two selections (symmetric difference) are the
  loop's "loose" buckets; a loop with any loose bucket is counted as tied.
- Candidates. They equal the oracle's when no loop is tied. Otherwise every
  frequency in the symmetric difference must hash, in some tied loop, to a loose
  bucket (or have its residue in a loose comb residue). The GPU's candidates must
  also be exactly the frequencies that its own selections vote for (recounted
  here with plain NumPy).
- Support. The oracle's entries whose |v|^2 clears the largest excluded one (the
  (K+1)-th) by more than FINAL_MARGIN relative are "certain". Each must be in the
  GPU's support, unless the GPU lacks it as a candidate (explained) or a candidate
  only the GPU has took its place (counted). Entries more than FINAL_MARGIN below
  the K-th are out and must not be in it. The remaining slots are filled from the
  tie band between the two (counted). So the certain prefix and the validity of
  every choice are checked even when the K-th and (K+1)-th are a near-tie.
- Values of every frequency in both the GPU's support and the oracle's candidates
  agree within VAL_RTOL relative. Two counted exceptions remain. Median
  cancellation: |v_ref| < 1e-3 of the median |e_r| over the loops (ill-conditioned).
  Leakage level: the error is within the propagated bound of the measured bucket
  differences (sqrt2 max_r delta_r / min |Gtab|; the coordinate-wise median and the
  mean move by at most their inputs' largest change), and that bound is above
  VAL_RTOL |v_ref|.

compare() returns a Parity record. It asserts that something was compared: at least
one certain entry and one value, unless the oracle returns nothing.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

VAL_RTOL = 1e-4           # values, relative
UHAT_TOL = 1e-5           # bucket spectra, relative to the loop's largest |u|
FINAL_MARGIN = 1e-3       # relative |v|^2 gap that makes a support entry certain

RECORDS = []              # (test id, Parity) of every comparison, reported at the end of the run


def record(p):
    import os
    RECORDS.append((os.environ.get("PYTEST_CURRENT_TEST", "?").split(" ")[0], p))
    return p


@dataclass
class Parity:
    loops: int = 0                 # loops whose spectra and selections were compared
    loops_tied: int = 0            # of them, loops whose selection differs inside the tie band
    cand_equal: bool = True        # candidate sets equal
    cand_explained: int = 0        # candidates in the symmetric difference (each explained)
    certain: int = 0               # certain support entries found in the GPU's support
    certain_displaced: int = 0     # certain entries displaced by a GPU-only candidate
    certain_uncandidate: int = 0   # certain entries that are no GPU candidate (explained)
    band: int = 0                  # support entries chosen from the tie band at the K-boundary
    support_equal: bool = False    # whole supports equal
    values: int = 0                # values compared within VAL_RTOL
    values_ill: int = 0            # values excused by median cancellation
    values_leak: int = 0           # values within the propagated bucket-difference bound only
    values_tied: int = 0           # values not compared: the loops that estimate them are a near-tie
    skipped: str = ""              # why a round was not comparable (empty: compared)

    @property
    def ambiguous(self) -> bool:
        return bool(self.skipped or self.loops_tied or not self.cand_equal or not self.support_equal)


def hash_buckets(f, sigma: int, N: int, B: int):
    """Bucket of frequency f in a loop with scaling sigma (round half up, top wraps)."""
    M = N // B
    return ((((sigma * np.asarray(f, dtype=np.int64)) % N) + M // 2) // M) % B


def energy_band(E, delta):
    """Largest change of |u|^2 when u moves by delta, plus FP32 rounding of the square."""
    return 4.0 * np.sqrt(E) * delta + 4.0 * delta * delta + 1e-6 * E


def selection_check(jl, E, dK, delta):
    """jl: the GPU's selected buckets, E: the oracle's energies. Asserts the firm
    decisions and returns the loose buckets (symmetric difference)."""
    B = E.shape[0]
    if dK >= B:
        assert np.array_equal(np.sort(jl), np.arange(B)), "every bucket is selected when d*K = B"
        return set()
    e = np.sort(E)[::-1]
    a, b = e[dK - 1], e[dK]
    firm_in = E - energy_band(E, delta) > b + energy_band(b, delta)
    firm_out = E + energy_band(E, delta) < a - energy_band(a, delta)
    js = set(int(h) for h in jl)
    missing = [h for h in np.nonzero(firm_in)[0].tolist() if h not in js]
    assert not missing, f"firmly selected buckets not selected: {missing[:8]}"
    wrong = [h for h in js if firm_out[h]]
    assert not wrong, f"firmly excluded buckets selected: {wrong[:8]}"
    ref = set(np.lexsort((np.arange(B), -E))[:dK].tolist())
    return js ^ ref


def voted_frequencies(jlists, sigma, N: int, B: int, T: int, comb_mask=None, exclude=None):
    """Frequencies with at least T votes from the given selections (plain NumPy),
    restricted to residues the comb mask keeps; excluded frequencies removed."""
    f = np.arange(N, dtype=np.int64)
    votes = np.zeros(N, dtype=np.int32)
    for r, jl in enumerate(jlists):
        sel = np.zeros(B, dtype=bool)
        sel[np.asarray(jl, dtype=np.int64)] = True
        votes += sel[hash_buckets(f, int(sigma[r]), N, B)]
    ok = votes >= T
    if comb_mask is not None:
        ok &= comb_mask[f % comb_mask.shape[0]]
    if exclude is not None and len(exclude):
        ok[np.asarray(exclude, dtype=np.int64)] = False
    return np.nonzero(ok)[0]


def bitmap_rows(bits, nbits: int):
    return np.array([(bits[h >> 5] >> (h & 31)) & 1 for h in range(nbits)], dtype=bool)


def support_and_values(p: Parity, idx_g, val_g, I_ref, v_ref, e_ref, K: int, gpu_only, uncandidate,
                       delta_v: float, value_tied=frozenset()):
    """Support comparison around the K-boundary and value comparison (see the module
    text). I_ref, v_ref: the oracle's candidates and their estimates; e_ref: the
    per-loop estimates [loops][candidates] (NaN where a loop does not estimate the
    candidate); gpu_only: candidates only the GPU has;
    uncandidate: oracle candidates the GPU does not have (explained by ties);
    delta_v: the leakage bound of a value; value_tied: frequencies whose estimate may
    legitimately differ (phase location: a pair's decode is a near-tie), counted only.
    Returns the certain entries."""
    I_ref = np.asarray(I_ref, dtype=np.int64)
    ok = idx_g >= 0
    assert np.all(val_g[~ok] == 0) and np.all(idx_g[~ok] == -1), "padding"
    S_g = idx_g[ok]
    assert np.all(np.diff(S_g) > 0), "support not ascending"
    pos = {int(f): k for k, f in enumerate(I_ref.tolist())}
    mag = v_ref.real ** 2 + v_ref.imag ** 2
    order = np.lexsort((I_ref, -mag))
    top = order[:K]
    m = FINAL_MARGIN
    b = mag[order[K]] if I_ref.shape[0] > K else 0.0      # largest excluded |v|^2
    aK = mag[order[K - 1]] if I_ref.shape[0] >= K else 0.0  # K-th largest |v|^2
    # certain: clears the largest excluded entry; out: firmly below the K-th; the rest is
    # the tie band around the boundary, from which the remaining slots may be filled
    certain = [int(I_ref[k]) for k in top if mag[k] - b > m * mag[k]]
    out = {int(I_ref[k]) for k in range(I_ref.shape[0]) if aK - mag[k] > m * aK}
    sg = set(int(f) for f in S_g)
    displaced_allowed = len(sg & set(int(f) for f in gpu_only))
    for f in certain:
        if f in sg:
            p.certain += 1
        elif f in uncandidate:
            p.certain_uncandidate += 1
        else:
            p.certain_displaced += 1
    assert p.certain_displaced <= displaced_allowed, \
        f"{p.certain_displaced} certain entries missing from the support, {displaced_allowed} GPU-only candidates in it"
    # entries firmly below the K-th only in place of oracle top-K entries the GPU does not have
    low = sorted(f for f in sg if f in out)
    lost = sum(1 for k in top if int(I_ref[k]) in uncandidate)
    assert len(low) <= lost, f"frequencies firmly below the K-th entry in the support: {low[:8]}"
    cs = set(certain)
    p.band = sum(1 for f in sg if f in pos and f not in cs and f not in out)
    n_cand = len(set(I_ref.tolist()) - uncandidate) + len(gpu_only)
    assert S_g.shape[0] == min(K, n_cand), f"support size {S_g.shape[0]}, candidates {n_cand}"
    ref_support = np.sort(I_ref[top])
    p.support_equal = np.array_equal(S_g, ref_support)
    # values
    for f, v in zip(S_g.tolist(), val_g[ok].tolist()):
        if f not in pos:
            continue
        if f in value_tied:
            p.values_tied += 1
            continue
        k = pos[f]
        vr = complex(v_ref[k])
        err = abs(v - vr)
        if err <= VAL_RTOL * abs(vr):
            p.values += 1
            continue
        m_f = float(np.nanmedian(np.abs(e_ref[:, k])))
        if abs(vr) < 1e-3 * m_f:
            p.values_ill += 1
        elif err <= delta_v:
            p.values_leak += 1
        else:
            raise AssertionError(f"value of {f}: rel err {err / abs(vr):.2e} (bound {delta_v:.2e} abs)")
    return certain


def compare(g, r, K: int, B: int, L: int, w: int = 0, seed: int = 0, cand_exact: bool = True,
            comb_b: int = 0, min_certain: int = 1) -> Parity:
    """Voting path: the GPU run g (outputs, trace, perms) against the oracle result r.
    cand_exact=False when a comb prefilter's selection was a rounding-level tie."""
    tr = r.trace
    N = int(tr["counts"].shape[0])
    p = Parity()
    sigma, sigma_inv, tau = g["perms"]
    assert np.array_equal(sigma, tr["sigma"].astype(np.uint32)), "sigma"
    assert np.array_equal(tau, tr["tau"].astype(np.uint32)), "tau"
    assert np.array_equal(sigma_inv, tr["sigma_inv"].astype(np.uint32)), "sigma^-1"
    uh = g["trace"]["uhat"]
    dK = len(tr["J"][0])
    loose = []
    delta_max = 0.0
    jl_g = []
    for rr in range(L):
        ref = tr["uhat"][rr]
        scale = max(float(np.max(np.abs(ref))), 1e-30)
        err = float(np.max(np.abs(uh[rr] - ref)))
        assert err <= UHAT_TOL * scale, f"loop {rr} bucket spectra: {err / scale:.2e}"
        delta = max(err, 1e-7 * scale)
        delta_max = max(delta_max, delta)
        jl = np.sort(g["trace"]["jlist"][rr])
        assert len(np.unique(jl)) == jl.shape[0], "duplicate selected buckets"
        assert np.array_equal(np.nonzero(bitmap_rows(g["trace"]["jbits"][rr], B))[0], jl), "bitmap and list disagree"
        lz = selection_check(jl, np.abs(ref) ** 2, dK, delta)
        loose.append(lz)
        jl_g.append(jl)
        p.loops += 1
        p.loops_tied += bool(lz)
    # candidates: valid for the GPU's own selections, and equal to the oracle's up to ties
    cand = np.sort(g["trace"]["cand"].astype(np.int64))
    assert len(np.unique(cand)) == cand.shape[0], "duplicate candidates"
    cmask_g = None
    comb_loose = set()
    if comb_b:
        rows = np.asarray(g["trace"]["comb_rows"], dtype=bool)
        cmask_g = rows.any(axis=0)
        comb_loose = set(np.nonzero(cmask_g ^ tr["comb_mask"])[0].tolist())
    want = voted_frequencies(jl_g, sigma, N, B, int(tr["T"]), cmask_g)
    assert np.array_equal(cand, want), "candidates are not the frequencies the GPU's selections vote for"
    I_ref = np.asarray(tr["I"], dtype=np.int64)
    diff = set(cand.tolist()) ^ set(I_ref.tolist())
    p.cand_equal = not diff
    if diff:
        assert p.loops_tied or comb_loose or not cand_exact, "candidate sets differ with no tied selection"
        for f in diff:
            ok = any(int(hash_buckets(f, int(sigma[rr]), N, B)) in loose[rr] for rr in range(L))
            ok = ok or (comb_b and f % comb_b in comb_loose)
            assert ok, f"candidate {f} differs without a tied bucket"
        p.cand_explained = len(diff)
    uncandidate = set(I_ref.tolist()) - set(cand.tolist())
    gpu_only = set(cand.tolist()) - set(I_ref.tolist())
    # leakage bound of a value: the largest measured bucket difference over the smallest gain
    # (the estimation-only loops' buckets are not read back; their values must meet VAL_RTOL)
    delta_v = 1.5 * np.sqrt(2.0) * delta_max / float(np.min(np.abs(tr["G"])))
    certain = support_and_values(p, g["idx"], g["val"], I_ref, tr["v"], tr["e"], K, gpu_only, uncandidate,
                                 delta_v)
    if I_ref.shape[0]:
        assert len(certain) >= min_certain or p.loops_tied, f"only {len(certain)} certain entries"
        assert p.certain + p.certain_uncandidate + p.certain_displaced == len(certain)
        assert p.values + p.values_ill + p.values_leak >= 1, "no value compared"
    if p.cand_equal and tr["final_margin"] > FINAL_MARGIN:
        assert p.support_equal, "recovered support"
    return record(p)


RES_TOL = 1e-4   # residual buckets: the subtracted contributions carry the first round's value error


class _FirstRound:
    """The oracle's first round of an iterating run, as a result of its own."""

    def __init__(self, r):
        self.trace = dict(r.trace, final_margin=r.trace["final_margin1"])
        self.idx, self.val = r.trace["idx1"], r.trace["val1"]


def compare_iterate(g, plain, r, K: int, B: int, L: int, comb_b: int = 0):
    """Voting path with the subtraction round. g: the GPU run with the round, plain: the
    same plan without it, r: the oracle with iterate=True. Returns (first, second): the
    Parity of each round; second is None when the first rounds' supports differ inside
    the tie band (the residual buckets then differ by whole coefficients)."""
    tr = r.trace
    N = int(tr["counts"].shape[0])
    first = compare(plain, _FirstRound(r), K, B, L, comb_b=comb_b)
    n1 = int(np.sum(plain["idx"] >= 0))
    assert np.array_equal(g["trace"]["rec_idx"], plain["idx"][:n1]), "first round differs from the plain plan"
    assert np.array_equal(g["trace"]["rec_val"].astype(np.complex64), plain["val"][:n1].astype(np.complex64))
    K1 = tr["idx1"][tr["idx1"] >= 0]
    if not np.array_equal(g["trace"]["rec_idx"], K1):
        assert first.ambiguous, "first-round supports differ with no tie"
        record(Parity(skipped="first-round supports differ"))
        return first, None
    p = Parity()
    sigma = g["perms"][0]
    dK = len(tr["J2"][0])
    loose, jl_g, delta_max = [], [], 0.0
    for rr in range(L):
        scale = max(float(np.max(np.abs(tr["uhat"][rr]))), 1e-30)
        err = float(np.max(np.abs(g["trace"]["uhat"][rr] - tr["ures"][rr])))
        assert err <= RES_TOL * scale, f"loop {rr} residual buckets: {err / scale:.2e}"
        delta = max(err, 1e-7 * scale)
        delta_max = max(delta_max, delta)
        jl = np.sort(g["trace"]["jlist"][rr])
        assert np.array_equal(np.nonzero(bitmap_rows(g["trace"]["jbits"][rr], B))[0], jl), "bitmap and list disagree"
        lz = selection_check(jl, np.abs(tr["ures"][rr]) ** 2, dK, delta)
        loose.append(lz)
        jl_g.append(jl)
        p.loops += 1
        p.loops_tied += bool(lz)
    cand = np.sort(g["trace"]["cand"].astype(np.int64))
    assert len(np.unique(cand)) == cand.shape[0], "duplicate candidates"
    cmask_g = None
    if comb_b:
        cmask_g = np.asarray(g["trace"]["comb_rows"], dtype=bool).any(axis=0)
    want = voted_frequencies(jl_g, sigma, N, B, int(tr["T"]), cmask_g, exclude=K1)
    assert np.array_equal(cand, want), "second-round candidates are not those the GPU's selections vote for"
    I2 = np.asarray(tr["I2"], dtype=np.int64)
    diff = set(cand.tolist()) ^ set(I2.tolist())
    p.cand_equal = not diff
    for f in diff:
        assert any(int(hash_buckets(f, int(sigma[rr]), N, B)) in loose[rr] for rr in range(L)), \
            f"second-round candidate {f} differs without a tied bucket"
    p.cand_explained = len(diff)
    uncandidate = set(I2.tolist()) - set(cand.tolist())
    gpu_only = set(cand.tolist()) - set(I2.tolist())
    # per-loop estimates of every final candidate: the new ones', and the recovered values
    # plus their residual estimates
    V1 = tr["val1"][tr["idx1"] >= 0]
    e_all = np.hstack([tr["e2"], tr["eK"] + V1[None, :]])
    rec_err = float(np.max(np.abs(g["trace"]["rec_val"] - V1))) if V1.shape[0] else 0.0
    delta_v = 1.5 * np.sqrt(2.0) * delta_max / float(np.min(np.abs(tr["G"]))) + rec_err
    support_and_values(p, g["idx"], g["val"], tr["I_all2"], tr["v_all2"], e_all, K, gpu_only, uncandidate,
                       delta_v)
    if p.cand_equal and tr["final_margin"] > FINAL_MARGIN:
        assert p.support_equal, "final support"
    assert p.values + p.values_ill + p.values_leak >= 1 or not np.any(g["idx"] >= 0), "no value compared"
    return first, record(p)
