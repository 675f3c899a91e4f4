"""Parity of phase-encoding location (paired loops at shifts tau and tau+1) on
the GPU with the FP64 oracle's sfft(..., location="phase").

Integer results are compared exactly wherever the oracle's decision is
decided beyond the measured difference of the GPU's bucket values: the
selected buckets (energy gap at the boundary), every decode (distance of
t = angle N / 2 pi from the rounding boundary), hence the candidate set and the
support around the K-boundary. Values within 1e-4 relative; a leakage-level value
(one below the propagated bound of the measured bucket differences) is counted.
"""
import math

import numpy as np
import pytest

import oracle.sfft_oracle as O
from paper_2012_08238_amd.signals import make_signal
from parity import FINAL_MARGIN, Parity, record, support_and_values

pytestmark = pytest.mark.gpu

UHAT_TOL = 1e-5


def _run(dev, x64, iterate=False, **kw):
    import torch
    import paper_2012_08238_amd as S
    N = x64.shape[0]
    flags = kw.pop("flags", 0) | S.SFFT_FLAG_PHASE_LOCATION | (S.SFFT_FLAG_ITERATE if iterate else 0)
    p = S.Plan(N, flags=flags, **kw)
    xt = torch.from_numpy(x64.astype(np.complex64)).to(dev)
    idx, val, res = p(xt, residual=True)
    torch.cuda.synchronize()
    out = dict(idx=idx.cpu().numpy(), val=val.cpu().numpy().astype(np.complex128), resid=res.cpu().numpy(),
               trace=p.trace(), perms=p.perms())
    p.close()
    return out


def _sel_robust(E, dK, delta):
    e = np.sort(E)[::-1]
    if dK >= e.shape[0]:
        return True
    a, b = e[dK - 1], e[dK]
    return a - b > 4.0 * np.sqrt(a) * delta + 4.0 * delta * delta


def _firm_selection(E, dK, delta):
    """Buckets whose energy clears the dK-boundary by more than the measured
    difference delta of the values could move it (ranked by the oracle)."""
    e = np.sort(E)[::-1]
    if dK >= e.shape[0]:
        return np.ones(E.shape[0], dtype=bool)
    bnd = e[dK]
    return E - bnd > 4.0 * np.sqrt(E) * delta + 4.0 * delta * delta


def _robust_decode(a, b, t, delta, N):
    """The decode of bucket values (a, b) at t cannot change by a difference delta."""
    if min(abs(a), abs(b)) <= 4.0 * delta:
        return False
    dt = 1.2 * (delta / abs(a) + delta / abs(b)) * N / (2 * math.pi)
    s = t + 0.5
    return abs(s - round(s)) > dt


def compare_phase(g, r, K, B, L, N, iterate=False):
    """Returns the Parity record (support around the K-boundary and values through
    parity.support_and_values; loops_tied counts the pairs with a near-boundary
    selection or decode)."""
    tr = r.trace
    sigma, sigma_inv, tau = g["perms"]
    assert np.array_equal(sigma, tr["sigma"].astype(np.uint32)) and np.array_equal(tau, tr["tau"].astype(np.uint32))
    assert np.all(sigma[1::2] == sigma[0::2]) and np.all(tau[1::2] == (tau[0::2] + 1) % N)
    M = N // B
    if iterate:
        # the recovered set must be the oracle's for the residual round to be comparable
        if not np.array_equal(g["trace"]["rec_idx"], tr["idx1"][tr["idx1"] >= 0]):
            return record(Parity(skipped="first-round supports differ"))
        uh_ref, J_ref, decs, I_ref = tr["ures"], tr["J2"], tr["decodes2"], tr["I2"]
    else:
        uh_ref, J_ref, decs, I_ref = tr["uhat"], tr["J"], tr["decodes"], tr["I"]
    # buckets (and residual buckets) within the measured difference
    delta = 0.0
    for rr in range(L):
        scale = max(np.max(np.abs(tr["uhat"][rr])), 1e-30)
        err = np.max(np.abs(g["trace"]["uhat"][rr] - uh_ref[rr]))
        assert err <= (1e-4 if iterate else UHAT_TOL) * scale, f"loop {rr} buckets: {err / scale:.2e}"
        delta = max(delta, err, 1e-7 * scale)
    # selections: firmly selected buckets are selected, the rest of the GPU's are near the boundary
    loose = set()
    for rr in range(L):
        jl = np.sort(g["trace"]["jlist"][rr])
        bits = g["trace"]["jbits"][rr]
        assert np.array_equal(np.nonzero([(bits[h >> 5] >> (h & 31)) & 1 for h in range(B)])[0], jl)
        firm = _firm_selection(np.abs(uh_ref[rr]) ** 2, 2 * K, delta)
        assert set(np.nonzero(firm)[0].tolist()) <= set(jl.tolist()), f"loop {rr}: firm bucket not selected"
        if rr % 2 == 0:
            loose |= {(rr // 2, h) for h in set(jl.tolist()) | set(J_ref[rr].tolist()) if not firm[h]}
    # decodes of firm buckets that cannot round differently
    located = set()
    for j, h, t, f, ok in decs:
        for k in range(h.shape[0]):
            hk = int(h[k])
            if (j, hk) in loose:
                continue
            if _robust_decode(uh_ref[2 * j][hk], uh_ref[2 * j + 1][hk], t[k], delta, N):
                if ok[k]:
                    located.add(int(f[k]))
            else:
                loose.add((j, hk))
    if iterate:
        located -= set(tr["idx1"].tolist())
    gset = set(g["trace"]["cand"].astype(np.int64).tolist())
    assert len(gset) == g["trace"]["cand"].shape[0], "duplicate candidates"
    assert located <= gset, f"missed decodes {sorted(located - gset)[:8]}"
    assert located <= set(I_ref.tolist())

    def explained(f):
        return any((j, int(((int(sigma[2 * j]) * f) % N + M // 2) // M % B)) in loose for j in range(L // 2))
    for f in (gset - located) | (set(I_ref.tolist()) - located):
        assert explained(f), f"candidate {f} not explained by a near-boundary decode"
    p = Parity(loops=L, cand_equal=gset == set(I_ref.tolist()),
               cand_explained=len(gset ^ set(I_ref.tolist())))
    p.loops_tied = len({j for j, _ in loose})
    # support around the K-boundary and values: each located frequency's estimate uses the
    # loops of the pairs that decode it (NaN elsewhere, for the cancellation guard)
    if iterate:
        I_all, v_all = tr["I_all2"], tr["v_all2"]
        V1 = tr["val1"][tr["idx1"] >= 0]
        e2 = np.where(tr["use2"], tr["e2"], np.nan)
        e_all = np.hstack([e2, np.broadcast_to(V1, (L, V1.shape[0]))])
    else:
        I_all, v_all = tr["I"], tr["v"]
        e_all = np.where(tr["use"], tr["e"], np.nan)
    delta_v = 1.5 * np.sqrt(2.0) * delta / float(np.min(np.abs(tr["G"])))
    tied = {f for f in gset | set(I_ref.tolist()) if explained(f)}
    support_and_values(p, g["idx"], g["val"], I_all, v_all, e_all, K, gset - set(I_ref.tolist()),
                       set(I_ref.tolist()) - gset, delta_v, value_tied=tied)
    assert p.values >= 1 or not np.any(g["idx"] >= 0), "no value compared"
    if p.cand_equal and tr["final_margin"] > FINAL_MARGIN:
        assert p.support_equal, "support"
    return record(p)


def check_residual(g, x64, tpos):
    er, ein = O.residual_energy(x64.astype(np.complex64).astype(np.complex128), g["idx"], g["val"], tpos)
    res = g["resid"]
    assert abs(res[1] - ein) <= 1e-9 * ein
    assert abs(res[0] - er) <= 1e-9 * max(ein, 1e-300)


CASES = [  # N, K, B, L, w, snr, seed
    (1 << 14, 20, 128, 4, 1024, None, 0),     # 2K/B = 31%: collisions in some pairs
    (1 << 14, 20, 128, 4, 1024, None, 1),
    (1 << 16, 30, 512, 6, 4096, None, 2),
    (1 << 18, 50, 1024, 4, 8192, None, 3),
    (1 << 12, 3, 64, 2, 512, None, 4),        # one pair
    (1 << 14, 10, 256, 4, 2048, 40.0, 5),     # light noise
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("iterate", [False, True])
def test_phase_parity(dev, case, iterate):
    N, K, B, L, w, snr, seed = case
    sig = make_signal(N, K, snr, seed=900 + seed)
    g = _run(dev, sig.x, iterate=iterate, K=K, B=B, L=L, w=w, seed=seed, n_resid=1000)
    r = O.sfft(sig.x.astype(np.complex64).astype(np.complex128), K, B, L, w, seed=seed, n_resid=1000,
               location="phase", iterate=iterate)
    p = compare_phase(g, r, K, B, L, N, iterate)
    if p.skipped:
        # the second round is not comparable only after a first round that tied
        plain = _run(dev, sig.x, K=K, B=B, L=L, w=w, seed=seed, n_resid=1000)
        r1 = O.sfft(sig.x.astype(np.complex64).astype(np.complex128), K, B, L, w, seed=seed, n_resid=1000,
                    location="phase")
        assert compare_phase(plain, r1, K, B, L, N).ambiguous, p.skipped
    check_residual(g, sig.x, r.trace["tpos"])


def test_phase_cases_comparable(dev):
    """The exactly sparse cases are compared through every stage (not skipped)."""
    n = 0
    for case in CASES[:4]:
        N, K, B, L, w, snr, seed = case
        sig = make_signal(N, K, snr, seed=900 + seed)
        g = _run(dev, sig.x, K=K, B=B, L=L, w=w, seed=seed, n_resid=1000)
        r = O.sfft(sig.x.astype(np.complex64).astype(np.complex128), K, B, L, w, seed=seed, n_resid=1000,
                   location="phase")
        p = compare_phase(g, r, K, B, L, N)
        n += p.cand_equal and p.support_equal
    assert n >= 3


def test_phase_exact_support_rate(dev):
    """Exactly sparse: the GPU recovers the exact support as often as the oracle,
    and the subtraction round recovers it in most cases."""
    N, K, B, L, w = 1 << 14, 20, 128, 4, 1024
    hits_g, hits_o = [0, 0], [0, 0]
    for s in range(12):
        sig = make_signal(N, K, None, seed=40 + s)
        for i, it in enumerate((False, True)):
            g = _run(dev, sig.x, iterate=it, K=K, B=B, L=L, w=w, seed=s, n_resid=0)
            hits_g[i] += set(g["idx"].tolist()) == set(sig.freqs.tolist())
            r = O.sfft(sig.x, K, B, L, w, seed=s, n_resid=0, location="phase", iterate=it)
            hits_o[i] += set(r.idx.tolist()) == set(sig.freqs.tolist())
    assert hits_g == hits_o
    assert hits_g[1] >= 8


def test_phase_in_batch_bitwise(dev):
    import torch
    import paper_2012_08238_amd as S
    P, I = S.SFFT_FLAG_PHASE_LOCATION, S.SFFT_FLAG_ITERATE
    cfgs = [(1 << 14, 20, 128, 4, 1024, 0, P), (1 << 16, 20, 512, 7, 4096, 1, 0),
            (1 << 18, 50, 1024, 4, 8192, 2, P | I), (1 << 16, 40, 256, 5, 2048, 3, I)]
    plans = [S.Plan(N, K, B, L, w, seed=sd, flags=fl, n_resid=700) for (N, K, B, L, w, sd, fl) in cfgs]
    xs = [torch.from_numpy(make_signal(c[0], c[1], None if c[6] & P else 20.0, seed=950 + j).x.astype(np.complex64))
          .to(dev) for j, c in enumerate(cfgs)]
    singles = [tuple(t.clone() for t in p(x, residual=True)) for p, x in zip(plans, xs)]
    torch.cuda.synchronize()
    for branches in (1, 2):
        batch = S.Batch(plans, branches=branches)
        outs = [p.outputs(dev) for p in plans]
        for rep in range(2):
            for o in outs:
                for t in o:
                    t.zero_()
            batch.run(xs, [o[0] for o in outs], [o[1] for o in outs], [o[2] for o in outs])
            torch.cuda.synchronize()
            for j, (o, s) in enumerate(zip(outs, singles)):
                for a, b in zip(o, s):
                    assert torch.equal(a, b), f"branches {branches} replay {rep} signal {j}"
        batch.close()
    for p in plans:
        p.close()


def test_phase_sixteen_pairs(dev):
    """L = 32 (16 pairs, the loop maximum) with the subtraction round."""
    N, K, B, L, w = 1 << 16, 200, 2048, 32, 16384
    sig = make_signal(N, K, None, seed=78)
    ps = []
    for it in (False, True):
        g = _run(dev, sig.x, iterate=it, K=K, B=B, L=L, w=w, seed=2, n_resid=500)
        r = O.sfft(sig.x.astype(np.complex64).astype(np.complex128), K, B, L, w, seed=2, n_resid=500,
                   location="phase", iterate=it)
        ps.append(compare_phase(g, r, K, B, L, N, it))
        check_residual(g, sig.x, r.trace["tpos"])
    # the second round is compared unless the first round (the plan without it) tied
    assert ps[0].values >= K // 2
    assert not ps[1].skipped or ps[0].ambiguous, ps
