"""Parity of the subtraction round (iterative framework) on the GPU with the
FP64 oracle's sfft(..., iterate=True), whose subtraction removes each recovered
coefficient from every bucket.

Compared, stage by stage (parity.compare_iterate): the first round's outputs
(bitwise those of the plan without the round, and against the oracle's first
round), the residual buckets after the subtraction, the re-selected buckets, the
new candidates, and the final outputs. Integer results are compared exactly
wherever the oracle's decision is not a near-tie at the precision the GPU works
in, and near-ties are checked for validity and counted; the residual buckets
agree within 1e-4 of the loop's largest original bucket (the subtracted
contributions carry the value error of the first round, <= 1e-4 relative, times a
gain <= 1, and the reach leaves <= 1e-6 of each coefficient outside it).
"""
import numpy as np
import pytest

import oracle.sfft_oracle as O
from paper_2012_08238_amd.signals import make_signal
from parity import compare_iterate

pytestmark = pytest.mark.gpu

def _run(dev, x64, iterate=True, **kw):
    import torch
    import paper_2012_08238_amd as S
    N = x64.shape[0]
    flags = kw.pop("flags", 0) | (S.SFFT_FLAG_ITERATE if iterate else 0)
    p = S.Plan(N, flags=flags, **kw)
    xt = torch.from_numpy(x64.astype(np.complex64)).to(dev)
    idx, val, res = p(xt, residual=True)
    torch.cuda.synchronize()
    out = dict(idx=idx.cpu().numpy(), val=val.cpu().numpy().astype(np.complex128), resid=res.cpu().numpy(),
               trace=p.trace(), perms=p.perms())
    p.close()
    return out


def check_residual(g, x64, tpos):
    er, ein = O.residual_energy(x64.astype(np.complex64).astype(np.complex128), g["idx"], g["val"], tpos)
    res = g["resid"]
    assert abs(res[1] - ein) <= 1e-9 * ein
    assert abs(res[0] - er) <= 1e-9 * max(ein, 1e-300)


CASES = [  # N, K, B, L, w, snr, seed
    (1 << 18, 60, 512, 7, 4096, 20.0, 0),     # 2K/B = 23%: many shared buckets
    (1 << 18, 60, 512, 7, 4096, 20.0, 3),
    (1 << 16, 40, 256, 5, 2048, 10.0, 1),     # heavier collisions, lower SNR
    (1 << 14, 10, 128, 5, 512, None, 2),      # exactly sparse: residual at rounding level
    (1 << 12, 4, 64, 4, 512, 20.0, 4),        # even L
    (256, 8, 16, 3, 32, 20.0, 5),             # d*K = B: every bucket selected in both rounds
    (1 << 12, 3, 8, 5, 64, 20.0, 6),          # B < 32
]


@pytest.mark.parametrize("case", CASES)
def test_iterate_parity(dev, case):
    N, K, B, L, w, snr, seed = case
    sig = make_signal(N, K, snr, seed=700 + seed)
    kw = dict(K=K, B=B, L=L, w=w, seed=seed, n_resid=1000)
    g = _run(dev, sig.x, **kw)
    plain = _run(dev, sig.x, iterate=False, **kw)
    r = O.sfft(sig.x.astype(np.complex64).astype(np.complex128), K, B, L, w, seed=seed, n_resid=1000, iterate=True)
    first, second = compare_iterate(g, plain, r, K, B, L)
    assert second is not None, f"first rounds tied: {first}"
    assert second.certain + second.band + second.certain_displaced + second.certain_uncandidate >= 1
    check_residual(g, sig.x, r.trace["tpos"])


def test_iterate_collision_cases_comparable(dev):
    """The collision-heavy cases are compared through every stage (not skipped)."""
    n_full = 0
    for s in range(4):
        N, K, B, L, w = 1 << 18, 60, 512, 7, 4096
        sig = make_signal(N, K, 20.0, seed=600 + s)
        kw = dict(K=K, B=B, L=L, w=w, seed=s, n_resid=1000)
        g = _run(dev, sig.x, **kw)
        plain = _run(dev, sig.x, iterate=False, **kw)
        r = O.sfft(sig.x.astype(np.complex64).astype(np.complex128), K, B, L, w, seed=s, n_resid=1000, iterate=True)
        first, second = compare_iterate(g, plain, r, K, B, L)
        n_full += second is not None and not first.ambiguous and not second.ambiguous
    assert n_full >= 3


def test_iterate_recovers_collided_tones(dev):
    """One subtraction round finds the tones the first round missed (2K/B = 23%)."""
    missed = [0, 0]
    for s in range(6):
        sig = make_signal(1 << 18, 60, 20.0, seed=600 + s)
        for i, it in enumerate((False, True)):
            g = _run(dev, sig.x, iterate=it, K=60, B=512, L=7, w=4096, seed=s, n_resid=0)
            missed[i] += len(set(sig.freqs.tolist()) - set(g["idx"].tolist()))
    assert missed[0] >= 5 and missed[1] == 0


def test_iterate_mean_and_comb(dev):
    """The round composes with the mean combiner and the comb prefilter."""
    import paper_2012_08238_amd as S
    N, K, B, L, w, seed = 1 << 16, 30, 256, 5, 2048, 7
    sig = make_signal(N, K, 20.0, seed=707)
    kw = dict(K=K, B=B, L=L, w=w, seed=seed, n_resid=500, comb_b=1024, comb_loops=2)
    g = _run(dev, sig.x, flags=S.SFFT_FLAG_MEAN_ESTIMATE, **kw)
    plain = _run(dev, sig.x, iterate=False, flags=S.SFFT_FLAG_MEAN_ESTIMATE, **kw)
    r = O.sfft(sig.x.astype(np.complex64).astype(np.complex128), K, B, L, w, seed=seed, n_resid=500,
               combine="mean", comb_b=1024, comb_loops=2, iterate=True)
    assert min(r.trace["comb_margin"]) > 1e-4
    first, second = compare_iterate(g, plain, r, K, B, L, comb_b=1024)
    assert second is not None
    check_residual(g, sig.x, r.trace["tpos"])


def test_iterate_in_batch_bitwise(dev):
    """Iterating and plain plans in one batch: each result is bitwise its single execution."""
    import torch
    import paper_2012_08238_amd as S
    cfgs = [(1 << 18, 60, 512, 7, 4096, 0, S.SFFT_FLAG_ITERATE), (1 << 16, 20, 512, 7, 4096, 1, 0),
            (1 << 16, 40, 256, 5, 2048, 2, S.SFFT_FLAG_ITERATE), (1 << 14, 10, 128, 5, 512, 3, 0)]
    plans = [S.Plan(N, K, B, L, w, seed=sd, flags=fl, n_resid=700) for (N, K, B, L, w, sd, fl) in cfgs]
    xs = [torch.from_numpy(make_signal(c[0], c[1], 20.0, seed=800 + j).x.astype(np.complex64)).to(dev)
          for j, c in enumerate(cfgs)]
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


def test_iterate_deterministic(dev):
    import torch
    import paper_2012_08238_amd as S
    sig = make_signal(1 << 18, 60, 20.0, seed=601)
    p = S.Plan(1 << 18, 60, 512, 7, 4096, seed=1, flags=S.SFFT_FLAG_ITERATE)
    x = torch.from_numpy(sig.x.astype(np.complex64)).to(dev)
    a = p(x, residual=True)
    b = p(x, residual=True)
    torch.cuda.synchronize()
    for u, v in zip(a, b):
        assert torch.equal(u, v)
    p.close()


def test_iterate_max_sizes(dev):
    """K = 4096 at B = 16384 (the subtraction's LDS at its 96 KB bound, sort of 4096 keys):
    the first round is bitwise the plan without the round, the outputs are valid and
    deterministic, and the residual buckets match the oracle's when the first rounds agree."""
    N, K, B, L, w = 1 << 16, 4096, 16384, 5, 32768
    sig = make_signal(N, K, 30.0, seed=77)
    kw = dict(K=K, B=B, L=L, w=w, seed=1, n_resid=500)
    g = _run(dev, sig.x, **kw)
    g2 = _run(dev, sig.x, **kw)
    plain = _run(dev, sig.x, iterate=False, **kw)
    assert np.array_equal(g["idx"], g2["idx"]) and np.array_equal(g["val"], g2["val"])
    n1 = int(np.sum(plain["idx"] >= 0))
    assert np.array_equal(g["trace"]["rec_idx"], plain["idx"][:n1])
    ok = g["idx"] >= 0
    got = g["idx"][ok]
    assert np.all(np.diff(got) > 0) and np.all(g["idx"][~ok] == -1) and np.all(g["val"][~ok] == 0)
    r = O.sfft(sig.x.astype(np.complex64).astype(np.complex128), K, B, L, w, seed=1, n_resid=500, iterate=True)
    first, second = compare_iterate(g, plain, r, K, B, L)
    assert first.values >= 1
    check_residual(g, sig.x, r.trace["tpos"])
