"""The two enumerations of the vote, by loop (the frequencies of loops 0..L-T, each tested
against the other loops) and by loop pair (the loops split into T-1 groups; each pair within a
group enumerates its first loop and tests its second, the rest only for those both voted for),
give the same candidate set: the frequencies with >= T votes (the voting location of Table 1).
Each form is compared with the FP64 oracle (candidates, supports, values, residual) and the two
forms' candidate lists with each other, over the vote kernel's instances and code paths: the
two-phase tests, one candidate per lane (N/B < 16), the generic instance (L > 16), fewer than 32
buckets, T = L and even L."""
import numpy as np
import pytest

import oracle.sfft_oracle as O
from paper_2012_08238_amd.signals import make_signal
from parity import compare

pytestmark = pytest.mark.gpu

CFGS = [
    dict(N=1 << 14, K=10, B=128, L=5, w=512, seed=1, snr=None),              # exactly sparse
    dict(N=1 << 20, K=50, B=1024, L=7, w=8192, seed=2, snr=20.0),            # 2K/B = 10%
    dict(N=1 << 20, K=16, B=2048, L=9, w=16384, seed=3, snr=20.0),           # dK/B = 1/64: two-phase by loop
    dict(N=1 << 16, K=10, B=512, L=20, w=4096, seed=4, snr=10.0),            # L > 16: generic instance
    dict(N=1 << 12, K=4, B=512, L=7, w=2048, seed=5, snr=10.0, T=3),         # N/B = 8: a candidate per lane
    dict(N=1 << 12, K=3, B=8, L=5, w=64, seed=6, snr=10.0),                  # B < 32: one bitmap word
    dict(N=1 << 14, K=8, B=256, L=6, w=2048, seed=7, snr=20.0, T=6),         # T = L: one pair
    dict(N=1 << 14, K=8, B=256, L=8, w=2048, seed=8, snr=20.0, T=3),         # even L, two groups of 4
]


def _run(dev, x64, flags, K, B, L, w, seed, T):
    import torch
    import paper_2012_08238_amd as S
    p = S.Plan(x64.shape[0], K, B, L, w, seed=seed, vote_threshold=T, flags=flags)
    xt = torch.from_numpy(x64.astype(np.complex64)).to(dev)
    idx, val, res = p(xt, residual=True)
    torch.cuda.synchronize()
    out = dict(idx=idx.cpu().numpy(), val=val.cpu().numpy().astype(np.complex128), resid=res.cpu().numpy(),
               trace=p.trace(), perms=p.perms(), desc=p.describe())
    p.close()
    return out


@pytest.mark.parametrize("cfg", CFGS, ids=[f"N{c['N'].bit_length() - 1}_B{c['B']}_L{c['L']}_T{c.get('T', 0)}"
                                           for c in CFGS])
def test_vote_by_loop_and_by_pair(dev, cfg):
    import paper_2012_08238_amd as S
    N, K, B, L, w, seed = (cfg[k] for k in ("N", "K", "B", "L", "w", "seed"))
    T = cfg.get("T", 0)
    sig = make_signal(N, K, cfg["snr"], seed=700 + seed)
    x = sig.x.astype(np.complex64).astype(np.complex128)
    r = O.sfft(x, K, B, L, w, seed=seed, T=T or None)
    got = {}
    for name, flags in (("loop", S.SFFT_FLAG_VOTE_BY_LOOP), ("pair", S.SFFT_FLAG_VOTE_BY_PAIR)):
        g = _run(dev, sig.x, flags, K, B, L, w, seed, T)
        assert (g["desc"]["vote_pairs"] > 0) == (name == "pair")
        compare(g, r, K, B, L, w, seed)
        er, ein = O.residual_energy(x, g["idx"], g["val"], r.trace["tpos"])
        assert abs(g["resid"][1] - ein) <= 1e-9 * ein
        assert abs(g["resid"][0] - er) <= 1e-9 * max(ein, 1e-300)
        got[name] = g
    # the same candidate set, each frequency once, in either enumeration
    ca = np.sort(got["loop"]["trace"]["cand"])
    cb = np.sort(got["pair"]["trace"]["cand"])
    assert np.array_equal(ca, cb)
    assert len(np.unique(cb)) == cb.shape[0]
    assert np.array_equal(got["loop"]["idx"], got["pair"]["idx"])
    assert np.array_equal(got["loop"]["val"], got["pair"]["val"])


def _run_kw(dev, x64, **kw):
    import torch
    import paper_2012_08238_amd as S
    p = S.Plan(x64.shape[0], **kw)
    xt = torch.from_numpy(x64.astype(np.complex64)).to(dev)
    idx, val, res = p(xt, residual=True)
    torch.cuda.synchronize()
    out = dict(idx=idx.cpu().numpy(), val=val.cpu().numpy().astype(np.complex128), resid=res.cpu().numpy(),
               trace=p.trace(), perms=p.perms(), desc=p.describe())
    p.close()
    return out


@pytest.mark.parametrize("cfg", [
    dict(N=1 << 16, K=20, B=512, L=7, w=4096, seed=33, comb_b=2, comb_loops=3, comb_keep=1, snr=10.0),
    dict(N=1 << 20, K=50, B=1024, L=7, w=8192, seed=31, comb_b=1024, comb_loops=2, snr=20.0),
])
def test_vote_by_pair_with_comb(dev, cfg):
    """By pair, the comb prefilter's residue test applies to the finished frequencies as by loop."""
    import paper_2012_08238_amd as S
    from test_gpu_comb import _check_comb
    cfg = dict(cfg)
    N, snr = cfg.pop("N"), cfg.pop("snr")
    sig = make_signal(N, cfg["K"], snr, seed=cfg["seed"] + 90)
    keep = cfg.get("comb_keep", 0) or 2 * cfg["K"]
    r = O.sfft(sig.x.astype(np.complex64).astype(np.complex128), cfg["K"], cfg["B"], cfg["L"], cfg["w"],
               seed=cfg["seed"], comb_b=cfg["comb_b"], comb_loops=cfg["comb_loops"], comb_keep=keep)
    got = {}
    for name, flags in (("loop", S.SFFT_FLAG_VOTE_BY_LOOP), ("pair", S.SFFT_FLAG_VOTE_BY_PAIR)):
        g = _run_kw(dev, sig.x, flags=flags, **cfg)
        assert (g["desc"]["vote_pairs"] > 0) == (name == "pair")
        exact = _check_comb(g, r, sig.x, cfg["comb_b"], keep)
        compare(g, r, cfg["K"], cfg["B"], cfg["L"], cfg["w"], cfg["seed"], cand_exact=exact, comb_b=cfg["comb_b"])
        got[name] = g
    assert np.array_equal(np.sort(got["loop"]["trace"]["cand"]), np.sort(got["pair"]["trace"]["cand"]))
    assert np.array_equal(got["loop"]["idx"], got["pair"]["idx"])


@pytest.mark.parametrize("case", [
    (1 << 18, 60, 512, 7, 4096, 20.0, 0),
    (1 << 14, 10, 128, 5, 512, None, 2),
])
def test_vote_by_pair_subtraction_round(dev, case):
    """By pair, the second round skips the first round's frequencies as by loop (the
    recovered set's exclusion in the finished frequencies)."""
    import paper_2012_08238_amd as S
    from parity import compare_iterate
    N, K, B, L, w, snr, seed = case
    sig = make_signal(N, K, snr, seed=700 + seed)
    kw = dict(K=K, B=B, L=L, w=w, seed=seed, n_resid=1000)
    r = O.sfft(sig.x.astype(np.complex64).astype(np.complex128), K, B, L, w, seed=seed, n_resid=1000, iterate=True)
    got = {}
    for name, vf in (("loop", S.SFFT_FLAG_VOTE_BY_LOOP), ("pair", S.SFFT_FLAG_VOTE_BY_PAIR)):
        g = _run_kw(dev, sig.x, flags=vf | S.SFFT_FLAG_ITERATE, **kw)
        plain = _run_kw(dev, sig.x, flags=vf, **kw)
        assert (g["desc"]["vote_pairs"] > 0) == (name == "pair")
        first, second = compare_iterate(g, plain, r, K, B, L)
        assert second is not None, f"first rounds tied: {first}"
        got[name] = g
    assert np.array_equal(np.sort(got["loop"]["trace"]["cand"]), np.sort(got["pair"]["trace"]["cand"]))
    assert np.array_equal(got["loop"]["idx"], got["pair"]["idx"])
