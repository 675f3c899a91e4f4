"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Both sides get the same complex64 signal. Integer work must match exactly:
permutations, the sampled index set, selected buckets, candidate sets and
recovered supports, wherever the oracle's decision is not a near-tie at FP32
precision; near-ties are checked for validity and counted (parity.compare).
Floating point: bucket spectra within 1e-5 of the loop's largest bucket,
values within |v - v_ref| <= 1e-4 |v_ref|, FP64 residual within 1e-9.
"""
import numpy as np
import pytest

import oracle.sfft_oracle as O
from paper_2012_08238_amd.signals import impulse, make_signal
from parity import VAL_RTOL, compare  # noqa: F401

pytestmark = pytest.mark.gpu

SEL_MARGIN = 1e-4         # a comb prefilter's selection is compared where its boundary gap exceeds this


def _run(dev, x64, **plan_kw):
    import torch
    import paper_2012_08238_amd as S
    N = x64.shape[0]
    p = S.Plan(N, **plan_kw)
    xt = torch.from_numpy(x64.astype(np.complex64)).to(dev)
    idx, val, res = p(xt, residual=True)
    torch.cuda.synchronize()
    out = dict(idx=idx.cpu().numpy(), val=val.cpu().numpy().astype(np.complex128),
               resid=res.cpu().numpy(), trace=p.trace(), perms=p.perms(), desc=p.desc)
    p.close()
    return out


def _oracle(x64, K, B, L, w, seed, d=2, vote_threshold=0, n_resid=4096, combine="median"):
    T = vote_threshold or None
    return O.sfft(x64.astype(np.complex64).astype(np.complex128), K, B, L, w, seed=seed, d=d, T=T,
                  n_resid=n_resid, combine=combine)


def check_residual(g, x64, tpos):
    er, ein = O.residual_energy(x64.astype(np.complex64).astype(np.complex128), g["idx"], g["val"], tpos)
    res = g["resid"]
    assert abs(res[1] - ein) <= 1e-9 * ein
    assert abs(res[0] - er) <= 1e-9 * max(ein, 1e-300)


# ------------------------------------------------------------------ small configurations
@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_c1_exact_sparse(dev, seed):
    """N=2^14, K=10, exactly sparse, B=128, L=5, w=512 (complex64 cast of the complex128 signal)."""
    sig = make_signal(1 << 14, 10, None, seed=100 + seed)
    g = _run(dev, sig.x, K=10, B=128, L=5, w=512, seed=seed)
    r = _oracle(sig.x, 10, 128, 5, 512, seed)
    p = compare(g, r, 10, 128, 5, 512, seed)
    # every one of the K slots is a certain entry or a valid choice from the tie band
    # (seeds 1 and 2: the 10th and 11th largest are true unit tones 4e-9 apart), and
    # every returned value is compared
    assert p.certain + p.band == 10 and p.values == 10, p
    assert p.certain == (1 if seed in (1, 2) else 10), p
    check_residual(g, sig.x, r.trace["tpos"])


def test_c1_exact_support_invariant(dev):
    """Exactly sparse noiseless: the GPU finds the exact support as often as the oracle does."""
    import torch
    import paper_2012_08238_amd as S
    N, K, B, L, w = 1 << 14, 10, 128, 5, 512
    ok_g = ok_o = 0
    for s in range(20):
        sig = make_signal(N, K, None, seed=1000 + s)
        p = S.Plan(N, K, B, L, w, seed=s)
        idx, _ = p(torch.from_numpy(sig.x.astype(np.complex64)).to(dev))
        ok_g += set(idx.cpu().numpy().tolist()) == set(sig.freqs.tolist())
        r = O.sfft(sig.x, K, B, L, w, seed=s, n_resid=0)
        ok_o += set(r.idx.tolist()) == set(sig.freqs.tolist())
        p.close()
    assert ok_g == ok_o


def test_impulse_probe_sampled_set(dev):
    """x = e_j: loop r's buckets are zero except bucket i mod B with value g_i
    when j = (sigma_r i + tau_r) mod N for some i < w; this pins the permuted
    index arithmetic and the window taps exactly."""
    N, K, B, L, w = 1 << 12, 2, 64, 6, 512
    g_or = O.flat_window(w, B)
    for j in (0, 1, 777, N - 1):
        x = impulse(N, j)
        g = _run(dev, x, K=K, B=B, L=L, w=w, seed=5, n_resid=0 + 64)
        sigma, sigma_inv, tau = g["perms"]
        for r in range(L):
            u = np.fft.ifft(g["trace"]["uhat"][r])       # back to the folded buckets
            i = (int(sigma_inv[r]) * ((j - int(tau[r])) % N)) % N
            if i < w:
                b = i % B
                assert np.argmax(np.abs(u)) == b
                assert abs(u[b] - g_or[i]) <= 1e-6 * abs(g_or[i]) + 1e-7 * np.max(np.abs(u))
                rest = np.delete(np.abs(u), b)
                assert np.all(rest <= 1e-6 * abs(u[b]) + 1e-30)
            else:
                assert np.max(np.abs(g["trace"]["uhat"][r])) == 0.0


@pytest.mark.parametrize("cfg", [
    dict(N=1 << 10, K=1, B=16, L=3, w=128, seed=1),            # K = 1
    dict(N=256, K=8, B=16, L=3, w=32, seed=2),                  # d*K = B: every bucket selected
    dict(N=1 << 12, K=4, B=64, L=1, w=512, seed=3),             # one loop, T = 1
    dict(N=1 << 12, K=4, B=64, L=4, w=512, seed=4),             # even L: mean of the middle two
    dict(N=1 << 12, K=5, B=64, L=5, w=96, seed=5),              # w not a multiple of B
    dict(N=1 << 10, K=3, B=32, L=5, w=2, seed=6),               # smallest window
    dict(N=1 << 10, K=3, B=32, L=3, w=1 << 10, seed=7),         # window = whole signal
    dict(N=16, K=1, B=2, L=3, w=4, seed=8),                     # smallest N
    dict(N=1 << 12, K=6, B=64, L=7, w=512, seed=9, vote_threshold=1),   # T = 1: large I'
    dict(N=1 << 14, K=20, B=256, L=9, w=2048, seed=10, n_resid=1000),   # ragged residual tail
    dict(N=1 << 14, K=20, B=256, L=9, w=2048, seed=12, n_resid=1003),   # last residual run partial
    dict(N=1 << 12, K=4, B=64, L=5, w=512, seed=13, n_resid=5),         # fewer samples than one run
    dict(N=1 << 16, K=10, B=512, L=20, w=4096, seed=14),        # L > 16: the vote's generic instance
    dict(N=1 << 16, K=10, B=512, L=32, w=4096, seed=15),        # the most loops
    dict(N=1 << 14, K=6, B=256, L=1, w=2048, seed=16),          # one loop: T = 1, every enumerated frequency
    dict(N=1 << 12, K=3, B=8, L=5, w=64, seed=11),              # B < 32 (one bitmap word)
])
def test_edge_cases(dev, cfg):
    cfg = dict(cfg)
    N = cfg.pop("N")
    sig = make_signal(N, cfg["K"], 10.0, seed=cfg["seed"] + 50)
    n_resid = cfg.get("n_resid", 4096)
    g = _run(dev, sig.x, **cfg)
    r = _oracle(sig.x, cfg["K"], cfg["B"], cfg["L"], cfg["w"], cfg["seed"],
                vote_threshold=cfg.get("vote_threshold", 0), n_resid=n_resid)
    compare(g, r, cfg["K"], cfg["B"], cfg["L"], cfg["w"], cfg["seed"])
    check_residual(g, sig.x, r.trace["tpos"])


@pytest.mark.parametrize("L,T", [(4, 0), (5, 0), (8, 0), (11, 0), (16, 0), (9, 6)])
def test_vote_two_phase(dev, L, T):
    """Few selected buckets (dK/B = 1/64) with the default majority, enumerated by loop: the
    vote tests the first L - T + 2 loops for every candidate and the rest only for those that
    can still reach T. Candidate sets, supports and values as the oracle; T = 6 of 9 (not the
    default) takes the one-phase tests."""
    N, K, B = 1 << 20, 16, 2048
    assert 2 * K * 32 <= B
    sig = make_signal(N, K, 20.0, seed=900 + L)
    import paper_2012_08238_amd as S
    g = _run(dev, sig.x, K=K, B=B, L=L, w=8 * B, seed=L, vote_threshold=T, flags=S.SFFT_FLAG_VOTE_BY_LOOP)
    r = _oracle(sig.x, K, B, L, 8 * B, L, vote_threshold=T)
    compare(g, r, K, B, L, 8 * B, L)
    check_residual(g, sig.x, r.trace["tpos"])
    assert set(g["idx"].tolist()) == set(sig.freqs.tolist())


def test_zero_signal(dev):
    """All-zero input: every bucket ties, so the lowest buckets are selected and
    the lowest candidate frequencies are returned with value 0."""
    N, K, B, L, w = 1 << 12, 4, 64, 5, 512
    x = np.zeros(N, dtype=np.complex128)
    g = _run(dev, x, K=K, B=B, L=L, w=w, seed=3)
    r = _oracle(x, K, B, L, w, 3)
    assert np.array_equal(g["idx"], r.idx)
    assert np.all(g["val"] == 0)
    for rr in range(L):
        assert np.array_equal(np.sort(g["trace"]["jlist"][rr]), np.arange(2 * K))


def test_deterministic_repeat(dev):
    import torch
    import paper_2012_08238_amd as S
    sig = make_signal(1 << 16, 20, 20.0, seed=3)
    p = S.Plan(1 << 16, 20, 512, 7, 4096, seed=9)
    x = torch.from_numpy(sig.x.astype(np.complex64)).to(dev)
    a = p(x, residual=True)
    b = p(x, residual=True)
    torch.cuda.synchronize()
    for u, v in zip(a, b):
        assert torch.equal(u, v)
    p.close()


# ------------------------------------------------------------------ full-size configurations
@pytest.mark.parametrize("seed", [0, 1])
def test_c2_general_sparse(dev, seed):
    """N=2^20, K=50, 20 dB, B=1024, L=7, w=8192 (gather form by default)."""
    sig = make_signal(1 << 20, 50, 20.0, seed=200 + seed)
    g = _run(dev, sig.x, K=50, B=1024, L=7, w=8192, seed=seed)
    assert g["desc"]["fold_mode"] == 0
    r = _oracle(sig.x, 50, 1024, 7, 8192, seed)
    compare(g, r, 50, 1024, 7, 8192, seed)
    check_residual(g, sig.x, r.trace["tpos"])
    assert set(g["idx"].tolist()) == set(sig.freqs.tolist())


def test_fold_forms_bitwise_identical(dev):
    """Strip and gather bucketizations sum the same taps in the same order."""
    import paper_2012_08238_amd as S
    for N, K, B, L, w in ((1 << 20, 50, 1024, 7, 8192), (1 << 16, 10, 256, 9, 4096), (1 << 12, 3, 8, 5, 64)):
        sig = make_signal(N, K, 20.0, seed=7)
        a = _run(dev, sig.x, K=K, B=B, L=L, w=w, seed=1, flags=S.SFFT_FLAG_FOLD_GATHER)
        b = _run(dev, sig.x, K=K, B=B, L=L, w=w, seed=1, flags=S.SFFT_FLAG_FOLD_STRIP)
        assert a["desc"]["fold_mode"] == 0 and b["desc"]["fold_mode"] == 1
        assert np.array_equal(a["trace"]["uhat"], b["trace"]["uhat"])
        assert np.array_equal(a["idx"], b["idx"]) and np.array_equal(a["val"], b["val"])


@pytest.mark.parametrize("strip_cols", [0, 2, 8, 64])
def test_strip_widths_bitwise_identical(dev, strip_cols):
    import paper_2012_08238_amd as S
    N, K, B, L, w = 1 << 18, 40, 2048, 9, 16384
    sig = make_signal(N, K, 20.0, seed=8)
    a = _run(dev, sig.x, K=K, B=B, L=L, w=w, seed=2, flags=S.SFFT_FLAG_FOLD_GATHER)
    b = _run(dev, sig.x, K=K, B=B, L=L, w=w, seed=2, flags=S.SFFT_FLAG_FOLD_STRIP, strip_cols=strip_cols)
    assert np.array_equal(a["trace"]["uhat"], b["trace"]["uhat"])
    assert np.array_equal(a["idx"], b["idx"])


def test_c3_k100_metric_point(dev):
    """N=2^22, K=100, 20 dB, B=16384, L=9, w=8B (strip form): the benchmark workload."""
    sig = make_signal(1 << 22, 100, 20.0, seed=300)
    g = _run(dev, sig.x, K=100, B=16384, L=9, w=131072, seed=1)
    assert g["desc"]["fold_mode"] == 1
    r = _oracle(sig.x, 100, 16384, 9, 131072, 1)
    compare(g, r, 100, 16384, 9, 131072, 1)
    check_residual(g, sig.x, r.trace["tpos"])
    assert set(g["idx"].tolist()) == set(sig.freqs.tolist())


@pytest.mark.parametrize("K,B", [(50, 8192), (50, 16384)])
def test_c3_other_k(dev, K, B):
    sig = make_signal(1 << 22, K, 20.0, seed=301)
    g = _run(dev, sig.x, K=K, B=B, L=9, w=8 * B, seed=2)
    r = _oracle(sig.x, K, B, 9, 8 * B, 2)
    compare(g, r, K, B, 9, 8 * B, 2)


# ------------------------------------------------------------------ estimator variants
@pytest.mark.parametrize("cfg", [
    dict(N=1 << 16, K=20, B=512, L=7, w=4096, seed=21, d=1),
    dict(N=1 << 16, K=20, B=512, L=7, w=4096, seed=22, d=3),
    dict(N=1 << 18, K=16, B=1024, L=9, w=8192, seed=23, d=4),
    dict(N=1 << 16, K=20, B=512, L=7, w=4096, seed=24, mean=True),
    dict(N=1 << 20, K=50, B=1024, L=8, w=8192, seed=25, mean=True),
    dict(N=1 << 14, K=10, B=128, L=5, w=512, seed=26, mean=True, d=3),
])
def test_estimator_variants(dev, cfg):
    """d != 2 buckets per loop, and the mean of the loop estimates in place of the median."""
    import paper_2012_08238_amd as S
    cfg = dict(cfg)
    N = cfg.pop("N")
    mean = cfg.pop("mean", False)
    d = cfg.get("d", 2)
    sig = make_signal(N, cfg["K"], 20.0, seed=cfg["seed"] + 70)
    g = _run(dev, sig.x, flags=S.SFFT_FLAG_MEAN_ESTIMATE if mean else 0, **cfg)
    r = _oracle(sig.x, cfg["K"], cfg["B"], cfg["L"], cfg["w"], cfg["seed"], d=d,
                combine="mean" if mean else "median")
    compare(g, r, cfg["K"], cfg["B"], cfg["L"], cfg["w"], cfg["seed"])
    check_residual(g, sig.x, r.trace["tpos"])
