"""CPU checks of the C ABI library: it loads, exports every declared entry
point, validates parameters, and its host-built FP64 tables and permutations
equal the oracle's."""
import os
import re

import numpy as np
import pytest

import oracle.sfft_oracle as O
import paper_2012_08238_amd as S
from paper_2012_08238_amd import _capi

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "sfft.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sfft_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = S.load()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), f"missing export {n}"
    assert {n for n, _, _ in _capi.SIGNATURES} == set(names)


def test_version_and_status_strings():
    lib = S.load()
    assert b"gfx950" in lib.sfft_version()
    assert lib.sfft_status_string(-1) == b"invalid argument"


@pytest.mark.parametrize("bad", [
    dict(comb_loops=1, comb_b=3), dict(comb_loops=1, comb_b=1 << 14), dict(comb_loops=9, comb_b=64),
    dict(comb_loops=1, comb_b=16), dict(comb_loops=1, comb_b=64, comb_keep=65), dict(comb_loops=-1),
    dict(N=1000), dict(N=8), dict(B=3), dict(B=1 << 14), dict(B=16), dict(K=0), dict(K=600), dict(L=0), dict(L=33),
    dict(w=511), dict(w=0), dict(w=1 << 15), dict(vote_threshold=9), dict(n_resid=-1)])
def test_parameter_validation(bad):
    kw = dict(N=1 << 14, K=10, B=128, L=5, w=512)
    kw.update(bad)
    with pytest.raises(S.SfftError) as e:
        S.host_tables(S.PlanParams(**kw))
    assert e.value.status in (_capi.SFFT_E_INVALID, _capi.SFFT_E_UNSUPPORTED)


def test_unsupported_large_B():
    with pytest.raises(S.SfftError) as e:
        S.host_tables(S.PlanParams(N=1 << 22, K=200, B=1 << 19, L=9, w=1 << 20))
    assert e.value.status == _capi.SFFT_E_UNSUPPORTED
    # up to 2^18 buckets run through the two-pass FFT
    t = S.host_tables(S.PlanParams(N=1 << 22, K=200, B=1 << 18, L=3, w=1 << 19, n_resid=8))
    assert t["gain"].shape[0] == 16


def test_phase_location_pairs_and_validation():
    N, L, seed = 1 << 14, 6, 21
    t = S.host_tables(S.PlanParams(N, 10, 128, L, 512, seed=seed, n_resid=64, flags=S.SFFT_FLAG_PHASE_LOCATION))
    sigma, tau, tpos = O.draw_permutations(N, L, seed, 64)
    ps, pt = O.pair_permutations(sigma, tau, N)
    assert np.array_equal(t["sigma"], ps.astype(np.uint32)) and np.array_equal(t["tau"], pt.astype(np.uint32))
    assert np.array_equal(t["tpos"], tpos.astype(np.uint32))
    kw = dict(N=N, K=10, B=128, w=512, flags=S.SFFT_FLAG_PHASE_LOCATION)
    for bad in (dict(L=5), dict(L=4, vote_threshold=3)):
        with pytest.raises(S.SfftError) as e:
            S.host_tables(S.PlanParams(**kw, **bad))
        assert e.value.status == _capi.SFFT_E_INVALID
    with pytest.raises(S.SfftError) as e:   # explicit loops must already be paired
        S.host_tables(S.PlanParams(**kw, L=2, sigma=np.array([3, 5], np.uint32), tau=np.array([1, 2], np.uint32)))
    S.host_tables(S.PlanParams(**kw, L=2, sigma=np.array([3, 3], np.uint32), tau=np.array([N - 1, 0], np.uint32)))
    with pytest.raises(S.SfftError) as e:
        S.host_tables(S.PlanParams(N=1 << 20, K=10, B=1 << 15, L=4, w=1 << 18, flags=S.SFFT_FLAG_PHASE_LOCATION))
    assert e.value.status == _capi.SFFT_E_UNSUPPORTED


def test_est_loops_perms_and_validation():
    N, L, seed, S_ = 1 << 14, 5, 33, 64
    for comb in (0, 2):
        kw = dict(seed=seed, n_resid=S_, est_loops=3, est_B=512)
        if comb:
            kw.update(comb_b=256, comb_loops=comb)
        t = S.host_tables(S.PlanParams(N, 10, 128, L, 512, **kw))
        sigma, tau, _ = O.draw_permutations(N, L, seed, S_)
        es, et = O.draw_est_permutations(N, L, seed, S_, comb, 3)
        assert np.array_equal(t["sigma"], np.concatenate([sigma, es]).astype(np.uint32))
        assert np.array_equal(t["tau"], np.concatenate([tau, et]).astype(np.uint32))
        inv = np.array([O.modinv(s_, N) for s_ in np.concatenate([sigma, es])], dtype=np.uint32)
        assert np.array_equal(t["sigma_inv"], inv)
    base = dict(N=N, K=10, B=128, L=5, w=512)
    for bad in (dict(est_loops=28, est_B=256), dict(est_loops=2, est_B=8), dict(est_loops=2, est_B=300),
                dict(est_loops=2, est_B=256, est_w=3), dict(est_loops=-1)):
        with pytest.raises(S.SfftError) as e:
            S.host_tables(S.PlanParams(**base, **bad))
        assert e.value.status == _capi.SFFT_E_INVALID
    for bad in (dict(N=1 << 17, est_loops=2, est_B=1 << 15), dict(est_loops=2, est_B=256, flags=S.SFFT_FLAG_ITERATE),
                dict(est_loops=2, est_B=256, flags=S.SFFT_FLAG_PHASE_LOCATION, L=4)):
        kw = dict(base)
        kw.update(bad)
        with pytest.raises(S.SfftError) as e:
            S.host_tables(S.PlanParams(**kw))
        assert e.value.status == _capi.SFFT_E_UNSUPPORTED
    S.host_tables(S.PlanParams(**dict(base, L=16), est_loops=16, est_B=64))   # 32 loops in all


def test_two_pass_fft_validation():
    base = dict(N=1 << 20, K=50, L=5, flags=S.SFFT_FLAG_FFT_TWO_PASS)
    for B in (4096, 8192, 16384):
        S.host_tables(S.PlanParams(**base, B=B, w=8 * B, n_resid=8))
    with pytest.raises(S.SfftError) as e:
        S.host_tables(S.PlanParams(**base, B=2048, w=16384))
    assert e.value.status == _capi.SFFT_E_INVALID
    with pytest.raises(S.SfftError) as e:
        S.host_tables(S.PlanParams(N=1 << 20, K=50, L=5, B=4096, w=32768,
                                   flags=S.SFFT_FLAG_FFT_TWO_PASS | S.SFFT_FLAG_ITERATE))
    assert e.value.status == _capi.SFFT_E_UNSUPPORTED


def test_vote_pairs_cover_every_threshold_set():
    """By pair, every T-subset of the L loops holds one of the plan's pairs (so every frequency
    with >= T votes is enumerated by a pair whose two loops voted for it); brute force over the
    subsets."""
    from itertools import combinations
    for L in range(2, 13):
        for T in range(2, L + 1):
            g = T - 1
            sizes = [L // g + (1 if i < L % g else 0) for i in range(g)]
            if sum(z * (z - 1) // 2 for z in sizes) > 32:
                continue
            d = S.params_describe(S.PlanParams(N=1 << 14, K=4, B=128, L=L, w=512, vote_threshold=T,
                                               flags=S.SFFT_FLAG_VOTE_BY_PAIR))
            pairs = d["vote_pair"]
            assert d["vote_pairs"] == len(pairs) >= 1
            assert all(0 <= a < b < L for a, b in pairs) and len(set(pairs)) == len(pairs)
            ps = [set(q) for q in pairs]
            for sub in combinations(range(L), T):
                ss = set(sub)
                assert any(q <= ss for q in ps), (L, T, sub)


def test_vote_mode_choice_and_validation():
    def desc(**kw):
        base = dict(N=1 << 22, K=100, B=16384, L=9, w=131072)
        base.update(kw)
        return S.params_describe(S.PlanParams(**base))
    # the benchmark shape: 4 groups (3, 2, 2, 2) of consecutive loops, 6 pairs
    assert desc()["vote_pair"] == [(0, 1), (0, 2), (1, 2), (3, 4), (5, 6), (7, 8)]
    assert desc(flags=S.SFFT_FLAG_VOTE_BY_LOOP)["vote_pairs"] == 0
    assert desc(vote_threshold=1)["vote_pairs"] == 0            # T = 1: no pair needed
    assert desc(vote_threshold=2)["vote_pairs"] == 0            # one group of 9: 36 pairs
    assert desc(vote_threshold=3, flags=S.SFFT_FLAG_VOTE_BY_PAIR)["vote_pairs"] == 16   # 5 + 4 loops
    for kw in (dict(vote_threshold=1, flags=S.SFFT_FLAG_VOTE_BY_PAIR),
               dict(vote_threshold=2, flags=S.SFFT_FLAG_VOTE_BY_PAIR),   # 36 pairs
               dict(flags=S.SFFT_FLAG_VOTE_BY_PAIR | S.SFFT_FLAG_VOTE_BY_LOOP)):
        with pytest.raises(S.SfftError) as e:
            desc(**kw)
        assert e.value.status == _capi.SFFT_E_INVALID
    # phase location has no vote
    assert desc(L=4, flags=S.SFFT_FLAG_PHASE_LOCATION)["vote_pairs"] == 0


def test_fused_validation():
    def desc(**kw):
        base = dict(N=1 << 16, K=20, B=512, L=7, w=4096, flags=S.SFFT_FLAG_FUSED)
        base.update(kw)
        return S.params_describe(S.PlanParams(**base))
    # the fused form gathers its buckets, whatever the per-stage path would choose
    assert desc()["fold_mode"] == 0   # 0 gather, 1 strip
    assert S.params_describe(S.PlanParams(N=1 << 16, K=20, B=512, L=7, w=4096))["fold_mode"] == 1
    assert desc(N=1 << 20, K=1000, B=4096, L=5, w=32768)["K"] == 1000
    for kw in (dict(K=4, B=16, w=128), dict(N=1 << 20, B=8192, w=65536), dict(L=17), dict(N=1 << 20, K=1025, B=4096),
               dict(flags=S.SFFT_FLAG_FUSED | S.SFFT_FLAG_ITERATE),
               dict(L=4, flags=S.SFFT_FLAG_FUSED | S.SFFT_FLAG_PHASE_LOCATION),
               dict(flags=S.SFFT_FLAG_FUSED | S.SFFT_FLAG_FOLD_STRIP),
               dict(flags=S.SFFT_FLAG_FUSED | S.SFFT_FLAG_FFT_TWO_PASS, B=4096, N=1 << 18, w=32768),
               dict(comb_b=256, comb_loops=2), dict(est_loops=2, est_B=2048)):
        with pytest.raises(S.SfftError) as e:
            desc(**kw)
        assert e.value.status == _capi.SFFT_E_UNSUPPORTED, kw


def test_iterate_validation_and_gain():
    # the subtraction round runs with the one-workgroup FFT only
    with pytest.raises(S.SfftError) as e:
        S.host_tables(S.PlanParams(N=1 << 20, K=100, B=1 << 15, L=5, w=1 << 17, flags=S.SFFT_FLAG_ITERATE))
    assert e.value.status == _capi.SFFT_E_UNSUPPORTED
    # the round widens the gain table to the buckets of its reach; the plain table within it
    # is the same, bitwise, at w = 4B (reach 2), 8B (reach 1) and w = B (every bucket)
    for N, B, w in ((1 << 14, 128, 512), (1 << 14, 128, 1024), (1 << 12, 64, 64)):
        kw = dict(N=N, K=10, B=B, L=5, w=w, n_resid=8)
        a = S.host_tables(S.PlanParams(**kw))
        b = S.host_tables(S.PlanParams(flags=S.SFFT_FLAG_ITERATE, **kw))
        assert np.array_equal(a["gain"], b["gain"])


def _outside_reach(N, B, lo, hi):
    # offsets o = o0 - j N/B (o0 in [-N/2B, N/2B), j in [-lo, hi]) reach buckets of the
    # reach; True for the offsets (mod N) that none of them produces
    M = N // B
    covered = np.zeros(N, bool)
    covered[np.arange(-(hi * M + M // 2), lo * M + M // 2) % N] = True
    return ~covered


@pytest.mark.parametrize("N,B,w,c_g", [
    (1 << 14, 128, 1024, 0), (1 << 14, 128, 512, 0), (1 << 14, 128, 256, 0), (1 << 14, 128, 192, 0),
    (1 << 12, 64, 96, 0), (1 << 18, 512, 4096, 0), (1 << 16, 1024, 2048, 0), (1 << 12, 8, 64, 0),
    (1 << 14, 256, 3072, 6.0), (1 << 14, 128, 1024, 4.0), (256, 16, 32, 0), (1 << 12, 64, 64, 0),
    (1 << 10, 16, 64, 2.0)])
def test_subtraction_reach_bounds_the_response(N, B, w, c_g):
    """The subtraction round's reach (the buckets a recovered coefficient is removed from):
    the oracle's complete window response (library inverse FFT of the padded window) beyond
    it stays within the plan's bound, which is at most 1e-6 of the centre gain; or the reach
    is every bucket."""
    d = S.params_describe(S.PlanParams(N, 2, B, 5, w, gauss_c=c_g, flags=S.SFFT_FLAG_ITERATE))
    lo, hi, bound = d["sub_reach_lo"], d["sub_reach_hi"], d["sub_tail_bound"]
    Gf = O.gain_full(O.flat_window(w, B, c_g) if c_g else O.flat_window(w, B), N)
    if lo + hi + 1 == B:
        assert (lo, hi, bound) == (B // 2 - 1, B // 2, 0.0)
        assert not _outside_reach(N, B, lo, hi).any()
        return
    assert 1 <= lo == hi and 2 * hi + 1 < B and 0 < bound <= 1e-6
    tail = np.max(np.abs(Gf[_outside_reach(N, B, lo, hi)])) / abs(Gf[0])
    assert tail <= bound
    # the reach also leaves out nothing the method needs: one bucket less leaves more than
    # the bound (the window's response is still falling off there)
    if hi > 1:
        assert np.max(np.abs(Gf[_outside_reach(N, B, hi - 1, hi - 1)])) / abs(Gf[0]) > bound


def test_subtraction_reach_values_and_refusal():
    it = S.SFFT_FLAG_ITERATE
    reach = lambda N, B, w: S.params_describe(S.PlanParams(N, 2, B, 5, w, flags=it))["sub_reach_hi"]  # noqa: E731
    # the response falls off over about 8/(w/B) buckets at the default Gaussian ratio
    assert [reach(1 << 16, 256, a * 256) for a in (16, 8, 4, 2)] == [1, 1, 2, 4]
    assert S.params_describe(S.PlanParams(1 << 14, 10, 128, 5, 512))["sub_reach_hi"] == 0   # no round
    # a window whose response stays above 1e-6 over more than 129 buckets: refused
    with pytest.raises(S.SfftError) as e:
        S.params_describe(S.PlanParams(1 << 20, 10, 1024, 5, 512, flags=it))
    assert e.value.status == _capi.SFFT_E_UNSUPPORTED
    with pytest.raises(S.SfftError) as e:
        S.params_describe(S.PlanParams(1 << 20, 10, 1024, 5, 8192, gauss_c=2.0, flags=it))
    assert e.value.status == _capi.SFFT_E_UNSUPPORTED


@pytest.mark.parametrize("N,K,B,L,w,seed", [
    (1 << 14, 10, 128, 5, 512, 0), (1 << 14, 10, 128, 5, 512, 12345),
    (1 << 20, 50, 1024, 7, 8192, 7), (1 << 12, 3, 64, 9, 256, 99)])
def test_permutations_match_oracle(N, K, B, L, w, seed):
    t = S.host_tables(S.PlanParams(N, K, B, L, w, seed=seed, n_resid=64))
    sigma, tau, tpos = O.draw_permutations(N, L, seed, 64)
    assert np.array_equal(t["sigma"], sigma.astype(np.uint32))
    assert np.array_equal(t["tau"], tau.astype(np.uint32))
    assert np.array_equal(t["tpos"], tpos.astype(np.uint32))
    inv = np.array([O.modinv(s, N) for s in sigma], dtype=np.uint32)
    assert np.array_equal(t["sigma_inv"], inv)


def test_explicit_permutations():
    sig = np.array([3, 5, 7], np.uint32)
    tau = np.array([1, 0, 100], np.uint32)
    t = S.host_tables(S.PlanParams(1 << 10, 2, 16, 3, 64, sigma=sig, tau=tau))
    assert np.array_equal(t["sigma"], sig) and np.array_equal(t["tau"], tau)
    with pytest.raises(S.SfftError):
        S.host_tables(S.PlanParams(1 << 10, 2, 16, 3, 64, sigma=np.array([2, 5, 7], np.uint32), tau=tau))


@pytest.mark.parametrize("N,B,w", [(1 << 14, 128, 512), (1 << 12, 64, 1024), (1 << 16, 256, 2048),
                                   (1 << 10, 16, 96)])
def test_window_and_gain_match_oracle(N, B, w):
    t = S.host_tables(S.PlanParams(N, 1, B, 3, w))
    g = O.flat_window(w, B)
    G = O.gain_table(g, N, B)
    assert np.max(np.abs(t["window"] - g)) <= 1e-13 * np.max(np.abs(g))
    assert np.max(np.abs(t["gain"] - G)) <= 1e-13 * np.max(np.abs(G))


def test_gauss_c_override():
    t = S.host_tables(S.PlanParams(1 << 12, 1, 32, 3, 256, gauss_c=3.0))
    g = O.flat_window(256, 32, 3.0)
    assert np.max(np.abs(t["window"] - g)) <= 1e-13 * np.max(np.abs(g))
