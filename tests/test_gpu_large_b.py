"""B > 16384: the two-pass FFT of the column-order bucket values, selection in
DFT order with buckets h = sigma m mod B, and estimates through the phase
relation X[h] = e^{+2 pi i (s tau h mod B)/B} V[s h mod B]. Same parity bar as
the one-workgroup path: exact permutations, selections, candidates and
supports; values within 1e-4; FP64 residual within 1e-9."""
import numpy as np
import pytest

from paper_2012_08238_amd.signals import make_signal
from parity import compare
from test_gpu_parity import _oracle, _run, check_residual

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("K,B", [(200, 1 << 15), (500, 1 << 15), (1000, 1 << 16)])
def test_c3_large_k(dev, K, B):
    """N=2^22, 20 dB, L=9, w=8B, B the power of two near sqrt(NK)."""
    sig = make_signal(1 << 22, K, 20.0, seed=310 + K)
    g = _run(dev, sig.x, K=K, B=B, L=9, w=8 * B, seed=3)
    r = _oracle(sig.x, K, B, 9, 8 * B, 3)
    compare(g, r, K, B, 9, 8 * B, 3)
    check_residual(g, sig.x, r.trace["tpos"])
    assert set(g["idx"].tolist()) == set(sig.freqs.tolist())


@pytest.mark.parametrize("N,K,B,L,wB", [
    (1 << 23, 400, 1 << 17, 7, 8),     # B = 2^17 (512 x 256)
    (1 << 22, 100, 1 << 18, 5, 4),     # B = 2^18 (512 x 512), N/B = 16
    (1 << 16, 30, 1 << 15, 5, 2),      # N/B = 2
])
def test_large_b_shapes(dev, N, K, B, L, wB):
    sig = make_signal(N, K, 20.0, seed=320 + L)
    g = _run(dev, sig.x, K=K, B=B, L=L, w=wB * B, seed=4)
    r = _oracle(sig.x, K, B, L, wB * B, 4)
    compare(g, r, K, B, L, wB * B, 4)
    check_residual(g, sig.x, r.trace["tpos"])


def test_large_b_zero_signal(dev):
    """Every energy ties: the selection streams every entry and keeps the dK lowest buckets."""
    N, K, B, L, w = 1 << 16, 4, 1 << 15, 5, 1 << 16
    x = np.zeros(N, dtype=np.complex128)
    g = _run(dev, x, K=K, B=B, L=L, w=w, seed=3)
    r = _oracle(x, K, B, L, w, 3)
    assert np.array_equal(g["idx"], r.idx)
    assert np.all(g["val"] == 0)
    for rr in range(L):
        assert np.array_equal(np.sort(g["trace"]["jlist"][rr]), np.arange(2 * K))


def test_large_b_many_selected(dev):
    """d*K = 4096 > B/16 group maxima: the selection streams every entry."""
    N, K, B, L, w = 1 << 20, 2048, 1 << 15, 5, 1 << 17
    sig = make_signal(N, K, 30.0, seed=330)
    g = _run(dev, sig.x, K=K, B=B, L=L, w=w, seed=5)
    r = _oracle(sig.x, K, B, L, w, 5)
    compare(g, r, K, B, L, w, 5)


def test_large_b_fold_forms_identical(dev):
    import paper_2012_08238_amd as S
    N, K, B, L, w = 1 << 20, 100, 1 << 15, 5, 1 << 17
    sig = make_signal(N, K, 20.0, seed=340)
    a = _run(dev, sig.x, K=K, B=B, L=L, w=w, seed=6, flags=S.SFFT_FLAG_FOLD_GATHER)
    b = _run(dev, sig.x, K=K, B=B, L=L, w=w, seed=6, flags=S.SFFT_FLAG_FOLD_STRIP)
    assert np.array_equal(a["trace"]["uhat"], b["trace"]["uhat"])
    assert np.array_equal(a["idx"], b["idx"]) and np.array_equal(a["val"], b["val"])


def test_large_b_in_batch(dev):
    """A batch mixing one-workgroup and two-pass FFT sizes: each result bitwise as alone."""
    import torch
    import paper_2012_08238_amd as S
    cfgs = [(1 << 22, 200, 1 << 15, 9), (1 << 20, 50, 1024, 7), (1 << 22, 1000, 1 << 16, 9),
            (1 << 22, 200, 1 << 15, 9)]
    plans = [S.Plan(N, K, B, L, 8 * B, seed=7) for N, K, B, L in cfgs]
    xs = [torch.from_numpy(make_signal(N, K, 20.0, seed=350 + i).x.astype(np.complex64)).to(dev)
          for i, (N, K, B, L) in enumerate(cfgs)]
    singles = [tuple(t.clone() for t in p(x, residual=True)) for p, x in zip(plans, xs)]
    torch.cuda.synchronize()
    b = S.Batch(plans)
    outs = [p.outputs(dev) for p in plans]
    for rep in range(2):
        b.run(xs, [o[0] for o in outs], [o[1] for o in outs], [o[2] for o in outs])
        torch.cuda.synchronize()
        for o, s1 in zip(outs, singles):
            for u, v in zip(o, s1):
                assert torch.equal(u, v)
    b.close()
    for p in plans:
        p.close()


@pytest.mark.parametrize("N,K,B,L", [(1 << 20, 50, 4096, 7), (1 << 20, 60, 8192, 5), (1 << 22, 100, 16384, 9)])
def test_two_pass_fft_below_2_15(dev, N, K, B, L):
    """The two-pass FFT on request for 4096 <= B <= 16384: same parity bar as the
    one-workgroup form, and the same support as it."""
    import paper_2012_08238_amd as S
    sig = make_signal(N, K, 20.0, seed=320 + L)
    g = _run(dev, sig.x, K=K, B=B, L=L, w=8 * B, seed=7, flags=S.SFFT_FLAG_FFT_TWO_PASS)
    one = _run(dev, sig.x, K=K, B=B, L=L, w=8 * B, seed=7)
    r = _oracle(sig.x, K, B, L, 8 * B, 7)
    compare(g, r, K, B, L, 8 * B, 7)
    check_residual(g, sig.x, r.trace["tpos"])
    assert np.array_equal(g["idx"], one["idx"])
