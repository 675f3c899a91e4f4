"""The one-launch form of small plans (SFFT_FLAG_FUSED): one workgroup carries a
signal through every stage. It runs the per-stage kernels' device code, so its
outputs, residual and intermediates (bucket spectra, selections, candidates) are
bitwise those of the per-stage path of the same plan, and they meet the oracle
parity bar; in batches, alone, beside per-stage signals, and with more signals
than persistent workgroups."""
import numpy as np
import pytest

import oracle.sfft_oracle as O
from paper_2012_08238_amd.signals import make_signal
from parity import compare
from test_gpu_parity import check_residual

pytestmark = pytest.mark.gpu

CASES = [  # N, K, B, L, w, snr, seed, extra flags
    (1 << 14, 10, 128, 5, 512, None, 0, 0),            # exactly sparse, the smallest benchmark shape
    (1 << 16, 20, 512, 7, 4096, 10.0, 1, 0),
    (1 << 16, 50, 1024, 7, 8192, 20.0, 2, 0),
    (1 << 18, 100, 4096, 9, 32768, 20.0, 3, 0),        # the largest transform of this form
    (1 << 18, 100, 4096, 9, 32768, 20.0, 4, 0x200),    # vote by loop pairs
    (1 << 16, 20, 512, 7, 4096, 10.0, 5, 0x100),       # vote by loop
    (1 << 12, 4, 32, 4, 256, 20.0, 6, 0),              # smallest B, even L
    (1 << 15, 8, 256, 16, 2048, 15.0, 7, 0),           # L = 16
    (1 << 20, 1000, 4096, 5, 32768, 30.0, 8, 0),       # K = 1000: 4 outputs per thread
    (1 << 16, 20, 512, 7, 4096, 15.0, 9, 0x10),        # mean of the loop estimates
    (1 << 14, 10, 128, 5, 512, None, 10, 0x1),         # no residual
]


def _run(dev, x64, flags, **kw):
    import torch
    import paper_2012_08238_amd as S
    N = x64.shape[0]
    p = S.Plan(N, flags=flags, **kw)
    idx, val, res = p(torch.from_numpy(x64.astype(np.complex64)).to(dev), residual=True)
    torch.cuda.synchronize()
    out = dict(idx=idx.cpu().numpy(), val=val.cpu().numpy(), resid=res.cpu().numpy(), trace=p.trace(),
               perms=p.perms(), desc=p.desc)
    p.close()
    return out


@pytest.mark.parametrize("case", CASES)
def test_fused_equals_staged_and_oracle(dev, case):
    import paper_2012_08238_amd as S
    N, K, B, L, w, snr, seed, extra = case
    sig = make_signal(N, K, snr, seed=seed + 300)
    print(f"fused N={N} K={K} B={B} L={L} seed={seed} flags={extra:#x}", flush=True)
    f = _run(dev, sig.x, S.SFFT_FLAG_FUSED | extra, K=K, B=B, L=L, w=w, seed=seed)
    s = _run(dev, sig.x, extra, K=K, B=B, L=L, w=w, seed=seed)
    assert np.array_equal(f["idx"], s["idx"])
    assert np.array_equal(f["val"].view(np.uint32), s["val"].view(np.uint32))
    if not extra & 0x1:
        assert np.array_equal(f["resid"].view(np.uint64), s["resid"].view(np.uint64))
    for key in ("uhat", "jbits", "jlist"):
        a, b = f["trace"][key], s["trace"][key]
        assert np.array_equal(a.view(np.uint32) if a.dtype != np.uint32 else a,
                              b.view(np.uint32) if b.dtype != np.uint32 else b), key
    assert np.array_equal(np.sort(f["trace"]["cand"]), np.sort(s["trace"]["cand"]))
    r = O.sfft(sig.x.astype(np.complex64).astype(np.complex128), K, B, L, w, seed=seed,
               combine="mean" if extra & 0x10 else "median")
    g = dict(f, val=f["val"].astype(np.complex128))
    compare(g, r, K, B, L, w, seed)
    if not extra & 0x1:
        check_residual(g, sig.x, r.trace["tpos"])


def _batch_check(dev, plans, xs, reps=3):
    import torch
    import paper_2012_08238_amd as S
    singles = [tuple(t.clone() for t in p(x, residual=True)) for p, x in zip(plans, xs)]
    torch.cuda.synchronize()
    batch = S.Batch(plans)
    outs = [p.outputs(dev) for p in plans]
    for rep in range(reps):
        for o in outs:
            for t in o:
                t.zero_()
        if rep == 0:
            batch.run(xs, [o[0] for o in outs], [o[1] for o in outs], [o[2] for o in outs])
        else:   # the same buffers marshalled once
            if rep == 1:
                batch.bind(xs, [o[0] for o in outs], [o[1] for o in outs], [o[2] for o in outs])
            batch.run_bound()
        _ = (xs[0].abs() ** 2).sum()   # eager work between replays
        torch.cuda.synchronize()
        for j, (o, s) in enumerate(zip(outs, singles)):
            for a, b in zip(o, s):
                assert torch.equal(a, b), f"replay {rep}, signal {j}"
    batch.close()


def test_fused_batch_beside_staged(dev):
    """Fused signals of three sizes share one launch per L; per-stage signals (one of
    them the benchmark shape) run beside them in the same graph."""
    import torch
    import paper_2012_08238_amd as S
    cfgs = [(1 << 14, 10, 128, 5, 512, S.SFFT_FLAG_FUSED), (1 << 16, 20, 512, 5, 4096, S.SFFT_FLAG_FUSED),
            (1 << 18, 100, 4096, 9, 32768, S.SFFT_FLAG_FUSED), (1 << 22, 100, 16384, 9, 131072, 0),
            (1 << 16, 20, 512, 7, 4096, 0), (1 << 15, 8, 256, 7, 2048, S.SFFT_FLAG_FUSED)]
    plans, xs = [], []
    for j, (N, K, B, L, w, fl) in enumerate(cfgs):
        plans.append(S.Plan(N, K, B, L, w, seed=10 + j, flags=fl, n_resid=900 + 11 * j))
        xs.append(torch.from_numpy(make_signal(N, K, 20.0, seed=600 + j).x.astype(np.complex64)).to(dev))
    _batch_check(dev, plans, xs)
    for p in plans:
        p.close()


def test_fused_batch_only_fused_persistent(dev):
    """A batch of fused signals only (no bucketization launch at all) with more signals
    than persistent workgroups, so each workgroup takes several signals in turn."""
    import torch
    import paper_2012_08238_amd as S
    n = 2048 + 37
    plan = S.Plan(1 << 12, 4, 64, 5, 512, seed=3, flags=S.SFFT_FLAG_FUSED)
    base = [torch.from_numpy(make_signal(1 << 12, 4, 20.0, seed=900 + j).x.astype(np.complex64)).to(dev)
            for j in range(7)]
    xs = [base[j % 7] * (1.0 + 0.001 * j) for j in range(n)]   # distinct signals, same support
    _batch_check(dev, [plan] * n, xs, reps=3)
    plan.close()
