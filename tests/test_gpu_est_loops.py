"""Estimation-only loops (location and estimation loops separated, each with its
own bucket count) on the GPU against the FP64 oracle's sfft(..., est_loops=...),
and bitwise across single, batched and served execution."""
import numpy as np
import pytest

import oracle.sfft_oracle as O
from paper_2012_08238_amd.signals import make_signal
from parity import compare
from test_gpu_parity import check_residual

pytestmark = pytest.mark.gpu


def _run(dev, x64, **kw):
    import torch
    import paper_2012_08238_amd as S
    N = x64.shape[0]
    p = S.Plan(N, **kw)
    xt = torch.from_numpy(x64.astype(np.complex64)).to(dev)
    idx, val, res = p(xt, residual=True)
    torch.cuda.synchronize()
    out = dict(idx=idx.cpu().numpy(), val=val.cpu().numpy().astype(np.complex128), resid=res.cpu().numpy(),
               trace=p.trace(), perms=p.perms(), desc=p.desc)
    p.close()
    return out


CASES = [  # N, K, B, L, w, snr, seed, est_loops, est_B, est_w, flags
    (1 << 16, 20, 256, 5, 2048, 10.0, 0, 4, 1024, 0, 0),      # collision-heavy location, 4x the buckets to estimate
    (1 << 16, 20, 256, 5, 2048, 10.0, 1, 4, 1024, 0, 0),
    (1 << 14, 10, 128, 5, 512, 20.0, 2, 1, 64, 0, 0),         # fewer buckets than location, one loop
    (1 << 14, 10, 128, 4, 512, 20.0, 3, 3, 256, 4096, 0),     # explicit window, even total
    (1 << 18, 40, 1024, 16, 8192, 20.0, 4, 16, 2048, 0, 0),   # 32 loops in all
    (1 << 16, 20, 256, 5, 2048, 10.0, 5, 4, 1024, 0, 0x10),   # mean combiner
    (1 << 20, 50, 1024, 7, 8192, 20.0, 6, 2, 4096, 0, 0),     # C2 shape
    (1 << 20, 50, 4096, 5, 32768, 20.0, 7, 3, 8192, 0, 0x80), # location loops through the two-pass FFT
]


@pytest.mark.parametrize("case", CASES)
def test_est_loops_parity(dev, case):
    N, K, B, L, w, snr, seed, el, eb, ew, flags = case
    sig = make_signal(N, K, snr, seed=1200 + seed)
    g = _run(dev, sig.x, K=K, B=B, L=L, w=w, seed=seed, n_resid=1000, est_loops=el, est_B=eb, est_w=ew, flags=flags)
    r = O.sfft(sig.x.astype(np.complex64).astype(np.complex128), K, B, L, w, seed=seed, n_resid=1000,
               est_loops=el, est_B=eb, est_w=ew, combine="mean" if flags & 0x10 else "median")
    sigma, sigma_inv, tau = g["perms"]
    assert np.array_equal(sigma[L:], r.trace["est_sigma"].astype(np.uint32))
    assert np.array_equal(tau[L:], r.trace["est_tau"].astype(np.uint32))
    g["perms"] = (sigma[:L], sigma_inv[:L], tau[:L])
    compare(g, r, K, B, L, w, seed)
    check_residual(g, sig.x, r.trace["tpos"])


def test_est_loops_repair_values(dev):
    """Collision-heavy location (2K/B = 16%, SNR 10 dB): loops with 4x the buckets that
    only estimate bring the L1 error down and every best-K frequency back."""
    import paper_2012_08238_amd  # noqa: F401
    for s in range(3):
        sig = make_signal(1 << 16, 20, 10.0, seed=300 + s)
        xh = np.fft.fft(sig.x) / (1 << 16)
        g0 = _run(dev, sig.x, K=20, B=256, L=5, w=2048, seed=s, n_resid=0)
        g1 = _run(dev, sig.x, K=20, B=256, L=5, w=2048, seed=s, n_resid=0, est_loops=4, est_B=1024)
        m0 = O.recovery_errors(xh, g0["idx"], g0["val"], 20)
        m1 = O.recovery_errors(xh, g1["idx"], g1["val"], 20)
        assert m1["L0"] == 0 and m1["L1"] < 0.05 and m0["L1"] > 2 * m1["L1"]


CFGS = [  # N, K, B, L, w, seed, est_loops, est_B
    (1 << 16, 20, 256, 5, 2048, 0, 4, 1024),
    (1 << 16, 20, 512, 7, 4096, 1, 0, 0),
    (1 << 14, 10, 128, 5, 512, 2, 1, 64),
    (1 << 20, 50, 1024, 7, 8192, 3, 2, 4096),
]


def _plan(S, c):
    N, K, B, L, w, seed, el, eb = c
    return S.Plan(N, K, B, L, w, seed=seed, n_resid=500, est_loops=el, est_B=eb)


def test_est_loops_batch_and_serve_bitwise(dev):
    import torch
    import paper_2012_08238_amd as S
    plans = [_plan(S, c) for c in CFGS]
    xs = [torch.from_numpy(make_signal(c[0], c[1], 15.0, seed=1300 + j).x.astype(np.complex64)).to(dev)
          for j, c in enumerate(CFGS)]
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
    # served in a mix (twice each), every result bitwise its single execution
    srv = S.Server(1 << 30, max_inflight=16, n_streams=2)
    tickets = []
    for rep in range(2):
        for j, c in enumerate(CFGS):
            N, K, B, L, w, seed, el, eb = c
            prm = S.PlanParams(N, K, B, L, w, seed=seed, n_resid=500, est_loops=el, est_B=eb)
            o = plans[j].outputs(dev)
            tickets.append((j, o, srv.submit(prm, xs[j], o[0], o[1], o[2])))
    for j, o, t in tickets:
        srv.wait(t)
        for a, b in zip(o, singles[j]):
            assert torch.equal(a, b), f"served signal {j}"
    srv.close()
    for p in plans:
        p.close()
