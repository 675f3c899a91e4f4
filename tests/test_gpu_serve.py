"""Serving loop on the GPU: every request's result is bitwise the one its
parameter set gives alone, whether it ran alone or in a mix of other sizes,
under a tight memory budget with table eviction, and with waves overlapping;
served results of C5's sizes (up to N = 2^24) against the FP64 oracle."""
import numpy as np
import pytest

from paper_2012_08238_amd.signals import make_signal

pytestmark = pytest.mark.gpu

MIX = [  # (N, K, B, L, w, seed, snr, flags)
    (1 << 14, 10, 128, 5, 512, 3, None, 0),
    (1 << 16, 20, 512, 7, 4096, 5, 10.0, 0),
    (1 << 20, 50, 1024, 7, 8192, 6, 20.0, 0),
    (1 << 18, 30, 2048, 9, 16384, 7, 20.0, 0x2),   # gather form
    (1 << 12, 4, 64, 4, 256, 8, 30.0, 0x1),        # even L, no residual
    (1 << 22, 100, 16384, 9, 131072, 1, 20.0, 0),  # strip form, the benchmark shape
    (1 << 15, 8, 256, 7, 2048, 9, 20.0, 0x400),    # fused one-launch form
]


def _params(S, cfg):
    N, K, B, L, w, seed, snr, flags = cfg
    return S.PlanParams(N, K, B, L, w, seed=seed, flags=flags)


def _alone(S, dev, cfgs, xs):
    """Reference results: each request on its own plan, executed alone."""
    import torch
    plans = {}
    refs = []
    for c, x in zip(cfgs, xs):
        if c not in plans:
            plans[c] = S.Plan.from_params(_params(S, c))
        p = plans[c]
        refs.append(tuple(t.clone() for t in p(x, residual=True)))
        torch.cuda.synchronize()
    for p in plans.values():
        p.close()
    return refs


def _outputs(dev, cfg):
    import torch
    K = cfg[1]
    return (torch.full((K,), -7, dtype=torch.int64, device=dev), torch.zeros(K, dtype=torch.complex64, device=dev),
            torch.zeros(2, dtype=torch.float64, device=dev))


def _signals(dev, cfgs, base):
    import torch
    return [torch.from_numpy(make_signal(c[0], c[1], c[6], seed=base + i).x.astype(np.complex64)).to(dev)
            for i, c in enumerate(cfgs)]


def _same(out, ref, cfg):
    import torch
    idx, val, res = out
    ri, rv, rr = ref
    assert torch.equal(idx, ri)
    assert torch.equal(val.view(torch.float32), rv.view(torch.float32))
    if not cfg[7] & 0x1:
        assert torch.equal(res, rr)


def test_serve_mix_matches_alone(dev):
    import torch
    import paper_2012_08238_amd as S
    cfgs = [MIX[i % len(MIX)] for i in range(30)]
    xs = _signals(dev, cfgs, 900)
    refs = _alone(S, dev, cfgs, xs)
    srv = S.Server(hbm_budget_bytes=2 << 30, max_inflight=64, n_streams=3)
    handles = {c: srv.prepare(_params(S, c)) for c in set(cfgs)}
    outs = [_outputs(dev, c) for c in cfgs]
    torch.cuda.synchronize()
    tickets = []
    # a first burst, a few completions, then more requests while others run
    for i in range(12):
        tickets.append(srv.submit(handles[cfgs[i]], xs[i], *outs[i]))
    lat0, st0 = srv.wait(tickets[0])
    assert st0 == 0 and lat0 > 0
    for i in range(12, 30):
        tickets.append(srv.submit(handles[cfgs[i]], xs[i], *outs[i]))
    for t in tickets[1:]:
        lat, st = srv.wait(t)
        assert st == 0 and lat > 0
    torch.cuda.synchronize()
    for i, c in enumerate(cfgs):
        _same(outs[i], refs[i], c)
    s = srv.stats()
    assert s["completed"] == 30 and s["failed"] == 0
    assert s["batches"] < 30 and s["max_batch"] > 1        # requests were batched
    assert s["hbm_peak"] <= s["hbm_budget"]
    assert s["p99_latency_s"] >= s["p50_latency_s"] > 0
    srv.close()


def test_serve_waves_overlap(dev):
    """Requests submitted while earlier waves run go out as further waves on the other
    streams: at least two waves are on the device at once, and every result is bitwise
    its single execution."""
    import torch
    import paper_2012_08238_amd as S
    c = MIX[5]
    n = 24
    xs = _signals(dev, [c] * 6, 950)
    refs = _alone(S, dev, [c] * 6, xs)
    srv = S.Server(hbm_budget_bytes=2 << 30, max_inflight=n, n_streams=4)
    h = srv.prepare(_params(S, c))
    outs = [_outputs(dev, c) for _ in range(n)]
    torch.cuda.synchronize()
    tickets = [srv.submit(h, xs[i % 6], *outs[i]) for i in range(n)]
    for t in tickets:
        assert srv.wait(t)[1] == 0
    for i in range(n):
        _same(outs[i], refs[i % 6], c)
    s = srv.stats()
    assert s["completed"] == n
    assert s["max_waves_in_flight"] >= 2, s
    srv.close()


# C5's sizes with the serving loop's parameter rule (B next to sqrt(N K), w = 8B, L = 9):
# (N, K, SNR dB, seed); N = 2^24 at both ends of K (two-pass and one-workgroup FFT)
C5_MIX = [(1 << 24, 1000, 20.0, 1), (1 << 24, 20, 5.0, 2), (1 << 18, 300, 0.0, 3),
          (1 << 20, 700, 30.0, 4), (1 << 22, 64, 12.0, 5)]


def test_served_results_match_oracle(dev):
    """Requests of C5's sizes (N = 2^18 .. 2^24) served in a mix, each twice: every
    served result is bitwise its plan executed alone, and is compared with the FP64
    oracle through the parity protocol (the alone execution supplies the trace of
    the same computation)."""
    import dataclasses

    import torch
    import oracle.sfft_oracle as O
    import paper_2012_08238_amd as S
    from paper_2012_08238_amd import autotune as A
    from parity import compare
    from test_gpu_parity import check_residual
    prms = [dataclasses.replace(A.rule_params(N, K, seed=sd), n_resid=1000) for N, K, _, sd in C5_MIX]
    sigs = [make_signal(N, K, snr, seed=1500 + sd) for N, K, snr, sd in C5_MIX]
    xs = [torch.from_numpy(sg.x.astype(np.complex64)).to(dev) for sg in sigs]
    order = [0, 2, 1, 4, 3, 1, 0, 3, 2, 4]
    srv = S.Server(hbm_budget_bytes=6 << 30, max_inflight=16, n_streams=3)
    outs = [(torch.full((prms[j].K,), -7, dtype=torch.int64, device=dev),
             torch.zeros(prms[j].K, dtype=torch.complex64, device=dev),
             torch.zeros(2, dtype=torch.float64, device=dev)) for j in order]
    torch.cuda.synchronize()
    tickets = [srv.submit(prms[j], xs[j], *o) for j, o in zip(order, outs)]
    for t in tickets:
        assert srv.wait(t)[1] == 0
    assert srv.stats()["completed"] == len(order)
    srv.close()
    for j, (prm, sg, x) in enumerate(zip(prms, sigs, xs)):
        plan = S.Plan.from_params(prm)
        ai, av, ar = plan(x, residual=True)
        torch.cuda.synchronize()
        for k in [k for k, jj in enumerate(order) if jj == j]:
            assert torch.equal(outs[k][0], ai) and torch.equal(outs[k][1].view(torch.float32), av.view(torch.float32))
            assert torch.equal(outs[k][2], ar)
        k = order.index(j)
        g = dict(idx=outs[k][0].cpu().numpy(), val=outs[k][1].cpu().numpy().astype(np.complex128),
                 resid=outs[k][2].cpu().numpy(), trace=plan.trace(), perms=plan.perms())
        plan.close()
        x64 = sg.x.astype(np.complex64).astype(np.complex128)
        r = O.sfft(x64, prm.K, prm.B, prm.L, prm.w, seed=prm.seed, n_resid=1000)
        p = compare(g, r, prm.K, prm.B, prm.L)
        assert p.values >= 1, p
        check_residual(g, sg.x, r.trace["tpos"])


def test_serve_tight_budget_evicts(dev):
    import torch
    import paper_2012_08238_amd as S
    a, b = MIX[2], MIX[3]
    pa, pb = S.Plan.from_params(_params(S, a)), S.Plan.from_params(_params(S, b))
    da, db = pa.describe(), pb.describe()
    pa.close()
    pb.close()
    r256 = lambda v: (v + 255) // 256 * 256  # noqa: E731
    # room for one plan's tables and one workspace of the larger request, not for both plans
    budget = max(r256(da["table_bytes"]) + r256(da["workspace_bytes"]),
                 r256(db["table_bytes"]) + r256(db["workspace_bytes"])) + 4096
    budget = max(budget, 1 << 20)
    need_both = r256(da["table_bytes"]) + r256(db["table_bytes"]) + max(r256(da["workspace_bytes"]),
                                                                       r256(db["workspace_bytes"]))
    cfgs = [a, b, a, a, b, b, a, b]
    xs = _signals(dev, cfgs, 970)
    refs = _alone(S, dev, cfgs, xs)
    srv = S.Server(hbm_budget_bytes=budget, max_inflight=4, n_streams=2)
    outs = [_outputs(dev, c) for c in cfgs]
    torch.cuda.synchronize()
    tickets = [srv.submit(_params(S, c), x, *o) for c, x, o in zip(cfgs, xs, outs)]
    for t in tickets:
        assert srv.wait(t)[1] == 0
    for i, c in enumerate(cfgs):
        _same(outs[i], refs[i], c)
    s = srv.stats()
    assert s["completed"] == 8 and s["hbm_peak"] <= budget
    if need_both > budget:
        assert s["plan_cache_evictions"] > 0
    srv.close()


def test_serve_errors(dev):
    import torch
    import paper_2012_08238_amd as S
    srv = S.Server(hbm_budget_bytes=1 << 20, max_inflight=2, n_streams=1)
    x = torch.zeros(1 << 22, dtype=torch.complex64, device=dev)
    o = _outputs(dev, MIX[5])
    with pytest.raises(S.SfftError) as e:
        srv.submit(_params(S, MIX[5]), x, *o)        # never fits 1 MiB
    assert e.value.status == -2
    with pytest.raises(S.SfftError) as e:
        srv.submit(S.PlanParams(1 << 14, 10, 100, 5, 512), x, *o)   # B not a power of two
    assert e.value.status == -1
    with pytest.raises(S.SfftError) as e:
        srv.poll(12345)
    assert e.value.status == -6
    s = srv.stats()
    assert s["rejected"] == 2 and s["submitted"] == 0
    srv.close()


def test_serve_submit_many(dev):
    """A burst queued in one call: results bitwise those of each request alone, tickets in
    order, waves of several requests; all or none on a bad pointer."""
    import torch
    import paper_2012_08238_amd as S
    cfg = MIX[1]
    n = 48
    xs = _signals(dev, [cfg] * n, 1200)
    refs = _alone(S, dev, [cfg] * n, xs)
    srv = S.Server(hbm_budget_bytes=1 << 30, max_inflight=32, n_streams=2)
    outs = [_outputs(dev, cfg) for _ in range(n)]
    torch.cuda.synchronize()
    params = _params(S, cfg)
    ts = srv.submit_many(params, xs, [o[0] for o in outs], [o[1] for o in outs], [o[2] for o in outs])
    assert len(set(ts)) == n and ts == sorted(ts)
    for t in ts:
        _, st = srv.wait(t)
        assert st == 0
    for o, r in zip(outs, refs):
        _same(o, r, cfg)
    s = srv.stats()
    assert s["submitted"] == n and s["completed"] == n and s["max_batch"] > 1
    bad = list(xs[:4])
    bad[2] = xs[2][1:]   # 8 bytes off the 16-byte alignment
    with pytest.raises(S.SfftError) as e:
        srv.submit_many(params, bad, [o[0] for o in outs[:4]], [o[1] for o in outs[:4]])
    assert e.value.status == -1
    assert srv.stats()["submitted"] == n      # nothing of the refused burst was queued
    assert srv.submit_many(params, [], [], []) == []
    srv.close()
