"""Serving loop on the GPU: every request's result is bitwise the one its
parameter set gives alone, whether it ran alone or in a mix of other sizes,
under a tight memory budget with table eviction, and with waves overlapping."""
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
    import torch
    import paper_2012_08238_amd as S
    c = MIX[5]
    cfgs = [c] * 6
    xs = _signals(dev, cfgs, 950)
    refs = _alone(S, dev, cfgs, xs)
    srv = S.Server(hbm_budget_bytes=1 << 30, max_inflight=8, n_streams=4)
    h = srv.prepare(_params(S, c))
    outs = [_outputs(dev, c) for _ in cfgs]
    torch.cuda.synchronize()
    tickets = []
    for i in range(6):
        tickets.append(srv.submit(h, xs[i], *outs[i]))
    for t in tickets:
        assert srv.wait(t)[1] == 0
    for i in range(6):
        _same(outs[i], refs[i], c)
    s = srv.stats()
    assert s["completed"] == 6
    srv.close()


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
