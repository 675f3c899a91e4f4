"""Batched execution: every signal's result is bitwise the one it gets alone,
on every replay of the captured graphs, with eager work in between."""
import numpy as np
import pytest

from paper_2012_08238_amd.signals import make_signal

pytestmark = pytest.mark.gpu

CONFIGS = [  # (N, K, B, L, w, seed, snr)
    (1 << 14, 10, 128, 5, 512, 0, None),
    (1 << 16, 20, 512, 7, 4096, 1, 10.0),
    (1 << 18, 40, 2048, 9, 16384, 2, 20.0),
    (1 << 20, 50, 1024, 7, 8192, 3, 20.0),      # gather form
    (1 << 22, 100, 16384, 9, 131072, 4, 20.0),  # strip form, the benchmark shape
    (1 << 12, 3, 8, 4, 64, 5, -5.0),
    (1 << 16, 10, 512, 20, 4096, 6, 15.0),      # L > 16: one vote launch for both of these,
    (1 << 15, 8, 256, 32, 2048, 7, 15.0),       # each signal with its own L
]


@pytest.mark.parametrize("branches", [1, 2, 3])
def test_batch_matches_single(dev, branches):
    import torch
    import paper_2012_08238_amd as S
    plans, xs = [], []
    for j, (N, K, B, L, w, seed, snr) in enumerate(CONFIGS):
        plans.append(S.Plan(N, K, B, L, w, seed=seed, n_resid=1000 + 7 * j))
        xs.append(torch.from_numpy(make_signal(N, K, snr, seed=500 + j).x.astype(np.complex64)).to(dev))
    # repeat two plans with other signals: each batch entry has its own workspace
    order = list(range(len(CONFIGS))) + [4, 0]
    extra = {4: torch.from_numpy(make_signal(1 << 22, 100, 20.0, seed=777).x.astype(np.complex64)).to(dev),
             0: torch.from_numpy(make_signal(1 << 14, 10, None, seed=778).x.astype(np.complex64)).to(dev)}
    bx = [xs[i] for i in range(len(CONFIGS))] + [extra[4], extra[0]]
    bplans = [plans[i] for i in order]
    singles = []
    for p, x in zip(bplans, bx):
        singles.append(tuple(t.clone() for t in p(x, residual=True)))
    torch.cuda.synchronize()
    batch = S.Batch(bplans, branches=branches)
    outs = [p.outputs(dev) for p in bplans]
    for rep in range(3):
        for o in outs:
            for t in o:
                t.zero_()
        batch.run(bx, [o[0] for o in outs], [o[1] for o in outs], [o[2] for o in outs])
        # eager work between replays: single executions and torch ops on the same stream
        _ = bplans[0](bx[0])
        _ = (bx[4].abs() ** 2).sum()
        torch.cuda.synchronize()
        for j, (o, s) in enumerate(zip(outs, singles)):
            for a, b in zip(o, s):
                assert torch.equal(a, b), f"replay {rep}, signal {j}"
    batch.close()
    for p in plans:
        p.close()


def test_batch_timed_events(dev):
    import torch
    import paper_2012_08238_amd as S
    N, K, B, L, w = 1 << 20, 50, 1024, 7, 8192
    p = S.Plan(N, K, B, L, w, seed=9, flags=S.SFFT_FLAG_FOLD_STRIP)
    xs = [torch.from_numpy(make_signal(N, K, 20.0, seed=s).x.astype(np.complex64)).to(dev) for s in range(4)]
    b = S.Batch([p] * 4)
    outs = [p.outputs(dev) for _ in range(4)]
    from paper_2012_08238_amd._hip import HipEvent
    e0, e1 = HipEvent(), HipEvent()
    b.run_timed(xs, [o[0] for o in outs], [o[1] for o in outs], [o[2] for o in outs], e0, e1)
    torch.cuda.synchronize()
    assert e0.elapsed_ms(e1) > 0
    for x, o in zip(xs, outs):
        ref = p(x, residual=True)
        torch.cuda.synchronize()
        for a, c in zip(o, ref):
            assert torch.equal(a, c)
    b.close()
    p.close()


def test_branched_batch_refuses_fold_events(dev):
    import torch
    import paper_2012_08238_amd as S
    from paper_2012_08238_amd._hip import HipEvent
    N, K, B, L, w = 1 << 16, 10, 512, 5, 4096
    p = S.Plan(N, K, B, L, w, seed=1)
    xs = [torch.from_numpy(make_signal(N, K, 20.0, seed=s).x.astype(np.complex64)).to(dev) for s in range(4)]
    b = S.Batch([p] * 4, branches=2)
    outs = [p.outputs(dev) for _ in range(4)]
    with pytest.raises(S.SfftError) as e:
        b.run_timed(xs, [o[0] for o in outs], [o[1] for o in outs], [o[2] for o in outs], HipEvent(), HipEvent())
    assert e.value.status == -4
    b.run(xs, [o[0] for o in outs], [o[1] for o in outs], [o[2] for o in outs])
    torch.cuda.synchronize()
    for x, o in zip(xs, outs):
        ref = p(x, residual=True)
        torch.cuda.synchronize()
        for a, c in zip(o, ref):
            assert torch.equal(a, c)
    b.close()
    p.close()
