"""Uneven batch: 256 signals with N = 2^16..2^22, K = 10..500 and SNR -10..40 dB
(about 2.4 GB resident), one plan per signal from the untuned rule (B next to
sqrt(N K), w = 8B, L = 9). The batched graph must give every signal bitwise the
result of its single execution, on repeated replays; a sample is checked
against the oracle; and the autotuner's table entries are valid plans."""
import numpy as np
import pytest

from paper_2012_08238_amd.signals import derive_seed, make_signal_torch, uneven_batch_specs
from parity import compare
from test_gpu_parity import _oracle

pytestmark = pytest.mark.gpu


def _setup(dev, n=256):
    import paper_2012_08238_amd as S
    from paper_2012_08238_amd import autotune as A
    specs = uneven_batch_specs(n, seed=4)
    plans, xs, truth = [], [], []
    for i, (N, K, snr) in enumerate(specs):
        plans.append(S.Plan.from_params(A.rule_params(N, K, seed=i)))
        x, f, _ = make_signal_torch(N, K, snr, derive_seed(40, i), dev)
        xs.append(x)
        truth.append(f)
    return specs, plans, xs, truth


def test_uneven_batch_matches_single(dev):
    import torch
    import paper_2012_08238_amd as S
    specs, plans, xs, truth = _setup(dev)
    singles = []
    for p, x in zip(plans, xs):
        singles.append(tuple(t.clone() for t in p(x, residual=True)))
    torch.cuda.synchronize()
    b = S.Batch(plans)
    outs = [p.outputs(dev) for p in plans]
    for rep in range(2):
        for o in outs:
            o[0].fill_(-7)
        b.run(xs, [o[0] for o in outs], [o[1] for o in outs], [o[2] for o in outs])
        torch.cuda.synchronize()
        for i, (o, s1) in enumerate(zip(outs, singles)):
            for u, v in zip(o, s1):
                assert torch.equal(u, v), f"replay {rep}, signal {i} {specs[i]}"
    # accuracy where the noise allows it: recall of the planted tones at SNR >= 10 dB
    rec = []
    for (N, K, snr), o, f in zip(specs, outs, truth):
        if snr >= 10.0:
            rec.append(len(set(o[0].cpu().numpy().tolist()) & set(f.tolist())) / K)
    assert np.mean(rec) > 0.98
    b.close()
    for p in plans:
        p.close()


def test_uneven_sample_vs_oracle(dev):
    """A sample of the batch's signals (single execution = batch result, bitwise)."""
    import torch
    import paper_2012_08238_amd as S
    from paper_2012_08238_amd import autotune as A
    specs = uneven_batch_specs(256, seed=4)
    picks = [0, 1, 2, 3, 17, 100]
    for i in picks:
        N, K, snr = specs[i]
        prm = A.rule_params(N, K, seed=i)
        x, f, _ = make_signal_torch(N, K, snr, derive_seed(40, i), dev)
        p = S.Plan.from_params(prm)
        idx, val, res = p(x, residual=True)
        torch.cuda.synchronize()
        g = dict(idx=idx.cpu().numpy(), val=val.cpu().numpy().astype(np.complex128), resid=res.cpu().numpy(),
                 trace=p.trace(), perms=p.perms(), desc=p.desc)
        p.close()
        x64 = x.cpu().numpy().astype(np.complex128)
        r = _oracle(x64, K, prm.B, prm.L, prm.w, i)
        compare(g, r, K, prm.B, prm.L, prm.w, i)


def test_autotune_small_classes(dev, tmp_path):
    import torch
    import paper_2012_08238_amd as S
    from paper_2012_08238_amd import autotune as A
    t = A.Table(str(tmp_path / "tune.json"))
    for N, K in ((1 << 16, 40), (1 << 18, 200)):
        e = t.get(N, K, dev, probes=2, reps=3)
        assert e["B"] in A.b_candidates(N, A.class_k(K)) and e["wB"] in (4, 8)
        assert e["recall"] > 0.9 and e["ms"] > 0
        prm = t.params(N, K, seed=3, tune=False)
        p = S.Plan.from_params(prm)
        x, f, _ = make_signal_torch(N, K, 20.0, 99, dev)
        idx, _ = p(x)
        torch.cuda.synchronize()
        assert len(set(idx.cpu().numpy().tolist()) & set(f.tolist())) >= 0.95 * K
        p.close()
    assert len(A.Table(t.path).entries) == 2
