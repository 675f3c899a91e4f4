"""The benchmark's timed step, in its own launch configuration: 64 resident signals
of N=2^22, K=100, SNR 20 dB through one batch graph per step (B=16384, L=9, w=8B),
three steps in flight on three streams; with the benchmark's default one-workgroup
B-point FFT and with the two-pass form it offers. Every batch output
is bitwise the signal's single execution; sampled signals are compared with the
FP64 oracle (spectra, selections, candidates, support, values, residual) and every
signal's support with its planted tones."""
import numpy as np
import pytest

from paper_2012_08238_amd.signals import derive_seed, make_signal_torch
from parity import compare
from test_gpu_parity import _oracle, check_residual

pytestmark = pytest.mark.gpu

N, K, B, L, M, INFLIGHT, SEED = 1 << 22, 100, 16384, 9, 64, 3, 1
W = 8 * B
SAMPLED = (0, 37, 63)


@pytest.mark.parametrize("fft", ["one-workgroup", "two-pass"])
def test_benchmark_step_configuration(dev, fft):
    import torch
    import paper_2012_08238_amd as S
    xs, truth = [], []
    for i in range(M):
        x, f, _ = make_signal_torch(N, K, 20.0, derive_seed(0, i), dev)
        xs.append(x)
        truth.append(np.sort(f))
    plan = S.Plan(N, K, B, L, W, seed=SEED, flags=S.SFFT_FLAG_FFT_TWO_PASS if fft == "two-pass" else 0)
    batches, outs, streams = [], [], []
    for j in range(INFLIGHT):
        batches.append(S.Batch([plan] * M, branches=1))
        idx = torch.full((M, K), -7, dtype=torch.int64, device=dev)
        val = torch.zeros((M, K), dtype=torch.complex64, device=dev)
        res = torch.zeros((M, 2), dtype=torch.float64, device=dev)
        outs.append((idx, val, res))
        streams.append(torch.cuda.current_stream() if j == 0 else torch.cuda.Stream(device=dev))
    torch.cuda.synchronize()
    for step in range(2 * INFLIGHT):   # consecutive steps alternate over the batches
        j = step % INFLIGHT
        idx, val, res = outs[j]
        batches[j].run(xs, [idx[i] for i in range(M)], [val[i] for i in range(M)], [res[i] for i in range(M)],
                       stream=streams[j])
    torch.cuda.synchronize()
    for b in batches:
        b.close()
    host = [tuple(t.cpu().numpy() for t in o) for o in outs]
    for j in range(1, INFLIGHT):
        for a, c in zip(host[0], host[j]):
            assert np.array_equal(a, c), f"batch {j} differs from batch 0"
    idx_h, val_h, res_h = host[0]
    for i in range(M):
        assert np.array_equal(idx_h[i], truth[i]), f"signal {i} support"
    for i in SAMPLED:
        ri, rv, rr = plan(xs[i], residual=True)
        torch.cuda.synchronize()
        assert np.array_equal(ri.cpu().numpy(), idx_h[i]), f"signal {i} index vs single execution"
        assert np.array_equal(rv.cpu().numpy(), val_h[i]), f"signal {i} values vs single execution"
        assert np.array_equal(rr.cpu().numpy(), res_h[i]), f"signal {i} residual vs single execution"
        g = dict(idx=idx_h[i], val=val_h[i].astype(np.complex128), resid=res_h[i],
                 trace=plan.trace(), perms=plan.perms(), desc=plan.desc)
        x64 = xs[i].cpu().numpy().astype(np.complex128)
        r = _oracle(x64, K, B, L, W, SEED)
        p = compare(g, r, K, B, L, W, SEED)
        assert p.certain == K and p.values == K, p
        check_residual(g, x64, r.trace["tpos"])
    plan.close()
