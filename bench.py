#!/usr/bin/env python3
"""Throughput benchmark of the gfx950 flat-window voting sparse FFT.

Workload: N = 2^22 complex64 signals with K = 100 unit tones at uniform random
positions and phases plus complex white noise at 20 dB SNR; B = 16384 buckets,
L = 9 random bucketizations, window w = 8B = 131072, 2K buckets kept per loop,
strict-majority vote, median estimate, FP64 residual on 4096 samples.
A step is one pass of the whole path over a batch of signals resident in HBM
(one HIP graph replay: bucketization, B-point FFT + selection in one workgroup's
LDS per loop, votes, estimation and output, residual); three steps are kept in
flight on three streams with their own workspaces and outputs, so one step's
last stages overlap the next step's bucketization (--fft two-pass selects the
two-pass FFT instead). value = signals recovered per second.

Also reported: the bucketization kernel's roofline against MI355X HBM peak
(algorithmic bytes 8 N (1 - (1 - w/N)^L) per signal, the sampled fraction of
Table 2 with log N -> L), beside its line-granular bound (the 128-byte lines
holding a sample) and its measured traffic; p50/p99 latency through the serving
loop under Poisson arrivals and its saturated throughput; the plain single-signal
path's throughput; single-request latency; FP32-vs-FP64 parity on a sample; the
one-launch fused form against the graph of stage launches on small plans; and
the FP64 CPU oracle timed on the host (one core, and a pool over every core).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N, K, B, L, SNR_DB = 1 << 22, 100, 16384, 9, 20.0
PLAN_SEED = 1
HBM_PEAK_GBPS = 8000.0
PROFILE_COUNTERS = os.path.join(ROOT, "profiles", "fold_strip_pf_kernel_n22_k100_b64_counters.md")
KERNEL_SRC = [os.path.join(ROOT, "paper_2012_08238_amd", "csrc", f) for f in ("fold.hip", "fold_dev.hpp")]  # the bucketization


def alg_bytes_per_signal(W: int) -> float:
    return 8.0 * N * (1.0 - (1.0 - W / N) ** L)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for path in KERNEL_SRC:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def vote_flags(args) -> int:
    import paper_2012_08238_amd as S
    return {"auto": 0, "loop": S.SFFT_FLAG_VOTE_BY_LOOP, "pair": S.SFFT_FLAG_VOTE_BY_PAIR}[args.vote]


def committed_traffic(batch: int):
    """HBM bytes per bucketization launch from the committed counter summary,
    or None when it is absent, for another batch, or the kernel source changed."""
    if not os.path.exists(PROFILE_COUNTERS):
        return None
    text = open(PROFILE_COUNTERS).read()
    h = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", text)
    t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    b = re.search(r"batch:\s*(\d+)", text)
    if not (h and t and b) or h.group(1) != kernel_source_hash() or int(b.group(1)) != batch:
        return None
    return float(t.group(1))


# Oracle timings beside the metric's: (N, K, SNR dB or None, B, L, w) of the exactly sparse
# N=2^14 case and the N=2^20 general-sparse case
ORACLE_CONFIGS = {"n14_k10_exact": (1 << 14, 10, None, 128, 5, 512),
                  "n20_k50_snr20": (1 << 20, 50, 20.0, 1024, 7, 8192)}


def _oracle_one(job):
    """Pool worker: the FP64 oracle on one complex64 signal; returns its seconds."""
    import numpy as np
    import oracle.sfft_oracle as O
    x, (k, b, l, w, seed) = job
    a = time.perf_counter()
    O.sfft(np.asarray(x).astype(np.complex128), k, b, l, w, seed=seed)
    return time.perf_counter() - a


def oracle_pool_seconds(signals, params, workers: int) -> float:
    """Wall time of the oracle over `signals` in a pool of single-threaded worker processes
    (fresh interpreters that never touch the GPU)."""
    import multiprocessing as mp
    env = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in env:
        os.environ[k] = "1"
    try:
        with mp.get_context("spawn").Pool(workers) as pool:
            pool.map(_oracle_one, [(signals[0][:16], (1, 2, 1, 2, 0))] * workers)   # start every worker
            a = time.perf_counter()
            pool.map(_oracle_one, [(x, params) for x in signals], chunksize=1)
            return time.perf_counter() - a
    finally:
        for k, v in env.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def oracle_config_seconds(n, k, snr, b, l, w, count: int = 20) -> dict:
    """Single-core oracle time per signal over `count` signals of one configuration."""
    import numpy as np
    import oracle.sfft_oracle as O
    from paper_2012_08238_amd.signals import derive_seed, make_signal
    ts = []
    for i in range(count):
        x = make_signal(n, k, snr, seed=derive_seed(7, i)).x.astype(np.complex64).astype(np.complex128)
        a = time.perf_counter()
        O.sfft(x, k, b, l, w, seed=i)
        ts.append(time.perf_counter() - a)
    return {"N": n, "K": k, "B": b, "L": l, "w": w, "snr_db": snr, "signals": count, "cores": 1,
            "signals_per_s": round(count / sum(ts), 3), "p50_s": round(percentile(ts, 0.5), 5),
            "p99_s": round(percentile(ts, 0.99), 5)}


def percentile(v, q):
    v = sorted(v)
    if not v:
        return None
    k = (len(v) - 1) * q
    lo = int(k)
    hi = min(lo + 1, len(v) - 1)
    return v[lo] + (v[hi] - v[lo]) * (k - lo)


def serve_measure(S, torch, dev, xs, truth, args) -> dict:
    """Serving loop on the resident signals: Poisson arrivals at --serve-rate
    requests/s for --serve-seconds (latency = submission to completion), then a
    saturated burst (every request queued at once) for served throughput."""
    import numpy as np
    M = len(xs)
    srv = S.Server(hbm_budget_bytes=args.serve_budget_gib << 30, max_inflight=args.serve_inflight,
                   n_streams=args.serve_streams)
    fflags = {"auto": 0, "strip": S.SFFT_FLAG_FOLD_STRIP, "gather": S.SFFT_FLAG_FOLD_GATHER}[args.fold]
    fflags |= S.SFFT_FLAG_FFT_TWO_PASS if args.fft == "two-pass" and 4096 <= B <= 16384 else 0
    fflags |= vote_flags(args)
    h = srv.prepare(S.PlanParams(N, K, B, L, args.w_over_b * B, seed=PLAN_SEED, strip_cols=args.strip_cols,
                                 flags=fflags))
    n = max(1, int(args.serve_rate * args.serve_seconds))
    nb = args.serve_burst
    idx = torch.empty((max(n, nb), K), dtype=torch.int64, device=dev)
    val = torch.empty((max(n, nb), K), dtype=torch.complex64, device=dev)
    res = torch.empty((max(n, nb), 2), dtype=torch.float64, device=dev)
    # warm the tables into the arena
    srv.wait(srv.submit(h, xs[0], idx[0], val[0], res[0]))
    rng = np.random.default_rng(2000)
    arrivals = np.cumsum(rng.exponential(1.0 / args.serve_rate, n))
    tickets = []
    t0 = time.perf_counter()
    for i in range(n):
        target = t0 + arrivals[i]
        while True:
            d = target - time.perf_counter()
            if d <= 0:
                break
            if d > 2e-4:
                time.sleep(d - 1.5e-4)
        tickets.append(srv.submit(h, xs[i % M], idx[i], val[i], res[i]))
    lats = [srv.wait(t)[0] for t in tickets]
    t_open = time.perf_counter() - t0
    open_stats = srv.stats()
    ok = sum(set(idx[i].tolist()) == set(truth[i % M][0].tolist()) for i in range(min(n, 256)))
    # saturated: queue nb requests at once, time until the last completes
    burst = ([xs[i % M] for i in range(nb)], [idx[i] for i in range(nb)], [val[i] for i in range(nb)],
             [res[i] for i in range(nb)])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tickets = srv.submit_many(h, *burst)   # one call: the burst is admitted at once
    for t in tickets:
        srv.wait(t)
    t_sat = time.perf_counter() - t1
    st = srv.stats()
    srv.close()
    lat_ms = sorted(x * 1e3 for x in lats)
    return {
        "poisson": {"rate_req_s": args.serve_rate, "requests": n, "seconds": round(t_open, 3),
                    "p50_ms": round(percentile(lat_ms, 0.5), 4), "p99_ms": round(percentile(lat_ms, 0.99), 4),
                    "mean_ms": round(sum(lat_ms) / len(lat_ms), 4),
                    "waves": open_stats["batches"] - 1, "max_wave": open_stats["max_batch"],
                    "exact_support_sampled": f"{ok}/{min(n, 256)}"},
        "saturated": {"requests": nb, "signals_per_s": round(nb / t_sat, 1),
                      "waves": st["batches"] - open_stats["batches"], "max_wave": st["max_batch"],
                      "max_waves_in_flight": st["max_waves_in_flight"]},
        "config": {"hbm_budget_gib": args.serve_budget_gib, "max_inflight": args.serve_inflight,
                   "streams": args.serve_streams, "hbm_peak_bytes": st["hbm_peak"]},
    }


def snr_sweep(S, torch, dev, args) -> dict:
    """L0/L1/L2 error against the best K-term approximation (the dense FP64
    spectrum of each signal) versus SNR, median and mean of the loop estimates
    (the robustness experiment): N=2^20, K=50, B=1024, L=7, w=8B, signals per point."""
    from paper_2012_08238_amd.signals import derive_seed, make_signal_torch
    n, k, b, l = 1 << 20, 50, 1024, 7
    plans = {c: S.Plan(n, k, b, l, 8 * b, seed=11, flags=S.SFFT_FLAG_MEAN_ESTIMATE if c == "mean" else 0)
             for c in ("median", "mean")}
    out = {"N": n, "K": k, "B": b, "L": l, "w": 8 * b, "signals": args.sweep_signals, "points": []}
    for snr in (-10.0, 0.0, 10.0, 20.0, 30.0, 40.0):
        row = {"snr_db": snr}
        errs = {c: [0.0, 0.0, 0.0] for c in plans}
        for i in range(args.sweep_signals):
            x, _, _ = make_signal_torch(n, k, snr, derive_seed(60 + int(snr), i), dev)
            xh = torch.fft.fft(x.to(torch.complex128)) / n
            mag = xh.abs()
            best = torch.topk(mag, k).indices
            for c, p in plans.items():
                idx, val = p(x)
                got = idx[idx >= 0]
                est = torch.zeros(n, dtype=torch.complex128, device=dev)
                est[got] = val[idx >= 0].to(torch.complex128)
                ref = torch.zeros(n, dtype=torch.complex128, device=dev)
                ref[best] = xh[best]
                union = torch.unique(torch.cat([got, best]))
                d = (est - ref)[union]
                errs[c][0] += float(k - torch.isin(best, got).sum())
                errs[c][1] += float(d.abs().sum()) / k
                errs[c][2] += float((d.abs() ** 2).sum().sqrt())
        for c in plans:
            row[c] = {m: round(v / args.sweep_signals, 6) for m, v in zip(("L0", "L1", "L2"), errs[c])}
        out["points"].append(row)
    for p in plans.values():
        p.close()
    return out


def comb_measure(S, torch, dev, args) -> dict:
    """The comb prefilter (sFFT2.0 row) on batches of 64 resident signals: the
    C2 shape (N=2^20, K=50, B=1024, L=7, w=8B; 10% of the buckets kept per loop,
    so thousands of false frequencies pass the vote) and the benchmark shape with
    fewer buckets (N=2^22, K=100, B=4096, the comb disambiguating), each without
    and with the comb: signals/s, candidates per signal, exact supports."""
    from paper_2012_08238_amd.signals import derive_seed, make_signal_torch
    shapes = [("c2", 1 << 20, 50, 1024, 7, 0, 0), ("c2+comb", 1 << 20, 50, 1024, 7, 4096, 2),
              ("n22_b4096", 1 << 22, 100, 4096, 9, 0, 0), ("n22_b4096+comb", 1 << 22, 100, 4096, 9, 16384, 2)]
    out = {}
    m = args.comb_batch
    cache = {}
    for name, n, k, b, l, cb, cl in shapes:
        if (n, k) not in cache:
            cache[(n, k)] = [make_signal_torch(n, k, 20.0, derive_seed(70, i), dev) for i in range(m)]
        sigs = cache[(n, k)]
        plan = S.Plan(n, k, b, l, 8 * b, seed=13, comb_b=cb, comb_loops=cl)
        bt = S.Batch([plan] * m, branches=args.section_branches)
        outs = [plan.outputs(dev) for _ in range(m)]
        xs = [q[0] for q in sigs]
        for _ in range(2):
            bt.run(xs, [o[0] for o in outs], [o[1] for o in outs], [o[2] for o in outs])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.comb_steps):
            bt.run(xs, [o[0] for o in outs], [o[1] for o in outs], [o[2] for o in outs])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        exact = sum(set(o[0].cpu().numpy().tolist()) == set(q[1].tolist()) for o, q in zip(outs, sigs))
        plan.execute(xs[0], *outs[0])
        ncand = int(plan.trace()["cand"].shape[0])
        bt.close()
        plan.close()
        out[name] = {"N": n, "K": k, "B": b, "L": l, "w": 8 * b, "comb_b": cb, "comb_loops": cl,
                     "signals_per_s": round(m * args.comb_steps / el, 1), "candidates_signal0": ncand,
                     "exact_support": f"{exact}/{m}"}
    cache.clear()
    return out


def iterate_measure(S, torch, dev, args) -> dict:
    """One subtraction round of the iterative framework on batches of resident
    signals where the first recovery loses tones to shared buckets: N=2^22 with
    K=1000 in B=16384 buckets (2K/B = 12%), the C2 shape (N=2^20, K=50, B=1024,
    10%), and the benchmark shape (K=100, B=16384: the cost of the round where it
    is rarely needed); each without and with the round: signals/s, tones missed
    per signal (L0 against the planted support) and exact supports."""
    from paper_2012_08238_amd.signals import derive_seed, make_signal_torch
    shapes = [("n22_k1000_b16384", 1 << 22, 1000, 16384, 9), ("c2", 1 << 20, 50, 1024, 7),
              ("n22_k100_b16384", 1 << 22, 100, 16384, 9)]
    out = {}
    m = args.iter_batch
    for name, n, k, b, l in shapes:
        sigs = [make_signal_torch(n, k, 20.0, derive_seed(90, i), dev) for i in range(m)]
        xs = [q[0] for q in sigs]
        row = {"N": n, "K": k, "B": b, "L": l, "w": 8 * b, "snr_db": 20.0, "batch": m}
        for tag, fl in (("plain", 0), ("iterate", S.SFFT_FLAG_ITERATE)):
            plan = S.Plan(n, k, b, l, 8 * b, seed=17, flags=fl)
            bt = S.Batch([plan] * m, branches=args.section_branches)
            outs = [plan.outputs(dev) for _ in range(m)]
            for _ in range(2):
                bt.run(xs, [o[0] for o in outs], [o[1] for o in outs], [o[2] for o in outs])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.iter_steps):
                bt.run(xs, [o[0] for o in outs], [o[1] for o in outs], [o[2] for o in outs])
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            missed = [len(set(q[1].tolist()) - set(o[0].cpu().numpy().tolist())) for o, q in zip(outs, sigs)]
            row[tag] = {"signals_per_s": round(m * args.iter_steps / el, 1),
                        "missed_per_signal": round(sum(missed) / m, 3),
                        "exact_support": f"{sum(v == 0 for v in missed)}/{m}"}
            bt.close()
            plan.close()
        out[name] = row
        print(f"# subtraction round {name}: plain {row['plain']}, iterate {row['iterate']}", file=sys.stderr,
              flush=True)
    return out


def phase_measure(S, torch, dev, args) -> dict:
    """Phase-encoding location (the sFFT3.0 row) against voting on exactly sparse
    signals, N=2^22, K=100, w=8B, batches of resident signals: voting with the
    benchmark plan (B=16384, L=9) and phase location with two pairs (L=4) at
    B=16384 and B=4096, with and without the subtraction round: signals/s,
    exact supports and the largest value error against the planted tones."""
    import numpy as np
    from paper_2012_08238_amd.signals import derive_seed, make_signal_torch
    n, k = 1 << 22, 100
    m = args.phase_batch
    sigs = [make_signal_torch(n, k, None, derive_seed(110, i), dev) for i in range(m)]
    xs = [q[0] for q in sigs]
    P, I = S.SFFT_FLAG_PHASE_LOCATION, S.SFFT_FLAG_ITERATE
    runs = [("vote_b16384_L9", 16384, 9, 0), ("phase_b16384_L4", 16384, 4, P), ("phase_b16384_L4+iterate", 16384, 4, P | I),
            ("phase_b4096_L4", 4096, 4, P), ("phase_b4096_L4+iterate", 4096, 4, P | I)]
    out = {"N": n, "K": k, "snr_db": None, "batch": m}
    for name, b, l, fl in runs:
        plan = S.Plan(n, k, b, l, 8 * b, seed=19, flags=fl)
        bt = S.Batch([plan] * m, branches=args.section_branches)
        outs = [plan.outputs(dev) for _ in range(m)]
        for _ in range(2):
            bt.run(xs, [o[0] for o in outs], [o[1] for o in outs], [o[2] for o in outs])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.phase_steps):
            bt.run(xs, [o[0] for o in outs], [o[1] for o in outs], [o[2] for o in outs])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        exact, verr = 0, 0.0
        for o, q in zip(outs, sigs):
            gi, gv = o[0].cpu().numpy(), o[1].cpu().numpy()
            if set(gi.tolist()) == set(q[1].tolist()):
                exact += 1
                verr = max(verr, float(np.max(np.abs(gv - q[2][np.searchsorted(q[1], gi)]))))
        out[name] = {"B": b, "L": l, "signals_per_s": round(m * args.phase_steps / el, 1),
                     "exact_support": f"{exact}/{m}", "max_value_err_exact": verr}
        bt.close()
        plan.close()
        print(f"# phase location {name}: {out[name]}", file=sys.stderr, flush=True)
    return out


def est_loops_measure(S, torch, dev, args) -> dict:
    """Location and estimation loops separated: location with fewer buckets plus
    loops with 4x the buckets that only estimate, against the plain plan, on
    batches of resident signals at SNR 20 dB: signals/s, tones missed per signal
    and the median value error of the tones found (against the planted tones)."""
    import numpy as np
    from paper_2012_08238_amd.signals import derive_seed, make_signal_torch
    runs = [("c2_plain", 1 << 20, 50, 1024, 7, 0, 0), ("c2_loc512_est4x4096", 1 << 20, 50, 512, 7, 4, 4096),
            ("n22_plain_b16384", 1 << 22, 100, 16384, 9, 0, 0), ("n22_loc4096_est4x16384", 1 << 22, 100, 4096, 9, 4, 16384)]
    m = args.est_batch
    out = {"snr_db": 20.0, "batch": m}
    cache = {}
    for name, n, k, b, l, el, eb in runs:
        if (n, k) not in cache:
            cache.clear()
            cache[(n, k)] = [make_signal_torch(n, k, 20.0, derive_seed(130, i), dev) for i in range(m)]
        sigs = cache[(n, k)]
        xs = [q[0] for q in sigs]
        plan = S.Plan(n, k, b, l, 8 * b, seed=23, est_loops=el, est_B=eb)
        bt = S.Batch([plan] * m, branches=args.section_branches)
        outs = [plan.outputs(dev) for _ in range(m)]
        for _ in range(2):
            bt.run(xs, [o[0] for o in outs], [o[1] for o in outs], [o[2] for o in outs])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.est_steps):
            bt.run(xs, [o[0] for o in outs], [o[1] for o in outs], [o[2] for o in outs])
        torch.cuda.synchronize()
        el_s = time.perf_counter() - t0
        missed, errs = 0, []
        for o, q in zip(outs, sigs):
            gi, gv = o[0].cpu().numpy(), o[1].cpu().numpy()
            got = dict(zip(gi.tolist(), gv.tolist()))
            for f, tone in zip(q[1].tolist(), q[2].tolist()):
                if f in got:
                    errs.append(abs(got[f] - tone))
                else:
                    missed += 1
        out[name] = {"N": n, "K": k, "B": b, "L": l, "est_loops": el, "est_B": eb,
                     "signals_per_s": round(m * args.est_steps / el_s, 1), "missed_per_signal": round(missed / m, 3),
                     "median_value_err": float(np.median(errs)) if errs else None}
        bt.close()
        plan.close()
        print(f"# estimation loops {name}: {out[name]}", file=sys.stderr, flush=True)
    cache.clear()
    return out


def copy_bandwidth(torch, dev) -> float:
    """Achievable HBM bandwidth on this device: a 2 GiB device-to-device tensor
    copy (read + write bytes / time), best of 10."""
    n = 1 << 28   # complex64 elements: 2 GiB
    a = torch.empty(n, dtype=torch.complex64, device=dev)
    a.real.fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    best = 0.0
    for _ in range(10):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        best = max(best, 2.0 * 8 * n / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del a, b
    torch.cuda.empty_cache()
    return best


def dense_fft_context(torch, dev, xs) -> dict:
    """What the sparse path avoids: a dense N-point FFT of every signal of the
    batch on the same GPU (rocFFT through torch.fft, complex64), and one dense
    FP64 FFT of one signal on the host (numpy.fft, the fftw analogue)."""
    import numpy as np
    x = torch.stack(xs[:16])
    torch.fft.fft(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 5
    for _ in range(reps):
        torch.fft.fft(x)
    torch.cuda.synchronize()
    gpu = 16 * reps / (time.perf_counter() - t0)
    xh = xs[0].cpu().numpy().astype(np.complex128)
    np.fft.fft(xh)
    t0 = time.perf_counter()
    np.fft.fft(xh)
    cpu_s = time.perf_counter() - t0
    del x
    torch.cuda.empty_cache()
    return {"gpu_dense_fft_signals_per_s": round(gpu, 1), "gpu_dense_fft": "torch.fft.fft (rocFFT), complex64, 16 signals",
            "cpu_dense_fft_fp64_s": round(cpu_s, 4), "cpu_dense_fft": "numpy.fft.fft, one N=2^22 signal, FP64"}


def k_sweep_measure(S, torch, dev, args) -> dict:
    """The C3 sweep: N=2^22, SNR 20 dB, L=9, w=8B, K in {50, 100, 200, 500, 1000}
    with B = 2^round(log2 sqrt(N K)) (16384, 16384, 32768, 32768, 65536); batches of
    resident signals run as the benchmark step runs (--ksweep-inflight steps in flight on
    their own streams, workspaces, outputs and copies of the signals): signals/s, tones
    missed per signal, median value error against the planted tones (the FP32-vs-FP64
    parity of these shapes is a GPU test)."""
    import numpy as np
    from paper_2012_08238_amd.signals import derive_seed, make_signal_torch
    nf = max(1, args.ksweep_inflight)
    out = {"N": N, "L": L, "snr_db": SNR_DB, "batch": args.ksweep_batch, "steps_in_flight": nf, "points": []}
    m = args.ksweep_batch
    for k in (50, 100, 200, 500, 1000):
        b = 1 << int(round(np.log2(np.sqrt(N * k))))
        sigs = [make_signal_torch(N, k, SNR_DB, derive_seed(150 + k, i), dev) for i in range(m)]
        xs = [q[0] for q in sigs]
        xsets = [xs] + [[x.clone() for x in xs] for _ in range(nf - 1)]
        plan = S.Plan(N, k, b, L, 8 * b, seed=29)
        bts = [S.Batch([plan] * m, branches=args.branches) for _ in range(nf)]
        outsets = [[plan.outputs(dev) for _ in range(m)] for _ in range(nf)]
        streams = [torch.cuda.current_stream()] + [torch.cuda.Stream(device=dev) for _ in range(nf - 1)]
        for j in range(nf):
            bts[j].bind(xsets[j], [o[0] for o in outsets[j]], [o[1] for o in outsets[j]], [o[2] for o in outsets[j]])
        for _ in range(2):
            for j in range(nf):
                bts[j].run_bound(stream=streams[j])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for st in range(args.ksweep_steps):
            j = st % nf
            bts[j].run_bound(stream=streams[j])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        missed, errs = 0, []
        for o, q in zip(outsets[0], sigs):
            got = dict(zip(o[0].cpu().numpy().tolist(), o[1].cpu().numpy().tolist()))
            for f, tone in zip(q[1].tolist(), q[2].tolist()):
                if f in got:
                    errs.append(abs(got[f] - tone))
                else:
                    missed += 1
        pt = {"K": k, "B": b, "w": 8 * b, "signals_per_s": round(m * args.ksweep_steps / el, 1),
              "missed_per_signal": round(missed / m, 3), "median_value_err": float(np.median(errs)) if errs else None}
        out["points"].append(pt)
        for bt in bts:
            bt.close()
        plan.close()
        del sigs, xs, xsets, outsets
        print(f"# K sweep {pt}", file=sys.stderr, flush=True)
    return out


def fused_measure(S, torch, dev, args) -> dict:
    """The one-launch form (SFFT_FLAG_FUSED: one workgroup per signal, every stage in
    it) against the graph of batched stage launches, on small plans (the batch's
    small signals): time per replay of a batch of n signals, ten replays back to back
    between HIP events (median of three such runs after two warm replays), and
    single-signal latency (sfft_execute + stream sync, p50 of 30). Both forms give
    bitwise the same results (GPU test)."""
    import numpy as np
    from paper_2012_08238_amd.signals import derive_seed, make_signal_torch
    sizes = [int(v) for v in args.fused_batches.split(",") if v]
    out = {"batches": sizes, "shapes": []}
    for (ln, k, b, l, wb) in ((14, 10, 128, 5, 4), (16, 20, 512, 5, 8), (16, 50, 1024, 7, 8), (18, 100, 4096, 9, 8)):
        n = 1 << ln
        xs = [make_signal_torch(n, k, SNR_DB, derive_seed(170 + ln, i), dev)[0] for i in range(8)]
        row = {"N": n, "K": k, "B": b, "L": l, "w": wb * b}
        for name, fl in (("graph", 0), ("fused", S.SFFT_FLAG_FUSED)):
            plan = S.Plan(n, k, b, l, wb * b, seed=31, flags=fl)
            idx, val, res = plan.outputs(dev)
            for _ in range(3):
                plan.execute(xs[0], idx, val, res)
            torch.cuda.synchronize()
            lat = []
            for i in range(30):
                t0 = time.perf_counter()
                plan.execute(xs[i % 8], idx, val, res)
                torch.cuda.synchronize()
                lat.append(time.perf_counter() - t0)
            r = {"single_p50_us": round(percentile(lat, 0.5) * 1e6, 1)}
            for m in sizes:
                bx = [xs[j % 8] for j in range(m)]
                outs = [plan.outputs(dev) for _ in range(m)]
                cols = ([o[0] for o in outs], [o[1] for o in outs], [o[2] for o in outs])
                bt = S.Batch([plan] * m)
                bt.bind(bx, *cols)   # pointers marshalled once: the replays are not held up by the host
                for _ in range(2):
                    bt.run_bound()
                ts = []
                for _ in range(3):
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    for _ in range(10):
                        bt.run_bound()
                    e1.record()
                    e1.synchronize()
                    ts.append(e0.elapsed_time(e1) * 1e3 / 10)
                bt.close()
                us = float(np.median(ts))
                r[f"batch{m}_us"] = round(us, 1)
                r[f"batch{m}_signals_per_s"] = round(m / (us * 1e-6))
            row[name] = r
            plan.close()
        out["shapes"].append(row)
        print(f"# fused vs graph {row}", file=sys.stderr, flush=True)
    return out


def serve_mix_measure(S, torch, dev, args) -> dict:
    """Serving mixed requests: a pool of --mix-pool signals resident in HBM with
    N = 2^18..2^24, K = 20..1000, SNR 0..30 dB and one parameter set each (the
    rule: B next to sqrt(N K), w = 8B, L = 9), plans prepared up front (device
    resident after first use); requests draw pool entries at random and arrive
    as a Poisson process at --serve-rate; then a saturated burst."""
    import numpy as np
    from paper_2012_08238_amd import autotune as A
    from paper_2012_08238_amd.signals import derive_seed, make_signal_torch, poisson_arrivals, uneven_batch_specs
    specs = uneven_batch_specs(args.mix_pool, seed=5, log2n=(18, 24), k=(20, 1000), snr=(0.0, 30.0))
    srv = S.Server(hbm_budget_bytes=args.mix_budget_gib << 30, max_inflight=args.serve_inflight,
                   n_streams=args.serve_streams)
    pool = []
    for i, (n, k, snr) in enumerate(specs):
        x, f, _ = make_signal_torch(n, k, snr, derive_seed(50, i), dev)
        h = srv.prepare(A.rule_params(n, k, seed=i))
        pool.append((x, f, h, k, snr))
    nreq = max(1, int(args.serve_rate * args.serve_seconds))
    rng = np.random.default_rng(6)
    pick = rng.integers(0, len(pool), max(nreq, args.serve_burst))
    kmax = max(k for _, _, _, k, _ in pool)
    m = max(nreq, args.serve_burst)
    idx = torch.empty((m, kmax), dtype=torch.int64, device=dev)
    val = torch.empty((m, kmax), dtype=torch.complex64, device=dev)
    # make every plan resident once
    for j, (x, f, h, k, snr) in enumerate(pool):
        srv.wait(srv.submit(h, x, idx[j, :k], val[j, :k]))
    torch.cuda.synchronize()
    base = srv.stats()
    arrivals = poisson_arrivals(args.serve_rate, nreq, seed=2001)
    tickets = []
    t0 = time.perf_counter()
    for i in range(nreq):
        target = t0 + arrivals[i]
        while True:
            dt = target - time.perf_counter()
            if dt <= 0:
                break
            if dt > 2e-4:
                time.sleep(dt - 1.5e-4)
        x, f, h, k, snr = pool[pick[i]]
        tickets.append(srv.submit(h, x, idx[i, :k], val[i, :k]))
    lats = sorted(srv.wait(t)[0] * 1e3 for t in tickets)
    t_open = time.perf_counter() - t0
    mid = srv.stats()
    rec = []
    for i in range(min(nreq, 512)):
        x, f, h, k, snr = pool[pick[i]]
        if snr >= 10.0:
            rec.append(len(set(idx[i, :k].cpu().numpy().tolist()) & set(f.tolist())) / k)
    t1 = time.perf_counter()
    tickets = []
    for i in range(args.serve_burst):
        x, f, h, k, snr = pool[pick[i]]
        tickets.append(srv.submit(h, x, idx[i, :k], val[i, :k]))
    for t in tickets:
        srv.wait(t)
    t_sat = time.perf_counter() - t1
    st = srv.stats()
    srv.close()
    return {
        "pool": {"signals": len(pool), "resident_bytes": sum(n for n, _, _ in specs) * 8,
                 "N": "2^18..2^24", "K": "20..1000", "snr_db": "0..30", "params": "rule: B~sqrt(NK), w=8B, L=9"},
        "poisson": {"rate_req_s": args.serve_rate, "requests": nreq, "seconds": round(t_open, 3),
                    "p50_ms": round(percentile(lats, 0.5), 4), "p99_ms": round(percentile(lats, 0.99), 4),
                    "mean_ms": round(sum(lats) / len(lats), 4), "waves": mid["batches"] - base["batches"],
                    "mean_recall_snr_ge_10db": round(float(np.mean(rec)), 5) if rec else None},
        "saturated": {"requests": args.serve_burst, "signals_per_s": round(args.serve_burst / t_sat, 1),
                      "waves": st["batches"] - mid["batches"], "max_wave": st["max_batch"],
                      "max_waves_in_flight": st["max_waves_in_flight"]},
        "hbm": {"budget_bytes": st["hbm_budget"], "peak_bytes": st["hbm_peak"],
                "plan_cache_evictions": st["plan_cache_evictions"]},
    }


def uneven_measure(S, torch, dev, args) -> dict:
    """The uneven batch: --uneven signals with N = 2^16..2^22, K = 10..500, SNR
    -10..40 dB, resident in HBM, one plan per signal (tuned table if given, else
    the rule: B next to sqrt(N K), w = 8B, L = 9), one graph replay per step."""
    import numpy as np
    from paper_2012_08238_amd import autotune as A
    from paper_2012_08238_amd.signals import derive_seed, make_signal_torch, uneven_batch_specs
    specs = uneven_batch_specs(args.uneven, seed=4)
    table = A.Table(args.tune_table) if args.tune_table and os.path.exists(args.tune_table) else None
    t0 = time.perf_counter()
    plans, xs, truth = [], [], []
    for i, (n, k, snr) in enumerate(specs):
        prm = table.params(n, k, seed=i, device=dev) if table else A.rule_params(n, k, seed=i)
        plans.append(S.Plan.from_params(prm))
        x, f, _ = make_signal_torch(n, k, snr, derive_seed(40, i), dev)
        xs.append(x)
        truth.append(f)
    # steps in flight as in the main step: batches with their own workspaces and outputs
    # alternate over streams
    nf = max(1, args.uneven_inflight)
    # each step in flight reads its own copy of the signals (as in the main step)
    xsets = [xs] + [[x.clone() for x in xs] for _ in range(nf - 1)]
    bs = [S.Batch(plans, branches=args.uneven_branches) for _ in range(nf)]
    outsets = [[p.outputs(dev) for p in plans] for _ in range(nf)]
    streams = [torch.cuda.current_stream()] + [torch.cuda.Stream(device=dev) for _ in range(nf - 1)]
    outs = outsets[0]
    setup = time.perf_counter() - t0

    for j in range(nf):   # resident buffers: their pointers are marshalled once
        o = outsets[j]
        bs[j].bind(xsets[j], [q[0] for q in o], [q[1] for q in o], [q[2] for q in o])

    def run(j):
        bs[j].run_bound(stream=streams[j])
    for _ in range(2):
        for j in range(nf):
            run(j)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for s in range(args.uneven_steps):
        run(s % nf)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    rec = [len(set(o[0].cpu().numpy().tolist()) & set(f.tolist())) / k
           for (n, k, snr), o, f in zip(specs, outs, truth) if snr >= 10.0]
    # the plain single-signal path over the same batch
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for p, x, o in zip(plans, xs, outs):
        p.execute(x, o[0], o[1], o[2])
    torch.cuda.synchronize()
    single = len(plans) / (time.perf_counter() - t2)
    nbytes = sum(n for n, _, _ in specs) * 8
    for b in bs:
        b.close()
    for p in plans:
        p.close()
    del xsets[1:]
    return {"signals": len(specs), "resident_bytes": nbytes, "steps": args.uneven_steps, "steps_in_flight": nf,
            "graph_branches": args.uneven_branches,
            "ms_per_step": round(el / args.uneven_steps * 1e3, 4),
            "signals_per_s": round(len(specs) * args.uneven_steps / el, 1),
            "single_signal_path_signals_per_s": round(single, 1),
            "mean_recall_snr_ge_10db": round(float(np.mean(rec)), 5) if rec else None,
            "params": "autotuned table" if table else "rule: B next to sqrt(NK), w=8B, L=9",
            "setup_s": round(setup, 1)}


def main() -> int:
    global N, K, B, L
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--shape", default="22,100,16384,9",
                    help="log2 N, K, B, L of the step's workload (default: the metric's configuration; other "
                         "shapes are for profiling the same path)")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--batch", type=int, default=64, help="signals per step (64 x 32 MB = 2 GB, beyond the 256 MB cache)")
    ap.add_argument("--latency-runs", type=int, default=100)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the CPU oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--strip-cols", type=int, default=0, help="bucketization tile width (0 = plan default)")
    ap.add_argument("--w-over-b", type=int, default=8, help="window length w as a multiple of B")
    ap.add_argument("--fold", choices=["auto", "strip", "gather"], default="auto", help="bucketization form")
    ap.add_argument("--fft", choices=["two-pass", "one-workgroup"], default="one-workgroup",
                    help="B-point FFT form of the step's plan (two passes of small workgroups share compute units "
                         "with the next step's bucketization)")
    ap.add_argument("--vote", choices=["auto", "loop", "pair"], default="auto",
                    help="vote enumeration: by loop, by loop pair, or the plan's choice")
    ap.add_argument("--xcd-order", action="store_true", help="XCD-grouped workgroup order for the bucketization")
    ap.add_argument("--single-passes", type=int, default=3, help="passes over the batch through sfft_execute alone")
    ap.add_argument("--branches", type=int, default=1, help="parallel stream branches of the step's batch graph")
    ap.add_argument("--inflight", type=int, default=3, help="steps in flight (batches alternating over streams)")
    ap.add_argument("--section-branches", type=int, default=4, help="graph branches of the other sections' batches")
    ap.add_argument("--serve-seconds", type=float, default=2.0, help="duration of the Poisson serving run (0 = skip)")
    ap.add_argument("--serve-rate", type=float, default=2000.0, help="Poisson arrival rate, requests/s")
    ap.add_argument("--serve-burst", type=int, default=4096,
                    help="requests of the saturated serving run (enough waves that start-up and drain weigh little)")
    ap.add_argument("--serve-budget-gib", type=int, default=8)
    ap.add_argument("--serve-inflight", type=int, default=256)
    ap.add_argument("--serve-streams", type=int, default=4)
    ap.add_argument("--mix-pool", type=int, default=64, help="pool of mixed-size served signals (0 = skip)")
    ap.add_argument("--sweep-signals", type=int, default=8, help="signals per SNR point of the error sweep (0 = skip)")
    ap.add_argument("--comb-batch", type=int, default=64, help="signals per batch of the comb prefilter runs (0 = skip)")
    ap.add_argument("--comb-steps", type=int, default=10)
    ap.add_argument("--mix-budget-gib", type=int, default=16)
    ap.add_argument("--iter-batch", type=int, default=16, help="signals per batch of the subtraction-round runs (0 = skip)")
    ap.add_argument("--iter-steps", type=int, default=5)
    ap.add_argument("--phase-batch", type=int, default=64, help="signals per batch of the phase-location runs (0 = skip)")
    ap.add_argument("--phase-steps", type=int, default=10)
    ap.add_argument("--est-batch", type=int, default=32, help="signals per batch of the estimation-loop runs (0 = skip)")
    ap.add_argument("--est-steps", type=int, default=10)
    ap.add_argument("--ksweep-batch", type=int, default=64, help="signals per batch of the K sweep (0 = skip)")
    ap.add_argument("--ksweep-steps", type=int, default=60)
    ap.add_argument("--ksweep-inflight", type=int, default=3, help="steps in flight of the K sweep")
    ap.add_argument("--fused-batches", default="16,256,1024",
                    help="batch sizes of the fused-launch vs graph comparison on small plans (empty = skip)")
    ap.add_argument("--no-context", action="store_true", help="skip the copy-bandwidth and dense-FFT context")
    ap.add_argument("--uneven", type=int, default=256, help="signals of the uneven batch (0 = skip)")
    ap.add_argument("--uneven-steps", type=int, default=60)
    ap.add_argument("--uneven-inflight", type=int, default=2, help="steps in flight of the uneven batch")
    ap.add_argument("--uneven-branches", type=int, default=2,
                    help="graph branches of the uneven batch (measured: 2 -> 257k, 4 -> 242k signals/s)")
    ap.add_argument("--tune-table", default=os.path.join(ROOT, "paper_2012_08238_amd", "tuned", "mi355x_uneven.json"),
                    help="autotuner JSON table for the uneven batch ('' = the untuned rule; missing classes are tuned)")
    args = ap.parse_args()
    ln, K, B, L = (int(v) for v in args.shape.split(","))
    N = 1 << ln
    metric_shape = (N, K, B, L) == (1 << 22, 100, 16384, 9)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "how the path would shard over GPUs is described, not implemented", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2012_08238_amd as S
    from paper_2012_08238_amd.signals import derive_seed, make_signal_torch

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    M = args.batch
    t_setup = time.perf_counter()
    xs, truth = [], []
    for i in range(M):
        x, f, tones = make_signal_torch(N, K, SNR_DB, derive_seed(0, i), dev)
        xs.append(x)
        truth.append((f, tones))
    W = args.w_over_b * B
    fflags = {"auto": 0, "strip": S.SFFT_FLAG_FOLD_STRIP, "gather": S.SFFT_FLAG_FOLD_GATHER}[args.fold]
    plan = S.Plan(N, K, B, L, W, seed=PLAN_SEED, strip_cols=args.strip_cols,
                  flags=fflags | (S.SFFT_FLAG_XCD_ORDER if args.xcd_order else 0) | vote_flags(args) |
                  (S.SFFT_FLAG_FFT_TWO_PASS if args.fft == "two-pass" and 4096 <= B <= 16384 else 0))
    desc = plan.desc
    batch = S.Batch([plan] * M, branches=args.branches)
    idx = torch.empty((M, K), dtype=torch.int64, device=dev)
    val = torch.empty((M, K), dtype=torch.complex64, device=dev)
    res = torch.empty((M, 2), dtype=torch.float64, device=dev)
    idxs, vals, ress = [idx[i] for i in range(M)], [val[i] for i in range(M)], [res[i] for i in range(M)]
    torch.cuda.synchronize()
    print(f"# setup {time.perf_counter() - t_setup:.1f}s: {M} signals of N=2^{ln} resident, "
          f"fold_mode={desc['fold_mode']} strip_cols={desc['strip_cols']}", file=sys.stderr, flush=True)

    # steps in flight: consecutive steps alternate over `inflight` batches (own workspaces and
    # outputs) on their own streams, so one step's last stages overlap the next step's
    # bucketization; every step still runs every stage over all M signals
    nf = max(1, args.inflight)
    # each step in flight reads its own copy of the signals (distinct memory, same content), so
    # that no step can find another's signals in a cache
    xsets = [xs] + [[x.clone() for x in xs] for _ in range(nf - 1)]
    batches, outsets, streams = [batch], [(idxs, vals, ress)], [torch.cuda.current_stream()]
    for _ in range(nf - 1):
        batches.append(S.Batch([plan] * M, branches=args.branches))
        oi = torch.empty((M, K), dtype=torch.int64, device=dev)
        ov = torch.empty((M, K), dtype=torch.complex64, device=dev)
        orr = torch.empty((M, 2), dtype=torch.float64, device=dev)
        outsets.append(([oi[i] for i in range(M)], [ov[i] for i in range(M)], [orr[i] for i in range(M)]))
        streams.append(torch.cuda.Stream(device=dev))
    for j in range(nf):   # resident buffers: their pointers are marshalled once
        batches[j].bind(xsets[j], *outsets[j])
    for _ in range(args.warmup):
        for j in range(nf):
            batches[j].run_bound(stream=streams[j])
    torch.cuda.synchronize()
    from paper_2012_08238_amd._hip import HipEvent
    ev = [(HipEvent(), HipEvent()) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        if args.branches == 1 and nf == 1:
            batch.run_timed(xs, idxs, vals, ress, ev[k][0], ev[k][1])
        else:
            j = k % nf
            batches[j].run_bound(stream=streams[j])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    for b_ in batches[1:]:
        b_.close()
    del xsets[1:]
    launch_source = "bucketization launches of the timed steps"
    if args.branches > 1 or nf > 1:
        # branches and steps in flight run the bucketization beside other stages:
        # time the kernel over the whole batch in an unbranched graph instead
        kb = S.Batch([plan] * M)
        kb.run(xs, idxs, vals, ress)
        for k in range(args.steps):
            kb.run_timed(xs, idxs, vals, ress, ev[k][0], ev[k][1])
        torch.cuda.synchronize()
        kb.close()
        launch_source = "bucketization launches of an unbranched replay of the same batch, after the timed steps"
    fold_ms = [a.elapsed_ms(b) for a, b in ev]
    fold_avg_s = sum(fold_ms) / len(fold_ms) / 1e3
    print(f"# timed {args.steps} steps in {elapsed:.3f}s; bucketization {fold_avg_s * 1e6:.1f} us/launch",
          file=sys.stderr, flush=True)

    # accuracy of the last step against the planted tones
    idx_h, val_h, res_h = idx.cpu().numpy(), val.cpu().numpy(), res.cpu().numpy()
    exact = sum(set(idx_h[i].tolist()) == set(truth[i][0].tolist()) for i in range(M))
    resid_ratio = float(np.median(res_h[:, 0] / res_h[:, 1]))

    # single-request latency (one signal, alone, synchronised)
    lat = []
    li, lv, lr = plan.outputs(dev)
    for r in range(args.latency_runs + 3 if args.latency_runs > 0 else 0):
        torch.cuda.synchronize()
        a = time.perf_counter()
        plan.execute(xs[r % M], li, lv, lr)
        torch.cuda.synchronize()
        if r >= 3:
            lat.append(time.perf_counter() - a)

    # the plain single-signal path: one execution after another on one stream
    single = None
    if args.single_passes > 0:
        outs1 = [plan.outputs(dev) for _ in range(M)]
        for i in range(M):
            plan.execute(xs[i], *outs1[i])
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(args.single_passes):
            for i in range(M):
                plan.execute(xs[i], *outs1[i])
        torch.cuda.synchronize()
        single = M * args.single_passes / (time.perf_counter() - a)
        print(f"# single-signal path {single:.0f} signals/s", file=sys.stderr, flush=True)

    serving = None
    if args.serve_seconds > 0:
        serving = serve_measure(S, torch, dev, xs, truth, args)
    serving_mix = None
    if args.serve_seconds > 0 and args.mix_pool > 0:
        serving_mix = serve_mix_measure(S, torch, dev, args)
        print(f"# mixed serving p50 {serving_mix['poisson']['p50_ms']} ms p99 {serving_mix['poisson']['p99_ms']} ms",
              file=sys.stderr, flush=True)
    sweep = snr_sweep(S, torch, dev, args) if args.sweep_signals > 0 else None
    comb = comb_measure(S, torch, dev, args) if args.comb_batch > 0 else None
    iterate = iterate_measure(S, torch, dev, args) if args.iter_batch > 0 else None
    phase = phase_measure(S, torch, dev, args) if args.phase_batch > 0 else None
    est_loops = est_loops_measure(S, torch, dev, args) if args.est_batch > 0 else None
    ksweep = k_sweep_measure(S, torch, dev, args) if args.ksweep_batch > 0 else None
    fused = fused_measure(S, torch, dev, args) if args.fused_batches else None
    context = None
    if not args.no_context:
        context = dense_fft_context(torch, dev, xs)
        context["hbm_copy_GBps"] = round(copy_bandwidth(torch, dev), 1)
        print(f"# context {context}", file=sys.stderr, flush=True)
    uneven = None
    if args.uneven > 0:
        uneven = uneven_measure(S, torch, dev, args)
        print(f"# uneven batch {uneven['signals_per_s']:.0f} signals/s", file=sys.stderr, flush=True)

    alg = alg_bytes_per_signal(W) * M
    achieved = alg / fold_avg_s / 1e9
    traffic = committed_traffic(M) if metric_shape else None   # the counters cover the metric's shape
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                "kernel": "fold_strip_pf_kernel (bucketization)", "alg_bytes_per_launch": alg,
                "launch_us": round(fold_avg_s * 1e6, 2), "launch_timing": launch_source}
    # line-granular bound: the distinct 128-byte lines (the unit in which L2 reads HBM) and
    # 64-byte lines holding a sample of some loop, from the plan's sigma, tau and w
    sig_p, _, tau_p = plan.perms()
    ii = np.arange(W, dtype=np.int64)
    pos = np.concatenate([(int(sig_p[r]) * ii + int(tau_p[r])) % N for r in range(L)])
    lines128 = int(np.unique(pos >> 4).shape[0])
    lines64 = int(np.unique(pos >> 3).shape[0])
    lb = lines128 * 128 * M
    roofline["line_granular"] = {
        "line_bytes": 128, "bytes_per_launch": lb, "achieved": round(lb / fold_avg_s / 1e9, 1),
        "frac": round(lb / fold_avg_s / 1e9 / HBM_PEAK_GBPS, 4), "lines_touched_frac": round(lines128 * 16 / N, 4),
        "bytes_per_launch_64B_lines": lines64 * 64 * M,
        "note": "L2 reads HBM in 128-byte lines (TCC_EA0_RDREQ x 128 B equals the calibrated FETCH_SIZE)"}
    if traffic:
        roofline["effective_GBps"] = round(traffic / fold_avg_s / 1e9, 1)
    if context:
        # the same kernel against what a plain copy reaches on this device
        roofline["achievable_copy_GBps"] = context["hbm_copy_GBps"]
        if traffic:
            roofline["effective_frac_of_copy"] = round(traffic / fold_avg_s / 1e9 / context["hbm_copy_GBps"], 4)

    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        import oracle.sfft_oracle as O
        # one core: at least 20 of the benchmark signals, per-signal times kept
        n, ts, errs, sup_eq = 0, [], [], 0
        while n < M and (sum(ts) < args.cpu_seconds or n < 20):
            xh = xs[n].cpu().numpy().astype(np.complex128)
            a = time.perf_counter()
            r = O.sfft(xh, K, B, L, W, seed=PLAN_SEED)
            ts.append(time.perf_counter() - a)
            gi = idx_h[n]
            if np.array_equal(gi, r.idx):
                sup_eq += 1
                ok = r.idx >= 0
                errs.append(float(np.max(np.abs(val_h[n][ok] - r.val[ok]) / np.abs(r.val[ok]))))
            n += 1
        parity = {"signals": n, "support_equal": sup_eq,
                  "max_rel_value_err_fp32_vs_fp64": max(errs) if errs else None}
        # every core: a process pool over 2 signals per worker
        cores = min(16, len(os.sched_getaffinity(0)))
        npool = min(M, 2 * cores)
        pool_s = oracle_pool_seconds([xs[i].cpu().numpy() for i in range(npool)], (K, B, L, W, PLAN_SEED), cores)
        others = {name: oracle_config_seconds(*cfg) for name, cfg in ORACLE_CONFIGS.items()}
        cpu = {"value": round(npool / pool_s, 4), "unit": "signals/s", "cores": cores, "kind": "oracle",
               "sample": f"{npool} of the {M} benchmark signals (N=2^{ln}, K={K}) over a pool of {cores} "
                         f"single-threaded FP64 NumPy oracle processes, {pool_s:.1f}s wall",
               "single_core": {"value": round(n / sum(ts), 4), "unit": "signals/s", "cores": 1, "signals": n,
                               "p50_s": round(percentile(ts, 0.5), 4), "p99_s": round(percentile(ts, 0.99), 4),
                               "seconds": round(sum(ts), 2)},
               "other_configs": others}

    out = {
        "metric": "sparse spectra recovered/sec + p50/p99 latency, N=2^22 K=100, % HBM peak",
        "value": round(M * args.steps / elapsed, 2),
        "unit": "signals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"sFFT N=2^{ln} K={K} SNR20dB B={B} L={L} w={W}, batch of resident signals",
                   "N": N, "K": K, "B": B, "L": L, "w": W, "snr_db": SNR_DB, "batch": M,
                   "fold_mode": "strip" if desc["fold_mode"] == 1 else "gather",
                   "strip_cols": desc["strip_cols"], "graph_branches": args.branches, "steps_in_flight": nf,
                   "fft": args.fft, "vote_pairs": desc["vote_pairs"],
                   "parallelism": "single-gpu"},
        "latency": ({"p50_ms": serving["poisson"]["p50_ms"], "p99_ms": serving["poisson"]["p99_ms"],
                     "source": f"serving loop, Poisson arrivals at {serving['poisson']['rate_req_s']:.0f} req/s, "
                               "submission to completion"} if serving else None),
        "single_request_latency": ({"p50_ms": round(percentile(lat, 0.5) * 1e3, 4),
                                    "p99_ms": round(percentile(lat, 0.99) * 1e3, 4),
                                    "source": "sfft_execute alone + stream sync", "runs": len(lat)}
                                   if lat else None),
        "single_signal_path_signals_per_s": round(single, 1) if single else None,
        "serving": serving,
        "serving_mixed_sizes": serving_mix,
        "uneven_batch": uneven,
        "error_vs_snr": sweep,
        "comb_prefilter": comb,
        "subtraction_round": iterate,
        "phase_location": phase,
        "estimation_loops": est_loops,
        "k_sweep_c3": ksweep,
        "fused_vs_graph_small": fused,
        "context": context,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "accuracy": {"exact_support": f"{exact}/{M}", "median_residual_ratio": resid_ratio,
                     "parity_vs_oracle": parity},
        "sampled_fraction": desc["sampled_fraction_expected"],
    }
    print(json.dumps(out), flush=True)
    batch.close()
    plan.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
