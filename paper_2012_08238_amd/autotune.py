"""Autotuner of plan parameters per size class.

A size class is (log2 N, the octave of K). For a class the tuner tries the
bucket counts B next to sqrt(N K) (powers of two with d*K <= B/4 and N/B >= 2)
and windows w = 4B and 8B on seeded probe signals with planted tones at a
reference SNR:

* accuracy: the recall of the planted supports, averaged over the probes; the
  configurations within ``tol`` of the best recall are kept;
* speed: device time of one batched execution of the probes, repeated to
  about 256 MB of signal (graph replay, median of a few), the fastest kept
  configuration wins;
* execution form: for the winner, the gather form, strip widths around the
  default and (small plans) the fused one-launch form are timed. They never
  change results (every form sums the same taps in the same order and runs the
  same stage code), so only time decides.

The table persists as JSON: {"<log2N>:<K octave>": {"B":, "wB":, "L":,
"strip_cols":, "flags":, "ms":, "recall":}}. Tuning runs the library's kernels
on the current device; it only chooses parameters.
"""
from __future__ import annotations

import json
import math
import os

from . import SFFT_FLAG_FOLD_GATHER, SFFT_FLAG_FOLD_STRIP, SFFT_FLAG_FUSED, Batch, Plan, PlanParams

MAX_B = 1 << 18


def class_key(N: int, K: int) -> str:
    return f"{int(N).bit_length() - 1}:{int(K).bit_length()}"


def class_k(K: int) -> int:
    """The K a class is tuned at: the top of K's octave (the most buckets needed)."""
    return (1 << int(K).bit_length()) - 1


def b_candidates(N: int, K: int, d: int = 2) -> list[int]:
    root = math.sqrt(N * K)
    lo = 1 << max(1, int(math.floor(math.log2(root))))
    out = []
    for B in (lo // 2, lo, 2 * lo, 4 * lo):
        if 4 * d * K <= B <= min(MAX_B, N // 2) and B not in out:
            out.append(B)
    # keep the two nearest sqrt(N K) in log scale
    out.sort(key=lambda B: abs(math.log2(B) - math.log2(root)))
    out = sorted(out[:2])
    if not out:
        B = 1 << max(1, int(math.ceil(math.log2(4 * d * K))))
        if B <= min(MAX_B, N // 2):
            out = [B]
    return out


def rule_params(N: int, K: int, L: int = 9, seed: int = 0) -> PlanParams:
    """Untuned default: B the candidate nearest sqrt(N K), w = 8B (capped at N)."""
    cands = b_candidates(N, K)
    if not cands:
        raise ValueError(f"no bucket count fits N={N}, K={K}")
    root = math.sqrt(N * K)
    B = min(cands, key=lambda b: abs(math.log2(b) - math.log2(root)))
    return PlanParams(N, K, B, L, min(8 * B, N), seed=seed)


def params_from(entry: dict, N: int, K: int, seed: int = 0) -> PlanParams:
    B = entry["B"]
    return PlanParams(N, K, B, entry["L"], min(entry["wB"] * B, N), seed=seed, strip_cols=entry["strip_cols"],
                      flags=entry["flags"])


def _time_batch(plan, xs, outs, reps: int, fill: int = 1) -> float:
    """Median device time of one batched execution of the probes, each repeated
    `fill` times (so that small signals still fill the device as in a real batch)."""
    import torch
    xs = list(xs) * fill
    outs = [plan.outputs(xs[0].device) for _ in xs]
    b = Batch([plan] * len(xs))
    idx = [o[0] for o in outs]
    val = [o[1] for o in outs]
    b.run(xs, idx, val)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.run(xs, idx, val)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    b.close()
    ts.sort()
    return ts[len(ts) // 2]


def tune_class(N: int, K: int, device, L: int = 9, snr_db: float = 10.0, probes: int = 4, reps: int = 5,
               tol: float = 0.005, seed: int = 77) -> dict:
    """Tune one size class at its representative K; returns the table entry."""
    import torch

    from .signals import derive_seed, make_signal_torch
    Kc = min(class_k(K), N // 16)
    sigs = [make_signal_torch(N, Kc, snr_db, derive_seed(seed, i), device) for i in range(probes)]
    xs = [s[0] for s in sigs]
    # time batches of about 256 MB of signal (at most 64 signals), as in a full batch
    fill = max(1, min(64, (1 << 28) // (8 * N)) // probes)
    trials = []
    for B in b_candidates(N, Kc):
        for wB in (4, 8):
            if wB * B > N:
                continue
            p = Plan(N, Kc, B, L, wB * B, seed=seed, n_resid=0, flags=1)
            outs = [p.outputs(device) for _ in xs]
            recall = 0.0
            for (x, f, _), o in zip(sigs, outs):
                p.execute(x, o[0], o[1])
                torch.cuda.synchronize()
                got = set(o[0].cpu().numpy().tolist())
                recall += len(got & set(f.tolist())) / len(f)
            recall /= len(xs)
            ms = _time_batch(p, xs, outs, reps, fill)
            trials.append(dict(B=B, wB=wB, recall=recall, ms=ms, plan=p))
    if not trials:
        raise ValueError(f"no configuration fits N={N}, K={K}")
    best = max(t["recall"] for t in trials)
    kept = [t for t in trials if t["recall"] >= best - tol]
    win = min(kept, key=lambda t: t["ms"])
    for t in trials:
        if t is not win:
            t["plan"].close()
    # bucketization form and tile, fused form: results are identical, time decides
    B, wB = win["B"], win["wB"]
    base = win["plan"]
    default_c = base.desc["strip_cols"]
    forms = [(base.desc["fold_mode"] and SFFT_FLAG_FOLD_STRIP or SFFT_FLAG_FOLD_GATHER, 0, win["ms"])]
    alt = [(SFFT_FLAG_FOLD_GATHER, 0)]
    for c in (default_c // 2, default_c * 2):
        if 2 <= c <= B:
            alt.append((SFFT_FLAG_FOLD_STRIP, c))
    alt.append((SFFT_FLAG_FUSED, 0))   # refused (skipped) outside the fused form's scope
    base.close()
    for flags, c in alt:
        try:
            p = Plan(N, Kc, B, L, wB * B, seed=seed, n_resid=0, flags=1 | flags, strip_cols=c)
        except Exception:
            continue
        forms.append((flags, c, _time_batch(p, xs, None, reps, fill)))
        p.close()
    flags, c, ms = min(forms, key=lambda f: f[2])
    return dict(B=B, wB=wB, L=L, strip_cols=c, flags=flags, ms=ms, recall=win["recall"], tuned_at_k=Kc,
                snr_db=snr_db, probes=probes, timed_signals=probes * fill)


class Table:
    """Tuned parameters per size class, persisted as JSON."""

    def __init__(self, path: str | None = None):
        self.path = path
        self.entries: dict[str, dict] = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.entries = json.load(f)

    def get(self, N: int, K: int, device=None, tune: bool = True, **kw) -> dict | None:
        key = class_key(N, K)
        if key not in self.entries and tune:
            self.entries[key] = tune_class(N, K, device, **kw)
            self.save()
        return self.entries.get(key)

    def params(self, N: int, K: int, seed: int = 0, device=None, tune: bool = True, **kw) -> PlanParams:
        e = self.get(N, K, device, tune, **kw)
        return params_from(e, N, K, seed) if e else rule_params(N, K, seed=seed)

    def save(self) -> None:
        if self.path:
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.entries, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)


def main(argv=None) -> int:
    """Tune the size classes of a workload recipe into a JSON table."""
    import argparse

    import torch

    from .signals import uneven_batch_specs
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--out", required=True)
    ap.add_argument("--log2n", default="16,22", help="range of log2 N (inclusive)")
    ap.add_argument("--k", default="10,500", help="range of K (inclusive)")
    ap.add_argument("--snr", type=float, default=10.0)
    ap.add_argument("--probes", type=int, default=4)
    a = ap.parse_args(argv)
    lo, hi = (int(v) for v in a.log2n.split(","))
    klo, khi = (int(v) for v in a.k.split(","))
    dev = torch.device("cuda:0")
    t = Table(a.out)
    specs = uneven_batch_specs(4096, seed=4, log2n=(lo, hi), k=(klo, khi))
    keys = sorted({(n, class_k(k)) for n, k, _ in specs})
    for n, k in keys:
        e = t.get(n, k, dev, snr_db=a.snr, probes=a.probes)
        print(f"{class_key(n, k)}: B={e['B']} w=B*{e['wB']} strip_cols={e['strip_cols']} flags={e['flags']} "
              f"recall={e['recall']:.4f} {e['ms']:.3f} ms", flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
