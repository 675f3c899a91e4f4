"""Host logic of the autotuner: size classes, bucket-count candidates, the
untuned rule, and the JSON table round trip (no device needed)."""
import json
import math

import pytest

from paper_2012_08238_amd import autotune as A
from paper_2012_08238_amd.signals import poisson_arrivals, uneven_batch_specs


@pytest.mark.parametrize("N,K", [(1 << 16, 10), (1 << 16, 500), (1 << 20, 50), (1 << 22, 100), (1 << 22, 1000),
                                 (1 << 24, 1000), (1 << 18, 20)])
def test_b_candidates(N, K):
    c = A.b_candidates(N, K)
    assert 1 <= len(c) <= 2
    root = math.sqrt(N * K)
    for B in c:
        assert B & (B - 1) == 0 and 8 * K <= B <= min(A.MAX_B, N // 2)
        assert abs(math.log2(B) - math.log2(root)) <= 1.0
    p = A.rule_params(N, K)
    assert p.B in c and p.w == min(8 * p.B, N)


def test_class_key():
    assert A.class_key(1 << 20, 50) == "20:6"
    assert A.class_key(1 << 20, 63) == A.class_key(1 << 20, 32)
    assert A.class_k(50) == 63 and A.class_k(64) == 127


def test_table_roundtrip(tmp_path):
    path = str(tmp_path / "t.json")
    t = A.Table(path)
    t.entries["20:6"] = dict(B=1024, wB=8, L=7, strip_cols=0, flags=2, ms=0.1, recall=1.0)
    t.save()
    t2 = A.Table(path)
    assert t2.get(1 << 20, 40, tune=False)["B"] == 1024
    p = t2.params(1 << 20, 40, seed=5, tune=False)
    assert (p.N, p.K, p.B, p.L, p.w, p.flags, p.seed) == (1 << 20, 40, 1024, 7, 8192, 2, 5)
    assert t2.get(1 << 21, 40, tune=False) is None
    q = t2.params(1 << 21, 40, tune=False)          # untuned class: the rule
    assert q.B in A.b_candidates(1 << 21, 40)
    json.load(open(path))


def test_workload_recipes():
    s = uneven_batch_specs(256, seed=4)
    assert len(s) == 256
    assert {N.bit_length() - 1 for N, _, _ in s} == set(range(16, 23))
    assert all(10 <= K <= 500 and -10 <= snr <= 40 for _, K, snr in s)
    assert s == uneven_batch_specs(256, seed=4)
    a = poisson_arrivals(2000.0, 20000, seed=1)
    gaps = a[1:] - a[:-1]
    assert abs(gaps.mean() - 1 / 2000) < 0.05 / 2000 and (gaps > 0).all()
