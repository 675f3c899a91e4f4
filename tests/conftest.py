import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def pytest_terminal_summary(terminalreporter):
    """Report every parity comparison's counted near-ties (tests/parity.py keeps them)."""
    parity = sys.modules.get("parity")
    recs = getattr(parity, "RECORDS", None)
    if not recs:
        return
    tot = {k: 0 for k in ("loops", "loops_tied", "certain", "band", "certain_displaced", "certain_uncandidate",
                          "values", "values_ill", "values_leak", "values_tied")}
    amb = 0
    for _, p in recs:
        for k in tot:
            tot[k] += getattr(p, k)
        amb += p.ambiguous
    tr = terminalreporter
    tr.write_sep("-", "parity against the FP64 oracle")
    tr.write_line(f"{len(recs)} comparisons, {amb} with a counted near-tie; "
                  + ", ".join(f"{k} {v}" for k, v in tot.items()))
    for node, p in recs:
        if p.ambiguous:
            tr.write_line(f"  {node}: tied loops {p.loops_tied}, candidates equal {p.cand_equal} "
                          f"(explained {p.cand_explained}), certain {p.certain} + band {p.band}, "
                          f"displaced {p.certain_displaced}, uncandidate {p.certain_uncandidate}"
                          + (f", skipped: {p.skipped}" if p.skipped else ""))
