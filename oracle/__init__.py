"""FP64 CPU oracle of the flat-window voting sparse FFT.

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call or run anything in this
package. It shares no code with the HIP library and the library never calls it.
"""
from .sfft_oracle import *  # noqa: F401,F403
from .sfft_oracle import C_G, OracleResult, sfft  # noqa: F401
