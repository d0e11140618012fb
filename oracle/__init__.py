"""FP64 CPU oracle for the graph Fourier transform (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline`` leg may
import this package.  The library never calls it.
"""
from .gft_oracle import *  # noqa: F401,F403
