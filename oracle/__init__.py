"""Plain FP64 CPU oracle for the ROKS hot path.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  The product library never imports,
links or executes anything here, and the oracle shares no code with it.
"""
from . import roks, xc  # noqa: F401
