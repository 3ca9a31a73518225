"""CPU oracle for the D2V19 FDLB step (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package. The GPU library never imports it and it
never imports the GPU library.
"""
from .oracle import *  # noqa: F401,F403
from .riemann import exact_riemann, sample_riemann  # noqa: F401
