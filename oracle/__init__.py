"""CPU oracle for the Log(Graph) packed-graph path -- TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps the plain C implementation in lg_oracle.c with
numpy arrays; it shares no code with the GPU library.
"""

from .oracle import *  # noqa: F401,F403
