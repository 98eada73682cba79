"""Plain CPU oracle of the AQR-HNSW method (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
may import this package.  The product library never does.
"""
from .oracle import *  # noqa: F401,F403
