"""CPU FP64 oracle for the particle-particle ladder (TEST INFRASTRUCTURE ONLY).

Plain, slow, obviously-correct NumPy implementations of what the GPU path
computes (the ladder terms and the vvvv two-body-density contraction),
written from the paper's definitions. Only the test suite, the smoke
check and the CPU-baseline leg of the benchmark may import this package; the
library path never does. It shares no code with the HIP path.

Parity pins: every function here is checked in ``tests/test_oracle_pins.py``
and ``tests/test_oracle_density.py``
against brute force, closed forms, invariants and a spin-orbital derivation
(see each function's docstring).
"""
from .density import *  # noqa: F401,F403
from .ladder import *  # noqa: F401,F403
from .layout import OracleLayout  # noqa: F401
