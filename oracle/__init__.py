"""CPU FP64 oracle for the particle-particle ladder (TEST INFRASTRUCTURE ONLY).

Plain, slow, obviously-correct NumPy implementations of what the GPU path
computes (the ladder terms, the vvvv two-body-density contraction and the
O(O^3 V^3) contraction of the partial symmetric-antisymmetric scheme, and the
symmetry-adapted two-step Cholesky decomposition),
written from the paper's definitions. Only the test suite, the smoke
check and the CPU-baseline leg of the benchmark may import this package; the
library path never does. It shares no code with the HIP path.

Parity pins: every function here is checked in ``tests/test_oracle_pins.py``
``tests/test_oracle_density.py``, ``tests/test_oracle_partial.py`` and
``tests/test_oracle_cd.py``
against brute force, closed forms, invariants and a spin-orbital derivation
(see each function's docstring).
"""
from .cholesky import *  # noqa: F401,F403
from .density import *  # noqa: F401,F403
from .ladder import *  # noqa: F401,F403
from .partial import *  # noqa: F401,F403
from .layout import OracleLayout  # noqa: F401
