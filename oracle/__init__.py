"""CPU oracle for BootMMPM -- TEST INFRASTRUCTURE ONLY.

Plain, slow statements of what the method computes, used by ``tests/``, by the
smoke check and by the benchmark's CPU-baseline leg.  The product library never
imports this package, and this package never imports the product.

Every function is pinned by ``tests/test_oracle_*.py`` against facts the paper
or plain mathematics fix.  The Gaussian sampler is not part of the oracle
(errors are inputs drawn by ``synth``), so it has no pin here.
"""
from .api import *  # noqa: F401,F403
from .api import __all__  # noqa: F401
