"""FP64 CPU oracle for the QFactor instantiation sweep.

Test infrastructure only: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark are its only users.  Nothing in the GPU library imports
it, and it imports nothing from the library.
"""
from .qfactor_oracle import *  # noqa: F401,F403
from .qfactor_oracle import Options, Result, BuilderOracle, instantiate  # noqa: F401
