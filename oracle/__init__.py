"""CPU oracle for k-NN graph merge -- test infrastructure only.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark import this package.  The product path never imports it.
"""
from .oracle import *  # noqa: F401,F403
