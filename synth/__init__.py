"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark.  Holds no arithmetic of the merge method itself: only random
point sets with the shapes and value laws of the benchmark workloads, and
index-level perturbation of neighbour lists."""
from .gen import *  # noqa: F401,F403
