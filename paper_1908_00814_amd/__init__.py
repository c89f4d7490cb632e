"""k-NN graph merge (S-Merge, J-Merge) on one MI355X: hand-written HIP for
gfx950 behind a C ABI (include/knng_merge.h), with a thin Python binding."""
from . import knng  # noqa: F401
