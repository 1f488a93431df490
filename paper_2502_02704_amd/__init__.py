"""MI355X-native fine kinetic propagator of the multiscale kinetic/fluid
parareal method for the Vlasov-BGK equation (Laidin & Rey, arXiv 2502.02704).

The compute path lives in ``libbgk.so`` (hand-written HIP kernels for gfx950
behind a C ABI declared in ``include/bgk.h``); :mod:`.bgk` is the thin ctypes
binding on torch device tensors.  Importing this package does not load the
library; the first call into :mod:`.bgk` does, and raises if it is missing.
"""
from . import workloads  # noqa: F401

__all__ = ["workloads"]
