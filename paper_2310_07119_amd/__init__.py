"""MI355X-native truncated-Wigner Schrodinger-Poisson ensemble (arXiv 2310.07119).

The compute path is the HIP library ``libtw.so`` (C ABI in include/tw.h);
``twa.Plan`` is a thin ctypes binding that marshals torch device tensors and
the current HIP stream into it.
"""
from .twa import Batch, Fno, Plan, Problem, load_library  # noqa: F401
