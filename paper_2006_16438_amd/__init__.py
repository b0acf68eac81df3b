"""MI355X (gfx950) CP-ARLS-LEV mode-update library.

``CpArlsLev`` wraps the C ABI of ``include/cp_arls_lev.h``; ``synth`` draws
seeded synthetic workloads.  Importing the package does not load the HIP
library; the first ``CpArlsLev`` does, and fails loudly if it is missing.
"""
from . import synth  # noqa: F401


def __getattr__(name):
    if name == "CpArlsLev":
        from .api import CpArlsLev
        return CpArlsLev
    raise AttributeError(name)
