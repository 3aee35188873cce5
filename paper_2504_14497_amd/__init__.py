"""PC-MM over EC-ElGamal (P-256) on MI355X: the Python side of ``libpcmm``.

The compute path is the HIP library ``libpcmm.so`` built from ``csrc/``; this
package only marshals arguments into its C ABI (``pcmm.py``) and provides the
seeded workloads (``workloads.py``).  Importing the package does not load the
library; the first call into ``pcmm`` does, and fails loudly if it is missing.
"""
from . import workloads  # noqa: F401

__all__ = ["workloads", "pcmm"]


def __getattr__(name):
    if name == "pcmm":
        import importlib
        return importlib.import_module(__name__ + ".pcmm")
    raise AttributeError(name)
