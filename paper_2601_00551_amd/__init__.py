"""MI355X (gfx950) implementation of the SlingBAG Pro reconstruction hot path.

The forward model, its adjoint, zero-gradient filtering, the optimiser step,
the growth rule and the batched graph-captured iteration run as HIP kernels in
``libsbp.so`` behind the C-ABI of ``include/sbp.h``; this package is its
binding plus the host-side schedule driver.

Importing the package does not load the library; ``load()`` (or the first call
that needs it) does, and fails loudly if it has not been built.
"""
from __future__ import annotations

__all__ = ["load", "api", "synth"]


def load():
    """Load libsbp.so; raises RuntimeError if it is not built."""
    from . import _abi
    return _abi.lib()


def __getattr__(name):
    if name in ("api", "autograd", "recon", "autotune", "mlp", "synth"):
        import importlib
        return importlib.import_module(f".{name}", __name__)
    from . import api as _api
    if hasattr(_api, name):
        return getattr(_api, name)
    raise AttributeError(name)
