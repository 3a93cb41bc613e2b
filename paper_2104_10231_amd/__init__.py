"""MI355X-native RelRes Lennard-Jones hot path (arXiv:2104.10231, Eq. 20).

The compute path is the HIP library built from ``csrc/`` for gfx950 and its C
ABI (``include/relres.h``); ``relres`` is the Python binding.
"""
__all__ = ["RelRes", "RelResError", "load_library", "MIX_GEOMETRIC", "MIX_ARITHMETIC",
           "LIST_ATOM", "LIST_SITE"]


def __getattr__(name):
    # the binding imports torch; load it only when it is used
    if name in __all__:
        from . import relres as _r
        return getattr(_r, name)
    raise AttributeError(name)
