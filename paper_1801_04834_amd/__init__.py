"""MI355X-native FX correlator (LOFAR Cobalt hot path) behind the C ABI in ``include/cobalt.h``.

The compute path lives in ``libcobalt.so`` (HIP kernels for gfx950, built from ``csrc/``).
``binding`` marshals arguments to it; nothing in this package computes any step of the
chain in Python.  Importing the package does not load the library: creating a ``Plan``
does, and fails with a clear error when the library has not been built.
"""

__all__ = ["Plan", "CobaltError", "lib_path", "synth"]


def __getattr__(name):
    if name in ("Plan", "CobaltError", "lib_path", "estimate_bytes"):
        from . import binding
        return getattr(binding, name)
    raise AttributeError(name)
