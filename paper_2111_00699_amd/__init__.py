"""MI355X-native explicit MLS-MPM substep (arXiv 2111.00699 hot path).

The simulation runs in hand-written HIP kernels for gfx950 behind the C ABI
declared in ``include/mpm.h`` (``libmpm.so``).  ``paper_2111_00699_amd.mpm``
is the thin ctypes binding; ``paper_2111_00699_amd.scenes`` makes seeded
synthetic inputs.  Importing the package does not load the library.
"""
__all__ = ["mpm", "scenes"]


def __getattr__(name):
    if name in __all__:
        import importlib

        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
