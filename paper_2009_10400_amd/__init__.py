"""MI355X-native coupled TLED + Pennes bioheat solver (arXiv 2009.10400).

The solver lives in the HIP/C++ shared library ``csrc/libtled.so`` behind the
C-ABI declared in ``include/tled.h``; :mod:`paper_2009_10400_amd.tled` is the
thin ctypes binding.  :mod:`paper_2009_10400_amd.workloads` generates seeded
synthetic inputs.  The binding is imported lazily so that input generation
works on a machine without the built library.
"""

__all__ = ["tled", "workloads"]


def __getattr__(name):
    if name in ("tled", "workloads"):
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
