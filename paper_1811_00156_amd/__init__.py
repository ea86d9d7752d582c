"""MI355X-native random-forest performance prediction from AIWC feature vectors.

The package is deliberately small: ``synth`` generates seeded synthetic workloads
shaped like the paper's data (Sec. III-A), and ``rf`` is the ctypes binding of the
HIP library ``libaiwc_rf.so`` (quantile binning, forest fit, batched predict).
Submodules are imported lazily so that the pure-NumPy generator can be used
without touching the GPU library.
"""

__all__ = ["synth", "rf"]


def __getattr__(name):
    if name in __all__:
        import importlib

        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
