"""bcmg: ghost-point geometric multigrid on level-set domains for AMD MI355X.

The solver lives in libbcmg.so (HIP kernels for gfx950 behind the C ABI of
include/bcmg.h).  ``solver`` wraps it for torch device tensors, ``workloads``
holds the seeded synthetic inputs, ``batching`` the autotuned batched path and
``serving`` the continuous-batching request loop.  Submodules are imported on
first use so that ``workloads`` can be used without torch or a GPU.
"""
import importlib

__all__ = ["solver", "workloads", "build", "batching", "serving", "autotune"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
