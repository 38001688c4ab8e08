"""MI355X (gfx950) QAOA state-vector library for the dense sub-QUBOs of
distributed QAOA (arXiv 2506.10531).  The compute path is the HIP library
``libdqaoa.so`` behind the C ABI in ``include/dqaoa.h``; this package only
marshals arguments.  Importing it does not load the library; the first call
does, and fails loudly if it has not been built."""
import importlib

__all__ = ["api", "serve", "workloads"]

_API_NAMES = ("Context", "expect", "state", "sample", "grad", "QAOAExpect",
              "default_context", "host_context")


def __getattr__(name):
    if name in ("api", "serve", "workloads", "_lib"):
        return importlib.import_module(f".{name}", __name__)
    if name in _API_NAMES:
        return getattr(importlib.import_module(".api", __name__), name)
    if name == "SolveQueue":
        return importlib.import_module(".serve", __name__).SolveQueue
    raise AttributeError(name)
