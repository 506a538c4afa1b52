"""MI355X-native quantics-MPS Fresnel propagation (HIP kernels behind a C ABI).

Submodules load lazily so that importing the package does not require a GPU:
  build      compile libqtt.so in-tree with hipcc (gfx950)
  _lib       ctypes declarations of include/qtt.h
  api        PyTorch-facing entry points (tt_encode, mpo_apply, ...)
  mpo_build  host float64 construction of the Fresnel MPOs
"""
__all__ = ["build", "api", "mpo_build"]


def __getattr__(name):
    import importlib
    if name in ("build", "api", "mpo_build", "_lib", "autograd", "batch"):
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
