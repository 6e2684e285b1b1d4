"""MI355X (gfx950) library for the spatially mixed force evaluation of
ML-MIX (arXiv 2502.19081): C ABI in include/mlmix.h, HIP kernels in csrc/,
a ctypes binding (binding.py) and torch-facing wrappers (core.py,
autograd.py, md.py, serve.py)."""
__all__ = ["binding", "core"]


def __getattr__(name):
    import importlib
    if name in ("binding", "core", "autograd", "md", "serve"):
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
