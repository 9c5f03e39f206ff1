"""BootMMPM large-plaintext functional bootstrapping on MI355X (gfx950).

The compute lives in ``lib/libmmpm.so`` (HIP kernels + C ABI, include/mmpm.h);
``binding`` marshals numpy arrays and torch device tensors into it.  Importing
``Context`` without the built library raises ImportError: there is no CPU path.
"""

__all__ = ["Context", "Server", "MMError", "MM_DEVICE_PTRS", "MM_PLAIN"]


def __getattr__(name):
    if name in __all__:
        from . import binding
        return getattr(binding, name)
    raise AttributeError(name)
