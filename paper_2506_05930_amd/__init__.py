"""MI355X-native hot path of the neural visibility cache (Boksansky & Meister, JCGT 2025).

libnvc.so (HIP kernels for gfx950 behind the C ABI of include/nvc.h) does the
work; `api` marshals torch tensors into it and `cache.NVCache` strings the
calls into inference, sampling and online training.
"""
from . import _lib
from ._lib import NvcError, LIB_PATH

__all__ = ["_lib", "NvcError", "LIB_PATH", "load"]


def load():
    """Load libnvc.so (raises if it is not built)."""
    return _lib.load()
