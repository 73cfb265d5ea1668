"""MI355X labeling of discrete abstractions (Boolean product L = T (x) O).

The compute path is the HIP library liblbl.so (C ABI in include/lbl.h); the
module `lbl` is its ctypes binding.
"""
from . import lbl  # noqa: F401

__all__ = ["lbl"]
