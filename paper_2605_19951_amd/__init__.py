"""MI355X-native pole-shifted sparse solves for rational-approximation TEM.

The computation lives in libtem.so (HIP kernels for gfx950 behind the C ABI
of include/tem.h); ``tem`` is its thin binding and ``autograd`` wraps the
forward map d(ln sigma) with its adjoint as a torch.autograd.Function.
``rkfit`` (host-only, NumPy) computes the poles and residues the library
takes: RKFIT common poles for exp(-t z) over a set of times.
"""
from .tem import (FP32_IR, FP64, Tem, TemError, load_library, symbolic_host)  # noqa: F401

__all__ = ["Tem", "TemError", "FP64", "FP32_IR", "load_library", "symbolic_host"]
