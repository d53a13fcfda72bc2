"""MI355X-native adaptive-precision EAM-ACE force evaluation (arXiv:2411.03002).

The compute path lives in libapx.so (hand-written HIP for gfx950, C ABI in
include/apx.h).  ``binding`` declares the ABI for ctypes; ``ops`` wraps it on torch
tensors; ``autograd`` exposes the ACE adjoint as a torch.autograd.Function.  Nothing is
loaded at import time; the first call that needs the library loads it and fails loudly
if it has not been built.
"""

__all__ = ["binding", "ops"]
