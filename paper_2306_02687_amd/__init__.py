"""MI355X (gfx950) hyper-reduced RVE evaluation for the monolithic hyper ROM FE2 method.

The compute path is the HIP library ``libhrom.so`` (C ABI in include/hrom.h);
``binding`` marshals torch tensors into it, ``solve`` sequences its calls
(micro Newton, monolithic iterations) and ``autograd`` exposes the adjoint
backward as a ``torch.autograd.Function``.
"""
from . import binding  # noqa: F401
from .binding import (FP64, MIXED_BF16, MIXED_FP16, ClusterSpec, HromError, Plan,  # noqa: F401
                      load)
