"""MI355X-native Stolt-based (A)ASHRT operator and robust IRLS-CG source
separation (thesis of A. Ibrahim, 2015; Chapters 4-6).

The compute path is ``libashrt.so`` (HIP kernels for gfx950 behind a C ABI,
``include/ashrt.h``); this package is its ctypes binding with PyTorch tensors
as device memory.  Importing it loads the library and fails if it is missing.
"""
from . import _lib  # noqa: F401
from ._lib import AshrtError, OP_FORWARD, OP_ADJOINT, OP_INVERT, OP_FISTA, lib  # noqa: F401
from .ashrt import Plan, BatchPlan, Params, autotune, validate_desc, report_dict  # noqa: F401
from .unet import UNet, TrainParams  # noqa: F401

lib()  # load now: fail loudly when the HIP library is not built
