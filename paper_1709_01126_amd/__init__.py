"""MI355X-native FP64 point-Jacobi PCG for the spherical Laplace equation
(the potential-field solve of arXiv:1709.01126, Sec. 2).

The solver is the C-ABI library ``libpot3d.so``.  Its hand-written gfx950
kernels are in ``csrc/`` and its interface is in ``include/pot3d.h``.
``pot3d`` is the ctypes binding.  PyTorch is only used by callers for device
buffers and streams.
"""
from .pot3d import (EBREAKDOWN, EDEVICE, EINVAL, ENOCONV, ENOMEM, FP32_REFINED, FP64, ITER_ONE_SWEEP,  # noqa: F401
                    PC_JACOBI, PC_PHI_LINE,
                    ITER_TWO_PASS, OK, REFINE_RELIABLE, REFINE_RESTART, UPPER_CLOSED_WALL, UPPER_SOURCE_SURFACE, Pot3dError, Server, Solver, load)
