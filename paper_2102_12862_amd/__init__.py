"""MI355X (gfx950) shallow-water finite-volume step: HIP kernels behind a C ABI.

The product is ``libswe.so`` (sources in ``csrc/``, ABI in ``include/swe.h``);
``swe`` is its ctypes binding.  Building: ``python -m paper_2102_12862_amd.build``.
"""
from .swe import (BC_INFLOW_UNIFORM, BC_OUTFLOW_ZEROGRAD, BC_WALL, FP32, FP64, NEG_CLIP,  # noqa: F401
                  NEG_ERROR, Batch, Mesh, State, SweError, TorchDevice, load)
