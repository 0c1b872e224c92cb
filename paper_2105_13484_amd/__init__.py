"""MI355X (gfx950) implementation of the SSPRK2-SE / SSPRK3-SE split-explicit step.

The computation lives in ``libssprkse.so`` (HIP kernels behind the C ABI of
include/ssprkse.h); ``ssprkse`` is its ctypes binding.  There is no CPU
fallback: using the binding without the built library raises ImportError.
"""
from .ssprkse import (  # noqa: F401
    DeviceMesh, DeviceState, SSEError, load, state_from_case, LIB_PATH, EXPORTED,
    SSE_OK, SSE_EINVAL, SSE_ENOMEM, SSE_EDEVICE, SSE_ENONFINITE, SSE_ESTATE,
)
