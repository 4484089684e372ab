"""MI355X-native grouped multi-density J/K Fock builds (ESMF, arXiv:2002.00322).

The compute path is libesmf.so (hand-written HIP for gfx950 behind a C ABI,
``include/esmf.h``); this package only marshals arguments.  PyTorch supplies
device memory and streams."""
from ._native import (  # noqa: F401
    EsmfError, InvalidArgument, OutOfMemory, DeviceError, NotSupported,
    PREC_FP64, PREC_MIXED, PREC_STORE32, STORE_FP64, STORE_FP32, STORE_DIRECT,
)
from .api import (  # noqa: F401
    EriStore, Server, fock_build, fock_build_batched, fock_tune, batched_report, timing_enable, timing_collect,
    probe_peaks,
    nine_densities, energy_two_body, energy_gradient, ESMF_SYMMETRIC,
)
