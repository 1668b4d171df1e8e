"""MI355X-native plain-LWE KEM hot path (HIP kernels for gfx950 behind a C ABI).

The compute lives in ``liblwe_hip.so`` (see ``include/lwe.h``); this package holds its
ctypes binding (``lwe``), the build script (``build``), the batch-shape autotuner
(``tune``) and the continuous-batching server (``serve``).
"""
from .lwe import (  # noqa: F401
    Context,
    LweError,
    LweLibraryMissing,
    Params,
    NOALLOC_SCRATCH_BYTES,
    cdf_table,
    decaps_batch_noalloc,
    lib,
    param_id,
    param_id_paper,
    params,
    register_params,
)
