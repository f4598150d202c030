"""MI355X-native PRISM STEM-EELS map simulation (Brown, Ciston, Ophus; arXiv:1908.07628).

The compute path is the HIP library libeels.so (C ABI in include/eels.h); this package
holds its sources (csrc/), the in-tree build script and the ctypes binding.
"""
from .eels import (  # noqa: F401
    BF16_SPLIT,
    FP16_SPLIT,
    FP32,
    EelsError,
    Plan,
    cgemm,
    device_inputs,
    bf_corrected,
    load_library,
    map_mean,
    map_ratio,
    solve,
    solve_conventional,
    solve_with_images,
)

__version__ = "0.4"
