"""FP64 CPU oracle for the PRISM STEM-EELS method (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import, call or run anything in this package.  It shares no code with the
HIP library: it re-derives every quantity from the paper's equations with
numpy in float64 (numpy.fft for transforms, numpy matmul for products).

Modules
-------
physics     constants, grids, band limit, propagator, transmission, beam lists,
            probe coefficients, crop windows and probe eligibility
conventional  O1: the conventional multislice STEM-EELS algorithm (Sec. 3, first
            algorithm) -- the plain definition of the map
prism       O2: the PRISM STEM-EELS algorithm (Sec. 3, second algorithm) with
            the exact transposed multislice operator
models      operation-count, runtime and memory models of Sec. 3 (cost formulas)
metrics     the map error metric of Eq. nrmsse (as read: relative L2 norm)

The f > 1 (PRISM interpolation) semantics, which the paper does not state for EELS,
are pinned by the tiled-specimen identity described in prism.py.
"""
