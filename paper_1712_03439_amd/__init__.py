"""MI355X-native room-simulator hot path (arXiv:1712.03439): RIR tail cut-off,
overlap-add FFT filtering and SNR-scaled mixing in hand-written HIP kernels for
gfx950, behind the C ABI in include/rsim.h.

Import `paper_1712_03439_amd.rsim` for the binding; it loads librsim.so and
raises if the library has not been built.
"""
__version__ = "1.0.0"
