"""FP64 CPU oracle for the room-simulator hot path (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the GPU path.  `image_oracle`
holds the image-method RIR of eq. (1).
"""
from .rsim_oracle import (  # noqa: F401
    cut_scale,
    cut_rir,
    dry_power,
    snr_gains,
    convolve,
    mix,
    mix_at,
    mix_backward,
    mix_backward_at,
    out_length,
    reverb_energy,
    snr_gains_reverb,
    simulate,
)
