"""FP64 oracle of the image-method room impulse response (eq. 1).

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or run
this module.  It shares no code, tables or helpers with the GPU path.

The paper (Sec. 2.1, eq. 1) models a rectangular room whose walls reflect
uniformly with coefficient r: the room is mirrored across its walls into a
grid of virtual rooms, each holding one image of the source, and the RIR is
the sum over the V images of r^g / d placed at the tap ceil(d fs / c0), where
d is the image-to-microphone distance and g the number of reflections.  It
uses a 17 x 17 x 17 grid of virtual rooms (order K = 8), fs = 16 kHz and
c0 = 343 m/s.

Readings where the paper is silent:
* The virtual room (a, b, c), -K <= a, b, c <= K, holds the image at
  x = a Lx + xs for even a and a Lx + (Lx - xs) for odd a (likewise y, z),
  reached after g = |a| + |b| + |c| reflections.
* Taps at or beyond the requested length are dropped.
* Geometry: sides below 10 km, source and microphone at least 5 mm inside
  every wall and at least 1 cm apart, so every image is at least 1 cm from
  the microphone; 0 <= r <= 1.
* Arithmetic: binary64, no fused multiply-add, in this order:
  d = sqrt((dx dx + dy dy) + dz dz); n = ceil((d fs) / c0);
  r^g = r multiplied g times starting from 1; amplitude (r^g) / d.
* Accumulation: each amplitude is quantised to a multiple of 2^-40
  (rint(amplitude 2^40), half to even) and the taps sum these integers
  exactly, so the result does not depend on the order of the images; the
  sum is converted to binary64, scaled by 2^-40 and rounded once to float32.
  Each image adds at most 2^-41 of quantisation error.
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np

FIXED_SHIFT = 40


def image_taps(room: Sequence[float], src: Sequence[float], mic: Sequence[float], refl: float,
               order: int = 8, fs: float = 16000.0, c0: float = 343.0):
    """Every image of eq. (1): (tap n, amplitude r^g / d, g, d) as arrays, in
    the order a, then b, then c from -K to K."""
    K = int(order)
    if K < 0:
        raise ValueError("order must be >= 0")
    L = [float(v) for v in room]
    s = [float(v) for v in src]
    m = [float(v) for v in mic]
    idx = np.arange(-K, K + 1)
    # per axis: image coordinate minus the mic coordinate, and |index|
    deltas = []
    for ax in range(3):
        pos = np.where(idx % 2 == 0, idx * L[ax] + s[ax], idx * L[ax] + (L[ax] - s[ax]))
        deltas.append(pos - m[ax])
    dx, dy, dz = np.meshgrid(deltas[0], deltas[1], deltas[2], indexing="ij")
    ga, gb, gc = np.meshgrid(np.abs(idx), np.abs(idx), np.abs(idx), indexing="ij")
    d2 = (dx * dx + dy * dy) + dz * dz
    d = np.sqrt(d2).reshape(-1)
    # source and microphone at least 5 mm inside every wall and 1 cm apart
    for ax in range(3):
        if not (L[ax] < 1e4 and 0.005 <= s[ax] <= L[ax] - 0.005 and 0.005 <= m[ax] <= L[ax] - 0.005):
            raise ValueError("sides below 10 km; source and microphone at least 5 mm inside the room")
    if ((s[0] - m[0]) * (s[0] - m[0]) + (s[1] - m[1]) * (s[1] - m[1])) + (s[2] - m[2]) * (s[2] - m[2]) < 1e-4:
        raise ValueError("source and microphone must be at least 1 cm apart")
    if not 0.0 <= float(refl) <= 1.0:
        raise ValueError("the reflection coefficient must lie in [0, 1]")
    n = np.ceil((d * float(fs)) / float(c0)).astype(np.int64)
    g = (ga + gb + gc).reshape(-1)
    pw = np.empty(3 * K + 1)
    p = 1.0
    for k in range(3 * K + 1):
        pw[k] = p
        p = p * float(refl)
    amp = pw[g] / d
    return n, amp, g, d


def image_rir(room: Sequence[float], src: Sequence[float], mic: Sequence[float], refl: float, length: int,
              order: int = 8, fs: float = 16000.0, c0: float = 343.0) -> np.ndarray:
    """The RIR of eq. (1), `length` taps, float32 (readings in the module
    docstring)."""
    n, amp, _, _ = image_taps(room, src, mic, refl, order, fs, c0)
    q = np.rint(amp * float(2 ** FIXED_SHIFT)).astype(np.int64)
    acc = np.zeros(max(int(length), 0), np.int64)
    keep = n < length
    np.add.at(acc, n[keep], q[keep])
    return (acc.astype(np.float64) * math.ldexp(1.0, -FIXED_SHIFT)).astype(np.float32)


def image_rir_exact(room: Sequence[float], src: Sequence[float], mic: Sequence[float], refl: float,
                    length: int, order: int = 8, fs: float = 16000.0, c0: float = 343.0) -> np.ndarray:
    """Eq. (1) summed in binary64 without quantisation (for the error bound)."""
    n, amp, _, _ = image_taps(room, src, mic, refl, order, fs, c0)
    acc = np.zeros(max(int(length), 0), np.float64)
    keep = n < length
    np.add.at(acc, n[keep], amp[keep])
    return acc
