"""Pins of the image-method oracle (eq. 1), CPU only.

Each check fixes the oracle to something other than itself: a worked case with
exactly known distance and tap, an independent construction of the images by
explicit mirroring across the walls (pure Python), the reflection-free limit
r = 0, reciprocity of source and microphone, and the bound between the
quantised and the plain binary64 sums."""
import math

import numpy as np
import pytest

from oracle import image_oracle as im

FS, C0 = 16000.0, 343.0


def test_direct_path_of_a_3_4_5_triangle():
    # order 0: only the real source; |src - mic| = 5 m exactly, so the tap is
    # ceil(5 * 16000 / 343) = ceil(233.2361...) = 234 and the amplitude 1/5
    h = im.image_rir((6.0, 7.0, 3.0), (1.0, 1.0, 1.0), (4.0, 5.0, 1.0), 0.7, 400, order=0)
    assert np.count_nonzero(h) == 1
    assert h[234] == np.float32(0.2)


def _mirror_images(L, s, K):
    """Images of coordinate s in [0, L] after 0..K reflections, built by
    mirroring across the walls 0 and L in turn: (position, reflections)."""
    out = [(s, 0)]
    for first in (0, 1):
        p = s
        wall = first
        for k in range(1, K + 1):
            p = -p if wall == 0 else 2.0 * L - p
            out.append((p, k))
            wall = 1 - wall
    return out


def _brute_rir(room, src, mic, r, length, K):
    """Eq. (1) by explicit mirroring, summed in binary64 (pure Python)."""
    axes = [_mirror_images(room[a], src[a], K) for a in range(3)]
    h = [0.0] * length
    count = [0] * length
    for px, gx in axes[0]:
        for py, gy in axes[1]:
            for pz, gz in axes[2]:
                d = math.sqrt((px - mic[0]) ** 2 + (py - mic[1]) ** 2 + (pz - mic[2]) ** 2)
                n = math.ceil(d * FS / C0)
                if n < length:
                    h[n] += r ** (gx + gy + gz) / d
                    count[n] += 1
    return np.array(h), np.array(count)


@pytest.mark.parametrize("K", [0, 1, 2, 3])
def test_images_match_explicit_mirroring(K):
    room, src, mic, r = (4.3, 3.7, 2.9), (1.1, 2.6, 1.3), (3.2, 0.9, 1.7), 0.63
    length = 2000
    # per axis, the oracle's image set equals the mirrored one
    n, amp, g, d = im.image_taps(room, src, mic, r, order=K)
    assert n.size == (2 * K + 1) ** 3
    ref, cnt = _brute_rir(room, src, mic, r, length, K)
    got = im.image_rir(room, src, mic, r, length, order=K).astype(np.float64)
    # quantisation 2^-41 per image, then one float32 rounding
    bound = cnt * 2.0 ** -41 + np.abs(ref) * 2.0 ** -24 + 1e-12 * np.abs(ref)
    assert np.all(np.abs(got - ref) <= bound)
    assert np.count_nonzero(got) == np.count_nonzero(cnt)


def test_no_reflection_leaves_the_direct_path():
    room, src, mic = (5.0, 4.0, 3.0), (1.0, 2.0, 1.5), (3.5, 1.2, 1.1)
    h8 = im.image_rir(room, src, mic, 0.0, 3000, order=8)
    h0 = im.image_rir(room, src, mic, 0.9, 3000, order=0)
    assert np.array_equal(h8, h0)
    d = math.dist(src, mic)
    assert np.nonzero(h0)[0].tolist() == [math.ceil(d * FS / C0)]


def test_reciprocity_of_source_and_microphone():
    rng = np.random.default_rng(5)
    for _ in range(4):
        room = rng.uniform(3.0, 8.0, 3)
        a = rng.uniform(0.3, 0.7, 3) * room
        b = rng.uniform(0.3, 0.7, 3) * room
        r = float(rng.uniform(0.3, 0.9))
        h1 = im.image_rir(room, a, b, r, 4000).astype(np.float64)
        h2 = im.image_rir(room, b, a, r, 4000).astype(np.float64)
        # the two differ only by last-bit differences of the distances
        assert np.max(np.abs(h1 - h2)) <= 4 * 2.0 ** -40 + 2.0 ** -24 * np.max(np.abs(h1))


def test_quantised_sum_within_its_bound_of_the_plain_sum():
    room, src, mic, r = (7.1, 5.3, 3.1), (2.0, 1.5, 1.2), (5.5, 4.0, 1.6), 0.85
    n, _, _, _ = im.image_taps(room, src, mic, r)
    length = 6000
    cnt = np.bincount(n[n < length], minlength=length)
    ex = im.image_rir_exact(room, src, mic, r, length)
    got = im.image_rir(room, src, mic, r, length).astype(np.float64)
    assert np.all(np.abs(got - ex) <= cnt * 2.0 ** -41 + np.abs(ex) * 2.0 ** -24 + 1e-15)


def test_small_amplitudes_are_rounded_to_nearest():
    # with r = 0.01 the images after four or more reflections have amplitudes
    # of about 2^-27 and below, where float32 resolves far finer than the
    # 2^-40 quantum: at taps holding only such images the quantised sum stays
    # within count * 2^-41 of the plain binary64 sum, the bound of rounding
    # each image to nearest (truncating errs by up to twice as much)
    room, src, mic, r = (7.1, 5.3, 3.1), (2.0, 1.5, 1.2), (5.5, 4.0, 1.6), 0.01
    length = 6000
    n, _, g, _ = im.image_taps(room, src, mic, r)
    keep = n < length
    cnt = np.bincount(n[keep], minlength=length)
    gmin = np.full(length, 1 << 30)
    np.minimum.at(gmin, n[keep], g[keep])
    small = (cnt > 0) & (gmin >= 4)
    assert np.count_nonzero(small) > 100
    ex = im.image_rir_exact(room, src, mic, r, length)[small]
    got = im.image_rir(room, src, mic, r, length).astype(np.float64)[small]
    assert np.all(np.abs(got - ex) <= cnt[small] * 2.0 ** -41 + np.abs(ex) * (2.0 ** -24 + 1e-15))


def test_taps_beyond_the_length_are_dropped():
    room, src, mic, r = (6.0, 5.0, 3.0), (1.0, 1.0, 1.0), (4.0, 3.0, 2.0), 0.8
    long = im.image_rir(room, src, mic, r, 5000)
    short = im.image_rir(room, src, mic, r, 1234)
    assert np.array_equal(long[:1234], short)
    assert im.image_rir(room, src, mic, r, 0).size == 0


@pytest.mark.parametrize("src,mic,r", [
    ((1.0, 1.0, 1.0), (1.0, 1.0, 1.0), 0.5),        # source at the microphone
    ((1.0, 1.0, 1.0), (1.005, 1.0, 1.0), 0.5),      # 5 mm apart
    ((0.001, 1.0, 1.0), (2.0, 1.0, 1.0), 0.5),      # 1 mm from a wall
    ((1.0, 1.0, 1.0), (2.0, 1.0, 2.999), 0.5),      # 1 mm from the ceiling
    ((1.0, 1.0, 1.0), (2.0, 1.0, 1.0), 1.5),        # r outside [0, 1]
])
def test_invalid_geometry_is_rejected(src, mic, r):
    with pytest.raises(ValueError):
        im.image_rir((5.0, 4.0, 3.0), src, mic, r, 100)
