"""Pins of the crowded-flavour preprocessing oracle (Sec. 3.1), on the CPU.

Checked against things other than its own definitions: scipy's maximum
filter (wrap mode) for the footprint dilation, numpy's median / partition
for the tile backgrounds, and closed-form cases -- a constant sky with
saturated stars is restored to the sky exactly, an image without saturated
pixels is returned unchanged, a fully masked tile takes the median of the
other tiles, a non-finite pixel is masked.
"""
import numpy as np
import pytest
from scipy import ndimage

from oracle import mask as om


@pytest.mark.parametrize("g0,g1", [(0, 0), (1, 2), (3, 3), (5, 1)])
def test_dilation_is_the_wrapped_maximum_filter(g0, g1):
    rng = np.random.default_rng(g0 * 10 + g1)
    sat = rng.uniform(size=(37, 29)) < 0.02
    sat[0, 0] = sat[-1, 5] = sat[12, -1] = True   # footprints across the wrap
    want = ndimage.maximum_filter(sat.astype(np.uint8), size=(2 * g0 + 1, 2 * g1 + 1),
                                  mode="wrap").astype(bool)
    assert np.array_equal(om.dilate(sat, g0, g1), want)


@pytest.mark.parametrize("m", [1, 2, 7, 8, 1001])
def test_lower_median(m):
    rng = np.random.default_rng(m)
    v = rng.normal(size=m)
    k = (m - 1) // 2
    assert om.lower_median(v) == np.partition(v, k)[k]
    if m % 2:
        assert om.lower_median(v) == np.median(v)


def test_saturated_pixels_and_nonfinite():
    r = np.array([[1.0, 5.0], [np.nan, 2.0]])
    s = np.array([[1.0, 1.0], [1.0, 9.0]])
    got = om.saturated(r, s, 5.0, 9.0)
    assert np.array_equal(got, [[False, True], [True, True]])


def test_constant_sky_with_saturated_stars_is_restored():
    n0, n1, sky, u = 96, 80, 100.0, 5000.0
    img = np.full((n0, n1), sky)
    yy, xx = np.mgrid[:n0, :n1]
    for (y, x) in ((10, 10), (50, 70), (90, 3)):   # the last wraps
        img += 2e5 * np.exp(-(((yy - y + n0 // 2) % n0 - n0 // 2) ** 2 +
                              ((xx - x + n1 // 2) % n1 - n1 // 2) ** 2) / 2.0)
    r = np.minimum(img, u)          # clipped at saturation
    s = np.minimum(0.9 * img, u)
    # grow by the radius where the stars fall below 1e-12 of the sky
    rb, sb, mask = om.crowded_fit_pair(r, s, u, u, 12, 12, 32, 16)
    assert mask.any()
    assert np.array_equal(rb[~mask], r[~mask]) and np.array_equal(sb[~mask], s[~mask])
    # every tile's background is the sky (its unmasked pixels are the sky to
    # within 2e5 exp(-72) ~ 1e-26), so the masked pixels are restored to it
    assert np.abs(rb[mask] - sky).max() <= 1e-9
    assert np.abs(sb[mask] - 0.9 * sky).max() <= 1e-9


def test_no_saturation_is_the_identity():
    rng = np.random.default_rng(3)
    r = rng.normal(100, 10, (64, 48)).astype(np.float32)
    s = rng.normal(100, 10, (64, 48)).astype(np.float32)
    rb, sb, mask = om.crowded_fit_pair(r, s, 1e4, 1e4, 3, 3, 16, 16)
    assert not mask.any()
    assert np.array_equal(rb, r) and np.array_equal(sb, s) and rb.dtype == np.float32


def test_tile_backgrounds_against_numpy_and_empty_tile_fallback():
    rng = np.random.default_rng(9)
    n0, n1, t0, t1 = 40, 50, 16, 16      # ragged last tiles (8 and 2 pixels)
    img = rng.normal(0, 1, (n0, n1))
    mask = rng.uniform(size=(n0, n1)) < 0.3
    mask[16:32, 16:32] = True            # tile (1, 1) fully masked
    bg = om.tile_backgrounds(img, mask, t0, t1)
    assert bg.shape == (3, 4)
    for i in range(3):
        for j in range(4):
            if (i, j) == (1, 1):
                continue
            v = img[i * t0:(i + 1) * t0, j * t1:(j + 1) * t1][~mask[i * t0:(i + 1) * t0,
                                                                     j * t1:(j + 1) * t1]]
            k = (len(v) - 1) // 2
            assert bg[i, j] == np.partition(v, k)[k]
    others = np.delete(bg.ravel(), 1 * 4 + 1)
    k = (len(others) - 1) // 2
    assert bg[1, 1] == np.partition(others, k)[k]
    allm = om.tile_backgrounds(img, np.ones_like(mask), t0, t1)
    assert not allm.any()
