"""Crowded-flavour preprocessing (Sec. 3.1) -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this module; the GPU library never calls it.

Sec. 3.1 masks the pixels affected by saturated sources and replaces them with
the neighbouring background, giving the fit pair (R-breve, S-breve) while the
unmasked images are kept for the difference image. The paper fixes no
details; the reading written out here:

* saturated: a pixel where R >= u_R or S >= u_S (the upper valid fluxes of
  the pair, Table A2's -tu / -iu), or either value is not finite -- a pixel
  is masked in both images, since the model compares R (x) K with S pixel by
  pixel;
* affected: within the kernel footprint of a saturated pixel, i.e. pixel x is
  masked if a saturated pixel lies at x + (a, b) for some |a| <= g0,
  |b| <= g1, the offsets taken circularly like the convolution of Eq. 12;
* neighbouring background: the image is cut into tiles of t0 x t1 pixels (the
  last tile of each axis ragged); a tile's background is the lower median --
  element (m - 1) // 2 of its m unmasked values in ascending order -- and a
  tile with no unmasked pixel takes the lower median of the backgrounds of
  the other tiles (0 when every pixel is masked);
* the masked pixels of each image take their tile's background, every other
  pixel keeps its value.

Written from these definitions with plain numpy; FP64 decisions on FP64
images, FP32 values compared in FP32.
"""
from __future__ import annotations

import numpy as np


def saturated(r, s, u_r, u_s):
    """Boolean image: not (r < u_r and s < u_s) -- a NaN compares false."""
    r = np.asarray(r)
    s = np.asarray(s)
    return ~((r < r.dtype.type(u_r)) & (s < s.dtype.type(u_s)))


def dilate(sat, g0, g1):
    """mask(x) = any sat(x + (a, b)) over |a| <= g0, |b| <= g1, circular."""
    sat = np.asarray(sat, dtype=bool)
    out = np.zeros_like(sat)
    for a in range(-g0, g0 + 1):
        for b in range(-g1, g1 + 1):
            out |= np.roll(np.roll(sat, -a, axis=0), -b, axis=1)
    return out


def lower_median(values):
    """Element (m - 1) // 2 of the m values in ascending order."""
    v = np.sort(np.asarray(values).ravel())
    return v[(len(v) - 1) // 2]


def tile_backgrounds(img, mask, t0, t1):
    """[ceil(n0/t0)][ceil(n1/t1)] backgrounds of img (same dtype)."""
    img = np.asarray(img)
    n0, n1 = img.shape
    nt0, nt1 = -(-n0 // t0), -(-n1 // t1)
    bg = np.zeros((nt0, nt1), dtype=img.dtype)
    empty = np.zeros((nt0, nt1), dtype=bool)
    for i in range(nt0):
        for j in range(nt1):
            blk = img[i * t0:(i + 1) * t0, j * t1:(j + 1) * t1]
            keep = ~mask[i * t0:(i + 1) * t0, j * t1:(j + 1) * t1]
            if keep.any():
                bg[i, j] = lower_median(blk[keep])
            else:
                empty[i, j] = True
    if empty.all():
        bg[:] = 0
    elif empty.any():
        bg[empty] = lower_median(bg[~empty])
    return bg


def fill(img, mask, bg, t0, t1):
    """Masked pixels := their tile's background."""
    img = np.asarray(img)
    n0, n1 = img.shape
    ti = (np.arange(n0) // t0)[:, None]
    tj = (np.arange(n1) // t1)[None, :]
    return np.where(mask, bg[ti, tj], img).astype(img.dtype)


def crowded_fit_pair(r, s, u_r, u_s, g0, g1, t0, t1):
    """(R-breve, S-breve, mask) of the crowded flavour."""
    mask = dilate(saturated(r, s, u_r, u_s), g0, g1)
    rb = fill(r, mask, tile_backgrounds(r, mask, t0, t1), t0, t1)
    sb = fill(s, mask, tile_backgrounds(s, mask, t0, t1), t0, t1)
    return rb, sb, mask
