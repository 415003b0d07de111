"""Noise decorrelation of the difference image (App. C) -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this module; the GPU library never calls it.

App. C models the difference image of co-added images as
    D = sum_j S_j (x) G_j - [sum_i R_i (x) H_i] (x) K          (Eq. C21)
with independent white noise of standard deviation sigma_Sj, sigma_Ri in the
individual images S_j, R_i (G_j, H_i already include the 1/M, 1/N of the
average co-add). A kernel Q whitens D (Eq. C22-C23); the real, even
solution (Eq. C24) is
    Q0^(p) = sqrt( sigma_D^2 / { sum_j sigma_Sj^2 |G_j^(p)|^2
                                 + sum_i sigma_Ri^2 |K^(p)|^2 |H_i^(p)|^2 } ),
normalised to unit kernel sum (Q^(0) = 1, the flux-preserving choice), and
the decorrelated image is D (x) Q, one circular convolution. Kernels are
small stamps (offsets a in [-w0, w0], b in [-w1, w1]) whose transforms are
the DFTs of the stamps placed circularly on the N0 x N1 grid. The spatial
variation of the matching kernel is ignored (App. C): K is the kernel field
of the fit evaluated at one position.

Written from the definitions above, with ``numpy.fft`` as the DFT; FP64.
"""
from __future__ import annotations

import numpy as np


def stamp_on_grid(stamp, n0, n1):
    """The (2w0+1) x (2w1+1) stamp placed circularly on an n0 x n1 grid:
    entry (a, b) at pixel (a mod n0, b mod n1)."""
    stamp = np.asarray(stamp, dtype=np.float64)
    w0, w1 = (stamp.shape[0] - 1) // 2, (stamp.shape[1] - 1) // 2
    grid = np.zeros((n0, n1))
    for a in range(-w0, w0 + 1):
        for b in range(-w1, w1 + 1):
            grid[a % n0, b % n1] += stamp[a + w0, b + w1]
    return grid


def delta_stamp(w0, w1, scale=1.0):
    st = np.zeros((2 * w0 + 1, 2 * w1 + 1))
    st[w0, w1] = scale
    return st


def kernel_at(stamps, dk, u0, u1):
    """Matching kernel at normalised position (u0, u1): sum over the kernel
    terms k = (i, j) of stamp_k * u0^i * u1^j (Eq. 5-6 with the stamps of
    Eq. 3-4, the kernel at one point of the field)."""
    terms = [(i, j) for i in range(dk + 1) for j in range(dk + 1 - i)]
    k = np.zeros(np.asarray(stamps[0]).shape)
    for t, (i, j) in enumerate(terms):
        k += np.asarray(stamps[t], dtype=np.float64) * (u0 ** i) * (u1 ** j)
    return k


def noise_power(kernel, n0, n1, sigma_s, g, sigma_r, h):
    """The denominator of Eq. C23-C24 on the full DFT grid:
    sum_j sigma_Sj^2 |G_j^|^2 + |K^|^2 sum_i sigma_Ri^2 |H_i^|^2."""
    kh = np.fft.fft2(stamp_on_grid(kernel, n0, n1))
    den = np.zeros((n0, n1))
    for sj, gj in zip(sigma_s, g):
        den += sj * sj * np.abs(np.fft.fft2(stamp_on_grid(gj, n0, n1))) ** 2
    acc = np.zeros((n0, n1))
    for si, hi in zip(sigma_r, h):
        acc += si * si * np.abs(np.fft.fft2(stamp_on_grid(hi, n0, n1))) ** 2
    return den + np.abs(kh) ** 2 * acc


def decorrelation_spectrum(kernel, n0, n1, sigma_s, g, sigma_r, h):
    """Q^ of Eq. C24 normalised to unit kernel sum: sqrt(den(0) / den(p))."""
    den = noise_power(kernel, n0, n1, sigma_s, g, sigma_r, h)
    return np.sqrt(den[0, 0] / den)


def decorrelate(d, kernel, sigma_s, g, sigma_r, h):
    """D (x) Q, circular, with Q^ from decorrelation_spectrum."""
    d = np.asarray(d, dtype=np.float64)
    n0, n1 = d.shape
    q = decorrelation_spectrum(kernel, n0, n1, sigma_s, g, sigma_r, h)
    return np.real(np.fft.ifft2(np.fft.fft2(d) * q))
