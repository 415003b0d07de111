"""Seeded synthetic star-field image pairs.

This module is the single input source shared by the GPU path's tests and
benchmark and by the CPU oracle's tests. It renders physical scenes (stars,
sky, noise) and holds none of the subtraction method's arithmetic: no basis
images, no normal equations, no model convolution. The science image is
rendered directly with its own point-spread function (the reference PSF
broadened by a Gaussian matching kernel, analytically for Gaussian PSFs and as
a broadened Moffat otherwise), its own photometric scale and its own sky.

Recipes (all draws from ``numpy.random.Generator(PCG64(seed))``):

* star positions: uniform continuous on [0, N0) x [0, N1) (a Poisson process
  conditioned on the count);
* fluxes: dN/df ~ f^-2 on [1e2, 1e5], by inverse CDF
  f = 1 / (1/1e2 - u (1/1e2 - 1/1e5));
* PSFs sampled at pixel centres with periodic wrap and analytic
  normalisation; Gaussian f exp(-r^2 / 2 s^2) / (2 pi s^2) with stamp radius
  ceil(5 s); Moffat f (b-1)/(pi a^2) (1 + r^2/a^2)^-b with
  a = FWHM / (2 sqrt(2^(1/b) - 1)) and stamp radius ceil(4 FWHM) + 2;
* reference R = sky 100 + stars + N(0, 10^2); science
  S = s(x) (100 + stars_S) + B(x) + N(0, 10^2).

Axis 0 of every array is the paper's x (row index), axis 1 its y.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

FLUX_MIN = 1.0e2
FLUX_MAX = 1.0e5
SKY = 100.0
NOISE = 10.0


@dataclass
class Pair:
    """One synthetic image pair plus the fit parameters it is meant for."""

    r: np.ndarray
    s: np.ndarray
    w0: int
    w1: int
    dk: int
    db: int
    const_phot: int = 0
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.r.shape


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def draw_fluxes(rng, n):
    u = rng.random(n)
    return 1.0 / (1.0 / FLUX_MIN - u * (1.0 / FLUX_MIN - 1.0 / FLUX_MAX))


def draw_positions(rng, n, n0, n1):
    return rng.random(n) * n0, rng.random(n) * n1


def _render(n0, n1, x, y, flux, radius, profile, chunk=1024):
    """Sum per-star stamps on an n0 x n1 torus. ``profile(r2, idx)`` returns
    the normalised PSF value at squared distance r2 for the stars ``idx``."""
    img = np.zeros(n0 * n1, dtype=np.float64)
    order = np.argsort(radius, kind="stable")
    for c0 in range(0, len(order), chunk):
        idx = order[c0:c0 + chunk]
        rad = int(radius[idx].max())
        off = np.arange(-rad, rad + 1)
        cx = np.floor(x[idx]).astype(np.int64)
        cy = np.floor(y[idx]).astype(np.int64)
        px = cx[:, None, None] + off[None, :, None]
        py = cy[:, None, None] + off[None, None, :]
        dx = px + 0.5 - x[idx][:, None, None]
        dy = py + 0.5 - y[idx][:, None, None]
        r2 = dx * dx + dy * dy
        val = flux[idx][:, None, None] * profile(r2, idx)
        inside = (np.abs(px - cx[:, None, None]) <= radius[idx][:, None, None]) & \
                 (np.abs(py - cy[:, None, None]) <= radius[idx][:, None, None])
        val = np.where(inside, val, 0.0)
        flat = (px % n0) * n1 + (py % n1)
        img += np.bincount(flat.ravel(), weights=val.ravel(), minlength=n0 * n1)
    return img.reshape(n0, n1)


def render_gaussian(n0, n1, x, y, flux, sigma):
    sigma = np.broadcast_to(np.asarray(sigma, dtype=np.float64), x.shape).copy()
    radius = np.ceil(5.0 * sigma).astype(np.int64)

    def prof(r2, idx):
        s2 = sigma[idx][:, None, None] ** 2
        return np.exp(-r2 / (2.0 * s2)) / (2.0 * math.pi * s2)

    return _render(n0, n1, x, y, flux, radius, prof)


def render_moffat(n0, n1, x, y, flux, fwhm, beta=3.0):
    fwhm = np.broadcast_to(np.asarray(fwhm, dtype=np.float64), x.shape).copy()
    a = fwhm / (2.0 * math.sqrt(2.0 ** (1.0 / beta) - 1.0))
    radius = (np.ceil(4.0 * fwhm) + 2).astype(np.int64)

    def prof(r2, idx):
        a2 = a[idx][:, None, None] ** 2
        return (beta - 1.0) / (math.pi * a2) * (1.0 + r2 / a2) ** (-beta)

    return _render(n0, n1, x, y, flux, radius, prof)


def norm_coords(n0, n1):
    """Centred coordinates in [-1, 1] along each axis (column vectors)."""
    c0 = (2.0 * np.arange(n0) - (n0 - 1)) / max(n0 - 1, 1)
    c1 = (2.0 * np.arange(n1) - (n1 - 1)) / max(n1 - 1, 1)
    return c0[:, None], c1[None, :]


def sky_quadratic(n0, n1):
    c0, c1 = norm_coords(n0, n1)
    return 5.0 + 2.0 * c0 - 1.5 * c1 + 0.8 * c0 ** 2 - 0.5 * c0 * c1 + 0.3 * c1 ** 2


def _finish(rng, r_true, s_true, noise, dtype):
    r = r_true + (rng.normal(0.0, noise, r_true.shape) if noise > 0 else 0.0)
    s = s_true + (rng.normal(0.0, noise, s_true.shape) if noise > 0 else 0.0)
    return r.astype(dtype), s.astype(dtype)


def config1(seed=1, noise=NOISE, transients=True):
    """256x256 FP64, 300 Gaussian stars (sigma 1.5); S is R seen through a
    0.9-scaled Gaussian kernel of sigma 1.2 plus 5 + 0.01 x, three point
    transients; 11x11 kernel, DK=0, DB=0."""
    rng = rng_for(seed)
    n0 = n1 = 256
    x, y = draw_positions(rng, 300, n0, n1)
    f = draw_fluxes(rng, 300)
    sr, sk = 1.5, 1.2
    stars_r = render_gaussian(n0, n1, x, y, f, sr)
    stars_s = render_gaussian(n0, n1, x, y, f, math.hypot(sr, sk))
    xx = np.arange(n0, dtype=np.float64)[:, None]
    s_true = 0.9 * (SKY + stars_s) + 5.0 + 0.01 * xx
    tx, ty = draw_positions(rng, 3, n0, n1)
    if transients:
        s_true = s_true + render_gaussian(n0, n1, tx, ty, np.full(3, 5.0e3),
                                          math.hypot(sr, sk))
    r, s = _finish(rng, SKY + stars_r, s_true, noise, np.float64)
    return Pair(r, s, 5, 5, 0, 0, 0, "C1 256x256 w=5 DK=0 DB=0",
                {"transients": (tx, ty)})


def config2(seed=2, noise=NOISE, n=1024, nstars=3000):
    """1024x1024 FP32, 3000 Gaussian stars; PSF sigma 1.2 -> 2.2 along x,
    photometric scale 0.85 -> 1.05 along y, matching-kernel sigma
    0.9 -> 1.4 along x, quadratic sky; 11x11 kernel, DK=2, DB=2."""
    rng = rng_for(seed)
    n0 = n1 = n
    x, y = draw_positions(rng, nstars, n0, n1)
    f = draw_fluxes(rng, nstars)
    sr = 1.2 + 1.0 * x / (n0 - 1)
    sk = 0.9 + 0.5 * x / (n0 - 1)
    scale_star = 0.85 + 0.20 * y / (n1 - 1)
    stars_r = render_gaussian(n0, n1, x, y, f, sr)
    stars_s = render_gaussian(n0, n1, x, y, f * scale_star, np.hypot(sr, sk))
    scale_pix = 0.85 + 0.20 * np.arange(n1, dtype=np.float64)[None, :] / (n1 - 1)
    s_true = scale_pix * SKY + stars_s + sky_quadratic(n0, n1)
    r, s = _finish(rng, SKY + stars_r, s_true, noise, np.float32)
    return Pair(r, s, 5, 5, 2, 2, 0, f"C2 {n0}x{n1} w=5 DK=2 DB=2")


def _rho(x, y, n0, n1):
    c0, c1 = (n0 - 1) / 2.0, (n1 - 1) / 2.0
    return np.hypot(x - c0 - 0.5, y - c1 - 0.5) / math.hypot(c0, c1)


def config3(seed=3, noise=NOISE, n=4096, nstars=40000):
    """4096x4096 FP32, 40000 Moffat (beta=3) stars with FWHM 2 + 2 rho^2
    (rho = radius / corner radius); matching-kernel sigma 1.0 + 0.6 rho^2,
    photometric scale 0.85 -> 1.05 along y, quadratic sky; 15x15 kernel,
    DK=2, DB=2."""
    rng = rng_for(seed)
    n0 = n1 = n
    x, y = draw_positions(rng, nstars, n0, n1)
    f = draw_fluxes(rng, nstars)
    rho = _rho(x, y, n0, n1)
    fwhm_r = 2.0 + 2.0 * rho ** 2
    sk = 1.0 + 0.6 * rho ** 2
    fwhm_s = np.hypot(fwhm_r, 2.0 * math.sqrt(2.0 * math.log(2.0)) * sk)
    scale_star = 0.85 + 0.20 * y / (n1 - 1)
    stars_r = render_moffat(n0, n1, x, y, f, fwhm_r)
    stars_s = render_moffat(n0, n1, x, y, f * scale_star, fwhm_s)
    scale_pix = 0.85 + 0.20 * np.arange(n1, dtype=np.float64)[None, :] / (n1 - 1)
    s_true = scale_pix * SKY + stars_s + sky_quadratic(n0, n1)
    r, s = _finish(rng, SKY + stars_r, s_true, noise, np.float32)
    return Pair(r, s, 7, 7, 2, 2, 0, f"C3 {n0}x{n1} w=7 DK=2 DB=2")


def star_pair(seed, n0, n1, w=5, dk=1, db=1, density=2.0e-3, noise=NOISE,
              dtype=np.float32, const_phot=0):
    """Generic pair: Gaussian PSF sigma ~ U[1, 2.5], linear photometric scale
    and kernel-width variation, polynomial sky of degree ``db``."""
    rng = rng_for(seed)
    nst = max(1, int(rng.poisson(density * n0 * n1)))
    x, y = draw_positions(rng, nst, n0, n1)
    f = draw_fluxes(rng, nst)
    sr = rng.uniform(1.0, 2.5)
    g0, g1 = rng.uniform(-0.3, 0.3, 2)
    s0 = rng.uniform(0.8, 1.1)
    sl0, sl1 = rng.uniform(-0.1, 0.1, 2)
    cx = (2.0 * x - (n0 - 1)) / max(n0 - 1, 1)
    cy = (2.0 * y - (n1 - 1)) / max(n1 - 1, 1)
    sk = np.clip(0.6 + 0.3 * (1.0 + g0 * cx + g1 * cy), 0.3, None)
    stars_r = render_gaussian(n0, n1, x, y, f, sr)
    stars_s = render_gaussian(n0, n1, x, y, f * (s0 + sl0 * cx + sl1 * cy),
                              np.hypot(sr, sk))
    c0, c1 = norm_coords(n0, n1)
    scale_pix = s0 + sl0 * c0 + sl1 * c1
    bcoef = rng.uniform(-3.0, 3.0, 6)
    bg = bcoef[0] + (bcoef[1] * c0 + bcoef[2] * c1 if db >= 1 else 0.0) + \
        (bcoef[3] * c0 ** 2 + bcoef[4] * c0 * c1 + bcoef[5] * c1 ** 2 if db >= 2 else 0.0)
    s_true = scale_pix * SKY + stars_s + bg
    r, s = _finish(rng, SKY + stars_r, s_true, noise, dtype)
    return Pair(r, s, w, w, dk, db, const_phot, f"pair {n0}x{n1} w={w} DK={dk} DB={db}")


BATCH_SHAPES = [(512, 512), (1024, 1024), (2048, 2048), (2048, 4096)]


def config4(first_seed=100, count=64, sizes=None):
    """64 pairs with shapes drawn uniformly from BATCH_SHAPES; star density
    2e-3 per pixel, PSF sigma ~ U[1, 2.5]; 11x11 kernel, DK=1, DB=1."""
    rng = rng_for(first_seed)
    shapes = sizes or BATCH_SHAPES
    picks = rng.integers(0, len(shapes), count)
    return [star_pair(first_seed + i, *shapes[p], w=5, dk=1, db=1)
            for i, p in enumerate(picks)]


STREAM_SHAPES = [((2048, 2048), 0.6), ((4096, 4096), 0.3), ((6144, 6144), 0.1)]


def stream_requests(count, seed=7, first_req_seed=1000):
    """Request descriptors for a serving stream: shape drawn 60/30/10 from
    2048^2, 4096^2, 6144^2, kernel half-width 5 or 7 with probability 1/2,
    DK=DB=2. Images are rendered lazily by ``star_pair``."""
    rng = rng_for(seed)
    out = []
    probs = np.array([p for _, p in STREAM_SHAPES])
    for i in range(count):
        shp = STREAM_SHAPES[int(rng.choice(len(STREAM_SHAPES), p=probs))][0]
        w = int(rng.choice([5, 7]))
        out.append({"seed": first_req_seed + i, "shape": shp, "w": w, "dk": 2, "db": 2})
    return out


def poisson_arrivals(count, rate, seed=7):
    """Arrival times (s) of a Poisson stream with the given rate (1/s)."""
    rng = rng_for(seed + 1)
    return np.cumsum(rng.exponential(1.0 / rate, count))


def random_images(seed, n0, n1, dtype=np.float64, mean=0.0, scale=1.0):
    """Plain Gaussian random images (for tiny brute-force checks)."""
    rng = rng_for(seed)
    r = mean + scale * rng.standard_normal((n0, n1))
    s = mean + scale * rng.standard_normal((n0, n1))
    return r.astype(dtype), s.astype(dtype)


CONFIGS = {"c1": config1, "c2": config2, "c3": config3}
