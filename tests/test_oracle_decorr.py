"""Pins of the noise-decorrelation oracle (App. C, Eq. C21-C24), on the CPU.

The oracle computes Q^ = sqrt(den(0) / den(p)) and D (x) Q with numpy's FFT.
It is checked here against things other than its own formula:
  * the claim of App. C itself -- the decorrelated noise is white -- by the
    exact covariance of D (x) Q summed pixel by pixel from direct circular
    convolutions of the kernels (no FFT), for co-adds of several images;
  * the closed form of that white level, den(0), from kernel sums alone;
  * special cases that reduce to the identity (a delta or a pure shift as the
    matching kernel with equal noise);
  * a Monte Carlo whitening test on rendered white noise;
  * the kernel at one position against the oracle's kernel-sum field.
"""
import numpy as np
import pytest

import oracle
from oracle import decorr


def _conv_direct(a, b):
    """Circular convolution (a (x) b)(x) = sum_y a(y) b(x - y), by loops over
    the nonzero entries of a."""
    n0, n1 = b.shape
    out = np.zeros((n0, n1))
    for y0, y1 in zip(*np.nonzero(a)):
        out += a[y0, y1] * np.roll(np.roll(b, y0, axis=0), y1, axis=1)
    return out


def _autocov(f):
    """sum_x f(x) f(x + tau) for every lag tau (direct sums)."""
    n0, n1 = f.shape
    c = np.zeros((n0, n1))
    for t0 in range(n0):
        for t1 in range(n1):
            c[t0, t1] = np.sum(f * np.roll(np.roll(f, -t0, axis=0), -t1, axis=1))
    return c


def _random_stamp(rng, w0, w1):
    st = rng.uniform(0.0, 1.0, (2 * w0 + 1, 2 * w1 + 1))
    return st / st.sum() * rng.uniform(0.7, 1.3)


@pytest.mark.parametrize("m,n", [(1, 1), (2, 3)])
def test_decorrelated_noise_is_white_exactly(m, n):
    rng = np.random.default_rng(5 + m + n)
    n0, n1, w0, w1 = 14, 12, 2, 1
    K = _random_stamp(rng, w0, w1)
    G = [_random_stamp(rng, w0, w1) for _ in range(m)]
    H = [_random_stamp(rng, w0, w1) for _ in range(n)]
    ss = rng.uniform(5, 15, m)
    sr = rng.uniform(5, 15, n)
    q = decorr.decorrelation_spectrum(K, n0, n1, ss, G, sr, H)
    Q = np.real(np.fft.ifft2(q))
    grid = lambda st: decorr.stamp_on_grid(st, n0, n1)  # noqa: E731
    cov = np.zeros((n0, n1))
    for sj, gj in zip(ss, G):
        cov += sj * sj * _autocov(_conv_direct(grid(gj), Q))
    for si, hi in zip(sr, H):
        cov += si * si * _autocov(_conv_direct(grid(hi), _conv_direct(grid(K), Q)))
    # white: no covariance at any nonzero lag
    off = cov.copy()
    off[0, 0] = 0.0
    assert np.abs(off).max() <= 1e-12 * cov[0, 0]
    # the white level is den(0), from kernel sums alone
    den0 = sum(sj * sj * gj.sum() ** 2 for sj, gj in zip(ss, G)) + \
        K.sum() ** 2 * sum(si * si * hi.sum() ** 2 for si, hi in zip(sr, H))
    assert cov[0, 0] == pytest.approx(den0, rel=1e-12)
    # without decorrelation the same noise is strongly correlated
    raw = np.zeros((n0, n1))
    for sj, gj in zip(ss, G):
        raw += sj * sj * _autocov(grid(gj))
    for si, hi in zip(sr, H):
        raw += si * si * _autocov(_conv_direct(grid(hi), grid(K)))
    raw0 = raw[0, 0]
    raw[0, 0] = 0.0
    assert np.abs(raw).max() > 0.02 * raw0


def test_unit_kernel_sum_and_symmetry():
    rng = np.random.default_rng(2)
    n0, n1 = 32, 24
    K = _random_stamp(rng, 3, 3)
    q = decorr.decorrelation_spectrum(K, n0, n1, [10.0], [decorr.delta_stamp(3, 3)], [6.0],
                                      [decorr.delta_stamp(3, 3)])
    Q = np.fft.ifft2(q)
    assert np.abs(Q.imag).max() < 1e-14
    assert Q.real.sum() == pytest.approx(1.0, abs=1e-13)
    Qr = Q.real
    Qm = np.roll(np.roll(Qr[::-1, ::-1], 1, axis=0), 1, axis=1)   # Q(-x)
    assert np.abs(Qr - Qm).max() < 1e-14


@pytest.mark.parametrize("kernel", ["delta", "shift", "scaled_shift"])
def test_identity_cases(kernel):
    rng = np.random.default_rng(3)
    n0, n1, w = 20, 18, 2
    D = rng.normal(0, 10, (n0, n1))
    K = np.zeros((2 * w + 1, 2 * w + 1))
    c = 1.0
    if kernel == "delta":
        K[w, w] = 1.0
    elif kernel == "shift":
        K[w + 1, w - 2] = 1.0
    else:
        c = 0.8
        K[w - 1, w + 2] = c
    # equal white levels at every frequency: sigma_S^2 + c^2 sigma_R^2 constant
    out = decorr.decorrelate(D, K, [7.0], [decorr.delta_stamp(w, w)], [4.0],
                             [decorr.delta_stamp(w, w)])
    assert np.abs(out - D).max() <= 1e-12 * np.abs(D).max()


def test_monte_carlo_whitening():
    rng = np.random.default_rng(11)
    n0 = n1 = 192
    w = 4
    y, x = np.mgrid[-w:w + 1, -w:w + 1]
    K = np.exp(-(x * x + y * y) / (2 * 1.6 ** 2))
    K *= 0.9 / K.sum()
    ss, sr = 2.0, 12.0
    S = rng.normal(0, ss, (n0, n1))
    R = rng.normal(0, sr, (n0, n1))
    D = S - _conv_direct(decorr.stamp_on_grid(K, n0, n1), R)
    out = decorr.decorrelate(D, K, [ss], [decorr.delta_stamp(w, w)], [sr],
                             [decorr.delta_stamp(w, w)])

    def rho(img, t0, t1):
        a = img - img.mean()
        return float(np.mean(a * np.roll(np.roll(a, t0, 0), t1, 1)) / np.mean(a * a))

    bound = 5.0 / np.sqrt(n0 * n1)
    assert abs(rho(D, 1, 0)) > 10 * bound      # correlated before
    for t in ((1, 0), (0, 1), (1, 1), (2, 0), (0, 3)):
        assert abs(rho(out, *t)) < bound, t   # white after


def test_kernel_at_matches_the_kernel_sum_field():
    rng = np.random.default_rng(4)
    n0, n1, w0, w1, dk = 24, 20, 2, 3, 2
    nu = oracle.num_unknowns(w0, w1, dk, 1)
    coef = rng.normal(0, 1, nu)
    st = oracle.stamps(coef, w0, w1, dk)
    field = oracle.kernel_sum_field(coef, n0, n1, w0, w1, dk)
    c0, c1 = oracle.coords(n0, n1)
    for x, y in ((0, 0), (5, 17), (23, 3), (12, 10)):
        assert decorr.kernel_at(st, dk, c0[x], c1[y]).sum() == pytest.approx(field[x, y], rel=1e-12)
