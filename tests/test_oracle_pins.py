"""Pins of the FP64 oracle against things other than itself.

Each check targets a different plausible mistake:
* explicit design matrix built with ``numpy.roll`` (assembly case logic of
  Eq. B5-B16, offsets, unknown order);
* exact recovery of kernels injected with an FFT circular convolution
  (shift orientation, weights at the source pixel, background terms);
* the Fourier-space model of Eq. 13-14 with the closed-form basis DFT
  (sign of W, a = N0 N1 a-ring);
* correlation-theorem forms of the lag tables (what the GPU path computes);
* symmetry / positive definiteness / stationarity (Eq. 16-17);
* invariance of D under the coordinate convention;
* the unknown counts quoted for the workloads.
"""
import numpy as np
import pytest

import datagen
import oracle
from oracle import brute

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def fft_circular_conv(img, stamp):
    """Circular convolution out(x) = sum_a stamp(a) img(x - a), stamp centred."""
    n0, n1 = img.shape
    L0, L1 = stamp.shape
    w0, w1 = L0 // 2, L1 // 2
    k = np.zeros((n0, n1))
    for a in range(-w0, w0 + 1):
        for b in range(-w1, w1 + 1):
            k[a % n0, b % n1] += stamp[a + w0, b + w1]
    return np.real(np.fft.ifft2(np.fft.fft2(img) * np.fft.fft2(k)))


def coef_from_stamps(stamps, bcoef, const_phot=0):
    """Delta-basis coefficients of given stamps: off-centre entries are the
    stamp values, the centre entry is the stamp sum (Eq. 3-4)."""
    P, L0, L1 = stamps.shape
    w0, w1 = L0 // 2, L1 // 2
    out = []
    for k in range(P):
        for a in range(-w0, w0 + 1):
            for b in range(-w1, w1 + 1):
                if a == 0 and b == 0:
                    if const_phot and k > 0:
                        assert abs(stamps[k].sum()) < 1e-12
                        continue
                    out.append(stamps[k].sum())
                else:
                    out.append(stamps[k, a + w0, b + w1])
    return np.array(list(out) + list(bcoef))


PARAMS = [(1, 1, 1, 1, 0), (1, 2, 2, 1, 1), (2, 1, 0, 0, 0), (1, 1, 2, 2, 0), (2, 2, 1, 2, 1)]
# the largest polynomial degrees the library accepts (DK, DB up to 4), DB > DK
PARAMS_HIGH = [(1, 1, 4, 3, 0), (1, 1, 3, 4, 1), (1, 1, 0, 4, 0)]


@pytest.mark.parametrize("w0,w1,dk,db,cp", PARAMS + PARAMS_HIGH)
def test_assembly_matches_explicit_design_matrix(w0, w1, dk, db, cp):
    r, s = datagen.random_images(11, 9, 11, mean=3.0)
    G, h = oracle.build_system(r, s, w0, w1, dk, db, cp)
    Gb, hb = brute.normal_equations(r, s, w0, w1, dk, db, cp)
    assert G.shape == Gb.shape
    assert np.abs(G - Gb).max() <= 1e-12 * np.abs(Gb).max()
    assert np.abs(h - hb).max() <= 1e-12 * np.abs(hb).max()


@pytest.mark.parametrize("w0,w1,dk,db,cp", PARAMS)
def test_solution_matches_lstsq(w0, w1, dk, db, cp):
    r, s = datagen.random_images(12, 10, 9, mean=2.0)
    c = oracle.fit(r, s, w0, w1, dk, db, cp)
    cb = brute.lstsq(r, s, w0, w1, dk, db, cp)
    assert np.abs(c - cb).max() <= 1e-9 * np.abs(cb).max()
    d = oracle.subtract(r, s, c, w0, w1, dk, db, cp)
    assert np.abs(d - brute.difference(r, s, c, w0, w1, dk, db, cp)).max() < 1e-10


def test_exact_recovery_invariant_kernel():
    """DK=0, DB=0: S = kernel * R + b, built with an FFT convolution."""
    rng = np.random.default_rng(3)
    r = datagen.star_pair(31, 24, 28, w=2, dk=0, db=0, density=0.05, noise=0.0,
                          dtype=np.float64).r
    stamp = rng.uniform(-0.2, 1.0, (5, 5))
    s = fft_circular_conv(r, stamp) + 7.25
    c = oracle.fit(r, s, 2, 2, 0, 0)
    expect = coef_from_stamps(stamp[None], [7.25])
    assert np.abs(c - expect).max() <= 1e-9 * np.abs(expect).max()
    d = oracle.subtract(r, s, c, 2, 2, 0, 0)
    assert np.abs(d).max() <= 1e-9 * np.abs(s).max()
    kap = oracle.stamps(c, 2, 2, 0)
    # normal equations square the design matrix's condition number
    assert np.abs(kap[0] - stamp).max() < 1e-7


def test_gaussian_kernel_recovery():
    """A plain Gaussian matching kernel scaled by 0.9 is recovered exactly."""
    # a white-noise reference keeps the delta-basis system well conditioned
    r = datagen.random_images(32, 40, 36, mean=3.0)[0]
    g = np.exp(-(np.arange(-3, 4)[:, None] ** 2 + np.arange(-3, 4)[None, :] ** 2) / (2 * 1.2 ** 2))
    g = 0.9 * g / g.sum()
    s = fft_circular_conv(r, g) + 5.0
    c = oracle.fit(r, s, 3, 3, 0, 0)
    kap = oracle.stamps(c, 3, 3, 0)
    assert abs(c[3 * 7 + 3] - 0.9) < 1e-10          # kernel sum = a_00 (Eq. 3-4)
    assert np.abs(kap[0] - g).max() < 1e-10
    assert abs(c[-1] - 5.0) < 1e-8


@pytest.mark.parametrize("dk,db,cp", [(1, 1, 0), (2, 2, 0), (2, 1, 1), (3, 4, 0), (4, 2, 1)])
def test_exact_recovery_varying_kernel(dk, db, cp):
    """S = sum_k (c0^i c1^j R) conv kappa_k + sum_m b_m c0^p c1^q: weights at
    the source pixel (Eq. 11-12). Recovered to rounding."""
    rng = np.random.default_rng(40 + dk + db)
    n0, n1, w = 26, 30, 2
    if dk <= 2:
        r = datagen.star_pair(33, n0, n1, w=w, dk=dk, db=db, density=0.04, noise=0.0,
                              dtype=np.float64).r
    else:
        # at degrees 3-4 a sparse star field on a flat sky leaves the kernel
        # sums' polynomial nearly collinear with the background's; a
        # white-noise reference keeps the system well conditioned
        r = datagen.random_images(34 + dk, n0, n1, mean=3.0)[0]
    c0 = (2.0 * np.arange(n0) - (n0 - 1)) / (n0 - 1)
    c1 = (2.0 * np.arange(n1) - (n1 - 1)) / (n1 - 1)
    P = oracle.nterms(dk)
    stamps = rng.normal(0, 0.3, (P, 5, 5))
    stamps[0] += 0.5
    if cp:
        for k in range(1, P):
            stamps[k, 2, 2] -= stamps[k].sum()
    bcoef = rng.normal(0, 2.0, oracle.nterms(db))
    s = np.zeros((n0, n1))
    for k, (i, j) in enumerate(oracle.terms(dk)):
        s += fft_circular_conv(c0[:, None] ** i * c1[None, :] ** j * r, stamps[k])
    for m, (p, q) in enumerate(oracle.terms(db)):
        s += bcoef[m] * c0[:, None] ** p * c1[None, :] ** q
    c = oracle.fit(r, s, w, w, dk, db, cp)
    expect = coef_from_stamps(stamps, bcoef, cp)
    assert np.abs(c - expect).max() <= 1e-8 * np.abs(expect).max()
    assert np.abs(oracle.subtract(r, s, c, w, w, dk, db, cp)).max() < 1e-8 * np.abs(s).max()


def test_fourier_model_eq13_eq14():
    """D from the oracle equals the inverse DFT of Eq. 13 built with the
    closed-form basis DFT of Eq. 14 and a = N0 N1 a-ring."""
    n0, n1, w0, w1, dk, db = 12, 10, 1, 2, 1, 1
    r, s = datagen.random_images(21, n0, n1, mean=4.0)
    rng = np.random.default_rng(5)
    nu = oracle.num_unknowns(w0, w1, dk, db)
    coef = rng.normal(0, 0.5, nu)
    d = oracle.subtract(r, s, coef, w0, w1, dk, db)
    N = n0 * n1
    W0 = np.exp(-2j * np.pi / n0)
    W1 = np.exp(-2j * np.pi / n1)
    l = np.arange(n0)[:, None]
    m = np.arange(n1)[None, :]
    c0 = (2.0 * np.arange(n0) - (n0 - 1)) / (n0 - 1)
    c1 = (2.0 * np.arange(n1) - (n1 - 1)) / (n1 - 1)
    Dhat = np.fft.fft2(s).astype(complex)
    u = 0
    for (i, j) in oracle.terms(dk):
        Rh = np.fft.fft2(c0[:, None] ** i * c1[None, :] ** j * r)
        for a in range(-w0, w0 + 1):
            for b in range(-w1, w1 + 1):
                Kh = (W0 ** (l * a) * W1 ** (m * b) - 1.0) / N if (a or b) else np.full((n0, n1), 1.0 / N)
                Dhat -= N * coef[u] * Rh * Kh
                u += 1
    for (p, q) in oracle.terms(db):
        Dhat -= coef[u] * np.fft.fft2(c0[:, None] ** p * c1[None, :] ** q * np.ones((n0, n1)))
        u += 1
    assert np.abs(np.real(np.fft.ifft2(Dhat)) - d).max() < 1e-10


def test_lag_tables_correlation_theorem():
    """Omega, Theta, Lambda equal (1/n) Re IDFT of the spectral products that
    the GPU path forms: conj(R^kb) R^k, conj(R^kb) S, conj(R^kb) T^m."""
    n0, n1, w0, w1, dk, db = 14, 12, 1, 2, 2, 1
    r, s = datagen.random_images(22, n0, n1, mean=1.0)
    c0 = (2.0 * np.arange(n0) - (n0 - 1)) / (n0 - 1)
    c1 = (2.0 * np.arange(n1) - (n1 - 1)) / (n1 - 1)
    spec = [np.fft.fft2(c0[:, None] ** i * c1[None, :] ** j * r) for (i, j) in oracle.terms(dk)]
    tsp = [np.fft.fft2(c0[:, None] ** p * c1[None, :] ** q * np.ones((n0, n1)))
           for (p, q) in oracle.terms(db)]
    om = oracle.omega(r, dk, w0, w1)
    th = oracle.theta(r, s, dk, w0, w1)
    la = oracle.lam(r, dk, db, w0, w1)
    P = len(spec)
    pr = 0
    for kb in range(P):
        for k in range(kb, P):
            cc = np.real(np.fft.ifft2(np.conj(spec[kb]) * spec[k]))
            for d0 in range(-2 * w0, 2 * w0 + 1):
                for d1 in range(-2 * w1, 2 * w1 + 1):
                    assert abs(om[pr, d0 + 2 * w0, d1 + 2 * w1] - cc[d0 % n0, d1 % n1]) < 1e-10
            pr += 1
        ct = np.real(np.fft.ifft2(np.conj(spec[kb]) * np.fft.fft2(s)))
        for m_, t in enumerate(tsp):
            cl = np.real(np.fft.ifft2(np.conj(spec[kb]) * t))
            for d0 in range(-w0, w0 + 1):
                for d1 in range(-w1, w1 + 1):
                    assert abs(la[kb, m_, d0 + w0, d1 + w1] - cl[d0 % n0, d1 % n1]) < 1e-10
        for d0 in range(-w0, w0 + 1):
            for d1 in range(-w1, w1 + 1):
                assert abs(th[kb, d0 + w0, d1 + w1] - ct[d0 % n0, d1 % n1]) < 1e-10


def test_symmetry_spd_and_cholesky():
    p = datagen.star_pair(34, 48, 40, w=3, dk=2, db=2, noise=10.0, dtype=np.float64)
    G, h = oracle.build_system(p.r, p.s, 3, 3, 2, 2)
    assert np.abs(G - G.T).max() <= 1e-13 * np.abs(G).max()
    assert np.linalg.eigvalsh(0.5 * (G + G.T)).min() > 0
    c = oracle.solve(G, h)
    ref = np.linalg.solve(G, h)
    assert np.linalg.norm(c - ref) <= 1e-7 * np.linalg.norm(ref)


def test_stationarity_at_optimum():
    """Eq. 16-17: the gradient of the objective vanishes at the solution."""
    p = datagen.star_pair(35, 20, 22, w=2, dk=1, db=1, noise=10.0, dtype=np.float64)
    c = oracle.fit(p.r, p.s, 2, 2, 1, 1)
    phi = brute.design_matrix(p.r, 2, 2, 1, 1)
    resid = p.s.ravel() - phi @ c
    g = phi.T @ resid
    assert np.abs(g).max() <= 1e-8 * np.abs(phi).max() * np.abs(p.s).max() * p.s.size ** 0.5


def test_coordinate_convention_leaves_d_unchanged():
    """Raw pixel coordinates (as printed in Eq. 2, 6) span the same model: D
    is the same as with the centred coordinates the oracle uses."""
    p = datagen.star_pair(36, 14, 16, w=1, dk=1, db=1, noise=5.0, dtype=np.float64)
    c = oracle.fit(p.r, p.s, 1, 1, 1, 1)
    d = oracle.subtract(p.r, p.s, c, 1, 1, 1, 1)
    n0, n1 = p.r.shape
    x = np.arange(n0, dtype=float)[:, None]
    y = np.arange(n1, dtype=float)[None, :]
    cols = []
    for (i, j) in oracle.terms(1):
        rk = x ** i * y ** j * p.r
        for a in range(-1, 2):
            for b in range(-1, 2):
                col = np.roll(rk, (a, b), axis=(0, 1))
                cols.append((col - rk if (a or b) else col).ravel())
    for (pp, q) in oracle.terms(1):
        cols.append((x ** pp * y ** q * np.ones_like(p.r)).ravel())
    phi = np.stack(cols, 1)
    craw, *_ = np.linalg.lstsq(phi, p.s.ravel(), rcond=None)
    draw = p.s - (phi @ craw).reshape(p.s.shape)
    assert np.abs(draw - d).max() < 1e-7 * np.abs(p.s).max()


def test_single_entry_route_matches_table_route():
    p = datagen.star_pair(37, 40, 36, w=3, dk=2, db=2, noise=10.0, dtype=np.float64)
    G, _ = oracle.build_system(p.r, p.s, 3, 3, 2, 2)
    rng = np.random.default_rng(1)
    n = G.shape[0]
    for u, v in list(rng.integers(0, n, (12, 2))) + [(0, 0), (n - 1, 0), (24, n - 2), (n - 1, n - 1)]:
        e = oracle.g_entry(p.r, 3, 3, 2, 2, 0, int(u), int(v))
        assert abs(e - G[u, v]) <= 1e-11 * np.abs(G).max()


def test_not_spd_is_reported():
    r = np.zeros((16, 16))
    s = np.ones((16, 16))
    with pytest.raises(np.linalg.LinAlgError):
        oracle.fit(r, s, 1, 1, 0, 0)


def test_unknown_counts_for_workloads():
    assert oracle.num_unknowns(5, 5, 0, 0) == 122
    assert oracle.num_unknowns(5, 5, 2, 2) == 732
    assert oracle.num_unknowns(7, 7, 2, 2) == 1356
    assert oracle.num_unknowns(5, 5, 1, 1) == 366
    assert oracle.num_unknowns(7, 7, 2, 2, 1) == 1356 - 5


def test_pixel_route_and_kernel_sum_field():
    p = datagen.star_pair(38, 30, 26, w=2, dk=2, db=1, noise=10.0, dtype=np.float64)
    c = oracle.fit(p.r, p.s, 2, 2, 2, 1)
    d = oracle.subtract(p.r, p.s, c, 2, 2, 2, 1)
    pix = [(0, 0), (29, 25), (3, 24), (15, 1), (7, 13)]
    dp = oracle.subtract_pixels(p.r, p.s, c, 2, 2, 2, 1, 0, pix)
    assert np.abs(dp - np.array([d[a, b] for a, b in pix])).max() < 1e-11
    ks = oracle.kernel_sum_field(c, 30, 26, 2, 2, 2)
    kap = oracle.stamps(c, 2, 2, 2)
    c0 = (2.0 * np.arange(30) - 29) / 29
    c1 = (2.0 * np.arange(26) - 25) / 25
    ref = sum(kap[k].sum() * c0[:, None] ** i * c1[None, :] ** j for k, (i, j) in enumerate(oracle.terms(2)))
    assert np.abs(ks - ref).max() < 1e-12


def test_phi_dot_is_a_column_of_phi_transpose():
    p = datagen.star_pair(39, 18, 20, w=2, dk=2, db=1, noise=10.0, dtype=np.float64)
    phi = brute.design_matrix(p.r, 2, 2, 2, 1, 1)
    img = np.random.default_rng(4).normal(size=p.r.shape)
    ref = phi.T @ img.ravel()
    for u in [0, 5, 24, 25, 40, phi.shape[1] - 3, phi.shape[1] - 1]:
        assert abs(oracle.phi_dot(p.r, img, 2, 2, 2, 1, 1, u) - ref[u]) < 1e-10 * np.abs(ref).max()
