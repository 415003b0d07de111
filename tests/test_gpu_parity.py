"""GPU parity of the HIP path against the FP64 CPU oracle (through the C ABI).

Sizes span several FFT tiles and ragged tails (half-spectrum widths
N1/2 + 1 are odd; row counts are not multiples of the workgroup tiles).
Tolerances:
* FP64 form: lag tables and G within 1e-10 of the largest entry; coefficients
  within 1e-6 relative (normwise) and D within 1e-5 of the sky noise RMS;
* mixed form (FP32 FFTs and products, FP64 assembly / solve / one refinement
  step): the same coefficient and D tolerances after refinement; the FP32
  normal matrix alone within 2e-5 of the largest entry.
"""
import numpy as np
import pytest
import torch

import datagen
import oracle

pytestmark = pytest.mark.gpu

CASES = [
    # n0, n1, w, dk, db, const_phot
    (48, 64, 2, 1, 1, 0),
    (64, 96, 3, 2, 2, 0),
    (96, 48, 2, 2, 1, 1),
    (144, 192, 4, 0, 0, 0),
    # tall images: column transforms with 64, 128 and 192 threads per line
    (1024, 64, 3, 2, 2, 0),
    (2048, 48, 2, 1, 1, 1),
    (3072, 32, 2, 2, 1, 0),
]


def _pair(seed, n0, n1, w, dk, db, cp, noise=10.0):
    p = datagen.star_pair(seed, n0, n1, w=w, dk=dk, db=db, density=0.01, noise=noise,
                          dtype=np.float64, const_phot=cp)
    return p.r, p.s


def _dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


@pytest.fixture(scope="module")
def ctx(sfft):
    c = sfft.Context(0)
    yield c
    c.close()


def _params(sfft, n0, n1, w, dk, db, cp, prec, dtype):
    return sfft.Params(n0, n1, w, w, dk, db, cp, prec, dtype)


@pytest.mark.parametrize("n", [16, 48, 96, 256, 384, 1024, 4096, 6144, 8192])
@pytest.mark.parametrize("cdt", [torch.complex128, torch.complex64])
def test_fft_lines_vs_numpy(ctx, n, cdt):
    rng = np.random.default_rng(n)
    lines = 5
    x = rng.standard_normal((lines, n)) + 1j * rng.standard_normal((lines, n))
    xt = torch.from_numpy(x).to("cuda", cdt)
    ref_f = np.fft.fft(x, axis=-1)
    ref_i = np.fft.ifft(x, axis=-1) * n
    got_f = ctx.fft_lines(xt, -1).cpu().numpy()
    got_i = ctx.fft_lines(xt, +1).cpu().numpy()
    tol = (1e-13 if cdt == torch.complex128 else 2e-6) * np.abs(ref_f).max()
    assert np.abs(got_f - ref_f).max() <= tol
    assert np.abs(got_i - ref_i).max() <= tol


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_lag_tables_and_system(sfft, ctx, case, prec):
    n0, n1, w, dk, db, cp = case
    r, s = _pair(7 + n0, n0, n1, w, dk, db, cp)
    pr = sfft.FP64 if prec == "fp64" else sfft.MIXED
    p = _params(sfft, n0, n1, w, dk, db, cp, pr, sfft.F64)
    tab = ctx.lag_tables(p, _dev(r), _dev(s))
    om = oracle.omega(r, dk, w, w)
    th = oracle.theta(r, s, dk, w, w)
    la = oracle.lam(r, dk, db, w, w)
    cm, ev = oracle.background_blocks(s, db)
    tol = 1e-10 if prec == "fp64" else 2e-5
    for name, got, ref in (("omega", tab["omega"], om), ("theta", tab["theta"], th)):
        g = got.cpu().numpy()
        assert np.abs(g - ref).max() <= tol * np.abs(ref).max(), name
    # background blocks are FP64 in both forms
    assert np.abs(tab["lambda"].cpu().numpy() - la).max() <= 1e-11 * np.abs(la).max()
    assert np.abs(tab["cmat"].cpu().numpy() - cm).max() <= 1e-12 * np.abs(cm).max()
    assert np.abs(tab["evec"].cpu().numpy() - ev).max() <= 1e-11 * np.abs(ev).max()
    G, h = ctx.build_system(p, _dev(r), _dev(s))
    Go, ho = oracle.build_system(r, s, w, w, dk, db, cp)
    Gg = G.cpu().numpy()
    assert np.array_equal(Gg, Gg.T)
    assert np.abs(Gg - Go).max() <= tol * np.abs(Go).max()
    assert np.abs(h.cpu().numpy() - ho).max() <= tol * np.abs(ho).max()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_run_matches_oracle(sfft, ctx, case, prec, dtype):
    n0, n1, w, dk, db, cp = case
    r, s = _pair(11 + n1, n0, n1, w, dk, db, cp)
    if dtype == "f32":
        r = r.astype(np.float32).astype(np.float64)
        s = s.astype(np.float32).astype(np.float64)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    pr = sfft.FP64 if prec == "fp64" else sfft.MIXED
    p = _params(sfft, n0, n1, w, dk, db, cp, pr, sfft.F32 if dtype == "f32" else sfft.F64)
    coef, d = ctx.run(p, _dev(r, tdt), _dev(s, tdt))
    ctx.sync()
    co = oracle.fit(r, s, w, w, dk, db, cp)
    do = oracle.subtract(r, s, co, w, w, dk, db, cp)
    c = coef.cpu().numpy()
    nk = len(c) - oracle.nterms(db)
    assert _rel(c[:nk], co[:nk]) <= 1e-6
    assert _rel(c[nk:], co[nk:]) <= 1e-6
    rms = float(np.sqrt(np.mean((d.cpu().numpy().astype(np.float64) - do) ** 2)))
    # FP32 output images carry their own rounding of |D| ~ noise level
    floor = 0.0 if dtype == "f64" else 6e-8 * np.abs(do).max()
    assert rms <= 1e-5 * 10.0 + floor


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_separate_calls_match_run(sfft, ctx, prec):
    n0, n1, w, dk, db, cp = 64, 96, 3, 2, 2, 0
    r, s = _pair(5, n0, n1, w, dk, db, cp)
    pr = sfft.FP64 if prec == "fp64" else sfft.MIXED
    p = _params(sfft, n0, n1, w, dk, db, cp, pr, sfft.F64)
    R, S = _dev(r), _dev(s)
    G, h = ctx.build_system(p, R, S)
    coef = ctx.solve(p, G, h, R, S)
    d = ctx.subtract(p, R, S, coef)
    coef2, d2 = ctx.run(p, R, S)
    ctx.sync()
    # the build and solve are the same kernels on the same inputs
    assert torch.equal(coef, coef2)
    # sfft_subtract transforms the apply pair as given, sfft_run reuses the
    # pedestal-free transforms of the fit pair: equal up to rounding
    rms = float(torch.sqrt(torch.mean((d - d2) ** 2)))
    assert rms <= (1e-10 if prec == "fp64" else 1e-5) * 10.0


def test_apply_pair_differs_from_fit_pair(sfft, ctx):
    """Fit on masked images, apply to the unmasked ones (Sec. 3)."""
    n0, n1, w, dk, db = 64, 64, 2, 1, 1
    r, s = _pair(21, n0, n1, w, dk, db, 0)
    rm, sm = r.copy(), s.copy()
    rm[10:20, 30:40] = 0.0
    sm[10:20, 30:40] = 0.0
    p = _params(sfft, n0, n1, w, dk, db, 0, sfft.FP64, sfft.F64)
    coef, d = ctx.run(p, _dev(rm), _dev(sm), _dev(r), _dev(s))
    ctx.sync()
    co = oracle.fit(rm, sm, w, w, dk, db)
    do = oracle.subtract(r, s, co, w, w, dk, db)
    assert _rel(coef.cpu().numpy(), co) <= 1e-6
    assert np.sqrt(np.mean((d.cpu().numpy() - do) ** 2)) <= 1e-4


def test_config1_full(sfft, ctx):
    """256 x 256 FP64 pair, 11 x 11 kernel, DK = DB = 0 (both forms)."""
    pair = datagen.config1()
    co = oracle.fit(pair.r, pair.s, 5, 5, 0, 0)
    do = oracle.subtract(pair.r, pair.s, co, 5, 5, 0, 0)
    for pr in (sfft.FP64, sfft.MIXED):
        p = sfft.Params(256, 256, 5, 5, 0, 0, 0, pr, sfft.F64)
        coef, d = ctx.run(p, _dev(pair.r), _dev(pair.s))
        ctx.sync()
        assert _rel(coef.cpu().numpy(), co) <= 1e-6
        assert np.sqrt(np.mean((d.cpu().numpy() - do) ** 2)) <= 1e-4


def test_not_spd_and_nonfinite_are_reported(sfft, ctx):
    p = sfft.Params(32, 32, 1, 1, 0, 0, 0, sfft.FP64, sfft.F64)
    z = torch.zeros((32, 32), dtype=torch.float64, device="cuda")
    o = torch.ones((32, 32), dtype=torch.float64, device="cuda")
    ctx.run(p, z, o)
    with pytest.raises(sfft.SfftError) as ei:
        ctx.sync()
    assert ei.value.code == sfft.E_NOT_SPD
    bad = o.clone()
    bad[3, 4] = float("nan")
    ctx.run(p, bad, o)
    with pytest.raises(sfft.SfftError) as ei:
        ctx.sync()
    assert ei.value.code == sfft.E_NONFINITE
    ctx.sync()   # flags were cleared by the report
