"""GPU parity of the HIP path against the FP64 CPU oracle (through the C ABI).

Sizes span several FFT tiles and ragged tails (half-spectrum widths
N1/2 + 1 are odd; row counts are not multiples of the workgroup tiles).
Tolerances:
* FP64 form: lag tables and G within 1e-10 of the largest entry; coefficients
  within 1e-6 relative (normwise) and D within 1e-5 of the sky noise RMS;
* mixed form (FP32 FFTs and products, FP64 assembly / solve / one refinement
  step): the same coefficient and D tolerances after refinement; the FP32
  normal matrix alone within 2e-5 of the largest entry. The mixed form takes
  FP32 images and DK <= 3; other parameter sets must be refused with
  SFFT_E_UNSUPPORTED (checked here).
"""
import numpy as np
import pytest
import torch

import datagen
import oracle

pytestmark = pytest.mark.gpu

CASES = [
    # n0, n1, w0, w1, dk, db, const_phot
    (48, 64, 2, 2, 1, 1, 0),
    (64, 96, 3, 3, 2, 2, 0),
    (96, 48, 2, 2, 2, 1, 1),
    (144, 192, 4, 4, 0, 0, 0),
    # tall images: column transforms with 64, 128 and 192 threads per line
    (1024, 64, 3, 3, 2, 2, 0),
    (2048, 48, 2, 2, 1, 1, 1),
    (3072, 48, 2, 2, 2, 1, 0),
    (3072, 32, 2, 2, 2, 1, 0),    # (mixed form refused: 32 columns)
    # the rest of the parameter space the library accepts:
    # w0 != w1 (Eq. 3-4 allow independent half widths), DB > DK
    (64, 96, 2, 4, 1, 2, 0),
    (96, 64, 5, 1, 0, 3, 0),
    # half widths without a specialised stencil (1, 6, 9, 16), DK = 3, 4 (the
    # DK = DB = 4 case on 96^2 pixels: 2536 unknowns need a well-determined fit)
    (48, 48, 1, 1, 3, 1, 0),
    (96, 96, 6, 6, 4, 4, 1),
    # w0 >= 8 with N0 a multiple of 1024: the pruned lag pass with three and
    # five 16-lag blocks
    (1024, 48, 9, 2, 1, 1, 0),
    (2048, 64, 16, 8, 0, 0, 0),
    # largest and smallest line lengths
    (8192, 48, 2, 2, 1, 0, 0),
    (48, 8192, 3, 2, 1, 1, 0),
    (16, 16, 1, 3, 0, 0, 0),
    # lengths with factors other than 2 and 3 (Bluestein lines): 46 = 2 23,
    # 62 = 2 31, 94 = 2 47, 50 = 2 5^2, 110 = 2 5 11, 2046 = 2 3 11 31
    (46, 62, 2, 2, 1, 1, 0),
    (94, 50, 3, 3, 2, 2, 0),
    (110, 96, 4, 2, 2, 1, 1),
    (2046, 34, 9, 2, 1, 1, 0),    # (mixed form refused: 34 columns)
    (2046, 62, 9, 2, 1, 1, 0),
]


def _pair(seed, n0, n1, w, dk, db, cp, noise=10.0):
    p = datagen.star_pair(seed, n0, n1, w=w, dk=dk, db=db, density=0.01, noise=noise,
                          dtype=np.float64, const_phot=cp)
    return p.r, p.s


def _f32_floor(d_ref):
    """RMS of the FP32 output's own rounding: at most 2^-24 |D| per pixel."""
    return 2.0 ** -24 * float(np.sqrt(np.mean(d_ref ** 2)))


def _dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


@pytest.fixture(scope="module")
def ctx(sfft):
    c = sfft.Context(0)
    yield c
    c.close()


def _params(sfft, n0, n1, w0, w1, dk, db, cp, prec, dtype):
    return sfft.Params(n0, n1, w0, w1, dk, db, cp, prec, dtype)


def _mixed_refused(sfft, prec, dtype, dk, n0=64, n1=64):
    """The parameter sets the mixed form refuses (FP64 images, DK = 4, a side
    under 48 pixels)."""
    return prec == "mixed" and (dtype == "f64" or dk > 3 or min(n0, n1) < 48)


def _assert_refused(sfft, ctx, p, R, S):
    assert sfft.Context.check(p) == sfft.E_UNSUPPORTED
    with pytest.raises(sfft.SfftError) as ei:
        ctx.run(p, R, S)
    assert ei.value.code == sfft.E_UNSUPPORTED


@pytest.mark.parametrize("n", [16, 48, 96, 256, 384, 1024, 4096, 6144, 8192,
                               # Bluestein lines (lengths with factors other than 2, 3)
                               18, 46, 62, 100, 1000, 2046, 4094, 4095])
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
    n0, n1, w0, w1, dk, db, cp = case
    r, s = _pair(7 + n0, n0, n1, w0, dk, db, cp)
    pr = sfft.FP64 if prec == "fp64" else sfft.MIXED
    # the mixed form transforms FP32 images
    dt = sfft.F64 if prec == "fp64" else sfft.F32
    if prec == "mixed":
        r = r.astype(np.float32).astype(np.float64)
        s = s.astype(np.float32).astype(np.float64)
    tdt = torch.float64 if prec == "fp64" else torch.float32
    p = _params(sfft, n0, n1, w0, w1, dk, db, cp, pr, dt)
    if _mixed_refused(sfft, prec, "f32", dk, n0, n1):
        _assert_refused(sfft, ctx, p, _dev(r, tdt), _dev(s, tdt))
        return
    tab = ctx.lag_tables(p, _dev(r, tdt), _dev(s, tdt))
    om = oracle.omega(r, dk, w0, w1)
    th = oracle.theta(r, s, dk, w0, w1)
    la = oracle.lam(r, dk, db, w0, w1)
    cm, ev = oracle.background_blocks(s, db)
    tol = 1e-10 if prec == "fp64" else 2e-5
    for name, got, ref in (("omega", tab["omega"], om), ("theta", tab["theta"], th)):
        g = got.cpu().numpy()
        assert np.abs(g - ref).max() <= tol * np.abs(ref).max(), name
    # background blocks are FP64 in both forms
    assert np.abs(tab["lambda"].cpu().numpy() - la).max() <= 1e-11 * np.abs(la).max()
    assert np.abs(tab["cmat"].cpu().numpy() - cm).max() <= 1e-12 * np.abs(cm).max()
    assert np.abs(tab["evec"].cpu().numpy() - ev).max() <= 1e-11 * np.abs(ev).max()
    G, h = ctx.build_system(p, _dev(r, tdt), _dev(s, tdt))
    Go, ho = oracle.build_system(r, s, w0, w1, dk, db, cp)
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
    n0, n1, w0, w1, dk, db, cp = case
    r, s = _pair(11 + n1, n0, n1, w0, dk, db, cp)
    if dtype == "f32":
        r = r.astype(np.float32).astype(np.float64)
        s = s.astype(np.float32).astype(np.float64)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    pr = sfft.FP64 if prec == "fp64" else sfft.MIXED
    p = _params(sfft, n0, n1, w0, w1, dk, db, cp, pr, sfft.F32 if dtype == "f32" else sfft.F64)
    if _mixed_refused(sfft, prec, dtype, dk, n0, n1):
        _assert_refused(sfft, ctx, p, _dev(r, tdt), _dev(s, tdt))
        return
    coef, d = ctx.run(p, _dev(r, tdt), _dev(s, tdt))
    ctx.sync()
    co = oracle.fit(r, s, w0, w1, dk, db, cp)
    do = oracle.subtract(r, s, co, w0, w1, dk, db, cp)
    c = coef.cpu().numpy()
    nk = len(c) - oracle.nterms(db)
    ek, eb = _rel(c[:nk], co[:nk]), _rel(c[nk:], co[nk:])
    rms = float(np.sqrt(np.mean((d.cpu().numpy().astype(np.float64) - do) ** 2)))
    print(f"case={case} prec={prec} dtype={dtype} coef_kernel={ek:.2e} coef_bg={eb:.2e} "
          f"d_rms={rms:.2e}")
    assert ek <= 1e-6
    assert eb <= 1e-6
    floor = 0.0 if dtype == "f64" else _f32_floor(do)
    assert rms <= 1e-5 * 10.0 + floor


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_separate_calls_match_run(sfft, ctx, prec):
    n0, n1, w, dk, db, cp = 64, 96, 3, 2, 2, 0
    r, s = _pair(5, n0, n1, w, dk, db, cp)
    pr = sfft.FP64 if prec == "fp64" else sfft.MIXED
    dt, tdt = (sfft.F64, torch.float64) if prec == "fp64" else (sfft.F32, torch.float32)
    p = _params(sfft, n0, n1, w, w, dk, db, cp, pr, dt)
    R, S = _dev(r, tdt), _dev(s, tdt)
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


@pytest.mark.parametrize("prec,dtype", [("fp64", "f64"), ("fp64", "f32"), ("mixed", "f32")])
def test_unaligned_caller_images_match_aligned(sfft, ctx, prec, dtype):
    """Row passes read 16-byte aligned image rows with vector loads and fall
    back to element loads otherwise: images that start one element past a
    16-byte boundary must give the same bits as aligned copies."""
    n0, n1, w, dk, db = 96, 128, 3, 2, 2
    r, s = _pair(11, n0, n1, w, dk, db, 0)
    pr = sfft.FP64 if prec == "fp64" else sfft.MIXED
    dt, tdt = (sfft.F64, torch.float64) if dtype == "f64" else (sfft.F32, torch.float32)
    p = _params(sfft, n0, n1, w, w, dk, db, 0, pr, dt)
    R, S = _dev(r, tdt), _dev(s, tdt)
    coef, d = ctx.run(p, R, S)
    ctx.sync()
    flat_r = torch.zeros(n0 * n1 + 1, dtype=tdt, device="cuda")
    flat_s = torch.zeros(n0 * n1 + 1, dtype=tdt, device="cuda")
    Ru, Su = flat_r[1:].view(n0, n1), flat_s[1:].view(n0, n1)
    Ru.copy_(R)
    Su.copy_(S)
    assert Ru.data_ptr() % 16 != 0 and Su.data_ptr() % 16 != 0
    coef_u, d_u = ctx.run(p, Ru, Su)
    ctx.sync()
    assert torch.equal(coef, coef_u)
    assert torch.equal(d, d_u)


APPLY_CASES = [
    # n0, n1, w, dk, db
    (64, 64, 2, 1, 1),
    (96, 128, 3, 2, 2),
    (1024, 64, 4, 2, 2),
]


@pytest.mark.parametrize("case", APPLY_CASES)
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_apply_pair_differs_from_fit_pair(sfft, ctx, case, prec, dtype):
    """Fit on masked images, apply to the unmasked ones (Sec. 3). The apply
    pair is transformed as given -- in the mixed form without the fit pair's
    pedestal -- so this is a rounding regime of its own."""
    n0, n1, w, dk, db = case
    r, s = _pair(21 + n0, n0, n1, w, dk, db, 0)
    if dtype == "f32":
        r = r.astype(np.float32).astype(np.float64)
        s = s.astype(np.float32).astype(np.float64)
    rm, sm = r.copy(), s.copy()
    # masked rectangles (zero outside the usable domain, as in Sec. 3)
    rm[10:20, 30:40] = 0.0
    sm[10:20, 30:40] = 0.0
    rm[n0 // 2:n0 // 2 + 7, 3:9] = 0.0
    sm[n0 // 2:n0 // 2 + 7, 3:9] = 0.0
    tdt = torch.float32 if dtype == "f32" else torch.float64
    pr = sfft.FP64 if prec == "fp64" else sfft.MIXED
    p = _params(sfft, n0, n1, w, w, dk, db, 0, pr, sfft.F32 if dtype == "f32" else sfft.F64)
    if _mixed_refused(sfft, prec, dtype, dk, n0, n1):
        _assert_refused(sfft, ctx, p, _dev(r, tdt), _dev(s, tdt))
        return
    coef, d = ctx.run(p, _dev(rm, tdt), _dev(sm, tdt), _dev(r, tdt), _dev(s, tdt))
    ctx.sync()
    co = oracle.fit(rm, sm, w, w, dk, db)
    do = oracle.subtract(r, s, co, w, w, dk, db)
    c = coef.cpu().numpy()
    nk = len(c) - oracle.nterms(db)
    ek, eb = _rel(c[:nk], co[:nk]), _rel(c[nk:], co[nk:])
    rms = float(np.sqrt(np.mean((d.cpu().numpy().astype(np.float64) - do) ** 2)))
    print(f"apply case={case} prec={prec} dtype={dtype} coef_kernel={ek:.2e} coef_bg={eb:.2e} "
          f"d_rms={rms:.2e}")
    assert ek <= 1e-6 and eb <= 1e-6
    floor = 0.0 if dtype == "f64" else _f32_floor(do)
    assert rms <= 1e-5 * 10.0 + floor
    # sfft_subtract on the apply pair with the same coefficients: the same
    # kernels, so the same image
    d2 = ctx.subtract(p, _dev(r, tdt), _dev(s, tdt), coef)
    ctx.sync()
    assert torch.equal(d, d2)


def test_config1_full(sfft, ctx):
    """256 x 256 FP64 pair, 11 x 11 kernel, DK = DB = 0: the FP64 form on the
    FP64 images, the mixed form on the pair rounded to FP32 (the oracle on the
    same rounded pair)."""
    pair = datagen.config1()
    for pr, dt, tdt in ((sfft.FP64, sfft.F64, torch.float64), (sfft.MIXED, sfft.F32, torch.float32)):
        r = pair.r if dt == sfft.F64 else pair.r.astype(np.float32).astype(np.float64)
        s = pair.s if dt == sfft.F64 else pair.s.astype(np.float32).astype(np.float64)
        co = oracle.fit(r, s, 5, 5, 0, 0)
        do = oracle.subtract(r, s, co, 5, 5, 0, 0)
        p = sfft.Params(256, 256, 5, 5, 0, 0, 0, pr, dt)
        coef, d = ctx.run(p, _dev(r, tdt), _dev(s, tdt))
        ctx.sync()
        assert _rel(coef.cpu().numpy(), co) <= 1e-6
        assert np.sqrt(np.mean((d.cpu().numpy().astype(np.float64) - do) ** 2)) <= 1e-4


def test_synchronous_solve_reports_not_spd(sfft, ctx):
    """sfft_solve on the null stream waits and returns the device status."""
    p = sfft.Params(32, 32, 1, 1, 0, 0, 0, sfft.FP64, sfft.F64)
    z = torch.zeros((32, 32), dtype=torch.float64, device="cuda")
    o = torch.ones((32, 32), dtype=torch.float64, device="cuda")
    G, h = ctx.build_system(p, z, o)
    with pytest.raises(sfft.SfftError) as ei:
        ctx.solve(p, G, h, stream=torch.cuda.default_stream(), sync=False)
    assert ei.value.code == sfft.E_NOT_SPD
    assert "sfft_solve" in str(ei.value)
    ctx.sync()   # reported once: the flag was cleared by the solve


def test_solve_wait_give_up_is_reported(sfft):
    """Force every block-to-block wait of the triangular solves to give up
    (a generation that is never published, a short bound): every workgroup
    still exits, the error is SFFT_E_HIP, the coefficients are NaN, and the
    next normal call is unaffected."""
    n0, n1, w, dk, db = 96, 128, 3, 2, 2     # 300 unknowns: 5 blocks per sweep
    r, s = _pair(44, n0, n1, w, dk, db, 0)
    with sfft.Context(0) as c:
        for pr, dt, tdt in ((sfft.FP64, sfft.F64, torch.float64),
                            (sfft.MIXED, sfft.F32, torch.float32)):
            R, S = _dev(r, tdt), _dev(s, tdt)
            p = sfft.Params(n0, n1, w, w, dk, db, 0, pr, dt)
            cref, dref = c.run(p, R, S)
            c.sync()
            c.debug_solve_stall(True)
            coef, d = c.run(p, R, S)
            with pytest.raises(sfft.SfftError) as ei:
                c.sync()
            assert ei.value.code == sfft.E_HIP
            assert torch.isnan(coef).all()
            c.debug_solve_stall(False)
            coef2, d2 = c.run(p, R, S)
            c.sync()
            assert torch.equal(coef2, cref) and torch.equal(d2, dref)


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
