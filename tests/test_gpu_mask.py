"""GPU crowded-flavour preprocessing (Sec. 3.1) against the oracle, bit for bit.

Every step is a comparison or a selection, so the mask and both filled
images must equal ``oracle.mask.crowded_fit_pair`` exactly, on seeded star
fields with stars clipped at a saturation level, in both image types, with
ragged tiles, footprints across the wrap, fully masked tiles and non-finite
pixels; then the whole path fitted on the masked pair and applied to the
unmasked one is checked against the oracle's fit and difference image.
"""
import numpy as np
import pytest
import torch

import datagen
import oracle
from oracle import mask as om

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(sfft):
    c = sfft.Context(0)
    yield c
    c.close()


def _saturated_pair(seed, n0, n1, u, dtype):
    pair = datagen.star_pair(seed, n0, n1, w=3, dk=1, db=1, density=0.004, dtype=np.float64)
    rng = np.random.default_rng(seed)
    r, s = pair.r.copy(), pair.s.copy()
    # a few very bright stars on top, clipped at the saturation level
    yy, xx = np.mgrid[:n0, :n1]
    for _ in range(6):
        y, x = rng.uniform(0, n0), rng.uniform(0, n1)
        dy = (yy - y + n0 / 2) % n0 - n0 / 2
        dx = (xx - x + n1 / 2) % n1 - n1 / 2
        blob = 5e5 * np.exp(-(dy * dy + dx * dx) / (2 * 1.8 ** 2))
        r += blob
        s += 0.95 * blob
    r, s = np.minimum(r, u), np.minimum(s, u)
    return r.astype(dtype), s.astype(dtype)


CASES = [
    # n0, n1, g0, g1, t0, t1
    (256, 256, 5, 5, 64, 64),
    (192, 160, 3, 7, 48, 40),
    (100, 130, 2, 4, 32, 64),     # ragged tiles
    (64, 64, 10, 10, 16, 16),     # large footprints: fully masked tiles
    (1024, 48, 6, 2, 64, 16),
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_crowded_mask_bit_exact(sfft, ctx, case, dtype):
    n0, n1, g0, g1, t0, t1 = case
    u = 3.0e4
    r, s = _saturated_pair(n0 + 3 * n1, n0, n1, u, dtype)
    r[5, 7] = np.nan                      # a bad pixel
    s[n0 - 1, n1 - 2] = np.inf
    rb, sb, m = om.crowded_fit_pair(r, s, u, u, g0, g1, t0, t1)
    print(f"case={case} dtype={np.dtype(dtype).name} masked={m.mean():.3f}", flush=True)
    R = torch.from_numpy(r).cuda()
    S = torch.from_numpy(s).cuda()
    Ro, So, M = ctx.crowded_mask(R, S, u, u, g0, g1, t0, t1, want_mask=True)
    torch.cuda.synchronize()
    assert np.array_equal(M.cpu().numpy().astype(bool), m)
    assert np.array_equal(Ro.cpu().numpy(), rb)
    assert np.array_equal(So.cpu().numpy(), sb)
    # in place (outputs = inputs)
    ctx.crowded_mask(R, S, u, u, g0, g1, t0, t1, r_out=R, s_out=S)
    torch.cuda.synchronize()
    assert np.array_equal(R.cpu().numpy(), rb) and np.array_equal(S.cpu().numpy(), sb)


def test_every_pixel_masked_and_none_masked(sfft, ctx):
    r = np.full((64, 80), 10.0, dtype=np.float32)
    s = np.full((64, 80), 20.0, dtype=np.float32)
    Ro, So = ctx.crowded_mask(torch.from_numpy(r).cuda(), torch.from_numpy(s).cuda(), 5.0, 5.0,
                              1, 1, 16, 16)
    assert not Ro.any() and not So.any()           # all masked: background 0
    Ro, So = ctx.crowded_mask(torch.from_numpy(r).cuda(), torch.from_numpy(s).cuda(), 1e9, 1e9,
                              1, 1, 16, 16)
    assert np.array_equal(Ro.cpu().numpy(), r) and np.array_equal(So.cpu().numpy(), s)


def test_fit_on_masked_pair_apply_to_unmasked(sfft, ctx):
    """The masked pair is the fit pair, the unmasked pair the apply pair
    (Sec. 3): the GPU path on the GPU-masked images against the oracle fit
    and difference image on the oracle-masked ones (the same arrays)."""
    n0 = n1 = 256
    w, dk, db = 4, 2, 2
    u = 3.0e4
    r, s = _saturated_pair(77, n0, n1, u, np.float32)
    rb, sb, m = om.crowded_fit_pair(r, s, u, u, w, w, 64, 64)
    R, S = torch.from_numpy(r).cuda(), torch.from_numpy(s).cuda()
    Rb, Sb = ctx.crowded_mask(R, S, u, u, w, w, 64, 64)
    torch.cuda.synchronize()
    assert np.array_equal(Rb.cpu().numpy(), rb) and np.array_equal(Sb.cpu().numpy(), sb)
    co = oracle.fit(rb.astype(np.float64), sb.astype(np.float64), w, w, dk, db)
    do = oracle.subtract(r.astype(np.float64), s.astype(np.float64), co, w, w, dk, db)
    for prec in (sfft.FP64, sfft.MIXED):
        p = sfft.Params(n0, n1, w, w, dk, db, 0, prec, sfft.F32)
        coef, d = ctx.run(p, Rb, Sb, R, S)
        ctx.sync()
        c = coef.cpu().numpy()
        nk = len(c) - oracle.nterms(db)
        ek = np.linalg.norm(c[:nk] - co[:nk]) / np.linalg.norm(co[:nk])
        eb = np.linalg.norm(c[nk:] - co[nk:]) / np.linalg.norm(co[nk:])
        rms = float(np.sqrt(np.mean((d.cpu().numpy().astype(np.float64) - do) ** 2)))
        print(f"masked fit prec={prec}: coef_kernel={ek:.2e} coef_bg={eb:.2e} d_rms={rms:.2e}",
              flush=True)
        assert ek <= 1e-6 and eb <= 1e-6
        # the apply pair keeps its saturated plateaus (RMS(S) ~ 2300 here):
        # besides the output's own rounding, the mixed form's FP32 transforms
        # of the raw apply pair round at ~1e-7 of RMS(S) (2^-22 allowed)
        floor = 2.0 ** -24 * float(np.sqrt(np.mean(do ** 2)))
        if prec == sfft.MIXED:
            floor += 2.0 ** -22 * float(np.sqrt(np.mean(s.astype(np.float64) ** 2)))
        assert rms <= 1e-4 + floor
