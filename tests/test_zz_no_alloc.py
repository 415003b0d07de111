"""sfft_run_noalloc, the allocation-free whole path, against sfft_run.

The allocation-free entry point carves its workspace and twiddle tables from
one static device array that keeps the previous call's contents. Two calls in
a row -- the second on a smaller image, in another precision and image type --
must each match sfft_run on the same inputs to the stated bar: coefficients
within 1e-6 relative (normwise, kernel block and background block) and the
difference image within an RMS of 1e-5 of the sky noise sigma (10). A
parameter set whose workspace exceeds the array is refused before anything
runs.
"""
import numpy as np
import pytest
import torch

import datagen

pytestmark = pytest.mark.gpu

SIGMA_SKY = 10.0


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _compare(tag, sfft, p, coef, d, coef_ref, d_ref):
    c, cr = coef.cpu().numpy(), coef_ref.cpu().numpy()
    nk = p.num_unknowns - (p.db + 1) * (p.db + 2) // 2
    ek, eb = _rel(c[:nk], cr[:nk]), _rel(c[nk:], cr[nk:])
    rms = float(torch.sqrt(torch.mean((d.double() - d_ref.double()) ** 2)))
    print(f"{tag}: coef_kernel={ek:.2e} coef_bg={eb:.2e} d_rms={rms:.2e}", flush=True)
    assert np.isfinite(c).all() and torch.isfinite(d).all()
    assert ek <= 1e-6 and eb <= 1e-6, (tag, ek, eb)
    assert rms <= 1e-5 * SIGMA_SKY, (tag, rms)


def test_noalloc_matches_run_twice_second_smaller(sfft):
    big = datagen.config2()        # 1024 x 1024, FP32 images, w = 5, DK = DB = 2
    small = datagen.config1()      # 256 x 256, FP64 images, w = 5, DK = DB = 0
    calls = [
        ("1024^2 mixed f32", big, sfft.Params(1024, 1024, 5, 5, 2, 2, 0, sfft.MIXED, sfft.F32),
         torch.float32),
        ("256^2 fp64 f64", small, sfft.Params(256, 256, 5, 5, 0, 0, 0, sfft.FP64, sfft.F64),
         torch.float64),
    ]
    with sfft.Context(0) as ctx:
        for tag, pair, p, tdt in calls:
            print(f"noalloc call: {tag}", flush=True)
            R = torch.from_numpy(pair.r).to("cuda", tdt)
            S = torch.from_numpy(pair.s).to("cuda", tdt)
            coef_ref, d_ref = ctx.run(p, R, S)
            ctx.sync()
            coef = torch.full((p.num_unknowns,), float("nan"), dtype=torch.float64, device="cuda")
            d = torch.full((p.n0, p.n1), float("nan"), dtype=tdt, device="cuda")
            ctx.run_noalloc(p, R, S, coef=coef, d=d)
            torch.cuda.synchronize()
            _compare(tag, sfft, p, coef, d, coef_ref, d_ref)


def test_noalloc_refuses_a_workspace_beyond_the_array(sfft):
    p = sfft.Params(4096, 4096, 7, 7, 2, 2, 0, sfft.MIXED, sfft.F32)
    R = torch.zeros((4096, 4096), dtype=torch.float32, device="cuda")
    with sfft.Context(0) as ctx:
        with pytest.raises(sfft.SfftError) as ei:
            ctx.run_noalloc(p, R, R)
        assert ei.value.code == sfft.E_NOMEM
