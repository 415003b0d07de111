"""GPU parity at the workload sizes, through the C ABI.

* 1024 x 1024 (DK = DB = 2, 11 x 11 kernel): the full FP64 oracle.
* the C4 sizes (512^2 .. 2048 x 4096, DK = DB = 1) and 6144 x 6144 (DK = DB =
  2) of the serving mix, through the engine: mixed vs FP64, sampled D,
  sampled stationarity.
* 4096 x 4096 (DK = DB = 2, 15 x 15 kernel, the benchmark's pair and launch
  configuration): entries of G and h sampled one by one from the oracle's
  basis-image definition, D sampled pixel by pixel, and stationarity of the
  GPU solution (Eq. 16-17: Phi^T (S - Phi c) = 0) on sampled components.
Tolerances as in test_gpu_parity: coefficients 1e-6 relative (normwise), D
within 1e-5 of the sky noise sigma = 10.
"""
import numpy as np
import pytest
import torch

import datagen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(sfft):
    c = sfft.Context(0)
    yield c
    c.close()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.timeout(600)
def test_config2_full_oracle(sfft, ctx):
    pair = datagen.config2()
    r64 = pair.r.astype(np.float64)
    s64 = pair.s.astype(np.float64)
    co = oracle.fit(r64, s64, 5, 5, 2, 2)
    do = oracle.subtract(r64, s64, co, 5, 5, 2, 2)
    R = torch.from_numpy(pair.r).cuda()
    S = torch.from_numpy(pair.s).cuda()
    nk = 6 * 121
    for prec in (sfft.FP64, sfft.MIXED):
        p = sfft.Params(1024, 1024, 5, 5, 2, 2, 0, prec, sfft.F32)
        coef, d = ctx.run(p, R, S)
        ctx.sync()
        c = coef.cpu().numpy()
        ek, eb = _rel(c[:nk], co[:nk]), _rel(c[nk:], co[nk:])
        rms = float(np.sqrt(np.mean((d.cpu().numpy().astype(np.float64) - do) ** 2)))
        print(f"C2 prec={prec} coef_kernel={ek:.2e} coef_bg={eb:.2e} d_rms={rms:.2e}")
        assert ek <= 1e-6 and eb <= 1e-6
        assert rms <= 1e-4


@pytest.fixture(scope="module")
def c3(sfft, ctx):
    pair = datagen.config3()
    R = torch.from_numpy(pair.r).cuda()
    S = torch.from_numpy(pair.s).cuda()
    out = {"pair": pair, "R": R, "S": S}
    for name, prec in (("fp64", sfft.FP64), ("mixed", sfft.MIXED)):
        p = sfft.Params(4096, 4096, 7, 7, 2, 2, 0, prec, sfft.F32)
        G, h = ctx.build_system(p, R, S)
        coef, d = ctx.run(p, R, S)
        ctx.sync()
        out[name] = {"G": G.cpu().numpy(), "h": h.cpu().numpy(), "coef": coef.cpu().numpy(),
                     "d": d.cpu().numpy()}
    return out


SAMPLES_G = [(0, 0), (112, 112), (112, 0), (500, 37), (1355, 1355), (1350, 200), (1351, 1352),
             (800, 799), (225, 224), (1000, 1353)]
SAMPLES_H = [0, 112, 113, 700, 1349, 1350, 1355]


@pytest.mark.timeout(900)
def test_config3_sampled_normal_equations(c3):
    r = c3["pair"].r.astype(np.float64)
    s = c3["pair"].s.astype(np.float64)
    for name, tol in (("fp64", 1e-10), ("mixed", 2e-5)):
        G = c3[name]["G"]
        scale = np.abs(np.diag(G)).max()
        assert np.array_equal(G, G.T)
        for u, v in SAMPLES_G:
            ref = oracle.g_entry(r, 7, 7, 2, 2, 0, u, v)
            assert abs(G[u, v] - ref) <= tol * scale, (name, u, v, G[u, v], ref)
        h = c3[name]["h"]
        hs = np.abs(h).max()
        for u in SAMPLES_H:
            ref = oracle.phi_dot(r, s, 7, 7, 2, 2, 0, u)
            assert abs(h[u] - ref) <= tol * hs, (name, u, h[u], ref)


@pytest.mark.timeout(900)
def test_config3_solution_and_difference(c3):
    r = c3["pair"].r.astype(np.float64)
    s = c3["pair"].s.astype(np.float64)
    c64 = c3["fp64"]["coef"]
    cm = c3["mixed"]["coef"]
    nk = 6 * 225
    # mixed vs the FP64 form (itself checked below through stationarity)
    assert _rel(cm[:nk], c64[:nk]) <= 1e-6
    assert _rel(cm[nk:], c64[nk:]) <= 1e-6
    # D at sampled pixels from the oracle with the GPU coefficients
    rng = np.random.default_rng(9)
    pix = np.concatenate([rng.integers(0, 4096, (40, 2)),
                          [[0, 0], [4095, 4095], [0, 4095], [7, 4090], [4093, 3]]])
    for name in ("fp64", "mixed"):
        ref = oracle.subtract_pixels(r, s, c3[name]["coef"], 7, 7, 2, 2, 0, pix)
        got = c3[name]["d"][pix[:, 0], pix[:, 1]].astype(np.float64)
        assert np.abs(got - ref).max() <= 1e-4 + 2e-7 * np.abs(s[pix[:, 0], pix[:, 1]]).max()
    # stationarity (Eq. 16-17) of both solutions: Phi_u^T D(c) = 0, measured
    # against the Cauchy-Schwarz scale ||Phi_u|| ||D|| with ||Phi_u||^2 = G_uu
    for name in ("fp64", "mixed"):
        d = oracle.subtract(r, s, c3[name]["coef"], 7, 7, 2, 2)
        dn = float(np.linalg.norm(d))
        for u in SAMPLES_H:
            g = oracle.phi_dot(r, d, 7, 7, 2, 2, 0, u)
            scale = np.sqrt(oracle.g_entry(r, 7, 7, 2, 2, 0, u, u)) * dn
            print(f"stationarity {name} u={u} g/scale={abs(g) / scale:.2e}")
            assert abs(g) <= 1e-6 * scale, (name, u, g, scale)


def _served(sfft, pr, p_params, dev="cuda"):
    """Both forms of one pair through the engine (the batched launch
    configuration: captured graphs per workspace); returns coef, D per form."""
    R = torch.from_numpy(pr.r).to(dev)
    S = torch.from_numpy(pr.s).to(dev)
    out = {}
    with sfft.Context(0) as c:
        c.engine_config(2)
        jobs = []
        for name, p in p_params.items():
            coef = torch.empty(p.num_unknowns, dtype=torch.float64, device=dev)
            d = torch.empty((p.n0, p.n1), dtype=torch.float32, device=dev)
            jobs.append((name, c.submit(p, R, S, R, S, coef, d), coef, d))
        for name, t, coef, d in jobs:
            assert c.wait(t) == sfft.OK
            out[name] = (coef.cpu().numpy(), d.cpu().numpy())
    return out


def _check_served(pr, out, w, dk, db, nk, pix_seed):
    """Mixed vs FP64 coefficients (1e-6), D at sampled pixels against the
    oracle with the GPU coefficients, and stationarity of the FP64 solution
    on sampled components."""
    n0, n1 = pr.r.shape
    r = pr.r.astype(np.float64)
    s = pr.s.astype(np.float64)
    c64, cm = out["fp64"][0], out["mixed"][0]
    assert _rel(cm[:nk], c64[:nk]) <= 1e-6
    assert _rel(cm[nk:], c64[nk:]) <= 1e-6
    rng = np.random.default_rng(pix_seed)
    pix = np.concatenate([np.stack([rng.integers(0, n0, 30), rng.integers(0, n1, 30)], 1),
                          [[0, 0], [n0 - 1, n1 - 1], [0, n1 - 1], [w, n1 - 1 - w]]])
    for name in ("fp64", "mixed"):
        ref = oracle.subtract_pixels(r, s, out[name][0], w, w, dk, db, 0, pix)
        got = out[name][1][pix[:, 0], pix[:, 1]].astype(np.float64)
        assert np.abs(got - ref).max() <= 1e-4 + 2e-7 * np.abs(s[pix[:, 0], pix[:, 1]]).max(), name
    d = oracle.subtract(r, s, c64, w, w, dk, db)
    dn = float(np.linalg.norm(d))
    nu = len(c64)
    for u in sorted({0, nk // 2, nk - 1, nk, nu - 1}):
        g = oracle.phi_dot(r, d, w, w, dk, db, 0, u)
        scale = np.sqrt(oracle.g_entry(r, w, w, dk, db, 0, u, u)) * dn
        assert abs(g) <= 1e-6 * scale, (u, g, scale)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("shape", datagen.BATCH_SHAPES)
def test_config4_sizes_through_engine(sfft, shape):
    """The C4 sizes (11x11 kernel, DK = DB = 1), both forms, served."""
    n0, n1 = shape
    pr = datagen.star_pair(100 + n0 + n1, n0, n1, w=5, dk=1, db=1)
    params = {name: sfft.Params(n0, n1, 5, 5, 1, 1, 0, prec, sfft.F32)
              for name, prec in (("fp64", sfft.FP64), ("mixed", sfft.MIXED))}
    out = _served(sfft, pr, params)
    _check_served(pr, out, 5, 1, 1, 3 * 121, 40 + n0)
    if n0 * n1 <= 1024 * 1024:   # the full oracle fit where it is quick
        co = oracle.fit(pr.r.astype(np.float64), pr.s.astype(np.float64), 5, 5, 1, 1)
        for name in ("fp64", "mixed"):
            assert _rel(out[name][0], co) <= 1e-6, name


@pytest.mark.timeout(900)
def test_config5_6144_through_engine(sfft):
    """The largest size of the serving mix: 6144 x 6144, 15x15 kernel,
    DK = DB = 2 (radix-3 line plans), both forms, served."""
    pr = datagen.star_pair(1000 + 6144, 6144, 6144, w=7, dk=2, db=2)
    params = {name: sfft.Params(6144, 6144, 7, 7, 2, 2, 0, prec, sfft.F32)
              for name, prec in (("fp64", sfft.FP64), ("mixed", sfft.MIXED))}
    out = _served(sfft, pr, params)
    _check_served(pr, out, 7, 2, 2, 6 * 225, 61)
