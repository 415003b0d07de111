"""Serving engine: continuous batching of independent pairs of uneven sizes.

Each result must be the same alone and in the mix (bit for bit: every
reduction has a fixed order and requests share no buffers), admission must
refuse a request that can never fit the HBM budget, and requests that fit
only one at a time must queue and complete.
"""
import numpy as np
import pytest
import torch

import datagen

pytestmark = pytest.mark.gpu

MIX = [
    # n0, n1, w, dk, db
    (64, 64, 2, 1, 1),
    (96, 128, 3, 2, 2),
    (256, 256, 5, 2, 2),
    (48, 96, 2, 0, 0),
    (192, 144, 4, 1, 2),
]


def _inputs(k, n0, n1, w, dk, db):
    p = datagen.star_pair(300 + k, n0, n1, w=w, dk=dk, db=db, density=0.01, dtype=np.float32)
    return torch.from_numpy(p.r).cuda(), torch.from_numpy(p.s).cuda()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_alone_equals_in_the_mix(sfft, prec):
    pr = sfft.FP64 if prec == "fp64" else sfft.MIXED
    alone = []
    with sfft.Context(0) as ctx:
        for k, (n0, n1, w, dk, db) in enumerate(MIX):
            p = sfft.Params(n0, n1, w, w, dk, db, 0, pr, sfft.F32)
            R, S = _inputs(k, n0, n1, w, dk, db)
            coef, d = ctx.run(p, R, S)
            ctx.sync()
            alone.append((p, R, S, coef.clone(), d.clone()))
    with sfft.Context(0) as ctx:
        ctx.engine_config(3)
        jobs = []
        for rep in range(3):
            for k, (p, R, S, _, _) in enumerate(alone):
                c = torch.full((p.num_unknowns,), float("nan"), dtype=torch.float64, device="cuda")
                d = torch.full((p.n0, p.n1), float("nan"), dtype=torch.float32, device="cuda")
                jobs.append((k, ctx.submit(p, R, S, R, S, c, d), c, d))
        for k, t, c, d in jobs:
            assert ctx.wait(t) == sfft.OK
        torch.cuda.synchronize()
        for k, t, c, d in jobs:
            assert torch.equal(c, alone[k][3]), (prec, k)
            assert torch.equal(d, alone[k][4]), (prec, k)
        for k, t, c, d in jobs:
            with pytest.raises(sfft.SfftError):
                ctx.poll(t)   # a finished ticket is reported once


def test_admission_refuses_what_can_never_fit(sfft):
    small = sfft.Params(64, 64, 2, 2, 1, 1, 0, sfft.MIXED, sfft.F32)
    big = sfft.Params(256, 256, 5, 5, 2, 2, 0, sfft.MIXED, sfft.F32)
    budget = sfft.Context.workspace_bytes(small) + 4096
    assert sfft.Context.workspace_bytes(big) > budget
    with sfft.Context(0, hbm_budget_bytes=budget) as ctx:
        R, S = _inputs(1, 256, 256, 5, 2, 2)
        c = torch.empty(big.num_unknowns, dtype=torch.float64, device="cuda")
        d = torch.empty((256, 256), dtype=torch.float32, device="cuda")
        with pytest.raises(sfft.SfftError) as ei:
            ctx.submit(big, R, S, R, S, c, d)
        assert ei.value.code == sfft.E_NOMEM


def test_requests_queue_until_memory_frees(sfft):
    p = sfft.Params(128, 128, 3, 3, 2, 2, 0, sfft.MIXED, sfft.F32)
    budget = int(sfft.Context.workspace_bytes(p) * 1.5)   # one workspace at a time
    R, S = _inputs(2, 128, 128, 3, 2, 2)
    with sfft.Context(0) as ref_ctx:
        cref, dref = ref_ctx.run(p, R, S)
        ref_ctx.sync()
    with sfft.Context(0, hbm_budget_bytes=budget) as ctx:
        ctx.engine_config(4)
        outs = []
        for _ in range(5):
            c = torch.empty(p.num_unknowns, dtype=torch.float64, device="cuda")
            d = torch.empty((128, 128), dtype=torch.float32, device="cuda")
            outs.append((ctx.submit(p, R, S, R, S, c, d), c, d))
        for t, c, d in outs:
            assert ctx.wait(t) == sfft.OK
            assert torch.equal(c, cref) and torch.equal(d, dref)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_graph_replays_match_eager(sfft, prec):
    """The engine replays one captured graph per workspace and variant (apply
    pair = fit pair, or not); the caller's buffers change on every replay and
    eager work runs between the replays. Every replay must equal the eager
    (directly launched) result bit for bit."""
    pr = sfft.FP64 if prec == "fp64" else sfft.MIXED
    shapes = [(96, 128, 3, 2, 2), (64, 64, 2, 1, 1)]
    with sfft.Context(0) as eager, sfft.Context(0) as ctx:
        ctx.engine_config(2)
        for rep in range(4):
            for k, (n0, n1, w, dk, db) in enumerate(shapes):
                p = sfft.Params(n0, n1, w, w, dk, db, 0, pr, sfft.F32)
                Rf, Sf = _inputs(10 * k + rep, n0, n1, w, dk, db)
                same = rep % 2 == 0
                if same:
                    R, S = Rf, Sf
                else:   # apply the fit to a second pair of the same shape
                    R, S = _inputs(100 + 10 * k + rep, n0, n1, w, dk, db)
                cref, dref = eager.run(p, Rf, Sf, R, S)
                eager.sync()
                want_coef = rep != 3
                c = torch.full((p.num_unknowns,), float("nan"), dtype=torch.float64,
                               device="cuda") if want_coef else None
                d = torch.full((n0, n1), float("nan"), dtype=torch.float32, device="cuda")
                t = ctx.submit(p, Rf, Sf, R, S, c, d)
                assert ctx.wait(t) == sfft.OK
                torch.cuda.synchronize()
                if want_coef:
                    assert torch.equal(c, cref), (prec, rep, k)
                assert torch.equal(d, dref), (prec, rep, k)


def test_one_workspace_alternating_image_types(sfft):
    """One slot, so every request reuses the same workspace: F32, F64, F32,
    F64 requests of one geometry (FP64 form) must each equal the direct call
    bit for bit (each image type replays its own captured graph). The mixed
    form refuses FP64 images at submit."""
    prec = "fp64"
    pr = sfft.FP64
    n0, n1, w, dk, db = 96, 128, 3, 2, 2
    R32, S32 = _inputs(7, n0, n1, w, dk, db)
    R64, S64 = R32.double(), S32.double()
    refs = {}
    with sfft.Context(0) as eager:
        for dt, (R, S) in ((sfft.F32, (R32, S32)), (sfft.F64, (R64, S64))):
            p = sfft.Params(n0, n1, w, w, dk, db, 0, pr, dt)
            c, d = eager.run(p, R, S)
            eager.sync()
            refs[dt] = (p, R, S, c, d)
    with sfft.Context(0) as ctx:
        ctx.engine_config(1)
        for dt in (sfft.F32, sfft.F64, sfft.F32, sfft.F64):
            p, R, S, cref, dref = refs[dt]
            c = torch.full((p.num_unknowns,), float("nan"), dtype=torch.float64, device="cuda")
            d = torch.full((n0, n1), float("nan"), dtype=p.torch_dtype, device="cuda")
            assert ctx.wait(ctx.submit(p, R, S, R, S, c, d)) == sfft.OK
            torch.cuda.synchronize()
            assert torch.equal(c, cref), (prec, dt)
            assert torch.equal(d, dref), (prec, dt)
        pm = sfft.Params(n0, n1, w, w, dk, db, 0, sfft.MIXED, sfft.F64)
        c = torch.empty(pm.num_unknowns, dtype=torch.float64, device="cuda")
        d = torch.empty((n0, n1), dtype=torch.float64, device="cuda")
        with pytest.raises(sfft.SfftError) as ei:
            ctx.submit(pm, R64, S64, R64, S64, c, d)
        assert ei.value.code == sfft.E_UNSUPPORTED


def test_submit_is_ordered_after_the_callers_stream(sfft):
    """Inputs written and outputs initialised on a side stream right before
    submit (no host synchronisation): the request must see them."""
    n0, n1, w, dk, db = 256, 256, 5, 2, 2
    p = sfft.Params(n0, n1, w, w, dk, db, 0, sfft.MIXED, sfft.F32)
    R, S = _inputs(9, n0, n1, w, dk, db)
    with sfft.Context(0) as eager:
        cref, dref = eager.run(p, R, S)
        eager.sync()
    side = torch.cuda.Stream()
    with sfft.Context(0) as ctx:
        ctx.engine_config(2)
        jobs = []
        for k in range(4):
            with torch.cuda.stream(side):
                # a long kernel first, so that a request that did not wait
                # for this stream would read the inputs before they exist
                big = torch.randn(4096, 4096, device="cuda")
                for _ in range(4):
                    big = big @ big * 1e-3
                R2 = R * 1.0 + big[0, 0] * 0.0
                S2 = S * 1.0 + big[0, 0] * 0.0
                c = torch.full((p.num_unknowns,), float("nan"), dtype=torch.float64, device="cuda")
                d = torch.full((n0, n1), float("nan"), dtype=torch.float32, device="cuda")
                jobs.append((ctx.submit(p, R2, S2, R2, S2, c, d), c, d))
            del R2, S2   # the binding holds them until the request is done
        for t, c, d in jobs:
            assert ctx.wait(t) == sfft.OK
        torch.cuda.synchronize()
        for t, c, d in jobs:
            assert torch.equal(c, cref) and torch.equal(d, dref)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_of_distinct_pairs_equals_alone(sfft, prec):
    """One slot held by a large request while distinct same-size requests
    queue up: they run as one batch (one launch per stage, one pair per
    blockIdx.z), fit-pair and apply-pair variants in separate batches. Each
    result must equal its direct call bit for bit -- with distinct inputs per
    pair, a pair reading another pair's buffers would show."""
    pr = sfft.FP64 if prec == "fp64" else sfft.MIXED
    n0, n1, w, dk, db = 96, 128, 3, 2, 2
    p = sfft.Params(n0, n1, w, w, dk, db, 0, pr, sfft.F32)
    big = sfft.Params(1024, 1024, 5, 5, 2, 2, 0, pr, sfft.F32)
    Rb, Sb = _inputs(600, 1024, 1024, 5, 2, 2)
    reqs = []
    for k in range(11):
        Rf, Sf = _inputs(500 + k, n0, n1, w, dk, db)
        if k % 3 == 2:   # apply the fit to another pair of the same shape
            R, S = _inputs(700 + k, n0, n1, w, dk, db)
        else:
            R, S = Rf, Sf
        reqs.append((Rf, Sf, R, S))
    refs = []
    with sfft.Context(0) as eager:
        for Rf, Sf, R, S in reqs:
            c, d = eager.run(p, Rf, Sf, R, S)
            eager.sync()
            refs.append((c, d))
    with sfft.Context(0) as ctx:
        ctx.engine_config(1, 8)
        for rnd in range(2):
            cb = torch.empty(big.num_unknowns, dtype=torch.float64, device="cuda")
            db_ = torch.empty((1024, 1024), dtype=torch.float32, device="cuda")
            tb = ctx.submit(big, Rb, Sb, Rb, Sb, cb, db_)
            jobs = []
            for k, (Rf, Sf, R, S) in enumerate(reqs):
                c = torch.full((p.num_unknowns,), float("nan"), dtype=torch.float64, device="cuda")
                d = torch.full((n0, n1), float("nan"), dtype=torch.float32, device="cuda")
                jobs.append((k, ctx.submit(p, Rf, Sf, R, S, c, d), c, d))
            assert ctx.wait(tb) == sfft.OK
            for k, t, c, d in jobs:
                assert ctx.wait(t) == sfft.OK
            torch.cuda.synchronize()
            for k, t, c, d in jobs:
                assert torch.equal(c, refs[k][0]), (prec, rnd, k)
                assert torch.equal(d, refs[k][1]), (prec, rnd, k)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_direct_batch_equals_each_run(sfft, prec):
    """sfft_run_batch: n distinct pairs of one variant as one launch per stage
    on the context's workspace; each result equals sfft_run on it bit for
    bit, for n = 5 (a workspace of 8 pairs) and then n = 3 on the same
    workspace, both apply-pair variants."""
    pr = sfft.FP64 if prec == "fp64" else sfft.MIXED
    n0, n1, w, dk, db = 96, 128, 3, 2, 2
    p = sfft.Params(n0, n1, w, w, dk, db, 0, pr, sfft.F32)
    with sfft.Context(0) as ctx:
        for n, same in ((5, True), (3, False), (5, False)):
            items, refs = [], []
            for k in range(n):
                Rf, Sf = _inputs(800 + 10 * n + k, n0, n1, w, dk, db)
                R, S = (Rf, Sf) if same else _inputs(900 + 10 * n + k, n0, n1, w, dk, db)
                cr, dr = ctx.run(p, Rf, Sf, R, S)
                ctx.sync()
                refs.append((cr.clone(), dr.clone()))
                c = torch.full((p.num_unknowns,), float("nan"), dtype=torch.float64, device="cuda")
                d = torch.full((n0, n1), float("nan"), dtype=torch.float32, device="cuda")
                items.append((Rf, Sf, R, S, c, d))
            ctx.run_batch(p, items)
            ctx.sync()
            for k, it in enumerate(items):
                assert torch.equal(it[4], refs[k][0]), (prec, n, same, k)
                assert torch.equal(it[5], refs[k][1]), (prec, n, same, k)


def test_direct_batch_reports_a_bad_pair(sfft):
    """A pair whose normal matrix is singular inside a batch: sfft_sync
    reports it, its coefficients are NaN, the other pairs are unaffected."""
    n0 = n1 = 32
    p = sfft.Params(n0, n1, 1, 1, 0, 0, 0, sfft.FP64, sfft.F64)
    rng = torch.Generator(device="cpu").manual_seed(5)
    good = [(torch.randn(n0, n1, generator=rng, dtype=torch.float64).cuda() + 100.0,
             torch.randn(n0, n1, generator=rng, dtype=torch.float64).cuda() + 100.0) for _ in range(3)]
    zero = torch.zeros((n0, n1), dtype=torch.float64, device="cuda")
    one = torch.ones((n0, n1), dtype=torch.float64, device="cuda")
    pairs = [good[0], (zero, one), good[1], good[2]]
    with sfft.Context(0) as ctx:
        refs = []
        for R, S in pairs:
            c, d = ctx.run(p, R, S)
            try:
                ctx.sync()
            except sfft.SfftError:
                pass
            refs.append(c.clone())
        items = [(R, S, R, S, torch.empty(p.num_unknowns, dtype=torch.float64, device="cuda"),
                  torch.empty((n0, n1), dtype=torch.float64, device="cuda")) for R, S in pairs]
        ctx.run_batch(p, items)
        with pytest.raises(sfft.SfftError) as ei:
            ctx.sync()
        assert ei.value.code == sfft.E_NOT_SPD
        assert torch.isnan(items[1][4]).all()
        for k in (0, 2, 3):
            assert torch.equal(items[k][4], refs[k])
        ctx.sync()   # reported once


def test_batch_of_bluestein_pairs_equals_alone(sfft):
    """A batch of pairs whose lengths need Bluestein lines (94 x 110) through
    the engine: each equals its direct call bit for bit."""
    n0, n1, w, dk, db = 94, 110, 3, 2, 2
    p = sfft.Params(n0, n1, w, w, dk, db, 0, sfft.MIXED, sfft.F32)
    with sfft.Context(0) as eager, sfft.Context(0) as ctx:
        ctx.engine_config(1, 4)
        refs, jobs = [], []
        for k in range(4):
            R, S = _inputs(950 + k, n0, n1, w, dk, db)
            c, d = eager.run(p, R, S)
            eager.sync()
            refs.append((c.clone(), d.clone()))
            co = torch.empty(p.num_unknowns, dtype=torch.float64, device="cuda")
            do = torch.empty((n0, n1), dtype=torch.float32, device="cuda")
            jobs.append((ctx.submit(p, R, S, R, S, co, do), co, do))
        for k, (t, co, do) in enumerate(jobs):
            assert ctx.wait(t) == sfft.OK
        torch.cuda.synchronize()
        for k, (t, co, do) in enumerate(jobs):
            assert torch.equal(co, refs[k][0]) and torch.equal(do, refs[k][1]), k


def test_many_slots_run_their_solves_concurrently(sfft):
    """Sixteen slots with batches of two: the dataflow triangular solves of
    many requests run at once, interleaved with every other stage, while
    their workgroups are spread over the XCDs in whatever order the hardware
    dispatches them. Every request must succeed and equal its direct call
    bit for bit, in both forms."""
    shapes = [(128, 128, 3, 2, 2), (256, 256, 5, 2, 2), (192, 256, 4, 1, 2), (96, 128, 3, 2, 1)]
    with sfft.Context(0) as eager, sfft.Context(0) as ctx:
        ctx.engine_config(16, 2)
        refs, jobs = {}, []
        for rep in range(6):
            for k, (n0, n1, w, dk, db) in enumerate(shapes):
                for pr in (sfft.MIXED, sfft.FP64):
                    p = sfft.Params(n0, n1, w, w, dk, db, 0, pr, sfft.F32)
                    R, S = _inputs(1200 + 10 * k + rep % 2, n0, n1, w, dk, db)
                    key = (k, pr, rep % 2)
                    if key not in refs:
                        c, d = eager.run(p, R, S)
                        eager.sync()
                        refs[key] = (c.clone(), d.clone())
                    co = torch.empty(p.num_unknowns, dtype=torch.float64, device="cuda")
                    do = torch.empty((n0, n1), dtype=torch.float32, device="cuda")
                    jobs.append((key, ctx.submit(p, R, S, R, S, co, do), co, do, R, S))
        for key, t, co, do, _, _ in jobs:
            assert ctx.wait(t) == sfft.OK, key
        torch.cuda.synchronize()
        for key, t, co, do, _, _ in jobs:
            assert torch.equal(co, refs[key][0]) and torch.equal(do, refs[key][1]), key
