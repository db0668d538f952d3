"""GPU parity of the batched context (length bins, persistent work queue, HIP
graphs, autotuned plan): bit-exact against the oracle and against the plain
one-launch path, including graph replays with eager work between them."""
import json
import os

import numpy as np
import pytest
import torch

import paper_1805_00106_amd as sw
from paper_1805_00106_amd import workloads as wl
from tests.gpu_util import SLOTS, assert_same, gpu_align, oracle_align, scoring_for

pytestmark = pytest.mark.gpu


def _ctx_run(batch, precision, ctx=None, max_read_len=None, repeats=1):
    refs = sw.RefSet.from_codes(torch.from_numpy(batch.ref_codes).cuda(), batch.ref_off, batch.ref_len)
    db = sw.DeviceBatch.upload(batch)
    sc = scoring_for(batch, precision, max_read_len=max_read_len)
    own = ctx is None
    if own:
        ctx = sw.Context(max(batch.n_reads, 1), max(batch.n_cals, 1))
    out = sw.Outputs(db.n_cals)
    results = []
    for _ in range(repeats):
        out.score.fill_(-7)
        out.ref_end.fill_(-7)
        out.read_end.fill_(-7)
        torch.cuda.synchronize()
        ctx.align(db, refs, sc, out)
        torch.cuda.synchronize()
        results.append(dict(score=out.score.cpu().numpy(), ref_end=out.ref_end.cpu().numpy(),
                            read_end=out.read_end.cpu().numpy()))
    plan = ctx.last_plan()
    if own:
        ctx.close()
    return results, plan


@pytest.mark.parametrize("precision", [sw.PREC_INT16, sw.PREC_INT32])
@pytest.mark.parametrize("seed", range(4))
def test_ctx_random_ragged(seed, precision):
    b = wl.random_small_batch(20 + seed, n_reads=120, read_len=(1, 120), band=12)
    exp, _ = oracle_align(b)
    res, plan = _ctx_run(b, precision, repeats=3)
    for k, r in enumerate(res):
        assert_same(r, exp, f"ctx seed {seed} replay {k} ({plan})", keys=SLOTS)


@pytest.mark.parametrize("band", [16, 32, 64])
def test_ctx_uneven_lengths_shape(band):
    """Uneven-lengths generator (L uniform 75..250, geometric CAL counts capped at 64)."""
    b = wl.uneven_lengths(n_reads=1200, band=band)
    exp, _ = oracle_align(b)
    res, plan = _ctx_run(b, sw.PREC_INT16, max_read_len=250, repeats=2)
    for r in res:
        assert_same(r, exp, f"uneven_lengths band {band} ({plan})", keys=SLOTS)
    # the tuner's pick: bins in either order, or input order without bins
    assert "longest first" in plan or "shortest first" in plan or "unbinned" in plan, plan


def test_ctx_equals_plain_on_chromosome_scale_shape():
    b = wl.chromosome_scale(n_reads=20000)
    plain = gpu_align(b, sw.PREC_INT16, reduce=False)
    res, plan = _ctx_run(b, sw.PREC_INT16, repeats=2)
    for r in res:
        assert_same(r, plain, f"ctx vs plain ({plan})")


def test_ctx_invalid_cals_and_capacity():
    b = wl.random_small_batch(30, n_reads=40, max_cals=3)
    b.cal_pos = b.cal_pos.copy()
    b.cal_ref = b.cal_ref.copy()
    b.cal_pos[0] = b.ref_len[int(b.cal_ref[0])] + 3
    b.cal_ref[1] = -1
    exp, errs = oracle_align(b)
    ctx = sw.Context(b.n_reads, b.n_cals)
    res, _ = _ctx_run(b, sw.PREC_INT16, ctx=ctx)
    assert_same(res[0], exp, "ctx invalid", keys=SLOTS)
    assert ctx.error_count() == errs > 0
    small = sw.Context(1, 1)
    with pytest.raises(sw.SwError) as ei:
        _ctx_run(b, sw.PREC_INT16, ctx=small)
    assert ei.value.code == -5
    small.close()
    ctx.close()


def _prepare(batch):
    refs = sw.RefSet.from_codes(torch.from_numpy(batch.ref_codes).cuda(), batch.ref_off, batch.ref_len)
    db = sw.DeviceBatch.upload(batch)
    return refs, db, sw.Outputs(db.n_cals)


def _host(out):
    torch.cuda.synchronize()
    return dict(score=out.score.cpu().numpy(), ref_end=out.ref_end.cpu().numpy(), read_end=out.read_end.cpu().numpy())


def test_ctx_shapes_change_and_graph_cache(tmp_path):
    """One context, alternating shapes: graphs are captured per shape and replayed."""
    cache = str(tmp_path / "tune.json")
    ctx = sw.Context(5000, 60000, tune_cache=cache)
    batches = [wl.random_small_batch(40 + k, n_reads=100 + 50 * k, read_len=(20, 200), band=16) for k in range(3)]
    exps = [oracle_align(b)[0] for b in batches]
    prepared = [_prepare(b) for b in batches]
    plans = []
    for rnd in range(2):
        for b, exp, (refs, db, out) in zip(batches, exps, prepared):
            out.score.fill_(-7)
            ctx.align(db, refs, scoring_for(b, sw.PREC_INT16, max_read_len=200), out)
            assert_same(_host(out), exp, f"round {rnd} {ctx.last_plan()}", keys=SLOTS)
            plans.append(ctx.last_plan())
    ctx.close()
    assert all("replay" in p for p in plans[3:]), plans
    with open(cache) as f:
        tuned = json.load(f)
    fields = ("unbinned", "bin_width", "descending", "strip_cap", "strip_slack", "grid_quarters", "ms")
    assert tuned and all(all(f in v for f in fields) for v in tuned.values())
    # the plan names the strip height each length range takes and how many plans were timed
    assert "heights 1-" in plans[0] and " plans)" in plans[0], plans[0]
    # a new context reads the cache and does not tune again
    ctx2 = sw.Context(5000, 60000, tune_cache=cache)
    refs, db, out = prepared[0]
    ctx2.align(db, refs, scoring_for(batches[0], sw.PREC_INT16, max_read_len=200), out)
    assert "tuned=cached" in ctx2.last_plan()
    assert_same(_host(out), exps[0], "cached plan", keys=SLOTS)
    ctx2.close()


@pytest.mark.parametrize("scoring,mrl", [((2, -3, 5, 2), 194), ((2, -500, 5, 2), 250), ((1, -1, 300, 2), 80),
                                         ((3, -1, 10, 29), 170)],
                         ids=["K6-top", "K4", "K6-gap-terms", "K4-row-offsets"])
def test_ctx_int16_tag_width_and_bias_edges(scoring, mrl):
    """The batched path at the edges of the int16 layout (tag width 6 at the top of
    its range, tag width 4, large gap terms, the largest row offsets at the top of
    tag width 4) on homopolymers with full windows (the largest values) and on
    mixed reads."""
    import dataclasses
    for seed, homo in ((23, True), (24, False)):
        b = wl.random_small_batch(seed, n_reads=150, read_len=(1, mrl), ref_len=(400, 1500), band=12,
                                  homopolymer=homo)
        b = dataclasses.replace(b, scoring=wl.Scoring(*scoring, 12))
        if homo:
            b = dataclasses.replace(b, cal_pos=np.full_like(b.cal_pos, 12), strand=np.full_like(b.strand, 3))
        exp, _ = oracle_align(b)
        res, plan = _ctx_run(b, sw.PREC_INT16, max_read_len=mrl, repeats=2)
        for r in res:
            assert_same(r, exp, f"{scoring} mrl {mrl} homopolymer={homo} ({plan})", keys=SLOTS)
        assert plan.startswith("int16-pairs")


@pytest.mark.parametrize("precision,mode", [(sw.PREC_INT16, sw.MODE_LOCAL), (sw.PREC_INT16, sw.MODE_FINAL_ROW),
                                            (sw.PREC_INT32, sw.MODE_LOCAL)])
def test_ctx_unbinned_plan(tmp_path, precision, mode):
    """The plan without bins (tasks in input order, the plain kernel popping tiles
    from the context's counter), forced through a tune cache entry for the call's
    shape class: same outputs as the oracle, on ragged reads and on one length."""
    import math
    for seed, lens in ((61, (1, 150)), (62, (100, 100))):
        b = wl.random_small_batch(seed, n_reads=400, read_len=lens, band=16, ref_len=(500, 3000))
        exp, _ = oracle_align(b, mode=mode)
        n_tasks = b.n_cals if precision == sw.PREC_INT16 else 2 * b.n_cals
        key = "gfx950/{}{}/L150/b16/t{}".format("int16" if precision == sw.PREC_INT16 else "int32",
                                              "-final-row" if mode == sw.MODE_FINAL_ROW else "",
                                              int(math.floor(math.log2(n_tasks))))
        cache = tmp_path / f"tune{seed}.json"
        cache.write_text('{\n  "%s": {"unbinned": 1, "bin_width": 4, "descending": 1, "strip_cap": 0, '
                         '"strip_slack": 0, "grid_quarters": 4, "ms": 1.0}\n}\n' % key)
        ctx = sw.Context(b.n_reads, b.n_cals, tune_cache=str(cache))
        refs, db, out = _prepare(b)
        for rnd in range(2):  # capture, then replay
            out.score.fill_(-7)
            ctx.align(db, refs, scoring_for(b, precision, max_read_len=150, mode=mode), out)
            plan = ctx.last_plan()
            assert "unbinned" in plan and "tuned=cached" in plan, plan
            assert_same(_host(out), exp, f"seed {seed} round {rnd} {plan}", keys=SLOTS)
        ctx.close()
