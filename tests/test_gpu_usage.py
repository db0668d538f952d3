"""The usage example of the design notes, run end to end on a small batch:
every call it shows works and agrees with the others."""
import pytest
import torch

import paper_1805_00106_amd as sw
from paper_1805_00106_amd import workloads as wl

pytestmark = pytest.mark.gpu


def test_usage_example_flow():
    b = wl.chromosome_scale(n_reads=2000)
    refs = sw.RefSet.from_codes(torch.from_numpy(b.ref_codes).cuda(), b.ref_off, b.ref_len)
    db = sw.DeviceBatch.upload(b)
    sc = sw.Scoring.make(2, -3, 5, 2, band=32, max_read_len=100)
    out = sw.align_batch(db, refs, sc)
    ctx = sw.Context(db.n_reads, db.n_cals)
    out_b = sw.Outputs(db.n_cals)
    ctx.align(db, refs, sc, out_b)
    assert torch.equal(out.score, out_b.score) and torch.equal(out.ref_end, out_b.ref_end)
    best, slot, tied = sw.reduce_best(db, b.n_refs, out.score)
    start, read_start, n_ops, cigar = sw.traceback(db, refs, sc, out, slot[:, 0])
    text = sw.cigar_text(cigar[0].cpu(), int(n_ops[0]))
    assert text and int(n_ops[0]) > 0
    ix = sw.SeedIndex(refs, seed_len=22)
    found = ix.find(db, stride=1, max_cals_per_seed=16, max_read_len=100)
    kept, cal_map = sw.cal_filter(found, bucket_bits=0)
    out2 = sw.align_batch(kept, refs, sc)
    best2, _, _ = sw.reduce_best(kept, b.n_refs, out2.score)
    # the seeds find the planted locus, whose score the synthetic CAL list also reaches
    assert (best2[:, 0] >= best[:, 0]).float().mean().item() > 0.99
    # served: submit host arrays, wait; the same outputs as the plain call
    srv = sw.Server(sc, memory_budget=1 << 30)
    srv.set_refs(refs)
    req = srv.submit_batch(b.subset_reads(range(1000)))
    assert srv.wait(req, 120000)
    n_cals = int(b.cal_ptr[1000])
    assert (req.score == out.score[:2 * n_cals].cpu().numpy()).all()
    assert (req.ref_end == out.ref_end[:2 * n_cals].cpu().numpy()).all()
    srv.close()
    ix.close()
    ctx.close()
