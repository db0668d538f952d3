"""GPU tests of the served path: results of every request are bit-identical
alone and in a concurrent mix (continuous batching), match the oracle, survive
admission under a tiny memory budget; oversize requests are rejected and
destroy drains every submitted request.  The served references of the
benchmark are longer than 2^31 bases; the last test serves requests on a
reference longer than 2^32 bases, through small steps (one wavefront per task)
and through the batched path."""
import threading

import numpy as np
import pytest
import torch

import paper_1805_00106_amd as sw
from oracle import oracle as orc
from paper_1805_00106_amd import workloads as wl

pytestmark = pytest.mark.gpu

_REFS = None


def refs_and_pack():
    global _REFS
    if _REFS is None:
        refs = wl.served_references(scale=0.002)        # 6.4 + 5.4 Mbp stand-ins
        pack = wl.concat_aligned(refs)
        _REFS = (refs, pack)
    return _REFS


def requests(n, seed0, sizes=None):
    refs, pack = refs_and_pack()
    rng = np.random.default_rng(seed0)
    sizes = sizes or [int(x) for x in np.clip(np.exp(rng.uniform(0, np.log(400), n)), 1, 400)]
    return [wl.served_request(refs, s, seed0 * 1000 + k, ref_pack=pack) for k, s in enumerate(sizes)]


def make_server(budget=256 << 20, max_step_reads=4096, max_step_cals=60000, depth=0):
    refs, pack = refs_and_pack()
    sc = sw.Scoring.make(2, -3, 5, 2, 32, sw.PREC_AUTO, max_read_len=250)
    srv = sw.Server(sc, memory_budget=budget, max_step_reads=max_step_reads, max_step_cals=max_step_cals,
                    max_steps_in_flight=depth)
    rs = sw.RefSet.from_codes(torch.from_numpy(pack[0]).cuda(), pack[1], pack[2])
    torch.cuda.synchronize()
    srv.set_refs(rs)
    return srv, rs


def outputs(req):
    return (req.score.copy(), req.ref_end.copy(), req.read_end.copy(), req.best_score.copy(), req.best_slot.copy(),
            req.n_tied.copy())


def test_served_matches_oracle():
    reqs = requests(6, 1)
    srv, rs = make_server()
    handles = [srv.submit_batch(b) for b in reqs]
    for h in handles:
        assert srv.wait(h, 60000)
    for b, h in zip(reqs, handles):
        s, r, e, _ = orc.align_batch(b, n_threads=8)
        bs, bl, nt = orc.reduce_best(b.cal_ptr, b.cal_ref, b.n_reads, b.n_refs, s)
        np.testing.assert_array_equal(h.score, s)
        np.testing.assert_array_equal(h.ref_end, r)
        np.testing.assert_array_equal(h.read_end, e)
        np.testing.assert_array_equal(h.best_score, bs.reshape(-1))
        np.testing.assert_array_equal(h.best_slot, bl.reshape(-1))
        np.testing.assert_array_equal(h.n_tied, nt.reshape(-1))
    srv.close()


def test_alone_equals_in_the_mix():
    reqs = requests(24, 2)
    srv, rs = make_server(max_step_reads=1500, max_step_cals=20000)
    alone = []
    for b in reqs:                         # one at a time: each request is alone on the GPU
        h = srv.submit_batch(b)
        assert srv.wait(h, 60000)
        alone.append(outputs(h))
    steps_alone = srv.stats()["steps"]
    # the same requests arriving concurrently from two threads, back to back, so
    # that requests arrive while earlier ones are on the GPU and share its steps
    mixed = [None] * len(reqs)
    prepared = [srv.prepare_batch(b) for b in reqs]

    def feeder(idx, seed):
        for k in idx:
            mixed[k] = srv.submit_prepared(prepared[k])

    th = [threading.Thread(target=feeder, args=(list(range(i, len(reqs), 2)), i)) for i in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for h in mixed:
        assert srv.wait(h, 60000)
    stats = srv.stats()
    for k, (a, h) in enumerate(zip(alone, mixed)):
        for x, y in zip(a, outputs(h)):
            np.testing.assert_array_equal(x, y, err_msg=f"request {k}")
    # requests shared steps: fewer steps than requests in the mixed phase
    assert stats["steps"] - steps_alone < len(reqs), (stats["steps"], steps_alone)
    srv.close()


@pytest.mark.parametrize("depth", [1, 3])
def test_fixed_steps_in_flight_match_oracle(depth):
    """Fixed step depths (the other tests run the adaptive default): requests
    from two threads share steps, and each matches the oracle."""
    reqs = requests(10, 7)
    srv, rs = make_server(max_step_reads=1500, max_step_cals=20000, depth=depth)
    prepared = [srv.prepare_batch(b) for b in reqs]

    def feeder(idx):
        for k in idx:
            srv.submit_prepared(prepared[k])

    th = [threading.Thread(target=feeder, args=(list(range(i, len(reqs), 2)),)) for i in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for h in prepared:
        assert srv.wait(h, 60000)
    for k, (b, h) in enumerate(zip(reqs, prepared)):
        s, r, e, _ = orc.align_batch(b, n_threads=8)
        bs, bl, nt = orc.reduce_best(b.cal_ptr, b.cal_ref, b.n_reads, b.n_refs, s)
        for x, y in zip(outputs(h), (s, r, e, bs.reshape(-1), bl.reshape(-1), nt.reshape(-1))):
            np.testing.assert_array_equal(x, y, err_msg=f"request {k}, depth {depth}")
    srv.close()


def test_tiny_budget_admission_and_rejection():
    reqs = requests(10, 3, sizes=[300] * 10)
    srv, rs = make_server(budget=1 << 20)                  # fits only a few requests at a time
    hs = [srv.submit_batch(b) for b in reqs]
    for h in hs:
        assert srv.wait(h, 60000)
    for b, h in zip(reqs, hs):
        s, r, e, _ = orc.align_batch(b, n_threads=8)
        np.testing.assert_array_equal(h.score, s)
        np.testing.assert_array_equal(h.ref_end, r)
    big = requests(1, 4, sizes=[3500])[0]
    with pytest.raises(sw.SwError) as ei:
        srv.submit_batch(big)
    assert ei.value.code == -9
    srv.close()


def test_destroy_drains_submitted_requests():
    reqs = requests(8, 5)
    srv, rs = make_server()
    hs = [srv.submit_batch(b) for b in reqs]
    srv.close()                                              # returns after every request is done
    for h in hs:
        assert (h.score != -7).all() and (h.read_end != -7).all()


def test_latency_timestamps_are_ordered():
    reqs = requests(5, 6)
    srv, rs = make_server()
    hs = [srv.submit_batch(b) for b in reqs]
    for h in hs:
        assert srv.wait(h, 60000)
        state, t_sub, t_adm, t_done = srv.info(h)
        assert state == 3 and t_sub <= t_adm <= t_done
    srv.close()


@pytest.mark.parametrize("precision", [sw.PREC_AUTO, sw.PREC_INT16])
def test_served_long_reference(precision):
    """Requests on a reference longer than 2^32 bases.  With AUTO precision a step
    of at most 16 CALs per compute unit takes the plain call, whose AUTO kernel
    runs one wavefront per task; int16 keeps every step on the batched path."""
    from tests.test_gpu_long_reference import batch_and_refs
    b, refs, exp = batch_and_refs()
    sc = sw.Scoring.make(2, -3, 5, 2, b.scoring.band, precision, max_read_len=int(b.read_len.max()))
    srv = sw.Server(sc, memory_budget=64 << 20, max_step_reads=4096, max_step_cals=60000)
    srv.set_refs(refs)
    parts = np.array_split(np.arange(b.n_reads), 4)
    subs = [b.subset_reads(idx) for idx in parts]
    hs = [srv.submit_batch(x) for x in subs]
    for h in hs:
        assert srv.wait(h, 120000)
    for idx, x, h in zip(parts, subs, hs):
        s, r, e, _ = orc.align_batch(x, n_threads=8)
        bs, bl, nt = orc.reduce_best(x.cal_ptr, x.cal_ref, x.n_reads, x.n_refs, s)
        np.testing.assert_array_equal(h.score, s)
        np.testing.assert_array_equal(h.ref_end, r)
        np.testing.assert_array_equal(h.read_end, e)
        np.testing.assert_array_equal(h.best_score, bs.reshape(-1))
        np.testing.assert_array_equal(h.best_slot, bl.reshape(-1))
        np.testing.assert_array_equal(h.n_tied, nt.reshape(-1))
    srv.close()
