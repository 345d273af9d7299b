"""GPU tests of the continuous-batching service and its hybrid NMS + OSD back
end: a request's result is the same alone and served among others."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from tests.helpers import ensure_built, oracle_code

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SERVE_CODES = [("bch63_36", 122), ("bch63_45", 33), ("bch127_64", 72), ("bch127_99", 33)]
NAMES = [n for n, _ in SERVE_CODES]


@pytest.fixture(scope="module")
def S():
    ensure_built()
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2412_20828_amd import serving
    return serving


def make_requests(S, n, seed, max_log2=12, engine_offsets=False):
    """engine_offsets: the requests bring no d_o; the engine draws them."""
    tr = synth.request_trace(n, seed, len(NAMES), 2.0, 5.0, max_log2=max_log2)
    reqs, cws = [], []
    for k, d in enumerate(tr):
        fr = synth.request_frames(NAMES, d, seed, k)
        reqs.append(S.Request(code=d.code, llr=fr.llr, d_o=None if engine_offsets else fr.d_o, rid=k))
        cws.append(fr.codewords)
    return tr, reqs, cws


def packed(cw):
    F, n = cw.shape
    p = np.zeros((F, 128), np.uint8)
    p[:, :n] = cw
    return np.packbits(p, axis=1, bitorder="little").view(np.uint64)


@pytest.mark.parametrize("osd_on,graph", [("device", True), ("device", False), ("host", True)])
def test_served_results_equal_alone(S, osd_on, graph):
    """Requests arriving at 20,000/s (several in flight on separate slots):
    every frame's decision, iteration count and flags equal those of the
    request decoded alone (its code's decoder, then host OSD-2 on its
    failures), with the service's OSD stage on the device or on the host, and
    each slot step replayed from its captured graph (one mixed-code kernel
    for all codes of the batch) or launched code by code.  With OSD on the
    device the requests bring no offsets: the engine draws them through the
    library, keyed by request id, and the alone decode draws the same."""
    eng = S.Engine(SERVE_CODES, slot_frames=8192, n_slots=3, osd_order=2, osd_on=osd_on, osd_threads=4, seed=3,
                   graph=graph, graph_min_frames=1500)
    if graph:
        assert eng.mix.kernel_name(8192) == "mix_63_36_m122_63_45_m33_127_64_m72_127_99_m33"
    tr, reqs, cws = make_requests(S, 48, 7, engine_offsets=osd_on == "device")
    done, wall = S.run_trace(eng, reqs, [d.t / 20000.0 for d in tr])
    assert len(done) == len(reqs) and eng.launches >= 2
    n_osd = 0
    for r, cw in zip(reqs, cws):
        bits, iters, fl = S.decode_alone(eng, r)
        assert np.array_equal(r.bits, bits), r.rid
        assert np.array_equal(r.iters, iters), r.rid
        assert np.array_equal(r.flags, fl), r.rid
        n_osd += int(((r.flags & S.FLAG_OSD) != 0).sum())
        assert r.t_done >= r.t_gpu >= r.t_admit >= r.arrival
    assert n_osd > 0  # the hybrid stage ran
    eng.close()


def test_hybrid_decisions(S):
    """OSD-2 outputs are codewords and equal the oracle's OSD-2 on the same
    channel LLRs; the hybrid's frame errors are at most the NMS stage's."""
    eng = S.Engine(SERVE_CODES, slot_frames=8192, n_slots=2, osd_order=2, osd_threads=4)
    tr, reqs, cws = make_requests(S, 24, 11, max_log2=10)
    for r in reqs:
        eng.submit(r)
    eng.drain()
    nms_err = hyb_err = 0
    for r, cw in zip(reqs, cws):
        name = NAMES[r.code]
        oc = oracle_code(name)
        N = oc.N
        truth = packed(cw)
        err = (r.bits != truth).any(1)
        hyb_err += int(err.sum())
        osd = np.nonzero(r.flags & S.FLAG_OSD)[0]
        if osd.size:
            ob = oracle.osd_batch(oc.G, r.llr[osd], 2)
            assert np.array_equal(packed(ob), r.bits[osd]), r.rid
            words = np.unpackbits(r.bits[osd].view(np.uint8), axis=1, bitorder="little")[:, :N]
            assert not ((words.astype(np.int64) @ oc.Hstd.T.astype(np.int64)) % 2).any()
            nms_err += int(err.sum()) - int(err[osd].sum()) + osd.size  # NMS failed on all of them
        else:
            nms_err += int(err.sum())
    assert hyb_err <= nms_err
    eng.close()


@pytest.mark.parametrize("graph", [True, False])
def test_admission_and_overlap(S, graph):
    """More frames than one slot holds are split over several launches in
    arrival order (each graph replay decodes exactly its batch: batches of
    every size follow each other on a slot); slots are in flight together; an
    oversized request or an unknown code is refused at submission."""
    eng = S.Engine(SERVE_CODES, slot_frames=4096, n_slots=3, osd_order=None, graph=graph, graph_min_frames=1)
    tr, reqs, cws = make_requests(S, 40, 5)
    for r in reqs:
        eng.submit(r)
    max_busy = 0
    done = []
    while eng.busy():
        done += eng.poll()
        max_busy = max(max_busy, sum(s.busy for s in eng.slots))
    assert len(done) == len(reqs)
    assert eng.launches >= sum(r.frames for r in reqs) // 4096
    assert eng.graph_steps == (eng.launches if graph else 0)
    assert max_busy >= 2
    admits = [r.t_admit for r in reqs]
    assert admits == sorted(admits)  # first come, first admitted
    for r in reqs:
        assert not (r.flags & S.FLAG_OSD).any()
        bits, iters, fl = S.decode_alone(eng, r)
        assert np.array_equal(r.bits, bits) and np.array_equal(r.flags, fl)
    big = S.Request(code=0, llr=np.zeros((4097, 64), np.float32), d_o=np.zeros(4097, np.uint8))
    with pytest.raises(Exception):
        eng.submit(big)
    with pytest.raises(Exception):
        eng.submit(S.Request(code=9, llr=np.zeros((1, 128), np.float32), d_o=np.zeros(1, np.uint8)))
    with pytest.raises(S.B.BchError):  # offsets outside [0, d_p)
        eng.submit(S.Request(code=2, llr=np.zeros((2, 128), np.float32), d_o=np.array([0, 42], np.uint8)))


def test_small_steps_skip_the_graph(S):
    """A step below graph_min_frames runs code by code (small-batch kernels),
    a step at or above it replays the slot's graph; both decode every frame
    as alone, and a replay after a larger one leaves the earlier batch's
    frames past its own end untouched."""
    eng = S.Engine(SERVE_CODES, slot_frames=4096, n_slots=1, osd_order=2, osd_threads=4, graph_min_frames=1000)
    tr, reqs, cws = make_requests(S, 12, 21, max_log2=11)
    small = [r for r in reqs if r.frames < 1000][:2]
    big = sorted([r for r in reqs if r.frames >= 200], key=lambda r: -r.frames)
    assert small and big
    eng.submit(small[0])
    eng.drain()
    assert (eng.launches, eng.graph_steps) == (1, 0)
    # a full slot, then a smaller replay on the same slot
    load, n = [], 0
    for r in big:
        if n + r.frames <= 4096:
            load.append(r)
            n += r.frames
    assert n >= 1000
    for r in load:
        eng.submit(r)
    eng.drain()
    assert eng.graph_steps == 1
    taken = {id(r) for r in load}
    last = [r for r in big if id(r) not in taken and r.frames >= 1000][:1] or [load[0]]
    again = S.Request(code=last[0].code, llr=last[0].llr, d_o=last[0].d_o, rid=999)
    eng.submit(again)
    eng.drain()
    assert eng.graph_steps == 2 and eng.launches == 3
    for r in [small[0]] + load + [again]:
        bits, iters, fl = S.decode_alone(eng, r)
        assert np.array_equal(r.bits, bits) and np.array_equal(r.iters, iters) and np.array_equal(r.flags, fl)
    eng.close()


def test_engine_offsets_follow_the_library_draw(S):
    """The engine's offsets of a request equal the oracle's Philox draw under
    the same key (engine seed, request id), and lie in [0, d_p)."""
    eng = S.Engine(SERVE_CODES[:1] + SERVE_CODES[2:3], slot_frames=4096, n_slots=1, osd_order=None, seed=77)
    for code, N, dp in ((0, 63, 21), (1, 127, 42)):
        r = S.Request(code=code, llr=np.zeros((1000, 128), np.float32), rid=12345 + code)
        d = eng.draw_offsets(r)
        assert np.array_equal(d, oracle.draw_offsets(N, 77, 12345 + code, 0, 1000))
        assert d.max() < dp and len(set(d.tolist())) == dp
