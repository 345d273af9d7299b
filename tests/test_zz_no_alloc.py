"""The allocation-free decode entry point against the ordinary one: the same
words, iteration counts, flags and posteriors on two calls in a row (the
second smaller, so stale scratch contents from the first would show), on a
nine-branch decoder of each code length, and the size limit reported as an
error before anything runs."""
import numpy as np
import pytest

import synth
from tests.helpers import HO_ROWS, ensure_built

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    b = ensure_built()
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return b


def _decoder(B, name, **kw):
    d = B.CODE_DEFS[name]
    c = B.Code(d.m, d.prim, d.t)
    p = B.Pcm.build(c, target_rows=HO_ROWS[name], seed=1)
    return c, p, B.Decoder(c, p, n_branches=9, max_iter=8, **kw)


def _outputs(F, W64, trace_shape=None):
    bits = torch.full((F, W64), -1, dtype=torch.int64, device="cuda")
    iters = torch.full((F,), 255, dtype=torch.uint8, device="cuda")
    flags = torch.full((F,), 255, dtype=torch.uint8, device="cuda")
    tr = torch.zeros(trace_shape, dtype=torch.float32, device="cuda") if trace_shape else None
    return bits, iters, flags, tr


@pytest.mark.parametrize("name,sizes", [("bch63_36", (70_000, 3_001)), ("bch127_64", (50_000, 129)),
                                        ("bch127_99", (4_096, 1))])
def test_noalloc_equals_allocating_entry(B, name, sizes):
    c, p, dec = _decoder(B, name)
    for k, F in enumerate(sizes):
        fr = synth.frames(name, F, 3.0, seed=40 + k)
        llr = torch.from_numpy(fr.llr).cuda()
        d_o = torch.from_numpy(fr.d_o).cuda()
        ld = llr.shape[1]
        trace = (F, 8, ld) if F <= 4096 else None
        ref = _outputs(F, dec.W64, trace)
        ws = torch.empty(max(1, dec.workspace_size(F)), dtype=torch.uint8, device="cuda")
        dec.decode_into(llr, d_o, *ref[:3], y_trace=ref[3], workspace=ws)
        got = _outputs(F, dec.W64, trace)
        dec.decode_noalloc(llr, d_o, *got[:3], y_trace=got[3])
        torch.cuda.synchronize()
        for a, b in zip(ref, got):
            if a is not None:
                assert torch.equal(a, b), (name, F)
        assert int(got[1].min()) >= 1 and int(got[1].max()) <= 8


def test_noalloc_fixed_point_and_limit(B):
    c, p, dec = _decoder(B, "bch63_45", precision=B.FIX8)
    F = 20_000
    fr = synth.frames("bch63_45", F, 3.5, seed=9)
    q = torch.empty((F, 64), dtype=torch.int8, device="cuda")
    B.quantize_llr(torch.from_numpy(fr.llr).cuda(), 63, 4.0, q)
    d_o = torch.from_numpy(fr.d_o).cuda()
    ref = _outputs(F, 1)
    dec.decode_into(q, d_o, *ref[:3], workspace=torch.empty(dec.workspace_size(F), dtype=torch.uint8, device="cuda"))
    got = _outputs(F, 1)
    dec.decode_noalloc(q, d_o, *got[:3])
    torch.cuda.synchronize()
    for a, b in zip(ref[:3], got[:3]):
        assert torch.equal(a, b)
    # beyond the scratch: refused on the host, nothing enqueued
    big = 1 << 23
    assert dec.workspace_size(big) > 17 << 20
    with pytest.raises(B.BchError, match="scratch"):
        dec.decode_noalloc(torch.empty((big, 64), dtype=torch.int8, device="cuda"),
                           torch.zeros(big, dtype=torch.uint8, device="cuda"), torch.empty((big, 1), dtype=torch.int64,
                                                                                           device="cuda"),
                           torch.empty(big, dtype=torch.uint8, device="cuda"),
                           torch.empty(big, dtype=torch.uint8, device="cuda"))
