"""The autotuner (run on an MI355X): it times the frames-per-wave layouts and
grids of a decoder, caches the fastest, and a decoder built from the cache
decodes every frame exactly as the default one does."""
import pytest

import synth
from tests.helpers import ensure_built

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    b = ensure_built()
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return b


@pytest.mark.parametrize("prec", ["fp32", "fix8"])
def test_tune_layout_cache_and_results(B, tmp_path, monkeypatch, prec):
    from paper_2412_20828_amd import autotune
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "tuning.json"))
    name, rows = "bch63_45", 33
    d = B.CODE_DEFS[name]
    code = B.Code(d.m, d.prim, d.t)
    pcm = B.Pcm.build(code, target_rows=rows, seed=1)
    precision = B.FIX8 if prec == "fix8" else B.FP32
    best, out = autotune.tune_layout(code, pcm, name, rows, precision, frames=200_000, reps=1)
    assert len(out) == (2 if prec == "fix8" else 1)
    assert best["waves_per_cu"] in autotune.WAVES
    assert best["frames_per_s"] == max(b["frames_per_s"] for b, _ in out)
    assert isinstance(best["packed16"], bool) and (prec == "fix8" or not best["packed16"])
    cached = autotune.load()[autotune.key(name, rows, precision, 9, autotune._gpu_name())]
    assert cached == best
    tuned = autotune.tuned_decoder(code, pcm, name, rows, precision=precision)
    assert bool(tuned.flags & B.PACKED16) == best["packed16"]
    plain = B.Decoder(code, pcm, n_branches=9, max_iter=8, precision=precision)
    fr = synth.frames(name, 20_000 + 17, 3.0, seed=21)
    llr = torch.from_numpy(fr.llr).cuda()
    if prec == "fix8":
        q = torch.empty(llr.shape, dtype=torch.int8, device="cuda")
        B.quantize_llr(llr, code.N, 4.0, q)
        llr = q
    d_o = torch.from_numpy(fr.d_o).cuda()
    a = tuned.decode(llr, d_o)
    b = plain.decode(llr, d_o)
    torch.cuda.synchronize()
    for x, y in zip(a[:3], b[:3]):
        assert torch.equal(x, y)
