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


def test_alpha_search_argmin_and_bracket(B, tmp_path, monkeypatch):
    """The alpha search returns the least frame error rate of its table, the
    table brackets it (the grid widened until it does), and the result is
    cached under the code, rows and I_m."""
    from paper_2412_20828_amd import autotune
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "tuning.json"))
    name, rows = "bch127_99", 33
    d = B.CODE_DEFS[name]
    code = B.Code(d.m, d.prim, d.t)
    pcm = B.Pcm.build(code, target_rows=rows, seed=1)
    e = autotune.search_alpha(code, pcm, name, rows, frames=60_000, grid=[0.9, 0.95, 1.0])
    fer = {float(a): v for a, v in e["fer"].items()}
    assert e["fer"]["%.2f" % e["alpha"]] == min(fer.values())
    assert e["bracketed"] and min(fer) < e["alpha"] < max(fer)
    assert e["ebn0"] == autotune.ALPHA_EBN0[127]
    assert autotune.tuned_alpha(name, rows) == e["alpha"]
    assert autotune.tuned_alpha(name, rows, max_iter=4) == 0.75  # nothing cached for I_m = 4


@pytest.mark.parametrize("name,rows", [("bch63_45", 33), ("bch63_36", 122), ("bch127_64", 72), ("bch127_99", 33)])
def test_parity_at_the_tuned_alpha(B, name, rows):
    """Each code decoded with the alpha the search cached (as the workloads'
    --alpha tuned does) against the oracle at that alpha."""
    import oracle
    from paper_2412_20828_amd import autotune
    from tests.helpers import compare_with_oracle, oracle_code, oracle_hopt
    alpha = autotune.tuned_alpha(name, rows)
    assert autotune.alpha_key(name, rows, 8) in autotune.load(), "no cached alpha for %s" % name
    d = B.CODE_DEFS[name]
    code = B.Code(d.m, d.prim, d.t)
    pcm = B.Pcm.build(code, target_rows=rows, seed=1)
    dec = B.Decoder(code, pcm, n_branches=9, alpha=alpha, max_iter=8)
    oc = oracle_code(name)
    H = oracle_hopt(name, rows)
    fr = synth.frames(name, 64 * 5 + 3, 3.0, seed=33)
    bits, it, fl, tr = dec.decode(torch.from_numpy(fr.llr).cuda(), torch.from_numpy(fr.d_o).cuda(), trace=True)
    torch.cuda.synchronize()
    res = oracle.decode_batch(H, oc.Hstd, fr.llr, fr.d_o, 9, alpha, 8, oracle.R1, threads=8, trace=True)
    words = B.unpack_bits(bits.cpu().numpy().view("uint64"), code.N)
    compare_with_oracle(words, it.cpu().numpy(), fl.cpu().numpy(), tr.cpu().numpy(), *res,
                        onestep=(H, oc.Hstd, fr.llr, fr.d_o, 9, alpha))
