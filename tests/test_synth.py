"""The seeded workload generator: valid codewords, LLR definition (eq. 1),
per-block reproducibility."""
import numpy as np
import pytest

import oracle
import synth


@pytest.mark.parametrize("name", list(synth.CODES))
def test_codewords_satisfy_oracle_parity_checks(name):
    m, p, t = synth.CODES[name]
    c = oracle.Code(m, p, t)
    spec = synth.code(name)
    assert (spec.N, spec.K) == (c.N, c.K)
    assert list(spec.g) == [int(x) for x in c.g]
    fr = synth.frames(name, 500, 3.0, seed=3)
    assert not ((fr.codewords.astype(int) @ c.Hstd.T.astype(int)) % 2).any()
    # systematic: message bits are the last K columns and are not all zero
    assert fr.codewords[:, c.N - c.K:].any()


def test_llr_definition_and_padding():
    spec = synth.code("bch63_45")
    fr = synth.frames("bch63_45", 2000, 3.0, seed=1)
    assert fr.llr.dtype == np.float32 and fr.llr.shape == (2000, 64)
    assert not fr.llr[:, 63:].any()
    s2 = synth.sigma2_of(3.0, spec.rate)
    y = fr.llr[:, :63] * s2 / 2.0
    noise = y - (1 - 2 * fr.codewords.astype(np.float64))
    assert abs(noise.mean()) < 0.02
    assert abs(noise.var() / s2 - 1.0) < 0.03
    assert fr.d_o.max() < 21 and fr.d_o.min() >= 0


def test_blocks_are_reproducible_and_independent():
    a = synth.frames("bch127_99", 100, 4.0, seed=9, block=2)
    b = synth.frames("bch127_99", 100, 4.0, seed=9, block=2)
    c = synth.frames("bch127_99", 100, 4.0, seed=9, block=3)
    assert np.array_equal(a.llr, b.llr) and np.array_equal(a.d_o, b.d_o)
    assert not np.array_equal(a.llr, c.llr)


def test_per_frame_snr():
    e = np.linspace(1.5, 5.0, 64)
    fr = synth.frames("bch63_36", 64, e, seed=2)
    assert np.allclose(fr.ebn0, e)


def test_mixed_frames_place_each_code_at_its_positions():
    names = ["bch127_64", "bch127_99", "bch63_36"]
    mf = synth.mixed_frames(names, 500, 5, [0.5, 0.25, 0.25], 1.5, 5.0)
    assert mf.llr.shape == (500, 128) and mf.code_idx.shape == (500,)
    assert set(np.unique(mf.code_idx)) == {0, 1, 2}
    for k, n in enumerate(names):
        sel = np.nonzero(mf.code_idx == k)[0]
        fr = synth.frames(n, sel.size, mf.ebn0[sel], 5)
        assert np.array_equal(mf.llr[sel, :fr.llr.shape[1]], fr.llr)
        assert (mf.d_o[sel] < synth.code(n).d_p).all()
        N = synth.code(n).N
        assert not mf.llr[sel, N:].any() and not mf.codewords[sel, N:].any()
    assert (mf.ebn0 >= 1.5).all() and (mf.ebn0 <= 5.0).all()


def test_request_trace_distribution():
    tr = synth.request_trace(20000, 1, 4, 2.0, 5.0)
    t = np.array([d.t for d in tr])
    gaps = np.diff(t)
    assert abs(gaps.mean() - 1.0) < 0.03 and abs(gaps.std() - 1.0) < 0.05   # exponential, rate 1
    sz = np.array([d.frames for d in tr])
    assert sz.min() >= 1 and sz.max() <= 4096
    lg = np.log2(sz[sz > 8])                                                  # log-uniform body
    assert abs(np.mean(lg) - (3 + 12) / 2) < 0.15
    assert set(np.unique([d.code for d in tr])) == {0, 1, 2, 3}
    e = np.array([d.ebn0 for d in tr])
    assert e.min() >= 2.0 and e.max() <= 5.0
    fr = synth.request_frames(["bch63_36", "bch63_45", "bch127_64", "bch127_99"], tr[5], 1, 5)
    assert fr.llr.shape[0] == tr[5].frames


def test_threaded_encoding_is_deterministic_with_torch_loaded():
    """Messages encoded side by side in threads (as the benchmark's generator
    threads do) give the codewords of a one-at-a-time encoding, and every one
    is valid.  With torch loaded, concurrent float BLAS calls from numpy
    threads have returned corrupted rows; the encoder is integer-only for that
    reason."""
    import torch  # noqa: F401  (loaded for its effect on the BLAS/OpenMP runtime)
    from concurrent.futures import ThreadPoolExecutor
    m, p, t = synth.CODES["bch127_99"]
    c = oracle.Code(m, p, t)
    spec = synth.code("bch127_99")
    msgs = [np.random.default_rng(k).integers(0, 2, (300000, spec.K), dtype=np.uint8) for k in range(8)]
    with ThreadPoolExecutor(8) as ex:
        par = list(ex.map(lambda x: synth.encode(spec, x), msgs))
    for x, cw in zip(msgs, par):
        assert np.array_equal(cw, synth.encode(spec, x))
        assert np.array_equal(cw[:, c.N - c.K:], x)
        assert not ((cw[:4096].astype(int) @ c.Hstd.T.astype(int)) % 2).any()
