"""The C-ABI library: it loads without a GPU, exports every entry point the
public header declares, and its host-side constructions (code matrices, H_o,
automorphism maps, OSD) agree exactly with the oracle."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from tests.helpers import HO_ROWS, ensure_built, header_symbols, oracle_code, oracle_hopt


@pytest.fixture(scope="module")
def B():
    return ensure_built()


def test_exports_every_declared_symbol(B):
    L = ctypes.CDLL(B.LIB_PATH)
    syms = header_symbols()
    assert len(syms) >= 18
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) == set(B.SYMBOLS)


@pytest.mark.parametrize("name", list(synth.CODES))
def test_code_matrices_match_oracle(B, name):
    d = B.CODE_DEFS[name]
    c = B.Code(d.m, d.prim, d.t)
    g, G, H = c.export()
    oc = oracle_code(name)
    assert (c.N, c.K) == (oc.N, oc.K)
    assert np.array_equal(g, oc.g) and np.array_equal(G, oc.G) and np.array_equal(H, oc.Hstd)


@pytest.mark.parametrize("name", ["bch63_45", "bch63_36", "bch127_99"])
def test_hopt_bit_exact_with_oracle(B, name):
    d = B.CODE_DEFS[name]
    c = B.Code(d.m, d.prim, d.t)
    p = B.Pcm.build(c, target_rows=HO_ROWS[name], seed=1)
    assert np.array_equal(p.dense(), oracle_hopt(name))
    assert p.c4 == oracle.count_4cycles(p.dense())


def test_hopt_beta_form_and_seed_bit_exact(B):
    d = B.CODE_DEFS["bch63_45"]
    c = B.Code(d.m, d.prim, d.t)
    oc = oracle_code("bch63_45")
    for beta, seed in [(2, 3), (5, 11)]:
        p = B.Pcm.build(c, beta=beta, seed=seed)
        H, mr1, used = oracle.build_hopt(oc, beta=beta, seed=seed)
        assert np.array_equal(p.dense(), H) and p.Mr1 == mr1 and p.seed_used == used


def test_pcm_import_validates(B):
    d = B.CODE_DEFS["bch63_45"]
    c = B.Code(d.m, d.prim, d.t)
    H = oracle_hopt("bch63_45")
    p = B.Pcm.from_dense(c, H)
    assert p.M == 33 and np.array_equal(p.dense(), H)
    bad = H.copy()
    bad[0, 0] ^= 1
    with pytest.raises(B.BchError):
        B.Pcm.from_dense(c, bad)
    with pytest.raises(B.BchError):
        B.Pcm.from_dense(c, H[:10])  # rank below N-K


@pytest.mark.parametrize("N,Bn", [(63, 9), (63, 3), (127, 9), (127, 1)])
def test_automorphisms_match_oracle(B, N, Bn):
    for d_o in ([0] if Bn == 1 else [0, 7, (21 if N == 63 else 42) - 1]):
        assert np.array_equal(B.make_automorphisms(N, Bn, d_o), oracle.branch_maps(N, Bn, d_o))
    with pytest.raises(B.BchError):
        B.make_automorphisms(N, 9, 50)


@pytest.mark.parametrize("name", ["bch63_45", "bch127_99"])
def test_host_osd_matches_oracle(B, name):
    d = B.CODE_DEFS[name]
    c = B.Code(d.m, d.prim, d.t)
    oc = oracle_code(name)
    fr = synth.frames(name, 120, 2.0, seed=5)
    for order in (0, 1, 2):
        words = B.unpack_bits(B.osd_decode(c, fr.llr, order, n_threads=4), c.N)
        ref = oracle.osd_batch(oc.G, fr.llr, order)
        assert (words == ref).all(1).mean() == 1.0


def test_host_osd_skip_leaves_frames(B):
    d = B.CODE_DEFS["bch63_45"]
    c = B.Code(d.m, d.prim, d.t)
    fr = synth.frames("bch63_45", 16, 2.0, seed=6)
    bits = np.full((16, 1), 12345, np.uint64)
    skip = np.zeros(16, np.uint8)
    skip[::2] = 1
    B.osd_decode(c, fr.llr, 2, skip=skip, bits=bits)
    assert (bits[::2, 0] == 12345).all() and (bits[1::2, 0] != 12345).any()


def test_argument_errors_are_reported(B):
    with pytest.raises(B.BchError):
        B.Code(6, 0b1000001, 3)  # not primitive
    with pytest.raises(B.BchError):
        B.Code(9, 0b1000010001, 3)  # N > 127
    d = B.CODE_DEFS["bch63_45"]
    c = B.Code(d.m, d.prim, d.t)
    p = B.Pcm.standard(c)
    assert p.M == 18 and p.E == 18 * 24


@pytest.mark.parametrize("N", [63, 127, 15])
def test_host_offset_draw_matches_oracle(B, N):
    for seed, key_hi, base, F in [(0, 0, 0, 1000), (2 ** 63 + 5, 77, 123456789, 300), (1, (3 << 32) | 9, 5, 1)]:
        got = B.draw_offsets(N, seed, key_hi, base, F)
        assert np.array_equal(got, oracle.draw_offsets(N, seed, key_hi, base, F))
    with pytest.raises(B.BchError):
        B.draw_offsets(N, 0, 0, -1, 4)


@pytest.mark.parametrize("N", [63, 127])
def test_keyed_offset_draw_matches_the_oracle_per_key(B, N):
    """One call over several keys equals the oracle's draw of each key's frames
    from uid 0, key after key (empty keys included)."""
    rng = np.random.default_rng(N)
    keys = rng.integers(0, 2 ** 63, 40, dtype=np.uint64)
    counts = rng.integers(0, 300, 40).astype(np.int64)
    counts[[3, 17]] = 0
    got = B.draw_offsets_keys(N, 2 ** 63 + 11, keys, counts)
    want = np.concatenate([oracle.draw_offsets(N, 2 ** 63 + 11, int(k), 0, int(c)) for k, c in zip(keys, counts)])
    assert np.array_equal(got, want)
    assert B.draw_offsets_keys(N, 1, keys[:0], counts[:0]).size == 0
    with pytest.raises(B.BchError):
        B.draw_offsets_keys(N, 0, keys[:2], np.array([4, -1], np.int64), out=np.zeros(3, np.uint8))


def test_synth_offsets_follow_the_library_draw(B):
    fr = synth.frames("bch63_36", 500, 3.0, seed=12, block=4)
    assert np.array_equal(fr.d_o, B.draw_offsets(63, 12, synth.offset_key("bch63_36", 4), 0, 500))


@pytest.mark.parametrize("name", list(HO_ROWS))
def test_pcm_stats_match_oracle(B, name):
    d = B.CODE_DEFS[name]
    c = B.Code(d.m, d.prim, d.t)
    for p in (B.Pcm.standard(c), B.Pcm.build(c, target_rows=HO_ROWS[name], seed=1)):
        got = p.stats()
        want = oracle.pcm_stats(p.dense())
        assert (got["M"], got["E"], got["c4"]) == (want["M"], want["edges"], want["c4"])
        for k in ("col_range", "row_range"):
            assert tuple(got[k]) == tuple(want[k])
        for k in ("col_mean", "col_std", "row_mean", "row_std"):
            assert abs(got[k] - want[k]) < 1e-12


def test_engine_draw_segment_equals_per_request_draws(B):
    """The serving engine's per-code draw (one keyed library call) writes each
    request's offsets where the per-request draw would, both for requests that
    lie back to back and for requests with caller-given offsets between them."""
    import types

    from paper_2412_20828_amd import serving
    eng = types.SimpleNamespace(codes=[(types.SimpleNamespace(N=127), None)], seed=31)
    sizes = [5, 300, 1, 77, 64]
    reqs = [types.SimpleNamespace(rid=1000 + k, frames=F) for k, F in enumerate(sizes)]
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    hd = np.full(sum(sizes), 0xff, np.uint8)
    serving.Engine._draw_segment(eng, 0, list(zip(reqs, offs)), hd)  # back to back: in place
    want = np.concatenate([B.draw_offsets(127, 31, r.rid, 0, r.frames) for r in reqs])
    assert np.array_equal(hd, want)
    hd[:] = 0xff
    gap = [(r, o) for k, (r, o) in enumerate(zip(reqs, offs)) if k != 2]  # request 2 brings its own
    serving.Engine._draw_segment(eng, 0, gap, hd)
    for r, o in gap:
        assert np.array_equal(hd[o:o + r.frames], B.draw_offsets(127, 31, r.rid, 0, r.frames))
    assert (hd[offs[2]:offs[2] + sizes[2]] == 0xff).all()
