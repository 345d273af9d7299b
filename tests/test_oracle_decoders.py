"""Pins for the oracle's decoders: hand-worked iterations on the (7,4) code,
literal vs min1/min2 forms, exact invariances of min-sum (scale, channel
symmetry), the branch merge of the enhanced decoder rebuilt from one-branch
runs, the fixed-point variant, and OSD against brute-force ML."""
import json
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")
PRIMS = {3: 0b1011, 4: 0b10011, 5: 0b100101, 6: 0b1000011, 7: 0b10001001}


@pytest.fixture(scope="module")
def hand():
    return json.load(open(os.path.join(GOLD, "hamming74_hand.json")))


def test_hamming_matrix_matches_code(hand):
    c = oracle.Code(3, PRIMS[3], 1)
    assert np.array_equal(c.Hstd, np.array(hand["H"], dtype=np.uint8))


@pytest.mark.parametrize("fn", [oracle.nms_literal, oracle.nms_fast])
@pytest.mark.parametrize("key,mode", [("plain_nms_R3", oracle.R3), ("restart_R1", oracle.R1)])
def test_hand_worked_iterations(hand, fn, key, mode):
    H = np.array(hand["H"], dtype=np.uint8)
    exp = hand[key]
    maps = oracle.branch_maps(7, 1, 0)
    r = fn(H, maps, np.array(hand["L"]), hand["alpha"], exp["max_iter"], mode, H, trace=True)
    assert r["iters"] == exp["iters"] and r["converged"] == exp["converged"]
    assert np.array_equal(r["y_trace"], np.array(exp["y_trace"]))  # dyadic: exact
    assert list(r["c_hat"]) == exp["c_hat"]


def test_hand_worked_fixed_point(hand):
    H = np.array(hand["H"], dtype=np.uint8)
    exp = hand["fixed_R1"]
    maps = oracle.branch_maps(7, 1, 0)
    r = oracle.nms_fixed(H, maps, np.array(exp["q"]), exp["max_iter"], oracle.R1, H, trace=True)
    assert r["iters"] == exp["iters"] and r["converged"] == exp["converged"]
    assert np.array_equal(r["y_trace"], np.array(exp["y_trace"]))
    assert list(r["c_hat"]) == exp["c_hat"]


def setup(NK=(63, 45), rows=33, seed=1):
    m = 6 if NK[0] == 63 else 7
    t = {(63, 45): 3, (63, 36): 5, (127, 99): 4, (127, 64): 10}[NK]
    c = oracle.Code(m, PRIMS[m], t)
    H, _, _ = oracle.build_hopt(c, target_rows=rows, seed=seed)
    return c, H


def noisy(c, rng, ebn0, n=1, codeword=True):
    sigma2 = 1.0 / (2 * c.K / c.N * 10 ** (ebn0 / 10))
    out = []
    cws = []
    for _ in range(n):
        msg = rng.integers(0, 2, c.K) if codeword else np.zeros(c.K, dtype=int)
        cw = (msg @ c.G.astype(int)) % 2
        y = (1 - 2 * cw) + np.sqrt(sigma2) * rng.standard_normal(c.N)
        out.append(2 * y / sigma2)
        cws.append(cw)
    return np.array(out), np.array(cws)


@pytest.mark.parametrize("mode", [oracle.R1, oracle.R2, oracle.R3])
@pytest.mark.parametrize("B", [1, 3, 9])
def test_literal_equals_fast(mode, B):
    c, H = setup()
    rng = np.random.default_rng(10 + mode + B)
    L, _ = noisy(c, rng, 2.5, n=6)
    for k, l in enumerate(L):
        maps = oracle.branch_maps(63, B, k % 21)
        a = oracle.nms_literal(H, maps, l, 0.75, 6, mode, c.Hstd, trace=True)
        b = oracle.nms_fast(H, maps, l, 0.75, 6, mode, c.Hstd, trace=True)
        assert a["iters"] == b["iters"] and np.array_equal(a["c_hat"], b["c_hat"])
        if mode == oracle.R2:
            np.testing.assert_allclose(a["y_trace"], b["y_trace"], rtol=1e-12, atol=1e-12)
        else:  # min-sum values are exact in both forms; sums run in the same order
            assert np.array_equal(a["y_trace"], b["y_trace"])


@pytest.mark.parametrize("mode", [oracle.R1, oracle.R2, oracle.R3])
def test_scale_invariance(mode):
    """Min-sum is positively homogeneous: 2^k L gives exactly 2^k messages (the
    choice of sigma^2 in eq. 1 does not matter)."""
    c, H = setup()
    rng = np.random.default_rng(3)
    L, _ = noisy(c, rng, 3.0, n=5)
    for k, l in enumerate(L):
        maps = oracle.branch_maps(63, 9, (5 * k) % 21)
        a = oracle.nms_fast(H, maps, l, 0.75, 8, mode, c.Hstd, trace=True)
        b = oracle.nms_fast(H, maps, l * 8.0, 0.75, 8, mode, c.Hstd, trace=True)
        assert a["iters"] == b["iters"] and np.array_equal(a["c_hat"], b["c_hat"])
        assert np.array_equal(a["y_trace"] * 8.0, b["y_trace"])


@pytest.mark.parametrize("mode", [oracle.R1, oracle.R3])
def test_channel_symmetry(mode):
    """Decoding L * (1 - 2c) for a codeword c gives the decision of L xor c and
    exactly sign-flipped messages (every check row and every branch map
    preserves the code)."""
    c, H = setup()
    rng = np.random.default_rng(4)
    L, _ = noisy(c, rng, 3.0, n=5, codeword=False)
    for k, l in enumerate(L):
        msg = rng.integers(0, 2, c.K)
        cw = (msg @ c.G.astype(int)) % 2
        s = 1 - 2 * cw
        maps = oracle.branch_maps(63, 9, (3 * k) % 21)
        a = oracle.nms_fast(H, maps, l, 0.75, 8, mode, c.Hstd, trace=True)
        b = oracle.nms_fast(H, maps, l * s, 0.75, 8, mode, c.Hstd, trace=True)
        assert a["iters"] == b["iters"]
        assert np.array_equal(a["c_hat"] ^ cw.astype(np.uint8), b["c_hat"])
        assert np.array_equal(a["y_trace"] * s, b["y_trace"])


@pytest.mark.parametrize("B", [1, 9])
def test_noiseless_codeword_converges_first_iteration(B):
    c, H = setup()
    rng = np.random.default_rng(5)
    for _ in range(4):
        cw = (rng.integers(0, 2, c.K) @ c.G.astype(int)) % 2
        L = 4.0 * (1 - 2 * cw)
        for mode in (oracle.R1, oracle.R2, oracle.R3):
            r = oracle.nms_fast(H, oracle.branch_maps(63, B, 7), L, 0.75, 8, mode, c.Hstd)
            assert r["converged"] and r["iters"] == 1
            assert np.array_equal(r["c_hat"], cw.astype(np.uint8))


def test_merge_rebuilt_from_single_branch_runs():
    """One enhanced iteration (R1) equals L + (1/B) sum_b pi_b^-1(S_b), where
    S_b comes from a one-branch run on the gathered input L[map_b] and the
    inverse permutation is applied here with plain numpy indexing."""
    c, H = setup()
    rng = np.random.default_rng(6)
    L, _ = noisy(c, rng, 2.0, n=4)
    ident = oracle.branch_maps(63, 1, 0)
    for k, l in enumerate(L):
        maps = oracle.branch_maps(63, 9, (7 * k + 2) % 21)
        full = oracle.nms_literal(H, maps, l, 0.75, 1, oracle.R1, c.Hstd, trace=True)
        acc = np.zeros(63)
        for mp in maps:
            Yb = l[mp]
            one = oracle.nms_literal(H, ident, Yb, 0.75, 1, oracle.R1, c.Hstd, trace=True)
            Sb = one["y_trace"][0] - Yb
            acc[mp] += Sb
        np.testing.assert_allclose(full["y_trace"][0], l + acc / 9.0, rtol=1e-12, atol=1e-12)


def test_identical_branches_reduce_to_one_branch():
    c, H = setup()
    rng = np.random.default_rng(7)
    L, _ = noisy(c, rng, 3.0, n=3)
    ident = oracle.branch_maps(63, 1, 0)
    nine = np.repeat(ident, 9, axis=0)
    for l in L:
        a = oracle.nms_fast(H, ident, l, 0.75, 4, oracle.R1, c.Hstd, trace=True)
        b = oracle.nms_fast(H, nine, l, 0.75, 4, oracle.R1, c.Hstd, trace=True)
        assert a["iters"] == b["iters"]
        np.testing.assert_allclose(a["y_trace"], b["y_trace"], rtol=1e-14)


def test_enhanced_beats_plain_nms_statistically():
    """The paper's claim: the automorphism merge improves on plain NMS on the
    same H_o.  300 frames at 3 dB; R1 with nine branches must fail less."""
    c, H = setup()
    rng = np.random.default_rng(8)
    L, cw = noisy(c, rng, 3.0, n=300)
    llr = np.zeros((300, 64), np.float32)
    llr[:, :63] = L
    d_o = rng.integers(0, 21, 300).astype(np.uint8)
    ch1, _, _ = oracle.decode_batch(H, c.Hstd, llr, d_o, 1, 0.75, 4, oracle.R3)
    ch9, _, _ = oracle.decode_batch(H, c.Hstd, llr, d_o, 9, 0.75, 4, oracle.R1)
    fer1 = (ch1 != cw).any(1).mean()
    fer9 = (ch9 != cw).any(1).mean()
    assert fer9 < 0.6 * fer1


# --------------------------------------------------------------- fixed point
def test_quantize_rounding_and_clamp():
    below = float(np.nextafter(np.float32(0.125), np.float32(0)))  # x 4 = 0.49999997: rounds to 0
    L = np.array([0.125, 0.124, -0.125, -0.126, 31.6, -40.0, 0.0, 31.874, below, -below], dtype=np.float32)
    q = oracle.quantize(L, 4.0)
    assert list(q) == [1, 0, -1, -1, 126, -127, 0, 127, 0, 0]


def test_fixed_point_saturation_and_range():
    c, H = setup()
    rng = np.random.default_rng(9)
    L, _ = noisy(c, rng, 2.0, n=20)
    for k, l in enumerate(L):
        q = oracle.quantize(l.astype(np.float32), 4.0)
        r = oracle.nms_fixed(H, oracle.branch_maps(63, 9, k % 21), q, 8, oracle.R1, c.Hstd,
                             trace=True)
        assert np.abs(r["y_trace"]).max() <= 32767
        # decisions follow the sign of the last posterior
        assert np.array_equal(r["c_hat"], (r["y_trace"][-1] < 0).astype(np.uint8))


def test_fixed_point_channel_symmetry_without_zeros():
    c, H = setup()
    rng = np.random.default_rng(11)
    L, _ = noisy(c, rng, 3.0, n=20, codeword=False)
    checked = 0
    for k, l in enumerate(L):
        q = oracle.quantize(l.astype(np.float32), 4.0)
        cw = ((rng.integers(0, 2, c.K) @ c.G.astype(int)) % 2).astype(np.uint8)
        s = (1 - 2 * cw.astype(np.int32))
        maps = oracle.branch_maps(63, 9, k % 21)
        a = oracle.nms_fixed(H, maps, q, 8, oracle.R1, c.Hstd, trace=True)
        if (q == 0).any() or (a["y_trace"] == 0).any():
            continue  # sgn(0) = +1 breaks the symmetry at exact zeros
        b = oracle.nms_fixed(H, maps, (q * s).astype(np.int8), 8, oracle.R1, c.Hstd, trace=True)
        assert a["iters"] == b["iters"]
        assert np.array_equal(a["y_trace"] * s, b["y_trace"])
        assert np.array_equal(a["c_hat"] ^ cw, b["c_hat"])
        checked += 1
    assert checked >= 5


def test_fixed_point_tracks_float_decisions():
    """With alpha = 3/4 rounded and int8 messages the decoder is only close to
    the float one; at 4 dB their frame outcomes agree on the large majority."""
    c, H = setup()
    rng = np.random.default_rng(12)
    L, cw = noisy(c, rng, 4.0, n=200)
    llr = np.zeros((200, 64), np.float32)
    llr[:, :63] = L
    d_o = rng.integers(0, 21, 200).astype(np.uint8)
    chf, _, _ = oracle.decode_batch(H, c.Hstd, llr, d_o, 9, 0.75, 8, oracle.R1)
    q = oracle.quantize(llr, 4.0)
    chq, _, _ = oracle.decode_batch(H, c.Hstd, q, d_o, 9, 0.75, 8, oracle.R1,
                                    kind=oracle.KIND_FIXED)
    okf = ~(chf != cw).any(1)
    okq = ~(chq != cw).any(1)
    assert (okf == okq).mean() > 0.95


# ---------------------------------------------------------------------- OSD
@pytest.mark.parametrize("m,t", [(3, 1), (4, 2), (4, 3), (5, 3)])
def test_osd_full_order_is_ml(m, t):
    c = oracle.Code(m, PRIMS[m], t)
    rng = np.random.default_rng(m * 10 + t)
    for _ in range(30):
        L = rng.standard_normal(c.N) * 2 + 0.5
        assert np.array_equal(oracle.osd(c.G, L, c.K), oracle.ml_bruteforce(c.G, L))


def test_osd2_finds_ml_within_two_mrb_flips():
    c = oracle.Code(5, PRIMS[5], 3)  # (31,16)
    rng = np.random.default_rng(13)
    hits = 0
    for _ in range(60):
        L = rng.standard_normal(c.N) * 1.5 + 1.0
        ml = oracle.ml_bruteforce(c.G, L)
        o2 = oracle.osd(c.G, L, 2)
        z = (L < 0).astype(np.uint8)
        r = np.abs(L)
        order = sorted(range(c.N), key=lambda i: (-r[i], i))
        # most reliable basis by greedy independence
        basis, rows = [], np.zeros((0, c.K), dtype=np.uint8)
        for p in order:
            cand = np.vstack([rows, c.G[:, p][None]])
            if oracle.rank(cand) > rows.shape[0]:
                rows = cand
                basis.append(p)
            if len(basis) == c.K:
                break
        flips = int((ml[basis] != z[basis]).sum())
        d = lambda w: r[w != z].sum()
        assert d(o2) >= d(ml) - 1e-12
        if flips <= 2:
            assert np.array_equal(o2, ml)
            hits += 1
    assert hits > 20


def test_osd_output_is_codeword():
    c = oracle.Code(6, PRIMS[6], 3)
    rng = np.random.default_rng(14)
    for _ in range(10):
        L = rng.standard_normal(63) * 2 + 1
        w = oracle.osd(c.G, L, 2)
        assert not ((c.Hstd.astype(int) @ w.astype(int)) % 2).any()


def test_hand_worked_fixed_point_three_branches():
    """B = 3 integer decoder against a hand-worked trajectory: v2c saturation
    at 127, the branch average rounding down and up, a positive average, then
    the closed form y^(t) = y^(4) - 63 (t - 4) until the posterior saturates
    at -32767 and stays there."""
    g = json.load(open(os.path.join(GOLD, "fixed_point_b3_hand.json")))
    H = np.array(g["H"], dtype=np.uint8)
    Hs = np.array(g["Hsyn"], dtype=np.uint8)
    maps = np.array(g["maps"], dtype=np.int16)
    r = oracle.nms_fixed(H, maps, np.array(g["q"], dtype=np.int8), g["max_iter"], oracle.R1, Hs, trace=True)
    assert r["iters"] == g["iters"] and r["converged"] == g["converged"]
    assert list(r["c_hat"]) == g["c_hat"]
    tr = r["y_trace"]
    first = np.array(g["y_first"])
    assert np.array_equal(tr[:4], first)
    t = np.arange(5, g["max_iter"] + 1)[:, None]
    want = np.maximum(first[3][None, :] + g["step_after"] * (t - 4), g["saturation"])
    assert np.array_equal(tr[4:], want)
    assert tr[519, 0] == -32723 and tr[520, 0] == -32767 and tr[520, 1] > -32767  # t = 520, 521
