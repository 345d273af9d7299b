"""Pins for the oracle's code algebra (system model, Section II; codes of
Table 1): closed forms, Table 1's standard-H attributes, true minimum
distances by enumeration, and the dual-code facts behind the
rank-deficiency discussion of Section III-A."""
import json
import math
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")
PRIMS = {3: 0b1011, 4: 0b10011, 5: 0b100101, 6: 0b1000011, 7: 0b10001001}


def gf_eval(poly, x, exp_t, log_t, N):
    """Evaluate a GF(2)-coefficient polynomial at a field element x (Horner)."""
    acc = 0
    for c in reversed(list(poly)):
        acc = (exp_t[log_t[acc] + log_t[x]] if acc and x else 0) ^ int(c)
    return acc


@pytest.mark.parametrize("m", [3, 4, 5, 6, 7])
def test_gf_tables_are_a_field(m):
    exp_t, log_t = oracle.gf_tables(m, PRIMS[m])
    N = (1 << m) - 1
    assert sorted(exp_t[:N]) == list(range(1, N + 1))  # alpha generates the group
    for i in range(N):
        assert log_t[exp_t[i]] == i
    # alpha^N = 1
    assert exp_t[N] == 1


@pytest.mark.parametrize("m,t", [(3, 1), (4, 1), (4, 2), (4, 3), (5, 2), (5, 3), (5, 5),
                                 (6, 3), (6, 5), (7, 4), (7, 7), (7, 10)])
def test_generator_zeros_and_check_polynomial(m, t):
    c = oracle.Code(m, PRIMS[m], t)
    N, K = c.N, c.K
    exp_t, log_t = oracle.gf_tables(m, PRIMS[m])
    # designed zeros alpha^1..alpha^2t are roots of g
    for j in range(1, 2 * t + 1):
        assert gf_eval(c.g, exp_t[j % N], exp_t, log_t, N) == 0
    # g * h = x^N + 1 over GF(2)
    prod = np.convolve(c.g.astype(int), c.h.astype(int)) % 2
    want = np.zeros(N + 1, dtype=int)
    want[0] = want[N] = 1
    assert np.array_equal(prod, want)
    # G H^T = 0, full ranks, systematic message part
    assert not ((c.G.astype(int) @ c.Hstd.T.astype(int)) % 2).any()
    assert oracle.rank(c.G) == K and oracle.rank(c.Hstd) == N - K
    assert np.array_equal(c.G[:, N - K:], np.eye(K, dtype=np.uint8))


def test_code_dimensions_of_table1():
    for m, t, K in [(6, 5, 36), (6, 3, 45), (7, 10, 64), (7, 7, 78), (7, 4, 99)]:
        assert oracle.Code(m, PRIMS[m], t).K == K


def test_table1_standard_h_attributes_exact():
    gold = json.load(open(os.path.join(GOLD, "table1_standard_h.json")))
    for row in gold["codes"]:
        c = oracle.Code(row["m"], row["prim"], row["t"])
        assert (c.N, c.K) == (row["N"], row["K"])
        s = oracle.pcm_stats(c.Hstd)
        assert s["M"] == row["M"]
        assert s["c4"] == row["c4"]
        assert list(s["col_range"]) == row["col_range"]
        assert list(s["row_range"]) == row["row_range"]
        assert round(s["col_mean"], 1) == row["col_mean"]
        assert round(s["col_std"], 1) == row["col_std"]
        assert round(s["row_mean"], 1) == row["row_mean"]


def test_four_cycle_count_brute_force():
    # count pairs of rows x pairs of columns directly on a small random matrix
    rng = np.random.default_rng(0)
    H = (rng.random((7, 12)) < 0.5).astype(np.uint8)
    brute = 0
    for a in range(7):
        for b in range(a + 1, 7):
            for c1 in range(12):
                for c2 in range(c1 + 1, 12):
                    brute += H[a, c1] & H[a, c2] & H[b, c1] & H[b, c2]
    assert oracle.count_4cycles(H) == brute


@pytest.mark.parametrize("m,t,d", [(3, 1, 3), (4, 1, 3), (4, 2, 5), (4, 3, 7), (5, 1, 3),
                                   (5, 2, 5), (5, 3, 7), (5, 5, 11)])
def test_minimum_distance_brute_force_tiny(m, t, d):
    c = oracle.Code(m, PRIMS[m], t)
    A = oracle.weight_distribution(c.G)
    assert A[0] == 1 and int(A.sum()) == 2 ** c.K
    dmin = min(w for w in range(1, c.N + 1) if A[w])
    assert dmin == d


def krawtchouk(k, x, n):
    return sum((-1) ** j * math.comb(x, j) * math.comb(n - x, k - j) for j in range(k + 1))


@pytest.mark.parametrize("m,t,d", [(6, 3, 7), (6, 5, 11), (7, 4, 9)])
def test_minimum_distance_by_macwilliams(m, t, d):
    """Enumerate the dual (2^(N-K) words), transform exactly to the code's
    low-weight coefficients: A_w = 2^-(N-K) sum_j B_j K_w(j)."""
    c = oracle.Code(m, PRIMS[m], t)
    B = [int(x) for x in oracle.weight_distribution(c.Hstd)]
    assert sum(B) == 2 ** (c.N - c.K)
    A = []
    for w in range(0, d + 1):
        s = sum(B[j] * krawtchouk(w, j, c.N) for j in range(c.N + 1))
        assert s % 2 ** (c.N - c.K) == 0
        A.append(s // 2 ** (c.N - c.K))
    assert A[0] == 1
    assert all(a == 0 for a in A[1:d])
    assert A[d] > 0


def test_dual_minimum_weight_rank_deficiency():
    """Section III-A: the (63,45) code has a full-rank H_o of uniform minimum-
    weight (16) rows; the (63,36) code's minimum-weight dual words cannot
    form a full-rank matrix."""
    c45 = oracle.Code(6, PRIMS[6], 3)
    A = oracle.weight_distribution(c45.Hstd)
    wmin = min(w for w in range(1, 64) if A[w])
    assert wmin == 16
    W = oracle.words_of_weight(c45.Hstd, 16)
    assert oracle.rank(W) == 18
    c36 = oracle.Code(6, PRIMS[6], 5)
    A = oracle.weight_distribution(c36.Hstd)
    wmin = min(w for w in range(1, 64) if A[w])
    assert wmin == 14
    W = oracle.words_of_weight(c36.Hstd, 14)
    assert oracle.rank(W) < 27
    # the next weight of Table 1's rows (16) completes the rank
    W16 = oracle.words_of_weight(c36.Hstd, 16)
    assert oracle.rank(np.vstack([W, W16])) == 27


def test_splitmix64_reference_sequence():
    # first outputs of the published SplitMix64 reference generator, seed 1234567
    assert oracle.splitmix64(1234567, 5) == [
        6457827717110365317, 3203168211198807973, 9817491932198370423,
        4593380528125082431, 16408922859458223821]
