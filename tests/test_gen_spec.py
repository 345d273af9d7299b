"""Host-side contracts of the row-function generator (no GPU): the sign-word
layout the 32-bit kernels build and the masks the generated row functions
apply to it must agree, and the generated parity (one popcount of the masked
words folded by XOR) must equal each row's sign parity."""
import numpy as np
import pytest

from paper_2412_20828_amd import gen_spec


def kernel_sign_words(signs):
    """The kernels' accumulation S = (S << 1) | sign, coordinate by
    coordinate, in words of 32 coordinates."""
    N = len(signs)
    S = [0] * ((N + 31) // 32)
    for i in range(N):
        S[i >> 5] = ((S[i >> 5] << 1) | int(signs[i])) & 0xFFFFFFFF
    return S


@pytest.mark.parametrize("N", [63, 127])
def test_sign_masks_select_the_row_coordinates(N):
    rng = np.random.default_rng(N)
    for _ in range(200):
        signs = rng.integers(0, 2, N)
        S = kernel_sign_words(signs)
        cols = sorted(rng.choice(N, int(rng.integers(2, 48)), replace=False).tolist())
        masks = gen_spec._sign_masks(cols, N)
        # the masked bits are exactly the row's sign bits
        assert sum(bin(S[k] & m).count("1") for k, m in enumerate(masks)) == int(signs[cols].sum())
        folded = 0
        for k, m in enumerate(masks):
            folded ^= S[k] & m
        assert bin(folded).count("1") & 1 == int(signs[cols].sum()) & 1


@pytest.mark.parametrize("N", [63, 127])
def test_sign_masks_one_bit_per_coordinate(N):
    seen = set()
    for c in range(N):
        masks = gen_spec._sign_masks([c], N)
        assert sum(bin(m).count("1") for m in masks) == 1
        key = tuple(masks)
        assert key not in seen
        seen.add(key)


def test_parity_expression_shape():
    e = gen_spec._parity("S", [0x5, 0, 0x80000000])
    assert e == "__builtin_popcount((S[0] & 0x00000005u) ^ (S[2] & 0x80000000u))"


def _run_min_steps(cols, vals, **kw):
    """Evaluate the generated statements of a min1/min2 search in Python:
    min, max and med3 (median of three) on the given integers."""
    env = {}
    med3 = lambda a, b, c: sorted([a, b, c])[1]  # noqa: E731
    glb = {"min": min, "max": max, "med3u": med3, "med3i": med3, "V": vals}
    for step in gen_spec._min_steps(cols, "_x", lambda c: "V[%d]" % c, **kw):
        for line in step:
            line = line.replace("const uint32_t ", "").replace("uint32_t ", "")
            for stmt in filter(None, (x.strip() for x in line.split(";"))):
                parts, depth, cur = [], 0, ""
                for ch in stmt:  # split "a = x, b = y" at top-level commas
                    depth += (ch == "(") - (ch == ")")
                    if ch == "," and depth == 0:
                        parts.append(cur)
                        cur = ""
                    else:
                        cur += ch
                parts.append(cur)
                for p in parts:
                    lhs, rhs = p.split("=", 1)
                    env[lhs.strip()] = eval(rhs, glb, env)
    return env["u1_x"], env["u2_x"]


@pytest.mark.parametrize("kw", [{}, {"tree": False}, {"pair_merge": False}])
def test_min_search_forms_give_the_two_least(kw):
    """Every form of the generated min1/min2 search (triples merged in pairs,
    one at a time, or the entry-by-entry chain) leaves the least and second
    least value of the row, for row weights 2..60, with many ties (values
    drawn from a handful) and without."""
    rng = np.random.default_rng(9)
    for w in range(2, 61):
        for _ in range(60):
            small = rng.random() < 0.5
            vals = [int(x) for x in (rng.integers(0, 4, w) if small else rng.integers(0, 1 << 31, w))]
            cols = rng.permutation(w).tolist()
            assert _run_min_steps(cols, vals, **kw) == tuple(sorted(vals)[:2]), (w, vals)


def test_min_search_instruction_counts():
    """The triple search spends 8 instructions per 6 entries where the chain
    spends 12: min/max/med3 calls in the generated statements, a min of a min
    counted once (the compiler's min3)."""
    import re
    cols = list(range(24))

    def count(kw):
        lines = [x for st in gen_spec._min_steps(cols, "", lambda c: "V[%d]" % c, **kw) for x in st]
        return sum(len(re.findall(r"\b(min|max|med3[ui])\(", x)) - x.count("min(min(") for x in lines)
    assert count({"tree": False}) == 2 * 24 - 2
    assert count({}) == 8 * 24 // 6 - 1  # the first two triples merge with three, not four


def _c2v_sums(H, Y):
    """Per coordinate, the sum over the rows containing it of the signed
    min-sum message (sign product of the row's other entries times their
    least magnitude), in row order: what one row function adds into U."""
    M, N = H.shape
    U = np.zeros(N)
    for r in range(M):
        cols = np.nonzero(H[r])[0]
        for c in cols:
            others = [k for k in cols if k != c]
            U[c] += np.prod(np.sign(Y[others])) * np.min(np.abs(Y[others]))
    return U


@pytest.mark.parametrize("N, dp", [(63, 21), (127, 42)])
def test_shift_matrices_fold_a_type_onto_one_gather(N, dp):
    """A nine-branch kernel runs shift s of permutation type p as the row
    function of shift_matrices(H)[s] on the type's shift-0 input
    B[k] = y[a (k - d_o)] and adds into U in B's frame.  That must equal the
    branch itself, H on Y[i] = y[a (i - s d_p - d_o)], with its sums read
    back through Y[i] = B[(i - s d_p) mod N]."""
    rng = np.random.default_rng(3)
    H = (rng.random((9, N)) < 0.2).astype(np.uint8)
    H[:, 0] = 1
    mats = gen_spec.shift_matrices(H, dp)
    assert len(mats) == 3 and np.array_equal(mats[0], H)
    for a in (1, 2, (N + 1) // 2):
        y = rng.normal(size=N)
        d_o = int(rng.integers(0, dp))
        Bp = y[(a * (np.arange(N) - d_o)) % N]
        folded = sum(_c2v_sums(Hs, Bp) for Hs in mats)
        direct = np.zeros(N)
        for s in range(3):
            Y = y[(a * (np.arange(N) - s * dp - d_o)) % N]
            U = _c2v_sums(H, Y)
            direct[(np.arange(N) - s * dp) % N] += U  # entry i of the branch is B[(i - s d_p) mod N]
        np.testing.assert_allclose(folded, direct, rtol=1e-12, atol=1e-12)


def test_packed_selection_by_saturating_difference():
    """The packed row function's c2v magnitude q1 + (q2 - q1) e, with
    e = (min1 + 1) - A saturated at 0 in unsigned 16 bits, must equal the
    fixed-point message of the entry, (3 m + 2) >> 2 of the least of the row's
    other entries (min2 at an entry holding min1, min1 elsewhere), for every
    min1 <= min2 <= 127 and every entry value the row can hold, ties at min1
    included."""
    q = lambda m: (3 * m + 2) >> 2  # noqa: E731
    for m1 in range(128):
        for m2 in range(m1, 128):
            q1, q2 = q(m1), q(m2)
            for A in [m1] + list(range(m2, 128)):
                e = max(0, (m1 + 1) - A) & 0xFFFF
                got = (q1 + ((q2 - q1) * e)) & 0xFFFF
                other = m2 if A == m1 else m1  # the least of the others
                assert got == q(other), (m1, m2, A)
    # the generated row function spends three packed instructions per two
    # frame-edges on it: the saturating difference, a multiply-add, an add
    H = np.zeros((2, 63), np.uint8)
    H[0, [0, 5, 9]] = 1
    H[1, [1, 5, 20, 40]] = 1
    src = gen_spec.body_source_pk16(H, 9)
    assert src.count("is_min(") == 7 and src.count(" + sq1;") == 7
