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
