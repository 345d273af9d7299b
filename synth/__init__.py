"""Seeded synthetic workloads for the BCH decoders: random information bits,
systematic BCH encoding, BPSK over AWGN and channel LLRs (the system model of
Section II, eq. 1), plus the per-frame random offset d_o that the enhanced
decoder's cyclic shifts draw (Section III-B).

This module is shared by the product path, the oracle-based tests and the
benchmark.  It holds none of the decoder's arithmetic.  The code's generator
polynomial is read from ``codes.json``, which ``make_codes.py`` writes from the
oracle's code construction.

Randomness: numpy's Philox counter-based generator, keyed by a SeedSequence of
(seed, code tag, stream, block) so that any block of frames is reproducible on
its own (a request's frames are the same alone and in a mix).
Streams: 0 information bits, 1 noise, 3 mixed-workload draws, 4 arrivals.
The offsets d_o follow the draw the decoder library offers
(bch_draw_offsets): word 0 of Philox4x64-10 at counter (frame uid, 0, 0, 0)
under key (seed, code tag << 32 | block), mapped to [0, d_p) by
((word >> 32) d_p) >> 32; here numpy's own Philox bit generator produces the
words.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))

# code name -> (m, primitive polynomial, t)
CODES = {
    "bch63_36": (6, 0b1000011, 5),
    "bch63_45": (6, 0b1000011, 3),
    "bch127_64": (7, 0b10001001, 10),
    "bch127_78": (7, 0b10001001, 7),
    "bch127_99": (7, 0b10001001, 4),
}
CODE_TAG = {"bch63_36": 1, "bch63_45": 2, "bch127_64": 3, "bch127_78": 4, "bch127_99": 5}


@dataclass(frozen=True)
class CodeSpec:
    name: str
    m: int
    prim: int
    t: int
    N: int
    K: int
    g: tuple  # generator polynomial coefficients, lowest degree first

    @property
    def rate(self) -> float:
        return self.K / self.N

    @property
    def ld(self) -> int:
        """Padded row stride of an LLR frame (64 or 128)."""
        return 64 if self.N <= 64 else 128

    @property
    def d_p(self) -> int:
        return 21 if self.N == 63 else 42


_specs = None


def code(name: str) -> CodeSpec:
    global _specs
    if _specs is None:
        with open(os.path.join(_HERE, "codes.json")) as fh:
            raw = json.load(fh)
        _specs = {}
        for k, v in raw["codes"].items():
            _specs[k] = CodeSpec(k, v["m"], v["prim"], v["t"], v["N"], v["K"], tuple(v["g"]))
    return _specs[name]


def sigma2_of(ebn0_db, rate):
    """Noise variance for Eb/N0 in dB at code rate K/N with unit-energy BPSK."""
    return 1.0 / (2.0 * rate * 10.0 ** (np.asarray(ebn0_db, dtype=np.float64) / 10.0))


def offsets(N: int, seed: int, key_hi: int, F: int, frame_base: int = 0) -> np.ndarray:
    """d_o of frames frame_base .. frame_base + F - 1: word 0 of Philox4x64-10
    at counter (uid, 0, 0, 0) under key (seed, key_hi), scaled to [0, d_p).
    numpy's Philox advances its counter before each block of four words, so it
    starts one step before frame_base (all ones wraps to zero)."""
    dp = 21 if N == 63 else (42 if N == 127 else N // 3)
    m64 = (1 << 64) - 1
    start = [frame_base - 1, 0, 0, 0] if frame_base > 0 else [m64] * 4
    bg = np.random.Philox(counter=np.array(start, dtype=np.uint64),
                          key=np.array([seed & m64, key_hi & m64], dtype=np.uint64))
    w = bg.random_raw(4 * F)[0::4] if F else np.zeros(0, np.uint64)
    return (((w >> np.uint64(32)) * np.uint64(dp)) >> np.uint64(32)).astype(np.uint8)


def offset_key(name: str, block: int) -> int:
    """key_hi of a code's frames in one block: code tag << 32 | block."""
    return (CODE_TAG[name] << 32) | (block & 0xFFFFFFFF)


def _rng(seed: int, tag: int, stream: int, block: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(np.random.SeedSequence([seed, tag, stream, block])))


def _parity_matrix(spec: CodeSpec) -> np.ndarray:
    """Row k = remainder of x^(N-K+k) divided by g(x): the parity bits that
    message bit k contributes to a systematic codeword."""
    N, K = spec.N, spec.K
    g = np.array(spec.g, dtype=np.uint8)
    r = N - K
    P = np.zeros((K, r), dtype=np.uint8)
    cur = g[:r].copy()  # x^r mod g, g monic of degree r
    for k in range(K):
        P[k] = cur
        top = cur[r - 1]  # multiply by x, reduce by g
        cur = np.concatenate([[0], cur[:-1]]).astype(np.uint8)
        if top:
            cur ^= g[:r]
    return P


_pmats = {}


def encode(spec: CodeSpec, msg: np.ndarray) -> np.ndarray:
    """Systematic codewords [F][N] (uint8): parity in columns 0..N-K-1, message
    bits in columns N-K..N-1 (coefficient of x^j in column j).

    The parity is the XOR of the parity rows of the set message bits, taken a
    message byte at a time from a 256-entry table per byte: exact integer work
    with no BLAS call, so that generator threads running side by side (several
    blocks of a workload at once) stay deterministic."""
    if spec.name not in _pmats:
        Pb = np.packbits(_parity_matrix(spec), axis=1, bitorder="little")  # [K][ceil(r/8)]
        nbytes = (spec.K + 7) // 8
        T = np.zeros((nbytes, 256, Pb.shape[1]), dtype=np.uint8)
        for j in range(nbytes):
            for b in range(8):
                k = 8 * j + b
                if k < spec.K:
                    sel = (np.arange(256) >> b) & 1 == 1
                    T[j, sel] ^= Pb[k]
        _pmats[spec.name] = T
    T = _pmats[spec.name]
    mp = np.packbits(msg.astype(np.uint8), axis=1, bitorder="little")  # [F][ceil(K/8)]
    par = np.zeros((msg.shape[0], T.shape[2]), dtype=np.uint8)
    for j in range(T.shape[0]):
        par ^= T[j][mp[:, j]]
    bits = np.unpackbits(par, axis=1, count=spec.N - spec.K, bitorder="little")
    return np.concatenate([bits, msg.astype(np.uint8)], axis=1)


@dataclass
class Frames:
    llr: np.ndarray        # [F][ld] float32, zero padding beyond N
    codewords: np.ndarray  # [F][N] uint8, transmitted
    d_o: np.ndarray        # [F] uint8, random cyclic offset in [0, d_p)
    ebn0: np.ndarray       # [F] float64


def frames(name: str, F: int, ebn0, seed: int, block: int = 0, zero_codeword: bool = False) -> Frames:
    """F frames of one code.  ebn0 is a scalar or a per-frame array (dB)."""
    spec = code(name)
    tag = CODE_TAG[name]
    N, K, ld = spec.N, spec.K, spec.ld
    if zero_codeword:
        msg = np.zeros((F, K), dtype=np.uint8)
    else:
        msg = _rng(seed, tag, 0, block).integers(0, 2, size=(F, K), dtype=np.uint8)
    cw = encode(spec, msg)
    e = np.broadcast_to(np.asarray(ebn0, dtype=np.float64), (F,)).copy()
    s2 = sigma2_of(e, spec.rate).astype(np.float32)[:, None]
    noise = _rng(seed, tag, 1, block).standard_normal(size=(F, N), dtype=np.float32)
    y = (1.0 - 2.0 * cw.astype(np.float32)) + np.sqrt(s2) * noise
    llr = np.zeros((F, ld), dtype=np.float32)
    llr[:, :N] = (2.0 / s2) * y
    d_o = offsets(N, seed, offset_key(name, block), F)
    return Frames(llr, cw, d_o, e)


def mixed_draws(F: int, seed: int, probs, ebn0_lo: float, ebn0_hi: float, block: int = 0):
    """Per-frame code index (drawn with the given probabilities) and Eb/N0
    uniform in [lo, hi], for mixed-code workloads."""
    r = _rng(seed, 0, 3, block)
    idx = r.choice(len(probs), size=F, p=np.asarray(probs, dtype=np.float64))
    e = r.uniform(ebn0_lo, ebn0_hi, size=F)
    return idx.astype(np.int32), e


@dataclass
class MixedFrames:
    llr: np.ndarray        # [F][ld] float32, ld = the widest code's row stride
    code_idx: np.ndarray   # [F] uint8 index into names
    codewords: np.ndarray  # [F][N_max] uint8 (zero beyond the frame's N)
    d_o: np.ndarray        # [F] uint8
    ebn0: np.ndarray       # [F] float64


def mixed_frames(names, F: int, seed: int, probs, ebn0_lo: float, ebn0_hi: float, block: int = 0) -> MixedFrames:
    """F frames of several codes interleaved: code and Eb/N0 drawn per frame
    (mixed_draws), then each code's frames generated by frames() at those
    Eb/N0 values and placed at their positions."""
    idx, e = mixed_draws(F, seed, probs, ebn0_lo, ebn0_hi, block)
    specs = [code(n) for n in names]
    ld = max(s.ld for s in specs)
    nmax = max(s.N for s in specs)
    llr = np.zeros((F, ld), dtype=np.float32)
    cw = np.zeros((F, nmax), dtype=np.uint8)
    d_o = np.zeros(F, dtype=np.uint8)
    for k, n in enumerate(names):
        sel = np.nonzero(idx == k)[0]
        if sel.size == 0:
            continue
        fr = frames(n, sel.size, e[sel], seed, block)
        llr[sel, :fr.llr.shape[1]] = fr.llr
        cw[sel, :specs[k].N] = fr.codewords
        d_o[sel] = fr.d_o
    return MixedFrames(llr, idx.astype(np.uint8), cw, d_o, e)


@dataclass
class RequestDraw:
    t: float               # arrival time at unit rate (seconds x requests/s)
    code: int              # index into names
    frames: int            # 1..2^max_log2, log-uniform
    ebn0: float            # dB, one value per request


def request_trace(n: int, seed: int, n_codes: int, ebn0_lo: float, ebn0_hi: float, max_log2: int = 12):
    """n requests of a Poisson stream at unit rate (divide t by the rate in
    requests/s): exponential gaps, size round(2^(max_log2 U)), code uniform,
    Eb/N0 uniform per request."""
    r = _rng(seed, 0, 4, 0)
    t = np.cumsum(r.exponential(1.0, size=n))
    size = np.rint(2.0 ** (max_log2 * r.uniform(0.0, 1.0, size=n))).astype(np.int64)
    code_i = r.integers(0, n_codes, size=n)
    e = r.uniform(ebn0_lo, ebn0_hi, size=n)
    return [RequestDraw(float(t[k]), int(code_i[k]), int(size[k]), float(e[k])) for k in range(n)]


def request_frames(names, draw: RequestDraw, seed: int, rid: int) -> Frames:
    """The frames of request rid (its own block of the code's streams)."""
    return frames(names[draw.code], draw.frames, draw.ebn0, seed, block=1000 + rid)
