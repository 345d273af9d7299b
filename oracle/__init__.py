"""CPU oracle for enhanced normalized min-sum decoding of short BCH codes.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use it; the product library never imports, links or calls
it, and it imports nothing from the product package.

Everything here is a thin numpy/ctypes wrapper around the plain C sources in
this directory (FP64 floating point, exact integers):

  * code algebra of binary primitive BCH codes (system model of Section II);
  * the optimised parity-check matrix H_o (Section III-A, steps 1-6; Table 1);
  * the automorphism block (Section III-B);
  * plain NMS (Section II-A, eqs. 2-5) and enhanced NMS (Algorithm 1), literal
    and min1/min2 forms, plus the integer fixed-point variant;
  * order-p OSD (Section II-B) and brute-force ML.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["oracle_code.c", "oracle_pcm.c", "oracle_perm.c", "oracle_nms.c",
            "oracle_osd.c", "oracle_batch.c"]

R1, R2, R3 = 1, 2, 3
KIND_LITERAL, KIND_FAST, KIND_FIXED = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile the oracle's C sources into liboracle.so (gcc, plain IEEE FP64:
    no FMA contraction, no fast-math)."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    if not force and os.path.exists(_LIB_PATH):
        newest = max(os.path.getmtime(s) for s in srcs + [os.path.join(_HERE, "oracle.h")])
        if os.path.getmtime(_LIB_PATH) >= newest:
            return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-o", tmp] + srcs + ["-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i32, u32, u64, dbl = ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
        L.orc_gf_tables.argtypes = [i32, u32, P, P]
        L.orc_bch_generator.argtypes = [i32, u32, i32, P, P]
        L.orc_bch_matrices.argtypes = [i32, u32, i32, P, P, P, P, P, P]
        L.orc_count_4cycles.argtypes = [P, i32, i32]
        L.orc_count_4cycles.restype = ctypes.c_int64
        L.orc_rank.argtypes = [P, i32, i32]
        L.orc_rref.argtypes = [P, i32, i32]
        L.orc_min_density.argtypes = [P, i32, i32, i32, P, i32]
        L.orc_build_hopt.argtypes = [P, i32, i32, i32, i32, i32, u64, i32, dbl, P, i32, P, P]
        L.orc_branch_maps.argtypes = [i32, i32, i32, P]
        L.orc_philox4x64_10.argtypes = [P, P, P]
        L.orc_philox4x64_10.restype = None
        L.orc_draw_offsets.argtypes = [i32, u64, u64, ctypes.c_int64, ctypes.c_int64, P]
        for fn in (L.orc_nms_literal, L.orc_nms_fast):
            fn.argtypes = [P, i32, i32, P, i32, P, dbl, i32, i32, P, i32, P, P, P, P]
        L.orc_nms_fixed.argtypes = [P, i32, i32, P, i32, P, i32, i32, P, i32, P, P, P, P]
        L.orc_osd.argtypes = [P, i32, i32, P, i32, P]
        L.orc_ml_bruteforce.argtypes = [P, i32, i32, P, P]
        L.orc_weight_distribution.argtypes = [P, i32, i32, P]
        L.orc_words_of_weight.argtypes = [P, i32, i32, i32, P, ctypes.c_int64]
        L.orc_words_of_weight.restype = ctypes.c_int64
        L.orc_splitmix64_next.argtypes = [P]
        L.orc_splitmix64_next.restype = u64
        L.orc_decode_batch.argtypes = [i32, P, i32, i32, i32, P, P, i32, i32, dbl, i32,
                                       i32, P, i32, P, P, P, P]
        L.orc_osd_batch.argtypes = [P, i32, i32, P, i32, i32, i32, P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int, what: str):
    if rc < 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")
    return rc


# --------------------------------------------------------------------------
# code algebra
# --------------------------------------------------------------------------
def gf_tables(m: int, prim: int):
    exp_t = np.zeros(2 * 128, dtype=np.int32)
    log_t = np.zeros(129, dtype=np.int32)
    _check(lib().orc_gf_tables(m, prim, _p(exp_t), _p(log_t)), "gf_tables")
    n = (1 << m) - 1
    return exp_t[:2 * n].copy(), log_t[:n + 1].copy()


class Code:
    """A binary primitive narrow-sense BCH code (N = 2^m - 1)."""

    def __init__(self, m: int, prim: int, t: int):
        N = ctypes.c_int()
        K = ctypes.c_int()
        n = (1 << m) - 1
        g = np.zeros(n + 1, dtype=np.uint8)
        h = np.zeros(n + 1, dtype=np.uint8)
        G = np.zeros(n * n, dtype=np.uint8)
        H = np.zeros(n * n, dtype=np.uint8)
        _check(lib().orc_bch_matrices(m, prim, t, ctypes.byref(N), ctypes.byref(K),
                                      _p(g), _p(h), _p(G), _p(H)), "bch_matrices")
        self.m, self.prim, self.t = m, prim, t
        self.N, self.K = N.value, K.value
        self.g = g[: self.N - self.K + 1].copy()
        self.h = h[: self.K + 1].copy()
        self.G = G[: self.K * self.N].reshape(self.K, self.N).copy()
        self.Hstd = H[: (self.N - self.K) * self.N].reshape(self.N - self.K, self.N).copy()

    @property
    def rate(self) -> float:
        return self.K / self.N


def count_4cycles(H: np.ndarray) -> int:
    H = np.ascontiguousarray(H, dtype=np.uint8)
    return int(lib().orc_count_4cycles(_p(H), H.shape[0], H.shape[1]))


def rank(H: np.ndarray) -> int:
    H = np.ascontiguousarray(H, dtype=np.uint8)
    return _check(lib().orc_rank(_p(H), H.shape[0], H.shape[1]), "rank")


def rref(H: np.ndarray):
    H = np.ascontiguousarray(H, dtype=np.uint8).copy()
    r = _check(lib().orc_rref(_p(H), H.shape[0], H.shape[1]), "rref")
    return H[:r].copy()


def min_density(Hr: np.ndarray, with_shifts: bool, cap: int = 8192) -> np.ndarray:
    Hr = np.ascontiguousarray(Hr, dtype=np.uint8)
    N = Hr.shape[1]
    out = np.zeros(cap * N, dtype=np.uint8)
    n = _check(lib().orc_min_density(_p(Hr), Hr.shape[0], N, int(with_shifts), _p(out), cap),
               "min_density")
    return out[: n * N].reshape(n, N).copy()


def build_hopt(code: Code, beta: int = 2, target_rows: int = 0, Q: int = 4, seed: int = 1,
               sa_steps_per_row: int = 200, sa_lambda: float = 10.0):
    """Steps 2-6 of Section III-A.  Returns (H_o, M_r1, seed actually used).
    target_rows > 0 pads to that many rows instead of beta * (M - M_r1)."""
    Hs = np.ascontiguousarray(code.Hstd)
    cap = 4096
    out = np.zeros(cap * code.N, dtype=np.uint8)
    mr1 = ctypes.c_int()
    used = ctypes.c_uint64()
    mo = _check(lib().orc_build_hopt(_p(Hs), Hs.shape[0], code.N, beta, target_rows, Q, seed,
                                     sa_steps_per_row, sa_lambda, _p(out), cap,
                                     ctypes.byref(mr1), ctypes.byref(used)), "build_hopt")
    return out[: mo * code.N].reshape(mo, code.N).copy(), mr1.value, used.value


def pcm_stats(H: np.ndarray) -> dict:
    """Table 1 attributes: dimensions, #length-4 cycles, column / row weight
    range, mean and (population) standard deviation."""
    H = np.asarray(H, dtype=np.uint8)
    cw = H.sum(axis=0).astype(np.float64)
    rw = H.sum(axis=1).astype(np.float64)
    return {
        "M": int(H.shape[0]), "N": int(H.shape[1]), "edges": int(H.sum()),
        "c4": count_4cycles(H),
        "col_range": (int(cw.min()), int(cw.max())), "col_mean": float(cw.mean()),
        "col_std": float(cw.std()),
        "row_range": (int(rw.min()), int(rw.max())), "row_mean": float(rw.mean()),
        "row_std": float(rw.std()),
    }


def weight_distribution(G: np.ndarray) -> np.ndarray:
    G = np.ascontiguousarray(G, dtype=np.uint8)
    A = np.zeros(G.shape[1] + 1, dtype=np.uint64)
    _check(lib().orc_weight_distribution(_p(G), G.shape[0], G.shape[1], _p(A)),
           "weight_distribution")
    return A


def words_of_weight(G: np.ndarray, w: int, cap: int = 1 << 16) -> np.ndarray:
    """Every codeword of Hamming weight w of the code spanned by the rows of G."""
    G = np.ascontiguousarray(G, dtype=np.uint8)
    N = G.shape[1]
    out = np.zeros(cap * N, dtype=np.uint8)
    n = _check(lib().orc_words_of_weight(_p(G), G.shape[0], N, w, _p(out), cap),
               "words_of_weight")
    if n > cap:
        raise RuntimeError("words_of_weight: %d words exceed cap %d" % (n, cap))
    return out[: n * N].reshape(n, N).copy()


def splitmix64(seed: int, n: int):
    st = ctypes.c_uint64(seed)
    return [int(lib().orc_splitmix64_next(ctypes.byref(st))) for _ in range(n)]


# --------------------------------------------------------------------------
# automorphisms and decoders
# --------------------------------------------------------------------------
def branch_maps(N: int, n_branches: int, d_o: int) -> np.ndarray:
    maps = np.zeros(9 * 128, dtype=np.int16)
    _check(lib().orc_branch_maps(N, n_branches, d_o, _p(maps)), "branch_maps")
    return maps[: n_branches * N].reshape(n_branches, N).copy()


def philox4x64_10(ctr, key):
    """One Philox4x64-10 block: four 64-bit counter words and two key words in,
    four output words out."""
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_p(c), _p(k), _p(out))
    return [int(v) for v in out]


def draw_offsets(N: int, seed: int, key_hi: int, frame_base: int, F: int) -> np.ndarray:
    """Random offsets d_o in [0, d_p) of frames frame_base .. frame_base + F - 1."""
    d = np.zeros(F, dtype=np.uint8)
    _check(lib().orc_draw_offsets(N, seed, key_hi, frame_base, F, _p(d)), "draw_offsets")
    return d


def _decode_one(fn, H, maps, L, alpha, max_iter, mode, Hsyn, trace):
    H = np.ascontiguousarray(H, dtype=np.uint8)
    Hsyn = np.ascontiguousarray(Hsyn, dtype=np.uint8)
    maps = np.ascontiguousarray(maps, dtype=np.int16)
    M, N = H.shape
    L = np.ascontiguousarray(L, dtype=np.float64)
    c = np.zeros(N, dtype=np.uint8)
    it = ctypes.c_int()
    cv = ctypes.c_int()
    tr = np.zeros((max_iter, N), dtype=np.float64) if trace else None
    _check(fn(_p(H), M, N, _p(maps), maps.shape[0], _p(L), alpha, max_iter, mode,
              _p(Hsyn), Hsyn.shape[0], _p(c), ctypes.byref(it), ctypes.byref(cv),
              _p(tr) if trace else None), "nms")
    res = {"c_hat": c, "iters": it.value, "converged": bool(cv.value)}
    if trace:
        res["y_trace"] = tr[: it.value].copy()
    return res


def nms_literal(H, maps, L, alpha, max_iter, mode, Hsyn, trace=False):
    return _decode_one(lib().orc_nms_literal, H, maps, L, alpha, max_iter, mode, Hsyn, trace)


def nms_fast(H, maps, L, alpha, max_iter, mode, Hsyn, trace=False):
    return _decode_one(lib().orc_nms_fast, H, maps, L, alpha, max_iter, mode, Hsyn, trace)


def nms_fixed(H, maps, q, max_iter, mode, Hsyn, trace=False):
    H = np.ascontiguousarray(H, dtype=np.uint8)
    Hsyn = np.ascontiguousarray(Hsyn, dtype=np.uint8)
    maps = np.ascontiguousarray(maps, dtype=np.int16)
    M, N = H.shape
    q = np.ascontiguousarray(q, dtype=np.int8)
    c = np.zeros(N, dtype=np.uint8)
    it = ctypes.c_int()
    cv = ctypes.c_int()
    tr = np.zeros((max_iter, N), dtype=np.int32) if trace else None
    _check(lib().orc_nms_fixed(_p(H), M, N, _p(maps), maps.shape[0], _p(q), max_iter, mode,
                               _p(Hsyn), Hsyn.shape[0], _p(c), ctypes.byref(it),
                               ctypes.byref(cv), _p(tr) if trace else None), "nms_fixed")
    res = {"c_hat": c, "iters": it.value, "converged": bool(cv.value)}
    if trace:
        res["y_trace"] = tr[: it.value].copy()
    return res


def quantize(llr: np.ndarray, scale: float) -> np.ndarray:
    """Fixed-point input: clamp(round-half-away(L * scale), -127, 127) as int8,
    the product L * scale formed in FP32 as the LLRs are FP32."""
    x = np.asarray(llr, dtype=np.float32) * np.float32(scale)
    r = np.sign(x) * np.floor(np.abs(x).astype(np.float64) + 0.5)
    return np.clip(r, -127, 127).astype(np.int8)


def decode_batch(H, Hsyn, llr, d_o, n_branches, alpha, max_iter, mode, kind=KIND_FAST,
                 threads: int = 1, trace: bool = False):
    """Decode every frame of llr ([F][ld] float32, or int8 for the fixed-point
    kind).  Returns (c_hat [F][N] uint8, iters [F] int32, converged [F] bool)
    and, with trace=True, also the [F][max_iter][N] posteriors (NaN / 0 past a
    frame's last iteration)."""
    H = np.ascontiguousarray(H, dtype=np.uint8)
    Hsyn = np.ascontiguousarray(Hsyn, dtype=np.uint8)
    M, N = H.shape
    llr = np.ascontiguousarray(llr)
    if kind == KIND_FIXED:
        assert llr.dtype == np.int8
    else:
        assert llr.dtype == np.float32
    F, ld = llr.shape
    d_o = np.ascontiguousarray(d_o if d_o is not None else np.zeros(F), dtype=np.uint8)
    c = np.zeros((F, N), dtype=np.uint8)
    it = np.zeros(F, dtype=np.int32)
    cv = np.zeros(F, dtype=np.uint8)
    tr = None
    if trace:
        tr = (np.zeros((F, max_iter, N), dtype=np.int32) if kind == KIND_FIXED
              else np.full((F, max_iter, N), np.nan))
    L = lib()

    def run(lo, hi):
        if hi <= lo:
            return
        rc = L.orc_decode_batch(kind, _p(H), M, N, n_branches, _p(d_o[lo:hi]),
                                _p(llr[lo:hi]), ld, hi - lo, alpha, max_iter, mode,
                                _p(Hsyn), Hsyn.shape[0], _p(c[lo:hi]), _p(it[lo:hi]),
                                _p(cv[lo:hi]), _p(tr[lo:hi]) if trace else None)
        _check(rc, "decode_batch")

    if threads <= 1 or F < 2 * threads:
        run(0, F)
    else:
        bounds = np.linspace(0, F, threads + 1).astype(int)
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(lambda k: run(bounds[k], bounds[k + 1]), range(threads)))
    if trace:
        return c, it, cv.astype(bool), tr
    return c, it, cv.astype(bool)


def osd(G, L, order):
    G = np.ascontiguousarray(G, dtype=np.uint8)
    K, N = G.shape
    L = np.ascontiguousarray(L, dtype=np.float64)
    c = np.zeros(N, dtype=np.uint8)
    _check(lib().orc_osd(_p(G), K, N, _p(L), order, _p(c)), "osd")
    return c


def osd_batch(G, llr, order, flags=None, c_hat=None):
    G = np.ascontiguousarray(G, dtype=np.uint8)
    K, N = G.shape
    llr = np.ascontiguousarray(llr, dtype=np.float32)
    F, ld = llr.shape
    c = np.zeros((F, N), dtype=np.uint8) if c_hat is None else np.ascontiguousarray(c_hat).copy()
    fl = None if flags is None else np.ascontiguousarray(flags, dtype=np.uint8)
    _check(lib().orc_osd_batch(_p(G), K, N, _p(llr), ld, F, order,
                               _p(fl) if fl is not None else None, _p(c)), "osd_batch")
    return c


def ml_bruteforce(G, L):
    G = np.ascontiguousarray(G, dtype=np.uint8)
    K, N = G.shape
    L = np.ascontiguousarray(L, dtype=np.float64)
    c = np.zeros(N, dtype=np.uint8)
    _check(lib().orc_ml_bruteforce(_p(G), K, N, _p(L), _p(c)), "ml_bruteforce")
    return c
