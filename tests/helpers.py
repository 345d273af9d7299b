"""Shared helpers of the test-suite: library/oracle set-up for the paper's
codes and the parity comparison between the HIP path and the oracle."""
from __future__ import annotations

import functools
import os
import re

import numpy as np

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bchnms.h")

# Table 1 dimensions of the optimised matrices used by the workloads
HO_ROWS = {"bch63_36": 122, "bch63_45": 33, "bch127_64": 72, "bch127_78": 57, "bch127_99": 33}

TRACE_TOL = 1e-5   # normwise relative tolerance per iteration
TIE_TOL = 1e-4     # |y_u| below this fraction of max|y| marks a possible sign tie


def ensure_built():
    from paper_2412_20828_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2412_20828_amd import build
        build.build(verbose=False)
    return binding


def header_symbols():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(bch_[a-z0-9_]+)\s*\(", txt)))


@functools.lru_cache(maxsize=None)
def oracle_code(name):
    m, p, t = synth.CODES[name]
    return oracle.Code(m, p, t)


@functools.lru_cache(maxsize=None)
def oracle_hopt(name, rows=None):
    c = oracle_code(name)
    H, _, _ = oracle.build_hopt(c, target_rows=rows or HO_ROWS[name], seed=1)
    return H


def compare_with_oracle(gpu_words, gpu_iters, gpu_flags, gpu_trace, orc_c, orc_it, orc_cv, orc_tr,
                        max_tie_frac=0.02, onestep=None):
    """Parity bar of the FP32 decoders against the FP64 oracle.

    Decisions: identical decoded words, iteration counts and flags on every
    frame that is not a tie (a frame whose oracle posterior comes within
    TIE_TOL of zero at or before the divergence); at most max_tie_frac ties.

    Posteriors, per iteration, normwise (max |gpu - ref| <= TRACE_TOL max |ref|):
      - onestep = (H, Hstd, llr, d_o, n_branches, alpha) for the restart mode,
        where an iteration is a function of y alone: every iteration t of the
        GPU trace, on every frame, is compared with one oracle iteration run
        from the GPU's own iterate t - 1 (the channel LLRs for t = 1).  The
        bound then holds for each iteration's arithmetic, while FP32 rounding
        compounded over a non-converging trajectory is not charged to it;
      - without onestep (edge-memory modes): the GPU trajectory against the
        oracle's, up to the first possible tie.
    Returns (n_frames, n_ties)."""
    F, N = orc_c.shape
    ties = 0
    for f in range(F):
        T = int(orc_it[f])
        tr = orc_tr[f, :T]
        scale = np.abs(tr).max(axis=1)
        near = (np.abs(tr) < TIE_TOL * scale[:, None]).any(axis=1)
        t_tie = int(np.argmax(near)) if near.any() else T
        same = (np.array_equal(gpu_words[f], orc_c[f]) and int(gpu_iters[f]) == T
                and bool(gpu_flags[f]) == bool(orc_cv[f]))
        if not same:
            assert near.any(), ("frame %d differs without a tie" % f)
            ties += 1
            continue
        if gpu_trace is not None and onestep is None:
            upto = min(T, t_tie + 1)
            g = gpu_trace[f, :upto, :N].astype(np.float64)
            err = np.abs(g - tr[:upto]).max(axis=1)
            assert (err <= TRACE_TOL * scale[:upto]).all(), (f, err / scale[:upto])
    assert ties <= max_tie_frac * F + 1, (ties, F)
    if gpu_trace is not None and onestep is not None:
        H, Hstd, llr, d_o, nb, alpha = onestep
        rows, src = [], []
        for f in range(F):
            for t in range(int(gpu_iters[f])):
                rows.append(llr[f] if t == 0 else gpu_trace[f, t - 1])
                src.append((f, t))
        X = np.ascontiguousarray(np.stack(rows), dtype=np.float32)
        X[:, N:] = 0.0
        dd = np.array([d_o[f] for f, _ in src], dtype=np.uint8)
        _, _, _, ref = oracle.decode_batch(H, Hstd, X, dd, nb, alpha, 1, oracle.R1, threads=8, trace=True)
        ref = ref[:, 0, :N]
        g = np.stack([gpu_trace[f, t, :N] for f, t in src]).astype(np.float64)
        err = np.abs(g - ref).max(axis=1)
        sc = np.abs(ref).max(axis=1)
        bad = np.nonzero(err > TRACE_TOL * sc)[0]
        assert bad.size == 0, [(src[i], err[i] / sc[i]) for i in bad[:5]]
    return F, ties
