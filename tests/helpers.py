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

TRACE_TOL = 1e-5   # normwise relative tolerance of one iteration (one-step check)
TIE_TOL = 1e-5     # |y_u| below this fraction of max|y| marks a possible sign tie
E2E_TOL = 1e-3     # normwise relative bound of the whole FP32 trajectory against FP64 (restart mode)
GROWTH = 3.0       # edge-memory modes: the bound at iteration t is TRACE_TOL GROWTH^(t-1)
PARITY_LOG = None  # a list to collect the statistics of every comparison, or None

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


def _first_divergence(g, tr, T, Tg):
    """First iteration (0-based) at which the GPU and oracle decisions differ,
    or the last common iteration when only the stop differs; None if the two
    runs are decision-for-decision equal."""
    n = min(T, Tg)
    for t in range(n):
        if not np.array_equal(g[t] < 0, tr[t] < 0):
            return t
    return None if T == Tg else n - 1


def compare_with_oracle(gpu_words, gpu_iters, gpu_flags, gpu_trace, orc_c, orc_it, orc_cv, orc_tr,
                        max_tie_frac=0.02, onestep=None, traj_tol=None):
    """Parity bar of the FP32 decoders against the FP64 oracle.

    Decisions: identical decoded words, iteration counts and flags on every
    frame that is not a tie; at most max_tie_frac ties.  A differing frame is
    a tie only if the oracle's posterior has a coordinate near zero
    (relative to the frame's largest magnitude at that iteration) at or
    before the first divergence.  With the GPU trace the divergence is the
    first iteration whose GPU and oracle decisions differ, "near" means within
    max(TIE_TOL, the GPU's normwise deviation from the oracle at that
    iteration), and that deviation must itself stay within the trajectory
    bound through the divergence: the flip is a sign decision inside the
    FP32 error envelope.  Without the trace the divergence is the last
    iteration both runs execute and "near" means within TIE_TOL.

    Posteriors (with a GPU trace), normwise, max_u |gpu - ref| <= tol max_u |ref|:
      - onestep = (H, Hstd, llr, d_o, n_branches, alpha) for the restart mode,
        where an iteration is a function of y alone: every iteration t of the
        GPU trace, on every frame, against one oracle iteration run from the
        GPU's own iterate t - 1 (the channel LLRs for t = 1), tol = TRACE_TOL;
      - the whole trajectory against the oracle's, on every iteration before
        the first divergence: it bounds the compounding of FP32 rounding over
        the iterations, which the one-step check does not charge.  Restart
        mode: within E2E_TOL.  Edge-memory modes, whose message state the GPU
        does not export, so that this is their only check of the posteriors:
        within TRACE_TOL GROWTH^(t-1) at iteration t, i.e. the one-step bound
        at the first iteration (which starts from the channel LLRs and zero
        messages on both sides) and at most three-fold amplification per
        iteration after it; measured, non-converging frames of plain NMS on
        the standard matrix grow about 2.5-fold per iteration, 1e-7 after one
        iteration and 1.7e-3 after twelve.  traj_tol overrides with a flat
        bound.
    Returns (n_frames, n_ties)."""
    F, N = orc_c.shape
    T_max = orc_tr.shape[1]
    if traj_tol is not None:
        bound = np.full(T_max, traj_tol)
    elif onestep is not None:
        bound = np.full(T_max, E2E_TOL)
    else:
        bound = TRACE_TOL * GROWTH ** np.arange(T_max)
    ties, tie_rho, worst_traj, worst_frac = 0, 0.0, 0.0, 0.0
    for f in range(F):
        T, Tg = int(orc_it[f]), int(gpu_iters[f])
        tr = orc_tr[f, :T]
        scale = np.abs(tr).max(axis=1)
        rho = np.abs(tr).min(axis=1) / np.where(scale > 0, scale, 1.0)
        same = (np.array_equal(gpu_words[f], orc_c[f]) and Tg == T
                and bool(gpu_flags[f]) == bool(orc_cv[f]))
        near = np.full(T, TIE_TOL)
        if gpu_trace is not None:
            g = gpu_trace[f, :Tg, :N].astype(np.float64)
            t_div = _first_divergence(g, tr, T, Tg)
            upto = T if t_div is None else t_div
            n = min(T, Tg)
            err = np.abs(g[:n] - tr[:n]).max(axis=1) / np.where(scale[:n] > 0, scale[:n], 1.0)
            if upto:
                worst_traj = max(worst_traj, float(err[:upto].max()))
                worst_frac = max(worst_frac, float((err[:upto] / bound[:upto]).max()))
                assert (err[:upto] <= bound[:upto]).all(), ("trajectory", f, err[:upto])
            if t_div is not None:
                assert err[t_div] <= bound[t_div], ("frame %d differs without a tie (deviation %.3g at the "
                                                    "divergence)" % (f, err[t_div]), t_div)
                near[:n] = np.maximum(TIE_TOL, err)
        else:
            t_div = None if same else min(T, Tg) - 1
        if not same:
            last = min(T, Tg) - 1 if t_div is None else t_div
            excess = rho[:last + 1] - near[:last + 1]
            assert float(excess.min()) < 0, ("frame %d differs without a tie" % f, float(rho[:last + 1].min()),
                                             last)
            ties += 1
            tie_rho = max(tie_rho, float(rho[:last + 1].min()))
    assert ties <= max_tie_frac * F + 1, (ties, F)
    worst_one = 0.0
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
        rel = err / np.where(sc > 0, sc, 1.0)
        worst_one = float(rel.max())
        bad = np.nonzero(err > TRACE_TOL * sc)[0]
        assert bad.size == 0, [(src[i], err[i] / sc[i]) for i in bad[:5]]
    if PARITY_LOG is not None:
        PARITY_LOG.append({"frames": F, "ties": ties, "tie_rho_max": tie_rho, "traj_max": worst_traj,
                           "traj_frac_of_bound": worst_frac, "onestep_max": worst_one})
    return F, ties


def adversarial_frames(N, ld, F, seed, kind):
    """Frames that probe the decoders' corner cases (FP32 [F][ld]):
      - "equal": every |L| equal (2.5) with random signs: all row minima tie
        and exact zeros of the posterior become possible;
      - "negzero": channel-like values with a fifth of the coordinates set to
        -0.0 and a tenth to +0.0 (sgn(-0.0) = +1, decision [y < 0]);
      - "denormal": channel-like values scaled by 2^-132, so that every
        magnitude is an FP32 subnormal;
      - "mixed": half the coordinates subnormal, the rest normal, some -0.0."""
    rng = np.random.default_rng(seed)
    x = np.zeros((F, ld), np.float32)
    base = (rng.standard_normal((F, N)) * 2.0 + 2.5).astype(np.float32) * np.where(
        rng.random((F, N)) < 0.15, -1, 1).astype(np.float32)
    if kind == "equal":
        x[:, :N] = np.where(rng.random((F, N)) < 0.5, -2.5, 2.5)
    elif kind == "negzero":
        v = base.copy()
        u = rng.random((F, N))
        v[u < 0.2] = -0.0
        v[(u >= 0.2) & (u < 0.3)] = 0.0
        x[:, :N] = v
    elif kind == "denormal":
        x[:, :N] = (base.astype(np.float64) * 2.0 ** -132).astype(np.float32)
    elif kind == "mixed":
        v = base.copy()
        u = rng.random((F, N))
        v[u < 0.5] = (v[u < 0.5].astype(np.float64) * 2.0 ** -132).astype(np.float32)
        v[u > 0.9] = -0.0
        x[:, :N] = v
    else:
        raise ValueError(kind)
    return x
