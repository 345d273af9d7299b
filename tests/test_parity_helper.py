"""CPU checks of the parity comparison used by the GPU tests: the oracle's own
trace, rounded to FP32, passes; a perturbation of one iteration beyond the
tolerance is caught by the one-step check."""
import numpy as np
import pytest

import oracle
import synth
from tests.helpers import compare_with_oracle, oracle_code, oracle_hopt


def _run(name="bch63_45", rows=33, F=150, ebn0=2.5, B=9):
    oc = oracle_code(name)
    H = oracle_hopt(name, rows)
    fr = synth.frames(name, F, ebn0, seed=5)
    res = oracle.decode_batch(H, oc.Hstd, fr.llr, fr.d_o, B, 0.75, 8, oracle.R1, threads=4, trace=True)
    c, it, cv, tr = res
    ld = fr.llr.shape[1]
    g_tr = np.zeros((F, 8, ld), np.float32)
    g_tr[:, :, :oc.N] = tr.astype(np.float32)
    onestep = (H, oc.Hstd, fr.llr, fr.d_o, B, 0.75)
    return (c, it, cv.astype(np.uint8), g_tr), res, onestep


def test_fp32_rounded_oracle_trace_passes():
    g, res, onestep = _run()
    compare_with_oracle(*g, *res, onestep=onestep)
    compare_with_oracle(*g, *res)


def test_one_step_check_catches_a_perturbed_iteration():
    g, res, onestep = _run()
    c, it, cv, g_tr = g
    f = int(np.argmax(it >= 3))
    assert it[f] >= 3
    scale = np.abs(g_tr[f, 1]).max()
    g_tr = g_tr.copy()
    g_tr[f, 1, 7] += np.float32(1e-4 * scale)  # iteration 2 of frame f, one coordinate
    with pytest.raises(AssertionError):
        compare_with_oracle(c, it, cv, g_tr, *res, onestep=onestep)


def test_decision_flip_without_tie_is_caught():
    """A frame whose decoded word differs while the oracle's posterior never
    comes near zero is not a tie, with or without the GPU trace."""
    g, res, onestep = _run()
    c, it, cv, g_tr = g
    tr = res[3]
    rho = np.array([np.nanmin(np.abs(tr[f, :it[f]]) / np.nanmax(np.abs(tr[f, :it[f]]), axis=1, keepdims=True))
                    for f in range(len(it))])
    f = int(np.argmax(rho > 1e-3))
    assert rho[f] > 1e-3
    bad = c.copy()
    bad[f, 3] ^= 1
    with pytest.raises(AssertionError, match="without a tie"):
        compare_with_oracle(bad, it, cv, None, *res)
    g2 = g_tr.copy()
    g2[f, 0, :] = -g2[f, 0, :]  # every decision of iteration 1 flipped
    with pytest.raises(AssertionError, match="without a tie"):
        compare_with_oracle(bad, it, cv, g2, *res)


def test_near_zero_after_the_divergence_does_not_excuse():
    """Hand-made 7-coordinate frame: the GPU's decision differs at iteration
    1, where every oracle |y| is at least half the largest; the oracle's only
    near-zero value comes at iteration 3, after the divergence."""
    N, T = 7, 3
    tr = np.array([[[4.0, -3.0, 2.5, 3.0, -2.0, 5.0, 2.0],
                    [5.0, -4.0, 3.0, 3.5, -2.5, 6.0, 2.5],
                    [6.0, -5.0, 1e-9, 4.0, -3.0, 7.0, 3.0]]])
    orc_c = (tr[:, -1] < 0).astype(np.uint8)
    orc_it, orc_cv = np.array([T]), np.array([False])
    g = np.zeros((1, T, 8), np.float32)
    g[0, :, :N] = tr[0]
    g[0, 0, 2] = -2.5  # flipped at iteration 1
    gw = orc_c.copy()
    gw[0, 2] ^= 1
    with pytest.raises(AssertionError, match="without a tie"):
        compare_with_oracle(gw, orc_it, np.array([0]), g, orc_c, orc_it, orc_cv, tr)
    # the same flip at iteration 3, where the oracle value is within 1e-5 of zero, is a tie
    g[0, 0, 2] = 2.5
    g[0, 2, 2] = -1e-9
    assert compare_with_oracle(gw, orc_it, np.array([0]), g, orc_c, orc_it, orc_cv, tr) == (1, 1)


def test_flip_inside_the_measured_drift_is_a_tie():
    """With the GPU trace, a coordinate at 3e-5 of the frame's scale that
    flips where the GPU trajectory deviates by 6e-5 is a tie under a 1e-3
    trajectory bound, not under the edge-memory bound at iteration 2 (3e-5),
    and not when the deviation elsewhere exceeds the bound."""
    N, T = 7, 2
    tr = np.array([[[4.0, -3.0, 2.5, 3.0, -2.0, 5.0, 2.0],
                    [5.0, -4.0, 1.5e-4, 3.5, -2.5, 5.0, 2.5]]])
    orc_c = (tr[:, -1] < 0).astype(np.uint8)
    orc_it, orc_cv = np.array([T]), np.array([False])
    g = np.zeros((1, T, 8), np.float32)
    g[0, :, :N] = tr[0]
    g[0, 1, 2] = -1.5e-4  # deviation 3e-4 / 5 = 6e-5 at iteration 2
    gw = orc_c.copy()
    gw[0, 2] ^= 1
    assert compare_with_oracle(gw, orc_it, np.array([0]), g, orc_c, orc_it, orc_cv, tr, traj_tol=1e-3) == (1, 1)
    # the edge-memory bound at iteration 2 is 3e-5: the same flip is beyond it
    with pytest.raises(AssertionError, match="without a tie"):
        compare_with_oracle(gw, orc_it, np.array([0]), g, orc_c, orc_it, orc_cv, tr)
    g[0, 1, 0] = 5.1  # plus a deviation of 0.1 / 5.1 = 2e-2 elsewhere: beyond the flat bound too
    with pytest.raises(AssertionError, match="without a tie"):
        compare_with_oracle(gw, orc_it, np.array([0]), g, orc_c, orc_it, orc_cv, tr, traj_tol=1e-3)
