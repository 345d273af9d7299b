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
