"""Parity of the HIP decoders with the oracle (run on an MI355X).

Every test decodes the same seeded synthetic frames with the C-ABI library on
the GPU and with the FP64 oracle on the CPU, and applies the bar of
tests/helpers.compare_with_oracle: identical decoded words, iteration counts and
convergence flags on all frames but ties (a near-zero oracle posterior at or
before the first divergence); in restart mode every iteration's posterior
within 1e-5 (normwise) of one oracle iteration from the GPU's own previous
iterate; and the whole FP32 trajectory within 1e-3 of the FP64 one up to the
divergence.  The fixed-point kernels are bit-exact against the integer
oracle."""
import numpy as np
import pytest

import oracle
import synth
from tests.helpers import HO_ROWS, adversarial_frames, compare_with_oracle, ensure_built, oracle_code, oracle_hopt

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    b = ensure_built()
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return b


def lib_objects(B, name, rows):
    d = B.CODE_DEFS[name]
    c = B.Code(d.m, d.prim, d.t)
    p = B.Pcm.standard(c) if rows == 0 else B.Pcm.build(c, target_rows=rows, seed=1)
    return c, p


def run_pair(B, name, rows, F, ebn0, seed, n_branches, mode, max_iter, alpha=0.75, flags=0, llr_h=None):
    c, p = lib_objects(B, name, rows)
    oc = oracle_code(name)
    H = oc.Hstd if rows == 0 else oracle_hopt(name, rows)
    assert np.array_equal(p.dense(), H)
    fr = synth.frames(name, F, ebn0, seed=seed)
    if llr_h is not None:
        fr.llr = llr_h
    dec = B.Decoder(c, p, n_branches=n_branches, mode=mode, alpha=alpha, max_iter=max_iter, flags=flags)
    llr = torch.from_numpy(fr.llr).cuda()
    d_o = torch.from_numpy(fr.d_o).cuda()
    bits, iters, flg, tr = dec.decode(llr, d_o, trace=True)
    torch.cuda.synchronize()
    words = B.unpack_bits(bits.cpu().numpy().view(np.uint64), c.N)
    res = oracle.decode_batch(H, oc.Hstd, fr.llr, fr.d_o, n_branches, alpha, max_iter, mode,
                              threads=8, trace=True)
    dec.onestep = (H, oc.Hstd, fr.llr, fr.d_o, n_branches, alpha) if mode == oracle.R1 else None
    return fr, (words, iters.cpu().numpy(), flg.cpu().numpy(), tr.cpu().numpy()), res, dec


@pytest.mark.parametrize("generic", [False, True])
@pytest.mark.parametrize("name,ebn0", [("bch63_45", 3.0), ("bch63_36", 3.5), ("bch127_99", 4.0),
                                       ("bch127_64", 4.0), ("bch127_78", 4.0)])
def test_enhanced_nms_restart_mode(B, name, ebn0, generic):
    F = 64 * 7 + 37  # several waves and a ragged tail
    fr, g, o, dec = run_pair(B, name, HO_ROWS[name], F, ebn0, 11, 9, oracle.R1, 8,
                             flags=B.FORCE_GENERIC if generic else 0)
    assert dec.specialized == (not generic)
    compare_with_oracle(*g, *o, onestep=dec.onestep)


def test_small_batch_kernel_selection(B):
    """N = 127: decodes of at most 128 frames per CU run the three-wave kernel,
    larger ones the kernel of one wave per 64 frames; the flags force either.
    N = 63 has the three-wave kernel only."""
    c, p = lib_objects(B, "bch127_64", 72)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    dec = B.Decoder(c, p, n_branches=9, mode=B.MODE_RESTART, alpha=0.75, max_iter=8)
    assert dec.kernel_name(128 * n_cu) == "spec_bch127_64_m72_b9_grp"
    assert dec.kernel_name(128 * n_cu + 1) == "spec_bch127_64_m72_b9"
    always = B.Decoder(c, p, n_branches=9, mode=B.MODE_RESTART, alpha=0.75, max_iter=8, flags=B.SMALL_ALWAYS)
    assert always.kernel_name(10 ** 7) == "spec_bch127_64_m72_b9_grp"
    never = B.Decoder(c, p, n_branches=9, mode=B.MODE_RESTART, alpha=0.75, max_iter=8, flags=B.SMALL_NEVER)
    assert never.kernel_name(100) == "spec_bch127_64_m72_b9"
    packed = B.Decoder(c, p, n_branches=9, max_iter=8, precision=B.FIX8, flags=B.PACKED16)
    assert packed.kernel_name(100) == "spec_bch127_64_m72_b9_fix8_pk16"
    # fixed point without flags: the packed 16-bit kernel from 4,000,000 frames (N = 127)
    fix = B.Decoder(c, p, n_branches=9, max_iter=8, precision=B.FIX8)
    assert fix.kernel_name(100) == "spec_bch127_64_m72_b9_fix8_grp"
    assert fix.kernel_name(3_999_999) == "spec_bch127_64_m72_b9_fix8"
    assert fix.kernel_name(4_000_000) == "spec_bch127_64_m72_b9_fix8_pk16"
    unp = B.Decoder(c, p, n_branches=9, max_iter=8, precision=B.FIX8, flags=B.UNPACKED16)
    assert unp.kernel_name(10 ** 8) == "spec_bch127_64_m72_b9_fix8"
    with pytest.raises(B.BchError):
        B.Decoder(c, p, n_branches=9, max_iter=8, precision=B.FIX8, flags=B.PACKED16 | B.UNPACKED16)
    c63, p63 = lib_objects(B, "bch63_36", 122)
    d63 = B.Decoder(c63, p63, n_branches=9, mode=B.MODE_RESTART, alpha=0.75, max_iter=8)
    assert d63.kernel_name(100) == d63.kernel_name(10 ** 7) == "spec_bch63_36_m122_b9"
    f63 = B.Decoder(c63, p63, n_branches=9, max_iter=8, precision=B.FIX8)
    assert f63.kernel_name(7_999_999) == "spec_bch63_36_m122_b9_fix8"
    assert f63.kernel_name(8_000_000) == "spec_bch63_36_m122_b9_fix8_pk16"
    gen = B.Decoder(c, p, n_branches=9, mode=B.MODE_RESTART, alpha=0.75, max_iter=8, flags=B.FORCE_GENERIC)
    assert gen.kernel_name(100) == "generic"
    for bad in (B.SMALL_ALWAYS | B.SMALL_NEVER, 256):
        with pytest.raises(B.BchError):
            B.Decoder(c, p, n_branches=9, mode=B.MODE_RESTART, alpha=0.75, max_iter=8, flags=bad)


@pytest.mark.parametrize("flags", ["SMALL_ALWAYS", "SMALL_NEVER"])
@pytest.mark.parametrize("name,ebn0", [("bch127_99", 4.0), ("bch127_64", 4.0), ("bch127_78", 4.0)])
def test_127_kernels_both_forms(B, name, ebn0, flags):
    """Both N = 127 kernels (three waves per 64 frames, and one) against the
    oracle on several waves and a ragged tail."""
    F = 64 * 7 + 37
    fr, g, o, dec = run_pair(B, name, HO_ROWS[name], F, ebn0, 13, 9, oracle.R1, 8, flags=getattr(B, flags))
    assert dec.kernel_name(F).endswith("_grp") == (flags == "SMALL_ALWAYS")
    compare_with_oracle(*g, *o, onestep=dec.onestep)


@pytest.mark.parametrize("flags", ["SMALL_ALWAYS", "SMALL_NEVER"])
@pytest.mark.parametrize("name,ebn0", [("bch127_99", 4.0), ("bch127_64", 3.5)])
def test_127_fixed_point_both_forms(B, name, ebn0, flags):
    """Both N = 127 fixed-point kernels bit-exact against the integer oracle,
    every frame, iteration count and per-iteration posterior."""
    F = 64 * 5 + 29
    fr, w, it, fl, tr, ow, oit, ocv, otr = run_fix8_pair(B, name, HO_ROWS[name], F, ebn0, 43,
                                                         flags=getattr(B, flags))
    assert np.array_equal(w, ow)
    assert np.array_equal(it, oit)
    assert np.array_equal(fl.astype(bool), ocv)
    for f in range(F):
        assert np.array_equal(tr[f, :oit[f], :w.shape[1]], otr[f, :oit[f]]), f


def test_small_batch_kernel_large_batch_sampled(B):
    """The three-wave N = 127 kernel forced onto a batch of 400,000 frames
    (many frames per lane, every bucket drained): sampled frames against the
    oracle, and every converged word passes the syndrome test."""
    name, rows, F = "bch127_64", 72, 400_000
    c, p = lib_objects(B, name, rows)
    oc = oracle_code(name)
    H = oracle_hopt(name, rows)
    dec = B.Decoder(c, p, n_branches=9, mode=B.MODE_RESTART, alpha=0.75, max_iter=8, flags=B.SMALL_ALWAYS)
    assert dec.kernel_name(F).endswith("_grp")
    parts = [synth.frames(name, F // 4, 3.5, seed=88, block=k) for k in range(4)]
    llr = torch.from_numpy(np.concatenate([q.llr for q in parts])).cuda()
    d_o = torch.from_numpy(np.concatenate([q.d_o for q in parts])).cuda()
    bits, iters, flg, _ = dec.decode(llr, d_o)
    ok = torch.empty(F, dtype=torch.uint8, device="cuda")
    B.syndrome_check(c, bits, ok)
    torch.cuda.synchronize()
    flg_h = flg.cpu().numpy()
    it_h = iters.cpu().numpy()
    assert np.array_equal(ok.cpu().numpy()[flg_h == 1], np.ones(int(flg_h.sum()), np.uint8))
    assert it_h.min() >= 1 and it_h.max() <= 8 and (it_h[flg_h == 0] == 8).all()
    idx = np.sort(np.random.default_rng(9).choice(F, 800, replace=False))
    res = oracle.decode_batch(H, oc.Hstd, llr[torch.from_numpy(idx).cuda()].cpu().numpy(), d_o.cpu().numpy()[idx],
                              9, 0.75, 8, oracle.R1, threads=8, trace=True)
    words = B.unpack_bits(bits.cpu().numpy().view(np.uint64)[idx], c.N)
    compare_with_oracle(words, it_h[idx], flg_h[idx], None, *res)


@pytest.mark.parametrize("F", [1, 2, 63, 64, 65, 300])
def test_specialised_small_and_ragged_batches(B, F):
    fr, g, o, dec = run_pair(B, "bch63_45", 33, F, 2.0, 30 + F, 9, oracle.R1, 8)
    assert dec.specialized
    compare_with_oracle(*g, *o, onestep=dec.onestep)


@pytest.mark.parametrize("name,rows,F,ebn0", [("bch63_45", 33, 1_000_000, 3.0),
                                              ("bch63_36", 122, 1_000_000, 3.5),
                                              ("bch127_64", 72, 4_000_000, 4.0)])
def test_full_size_batches_sampled(B, name, rows, F, ebn0):
    """Batch sizes of the paper-sized workloads (1,000,000 frames per point for
    the length-63 codes, 4,000,000 for length 127) in the benchmark's launch
    configuration; the oracle decodes a random sample of frames one by one and
    every converged frame's word must satisfy the syndrome test."""
    c, p = lib_objects(B, name, rows)
    oc = oracle_code(name)
    H = oracle_hopt(name, rows)
    dec = B.Decoder(c, p, n_branches=9, mode=B.MODE_RESTART, alpha=0.75, max_iter=8)
    assert dec.specialized
    blocks = 8
    per = F // blocks
    parts = [synth.frames(name, per, ebn0, seed=77, block=k) for k in range(blocks)]
    llr = torch.from_numpy(np.concatenate([q.llr for q in parts])).cuda()
    d_o = torch.from_numpy(np.concatenate([q.d_o for q in parts])).cuda()
    bits, iters, flg, _ = dec.decode(llr, d_o)
    ok = torch.empty(F, dtype=torch.uint8, device="cuda")
    B.syndrome_check(c, bits, ok)
    torch.cuda.synchronize()
    flg_h = flg.cpu().numpy()
    assert np.array_equal(ok.cpu().numpy()[flg_h == 1], np.ones(int(flg_h.sum()), np.uint8))
    it_h = iters.cpu().numpy()
    assert it_h.min() >= 1 and it_h.max() <= 8 and (it_h[flg_h == 0] == 8).all()
    rng = np.random.default_rng(5)
    idx = np.sort(rng.choice(F, 1500, replace=False))
    llr_h = llr[torch.from_numpy(idx).cuda()].cpu().numpy()
    d_h = d_o.cpu().numpy()[idx]
    res = oracle.decode_batch(H, oc.Hstd, llr_h, d_h, 9, 0.75, 8, oracle.R1, threads=8, trace=True)
    words = B.unpack_bits(bits.cpu().numpy().view(np.uint64)[idx], c.N)
    compare_with_oracle(words, it_h[idx], flg_h[idx], None, *res)


@pytest.mark.parametrize("name,rows,nb,precision,flags", [("bch127_64", 72, 9, "fp32", 0),
                                                         ("bch127_99", 33, 9, "fix8", "PACKED16"),
                                                         ("bch127_99", 33, 9, "fix8", "UNPACKED16"),
                                                         ("bch63_36", 122, 9, "fp32", 0),
                                                         ("bch63_45", 33, 1, "fp32", 0)])
def test_range_buckets_equal_chunked_calls(B, name, rows, nb, precision, flags):
    """With CHUNK_BUCKETS, from 1,048,576 frames the prepass also deals
    chunks of 65,536 frames to eight ranges, one per XCD.  Every frame of a
    1,300,000-frame call (ranges of two or three chunks, the last one ragged)
    must equal, in word, iteration count and flag, the same frame decoded in
    calls of at most 500,000 frames (no ranges): nothing is lost, repeated or
    decoded with another frame's offset (one branch: a single offset bucket
    per range)."""
    F, chunk = 1_300_000, 500_000
    c, p = lib_objects(B, name, rows)
    dec = B.Decoder(c, p, n_branches=nb, mode=B.MODE_RESTART, alpha=0.75, max_iter=8,
                    precision=B.FIX8 if precision == "fix8" else B.FP32,
                    flags=(getattr(B, flags) if flags else 0) | B.CHUNK_BUCKETS)
    assert dec.specialized
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(8) as ex:
        parts = list(ex.map(lambda k: synth.frames(name, 100_000, 2.5 + 0.1 * k, seed=91, block=k), range(13)))
    llr = torch.from_numpy(np.concatenate([q.llr for q in parts])).cuda()
    d_o = torch.from_numpy(np.concatenate([q.d_o for q in parts])).cuda()
    if precision == "fix8":
        q8 = torch.empty(llr.shape, dtype=torch.int8, device="cuda")
        B.quantize_llr(llr, c.N, 4.0, q8)
        llr = q8
    whole = dec.decode(llr, d_o)[:3]
    outs = [dec.decode(llr[k:k + chunk].contiguous(), d_o[k:k + chunk].contiguous())[:3] for k in range(0, F, chunk)]
    torch.cuda.synchronize()
    for j in range(3):
        assert torch.equal(whole[j], torch.cat([o[j] for o in outs])), j
    assert int(whole[1].min()) >= 1


@pytest.mark.parametrize("name,rows,per,grid,precision", [
    ("bch63_36", 122, 1_000_000, (1.0, 6.0, 0.5), "fp32"),
    ("bch127_64", 72, 4_000_000, (2.0, 5.0, 0.5), "fp32"),
    ("bch127_64", 72, 4_000_000, (2.0, 5.0, 0.5), "fix8"),
    ("bch127_64", 72, 4_000_000, (2.0, 5.0, 0.5), "fix8_packed16"),
    ("bch63_36", 122, 1_000_000, (1.0, 6.0, 0.5), "fix8_packed16")])
def test_sweep_in_one_call_sampled(B, name, rows, per, grid, precision):
    """A whole Eb/N0 sweep of one code in a single decode call, as the
    benchmark launches it by default: 11 x 1,000,000 frames for length 63 and
    7 x 4,000,000 for length 127.  Every converged word must pass the syndrome
    test; sampled frames of every point must equal the oracle (FP32: the
    tolerance of compare_with_oracle; int8: bit-exact)."""
    from concurrent.futures import ThreadPoolExecutor
    c, p = lib_objects(B, name, rows)
    oc = oracle_code(name)
    H = oracle_hopt(name, rows)
    lo, hi, st = grid
    points = [lo + k * st for k in range(int(round((hi - lo) / st)) + 1)]
    F = per * len(points)
    ld = 64 if c.N <= 64 else 128
    llr = torch.empty((F, ld), dtype=torch.float32, device="cuda")
    d_o = torch.empty(F, dtype=torch.uint8, device="cuda")
    blk = 500_000
    jobs = [(j, e, k) for j, e in enumerate(points) for k in range(per // blk)]
    with ThreadPoolExecutor(8) as ex:
        for (j, e, k), q in zip(jobs, ex.map(lambda a: synth.frames(name, blk, a[1], seed=123 + a[0], block=a[2]),
                                              jobs)):
            f0 = j * per + k * blk
            llr[f0:f0 + blk].copy_(torch.from_numpy(q.llr))
            d_o[f0:f0 + blk].copy_(torch.from_numpy(q.d_o))
    if precision.startswith("fix8"):
        inp = torch.empty(llr.shape, dtype=torch.int8, device="cuda")
        B.quantize_llr(llr, c.N, 4.0, inp)
        del llr
        dec = B.Decoder(c, p, n_branches=9, max_iter=8, precision=B.FIX8,
                        flags=B.PACKED16 if precision == "fix8_packed16" else B.UNPACKED16)
    else:
        inp = llr
        dec = B.Decoder(c, p, n_branches=9, mode=B.MODE_RESTART, alpha=0.75, max_iter=8)
    assert dec.specialized
    bits, iters, flg, _ = dec.decode(inp, d_o)
    ok = torch.empty(F, dtype=torch.uint8, device="cuda")
    B.syndrome_check(c, bits, ok)
    torch.cuda.synchronize()
    flg_h = flg.cpu().numpy()
    it_h = iters.cpu().numpy()
    assert np.array_equal(ok.cpu().numpy()[flg_h == 1], np.ones(int(flg_h.sum()), np.uint8))
    assert it_h.min() >= 1 and it_h.max() <= 8 and (it_h[flg_h == 0] == 8).all()
    rng = np.random.default_rng(17)
    idx = np.sort(np.concatenate([j * per + rng.choice(per, 150, replace=False) for j in range(len(points))]))
    x_h = inp[torch.from_numpy(idx).cuda()].cpu().numpy()
    d_h = d_o.cpu().numpy()[idx]
    words = B.unpack_bits(bits.cpu().numpy().view(np.uint64)[idx], c.N)
    if precision.startswith("fix8"):
        ow, oit, ocv = oracle.decode_batch(H, oc.Hstd, x_h, d_h, 9, 0.75, 8, oracle.R1,
                                           kind=oracle.KIND_FIXED, threads=8)
        assert np.array_equal(words, ow)
        assert np.array_equal(it_h[idx], oit)
        assert np.array_equal(flg_h[idx].astype(bool), ocv)
    else:
        res = oracle.decode_batch(H, oc.Hstd, x_h, d_h, 9, 0.75, 8, oracle.R1, threads=8, trace=True)
        compare_with_oracle(words, it_h[idx], flg_h[idx], None, *res)


@pytest.mark.parametrize("mode", [oracle.R2, oracle.R3])
def test_enhanced_nms_memory_modes(B, mode):
    """The edge-memory readings of eq. 2 (generic kernel, nine branches):
    every differing frame a tie at or before its divergence, and the FP32
    trajectory within the trajectory bound of the FP64 one up to it."""
    fr, g, o, _ = run_pair(B, "bch63_45", 33, 300, 3.0, 12, 9, mode, 6)
    compare_with_oracle(*g, *o)


def test_plain_nms_standard_matrix_config(B):
    """Plain flooding NMS (one branch, extrinsic messages) on the standard
    27 x 63 matrix of BCH(63,36), alpha 0.75, 12 iterations, 10,000 frames at
    3.0 dB, seed 0: the full parity bar (ties justified at or before the
    divergence, trajectory compared up to it) and equal frame error rates up
    to the ties."""
    fr, g, o, _ = run_pair(B, "bch63_36", 0, 10000, 3.0, 0, 1, oracle.R3, 12)
    _, ties = compare_with_oracle(*g, *o)
    words = g[0]
    err_g = int((words != fr.codewords).any(1).sum())
    err_o = int((o[0] != fr.codewords).any(1).sum())
    assert abs(err_g - err_o) <= ties


@pytest.mark.parametrize("generic", [False, True])
@pytest.mark.parametrize("name,ebn0,alpha,kind", [("bch63_36", 3.0, 0.75, None), ("bch63_45", 3.5, 0.75, None),
                                                  ("bch63_36", 2.0, 1.0, None), ("bch63_45", 2.5, 0.6, None),
                                                  ("bch63_36", 3.0, 0.75, "equal"), ("bch63_45", 3.0, 0.75, "mixed")])
def test_plain_nms_extrinsic_kernel(B, name, ebn0, alpha, kind, generic):
    """The specialised kernel of plain flooding NMS with extrinsic messages
    (one branch, standard matrix) and the generic kernel it replaces, on
    several waves with a ragged tail, at three values of alpha and on
    adversarial frames (equal magnitudes, -0.0 and subnormals): the parity bar
    of the edge-memory modes against the FP64 oracle."""
    N, ld, F = 63, 64, 64 * 5 + 23
    x = adversarial_frames(N, ld, F, 300, kind) if kind else None
    fr, g, o, dec = run_pair(B, name, 0, F, ebn0, 41, 1, oracle.R3, 12, alpha=alpha,
                             flags=B.FORCE_GENERIC if generic else 0, llr_h=x)
    rows = {"bch63_36": 27, "bch63_45": 18}[name]
    assert dec.kernel_name(F) == ("generic" if generic else "spec_%s_m%d_b1_ext" % (name, rows))
    compare_with_oracle(*g, *o, max_tie_frac=1.0 if kind else 0.02)


def test_plain_nms_extrinsic_kernel_matches_generic(B):
    """At 20,000 frames of BCH(63,36) at 2.5 dB (many frames run all 12
    iterations), the specialised and generic kernels take the same decisions
    except on frames whose posteriors pass within FP32 rounding of zero: at
    most 0.5% differ, and the frame error rates agree within that."""
    c, p = lib_objects(B, "bch63_36", 0)
    fr = synth.frames("bch63_36", 20000, 2.5, seed=43)
    llr = torch.from_numpy(fr.llr).cuda()
    out = []
    for flags in (0, B.FORCE_GENERIC):
        dec = B.Decoder(c, p, n_branches=1, mode=B.MODE_EXTRINSIC, max_iter=12, flags=flags)
        bits, iters, _, _ = dec.decode(llr)
        torch.cuda.synchronize()
        out.append((B.unpack_bits(bits.cpu().numpy().view(np.uint64), c.N), iters.cpu().numpy()))
    diff = (out[0][0] != out[1][0]).any(1) | (out[0][1] != out[1][1])
    assert diff.mean() <= 0.005
    errs = [int((w != fr.codewords).any(1).sum()) for w, _ in out]
    assert abs(errs[0] - errs[1]) <= int(diff.sum())


@pytest.mark.parametrize("name,alpha,flags", [("bch63_45", 0.55, 0), ("bch63_45", 1.0, 0), ("bch63_36", 0.55, 0),
                                              ("bch127_64", 1.0, "SMALL_NEVER"), ("bch127_64", 1.0, "SMALL_ALWAYS"),
                                              ("bch127_99", 1.0, "SMALL_NEVER"), ("bch127_99", 0.6, "SMALL_ALWAYS")])
def test_alpha_other_than_three_quarters(B, name, alpha, flags):
    """The normalisation factor of eq. 3 is a run-time parameter of the
    specialised kernels: alpha = 0.55, 0.6 and 1.0 (the bracket of the alpha
    search) on every kernel form, against the oracle at the same alpha."""
    F = 64 * 4 + 21
    fr, g, o, dec = run_pair(B, name, HO_ROWS[name], F, 3.0, 19, 9, oracle.R1, 8, alpha=alpha,
                             flags=getattr(B, flags) if flags else 0)
    assert dec.specialized
    compare_with_oracle(*g, *o, onestep=dec.onestep)


ADV_KINDS = ["equal", "negzero", "denormal", "mixed"]
ADV_FORMS = [("bch63_45", 0), ("bch63_36", 0), ("bch127_64", "SMALL_NEVER"), ("bch127_64", "SMALL_ALWAYS"),
             ("bch127_99", "SMALL_NEVER"), ("bch63_45", "FORCE_GENERIC")]


@pytest.mark.parametrize("kind", ADV_KINDS)
@pytest.mark.parametrize("name,flags", ADV_FORMS)
def test_adversarial_frames_fp32(B, name, flags, kind):
    """Equal magnitudes with random signs, -0.0 entries and FP32 subnormals on
    every FP32 kernel form, against the oracle with the full parity bar.
    Equal magnitudes make exact zeros of the posterior possible, and frames
    with half their coordinates subnormal put those coordinates within
    rounding of zero, so in these two kinds ties are not capped (each must
    still be justified at or before its divergence)."""
    N = 63 if name.startswith("bch63") else 127
    ld = 64 if N == 63 else 128
    F = 64 * 3 + 5
    x = adversarial_frames(N, ld, F, 100 + ADV_KINDS.index(kind), kind)
    fr, g, o, dec = run_pair(B, name, HO_ROWS[name], F, 3.0, 29, 9, oracle.R1, 8,
                             flags=getattr(B, flags) if flags else 0, llr_h=x)
    assert dec.specialized == (flags != "FORCE_GENERIC")
    compare_with_oracle(*g, *o, onestep=dec.onestep, max_tie_frac=1.0 if kind in ("equal", "mixed") else 0.02)


def int8_adversarial(N, ld, F, seed, kind):
    """int8 frames at the ends of the range: "sat" every |q| = 127 with random
    signs, "equal" every |q| = 10, "zeros" half the entries 0."""
    rng = np.random.default_rng(seed)
    q = np.zeros((F, ld), np.int8)
    sg = np.where(rng.random((F, N)) < 0.5, -1, 1)
    if kind == "sat":
        q[:, :N] = 127 * sg
    elif kind == "equal":
        q[:, :N] = 10 * sg
    else:
        v = rng.integers(-127, 128, (F, N))
        v[rng.random((F, N)) < 0.5] = 0
        q[:, :N] = v
    return q


@pytest.mark.parametrize("kind", ["sat", "equal", "zeros", "quant_equal", "quant_mixed"])
@pytest.mark.parametrize("name,flags", [("bch63_45", 0), ("bch63_36", "PACKED16"), ("bch127_64", "SMALL_NEVER"),
                                        ("bch127_64", "SMALL_ALWAYS"), ("bch127_99", "PACKED16")])
def test_adversarial_frames_fixed_point(B, name, flags, kind):
    """Saturated, equal-magnitude and zero-heavy int8 frames (and the
    quantised equal-magnitude and subnormal/-0.0 float frames) on every
    fixed-point kernel form: bit-exact words, iteration counts, flags and
    per-iteration posteriors against the integer oracle."""
    N = 63 if name.startswith("bch63") else 127
    ld = 64 if N == 63 else 128
    F = 128 * 2 + 9
    c, p = lib_objects(B, name, HO_ROWS[name])
    oc = oracle_code(name)
    H = oracle_hopt(name, HO_ROWS[name])
    if kind.startswith("quant_"):
        x = torch.from_numpy(adversarial_frames(N, ld, F, 7, kind[6:])).cuda()
        q = torch.empty(x.shape, dtype=torch.int8, device="cuda")
        B.quantize_llr(x, N, 4.0, q)
    else:
        q = torch.from_numpy(int8_adversarial(N, ld, F, 11, kind)).cuda()
    d_o_h = oracle.draw_offsets(N, 5, 6, 0, F)
    dec = B.Decoder(c, p, n_branches=9, max_iter=8, precision=B.FIX8, flags=getattr(B, flags) if flags else 0)
    assert dec.specialized
    bits, iters, flg, tr = dec.decode(q, torch.from_numpy(d_o_h).cuda(), trace=True)
    torch.cuda.synchronize()
    qh = q.cpu().numpy()
    ow, oit, ocv, otr = oracle.decode_batch(H, oc.Hstd, qh, d_o_h, 9, 0.75, 8, oracle.R1, kind=oracle.KIND_FIXED,
                                            threads=8, trace=True)
    w = B.unpack_bits(bits.cpu().numpy().view(np.uint64), N)
    it, fl, trh = iters.cpu().numpy(), flg.cpu().numpy(), tr.cpu().numpy()
    assert np.array_equal(w, ow) and np.array_equal(it, oit) and np.array_equal(fl.astype(bool), ocv)
    for f in range(F):
        assert np.array_equal(trh[f, :oit[f], :N], otr[f, :oit[f]]), f


@pytest.mark.parametrize("generic", [False, True])
@pytest.mark.parametrize("name,nb", [("bch63_45", 3), ("bch63_36", 3), ("bch63_45", 1), ("bch63_36", 1)])
def test_one_and_three_branch_variants(B, name, nb, generic):
    """Restart mode with 3 branches (the three shifts of y) and with 1 (NMS on
    H_o alone): the specialised kernels of the branch-count ablation and the
    generic kernel, against the oracle."""
    F = 64 * 3 + 9
    fr, g, o, dec = run_pair(B, name, HO_ROWS[name], F, 3.0, 13, nb, oracle.R1, 8,
                             flags=B.FORCE_GENERIC if generic else 0)
    assert dec.specialized == (not generic)
    compare_with_oracle(*g, *o, onestep=dec.onestep)


@pytest.mark.parametrize("name,rows,nb,mode", [("bch63_36", 0, 1, "MODE_EXTRINSIC"), ("bch63_45", 0, 1, "MODE_EXTRINSIC"),
                                               ("bch63_45", 33, 1, "MODE_RESTART"), ("bch63_36", 122, 3, "MODE_RESTART")])
def test_reserved_handout_covers_every_frame(B, name, rows, nb, mode):
    """The one- and three-branch kernels take frames with a private reserve
    of 64 slots per wave while their bucket is far from dry.  A 300,000-frame
    call (many reserves per wave, then exact grabs near the end) must decode
    every frame exactly as calls of 20,000 frames do, where the reserve rarely
    engages: nothing lost, repeated or decoded twice."""
    F, chunk = 300_000, 20_000
    c, p = lib_objects(B, name, rows)
    dec = B.Decoder(c, p, n_branches=nb, mode=getattr(B, mode), alpha=0.75, max_iter=8)
    assert dec.specialized
    fr = synth.frames(name, F, 2.5, seed=97)
    llr = torch.from_numpy(fr.llr).cuda()
    d_o = torch.from_numpy(fr.d_o).cuda()
    whole = dec.decode(llr, d_o)[:3]
    outs = [dec.decode(llr[k:k + chunk].contiguous(), d_o[k:k + chunk].contiguous())[:3] for k in range(0, F, chunk)]
    torch.cuda.synchronize()
    for j in range(3):
        assert torch.equal(whole[j], torch.cat([o[j] for o in outs])), j
    assert int(whole[1].min()) >= 1


def test_edge_cases(B):
    c, p = lib_objects(B, "bch63_45", 33)
    dec = B.Decoder(c, p, n_branches=9, max_iter=8)
    # F = 0 is a no-op
    e = torch.empty((0, 64), dtype=torch.float32, device="cuda")
    bits, its, flg, _ = dec.decode(e, torch.empty(0, dtype=torch.uint8, device="cuda"))
    assert bits.shape[0] == 0
    # all-zero LLRs: the zero word satisfies every check at once
    z = torch.zeros((65, 64), dtype=torch.float32, device="cuda")
    bits, its, flg, _ = dec.decode(z, torch.zeros(65, dtype=torch.uint8, device="cuda"))
    torch.cuda.synchronize()
    assert (bits.cpu() == 0).all() and (its.cpu() == 1).all() and (flg.cpu() == 1).all()
    # huge and tiny (normal) magnitudes decode like the unscaled frames
    fr = synth.frames("bch63_45", 130, 3.0, seed=21)
    d_o = torch.from_numpy(fr.d_o).cuda()
    ref = dec.decode(torch.from_numpy(fr.llr).cuda(), d_o)
    for s in (2.0 ** 60, 2.0 ** -60):
        out = dec.decode(torch.from_numpy(fr.llr * np.float32(s)).cuda(), d_o)
        torch.cuda.synchronize()
        assert torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1])


@pytest.mark.parametrize("prec,flags", [("fp32", "SMALL_ALWAYS"), ("fp32", "SMALL_NEVER"), ("fix8", "SMALL_ALWAYS"),
                                         ("fix8", "PACKED16")])
def test_edge_cases_127(B, prec, flags):
    """Empty, single-frame and all-zero batches on each N = 127 kernel."""
    c, p = lib_objects(B, "bch127_64", 72)
    precision = B.FIX8 if prec == "fix8" else B.FP32
    dec = B.Decoder(c, p, n_branches=9, max_iter=8, precision=precision, flags=getattr(B, flags))
    assert dec.specialized
    dt = torch.int8 if prec == "fix8" else torch.float32
    bits, its, flg, _ = dec.decode(torch.empty((0, 128), dtype=dt, device="cuda"),
                                   torch.empty(0, dtype=torch.uint8, device="cuda"))
    assert bits.shape[0] == 0
    for F in (1, 129):
        z = torch.zeros((F, 128), dtype=dt, device="cuda")
        d_o = torch.arange(F, dtype=torch.int32, device="cuda").remainder(42).to(torch.uint8)
        bits, its, flg, _ = dec.decode(z, d_o)
        torch.cuda.synchronize()
        assert (bits.cpu() == 0).all() and (its.cpu() == 1).all() and (flg.cpu() == 1).all()


def test_syndrome_kernel(B):
    c, _ = lib_objects(B, "bch127_99", 33)
    fr = synth.frames("bch127_99", 300, 4.0, seed=3)
    words = fr.codewords.copy()
    words[::3, 5] ^= 1
    packed = np.zeros((300, 2), np.uint64)
    for i in range(127):
        packed[:, i // 64] |= words[:, i].astype(np.uint64) << np.uint64(i % 64)
    bits = torch.from_numpy(packed.view(np.int64)).cuda()
    ok = torch.empty(300, dtype=torch.uint8, device="cuda")
    B.syndrome_check(c, bits, ok)
    torch.cuda.synchronize()
    oc = oracle_code("bch127_99")
    want = ~(((words.astype(int) @ oc.Hstd.T.astype(int)) % 2).any(1))
    assert np.array_equal(ok.cpu().numpy().astype(bool), want)


def test_quantizer_bit_exact(B):
    fr = synth.frames("bch63_36", 500, 2.0, seed=4)
    below = np.nextafter(np.float32(0.125), np.float32(0))  # x 4 = 0.49999997, rounds to 0
    fr.llr[0, :6] = [below, -below, 0.125, -0.125, 31.874, -31.875]
    llr = torch.from_numpy(fr.llr).cuda()
    q = torch.empty((500, 64), dtype=torch.int8, device="cuda")
    B.quantize_llr(llr, 63, 4.0, q)
    torch.cuda.synchronize()
    ref = oracle.quantize(fr.llr, 4.0)
    ref[:, 63:] = 0
    assert np.array_equal(q.cpu().numpy(), ref)


def test_results_independent_of_batch_composition(B):
    """A frame decodes the same alone, in a different batch position and in
    a mixed batch (per-frame randomness is an input, never the slot)."""
    c, p = lib_objects(B, "bch63_45", 33)
    dec = B.Decoder(c, p, n_branches=9, max_iter=8)
    fr = synth.frames("bch63_45", 257, 2.5, seed=8)
    llr = torch.from_numpy(fr.llr).cuda()
    d_o = torch.from_numpy(fr.d_o).cuda()
    full = dec.decode(llr, d_o)
    perm = torch.randperm(257, device="cuda")
    shuf = dec.decode(llr[perm].contiguous(), d_o[perm].contiguous())
    torch.cuda.synchronize()
    inv = torch.argsort(perm)
    for a, b in zip(full[:3], shuf[:3]):
        assert torch.equal(a, b[inv])
    one = dec.decode(llr[100:101].contiguous(), d_o[100:101].contiguous())
    torch.cuda.synchronize()
    assert torch.equal(one[0][0], full[0][100]) and torch.equal(one[1][0], full[1][100])


@pytest.mark.parametrize("precision", [0, 1])
def test_skewed_offsets_every_frame_decoded(B, precision):
    """Offsets concentrated in two buckets (d_o mod d_p), and a batch whose
    frames all share one offset: the workgroups of the grouped kernel crowd
    onto few buckets' cursors and move between buckets as they run dry.
    Every frame gets its outputs (iterations pre-filled with 0xff), and a
    sample equals the oracle (FP32: the parity bar; int8: bit-exact)."""
    name, rows, F = "bch63_45", 33, 300_000
    c, p = lib_objects(B, name, rows)
    oc = oracle_code(name)
    H = oracle_hopt(name, rows)
    dec = B.Decoder(c, p, n_branches=9, max_iter=8, precision=precision)
    assert dec.specialized
    fr = synth.frames(name, F, 2.5, seed=31)
    rng = np.random.default_rng(5)
    cases = [np.where(rng.random(F) < 0.85, 5, 17).astype(np.uint8), np.full(F, 19, np.uint8)]
    for d_o_h in cases:
        llr = torch.from_numpy(fr.llr).cuda()
        if precision:
            q = torch.empty(llr.shape, dtype=torch.int8, device="cuda")
            B.quantize_llr(llr, c.N, 4.0, q)
            llr = q
        bits = torch.empty((F, 1), dtype=torch.int64, device="cuda")
        iters = torch.full((F,), 255, dtype=torch.uint8, device="cuda")
        flg = torch.full((F,), 255, dtype=torch.uint8, device="cuda")
        ws = torch.empty(dec.workspace_size(F), dtype=torch.uint8, device="cuda")
        dec.decode_into(llr, torch.from_numpy(d_o_h).cuda(), bits, iters, flg, workspace=ws)
        torch.cuda.synchronize()
        it_h, fl_h = iters.cpu().numpy(), flg.cpu().numpy()
        assert ((it_h >= 1) & (it_h <= 8)).all() and (fl_h <= 1).all()
        pick = np.sort(rng.choice(F, 3000, replace=False))
        words = B.unpack_bits(bits.cpu().numpy().view(np.uint64)[pick], c.N)
        src = llr.cpu().numpy()[pick]
        if precision:
            oc_, oit, ocv = oracle.decode_batch(H, oc.Hstd, src, d_o_h[pick], 9, 0.75, 8, oracle.R1,
                                                kind=oracle.KIND_FIXED, threads=8)
            assert np.array_equal(words, oc_) and np.array_equal(it_h[pick], oit)
            assert np.array_equal(fl_h[pick].astype(bool), ocv)
        else:
            oc_, oit, ocv, otr = oracle.decode_batch(H, oc.Hstd, src, d_o_h[pick], 9, 0.75, 8, oracle.R1,
                                                     threads=8, trace=True)
            compare_with_oracle(words, it_h[pick], fl_h[pick], None, oc_, oit, ocv, otr)


# ------------------------------------------------------------ fixed point
def run_fix8_pair(B, name, rows, F, ebn0, seed, scale=4.0, flags=0):
    c, p = lib_objects(B, name, rows)
    oc = oracle_code(name)
    H = oracle_hopt(name, rows)
    fr = synth.frames(name, F, ebn0, seed=seed)
    llr = torch.from_numpy(fr.llr).cuda()
    q = torch.empty(llr.shape, dtype=torch.int8, device="cuda")
    B.quantize_llr(llr, c.N, scale, q)
    dec = B.Decoder(c, p, n_branches=9, mode=B.MODE_RESTART, max_iter=8, precision=B.FIX8, flags=flags)
    assert dec.specialized
    d_o = torch.from_numpy(fr.d_o).cuda()
    bits, iters, flg, tr = dec.decode(q, d_o, trace=True)
    torch.cuda.synchronize()
    qh = q.cpu().numpy()
    words = B.unpack_bits(bits.cpu().numpy().view(np.uint64), c.N)
    oc_, oit, ocv, otr = oracle.decode_batch(H, oc.Hstd, qh, fr.d_o, 9, 0.75, 8, oracle.R1,
                                             kind=oracle.KIND_FIXED, threads=8, trace=True)
    return fr, words, iters.cpu().numpy(), flg.cpu().numpy(), tr.cpu().numpy(), oc_, oit, ocv, otr


@pytest.mark.parametrize("name,ebn0,packed", [("bch63_45", 3.0, False), ("bch63_36", 3.5, False),
                                              ("bch63_45", 3.0, True), ("bch63_36", 3.5, True),
                                              ("bch127_99", 4.0, False), ("bch127_64", 3.5, False),
                                              ("bch127_99", 4.0, True), ("bch127_64", 3.5, True)])
def test_fixed_point_bit_exact(B, name, ebn0, packed):
    """int8 messages, (3m+2)>>2 c2v magnitudes, integer branch average:
    identical decoded words, iteration counts, flags and every per-iteration
    posterior as the integer oracle, on every frame (also for the packed
    16-bit kernel, two frames per lane)."""
    F = 128 * 3 + 17
    fr, w, it, fl, tr, ow, oit, ocv, otr = run_fix8_pair(B, name, HO_ROWS[name], F, ebn0, 41,
                                                         flags=B.PACKED16 if packed else 0)
    assert np.array_equal(w, ow)
    assert np.array_equal(it, oit)
    assert np.array_equal(fl.astype(bool), ocv)
    N = w.shape[1]
    for f in range(F):
        assert np.array_equal(tr[f, :oit[f], :N], otr[f, :oit[f]]), f


@pytest.mark.parametrize("packed", [False, True])
@pytest.mark.parametrize("name,rows", [("bch127_64", 72), ("bch127_99", 33)])
def test_fixed_point_full_size_sampled(B, name, rows, packed):
    """4,000,000 frames per point in one launch; 1000 sampled frames checked
    bit-exactly against the integer oracle (also for the packed 16-bit
    kernel)."""
    c, p = lib_objects(B, name, rows)
    oc = oracle_code(name)
    H = oracle_hopt(name, rows)
    F = 4_000_000
    parts = [synth.frames(name, F // 8, 3.0, seed=91, block=k) for k in range(8)]
    llr = torch.from_numpy(np.concatenate([q.llr for q in parts])).cuda()
    d_o_h = np.concatenate([q.d_o for q in parts])
    q = torch.empty(llr.shape, dtype=torch.int8, device="cuda")
    B.quantize_llr(llr, c.N, 4.0, q)
    del llr
    dec = B.Decoder(c, p, n_branches=9, max_iter=8, precision=B.FIX8, flags=B.PACKED16 if packed else B.UNPACKED16)
    assert dec.specialized and dec.kernel_name(F).endswith("_pk16") == packed
    bits, iters, flg, _ = dec.decode(q, torch.from_numpy(d_o_h).cuda())
    torch.cuda.synchronize()
    idx = np.sort(np.random.default_rng(3).choice(F, 1000, replace=False))
    qh = q[torch.from_numpy(idx).cuda()].cpu().numpy()
    ow, oit, ocv = oracle.decode_batch(H, oc.Hstd, qh, d_o_h[idx], 9, 0.75, 8, oracle.R1,
                                       kind=oracle.KIND_FIXED, threads=8)
    words = B.unpack_bits(bits.cpu().numpy().view(np.uint64)[idx], c.N)
    assert np.array_equal(words, ow)
    assert np.array_equal(iters.cpu().numpy()[idx], oit)
    assert np.array_equal(flg.cpu().numpy()[idx].astype(bool), ocv)


def test_fixed_point_without_kernel_is_rejected(B):
    c, p = lib_objects(B, "bch63_45", 0)  # standard matrix: no fixed-point kernel
    dec = B.Decoder(c, p, n_branches=1, mode=B.MODE_EXTRINSIC, max_iter=4, precision=B.FIX8)
    q = torch.zeros((64, 64), dtype=torch.int8, device="cuda")
    with pytest.raises(B.BchError):
        dec.decode(q)


# ------------------------------------------------------------ mixed-code batches
MIX = [("bch127_64", 72), ("bch127_99", 33), ("bch63_36", 122)]
MIX_P = [0.5, 0.25, 0.25]


def mixed_setup(B, precision, F, seed, lo=1.5, hi=5.0):
    objs = [lib_objects(B, n, r) for n, r in MIX]
    decs = [B.Decoder(c, p, n_branches=9, max_iter=8, precision=precision) for c, p in objs]
    assert all(d.specialized for d in decs)
    mf = synth.mixed_frames([n for n, _ in MIX], F, seed, MIX_P, lo, hi)
    llr = torch.from_numpy(mf.llr).cuda()
    if precision == B.FIX8:
        q = torch.empty(llr.shape, dtype=torch.int8, device="cuda")
        for k, (c, _) in enumerate(objs):
            qk = torch.empty(llr.shape, dtype=torch.int8, device="cuda")
            B.quantize_llr(llr, c.N, 4.0, qk)
            sel = torch.from_numpy(mf.code_idx == k).cuda()
            q[sel] = qk[sel]
        llr = q
    return objs, decs, mf, llr


@pytest.mark.parametrize("precision", [0, 1])
def test_mixed_batch_equals_each_code_alone(B, precision):
    """Interleaved frames of three codes in one call give, frame by frame,
    exactly the words, iteration counts and flags of each code's own call."""
    F = 3000
    objs, decs, mf, llr = mixed_setup(B, precision, F, seed=17)
    mix = B.MixedDecoder(decs)
    ci = torch.from_numpy(mf.code_idx).cuda()
    d_o = torch.from_numpy(mf.d_o).cuda()
    bits, iters, flg = mix.decode(ci, llr, d_o)
    torch.cuda.synchronize()
    for k, dec in enumerate(decs):
        sel = torch.from_numpy(np.nonzero(mf.code_idx == k)[0]).cuda()
        ab, ai, af, _ = dec.decode(llr[sel].contiguous(), d_o[sel].contiguous())
        torch.cuda.synchronize()
        assert torch.equal(bits[sel][:, :dec.W64], ab)
        assert torch.equal(iters[sel], ai) and torch.equal(flg[sel], af)
        assert int(ai.min()) >= 1


def test_mixed_batch_against_oracle(B):
    """Mixed FP32 batch against the FP64 oracle of every code (parity bar of
    the single-code tests), and the fixed-point mix bit-exact against the
    integer oracle."""
    F = 1200
    for precision in (0, 1):
        objs, decs, mf, llr = mixed_setup(B, precision, F, seed=23)
        mix = B.MixedDecoder(decs)
        bits, iters, flg = mix.decode(torch.from_numpy(mf.code_idx).cuda(), llr, torch.from_numpy(mf.d_o).cuda())
        torch.cuda.synchronize()
        bh, ih, fh = bits.cpu().numpy().view(np.uint64), iters.cpu().numpy(), flg.cpu().numpy()
        lh = llr.cpu().numpy()
        for k, (name, rows) in enumerate(MIX):
            sel = np.nonzero(mf.code_idx == k)[0]
            oc = oracle_code(name)
            H = oracle_hopt(name, rows)
            N = oc.N
            w = B.unpack_bits(bh[sel][:, :(N + 63) // 64], N)
            if precision == 0:
                res = oracle.decode_batch(H, oc.Hstd, lh[sel], mf.d_o[sel], 9, 0.75, 8, oracle.R1,
                                          threads=8, trace=True)
                compare_with_oracle(w, ih[sel], fh[sel], None, *res)
            else:
                ow, oit, ocv = oracle.decode_batch(H, oc.Hstd, lh[sel], mf.d_o[sel], 9, 0.75, 8, oracle.R1,
                                                   kind=oracle.KIND_FIXED, threads=8)
                assert np.array_equal(w, ow) and np.array_equal(ih[sel], oit)
                assert np.array_equal(fh[sel].astype(bool), ocv)


def test_mixed_batch_rejections(B):
    objs, decs, mf, llr = mixed_setup(B, 0, 64, seed=3)
    c, p = lib_objects(B, "bch63_45", 0)
    generic = B.Decoder(c, p, n_branches=3, mode=B.MODE_EXTRINSIC, max_iter=4)
    assert not generic.specialized
    ci = torch.from_numpy(mf.code_idx).cuda()
    d_o = torch.from_numpy(mf.d_o).cuda()
    with pytest.raises(B.BchError):
        B.MixedDecoder(decs + [generic]).decode(ci, llr, d_o)          # no specialised kernel
    fix = B.Decoder(*lib_objects(B, "bch63_45", 33), n_branches=9, max_iter=8, precision=B.FIX8)
    with pytest.raises(B.BchError):
        B.MixedDecoder(decs + [fix]).decode(ci, llr, d_o)              # precision differs
    with pytest.raises(B.BchError):
        B.MixedDecoder(decs).decode(ci, llr[:, :64].contiguous(), d_o)  # ld < 127
    # frames whose index names no decoder are left untouched
    ci2 = ci.clone()
    ci2[::2] = 7
    bits, iters, flg = B.MixedDecoder(decs).decode(ci2, llr, d_o)
    torch.cuda.synchronize()
    assert int(iters[::2].max()) == 0 and int(iters[1::2].min()) >= 1


def test_mixed_batch_graph_replay(B):
    """The mixed call captured in a HIP graph and replayed several times, with
    new inputs copied in and eager work between replays: every replay equals
    the eager call on the same inputs."""
    F = 4096
    objs, decs, mf, llr = mixed_setup(B, 0, F, seed=31)
    mix = B.MixedDecoder(decs)
    ci = torch.from_numpy(mf.code_idx).cuda()
    d_o = torch.from_numpy(mf.d_o).cuda()
    bits = torch.zeros((F, 2), dtype=torch.int64, device="cuda")
    iters = torch.zeros(F, dtype=torch.uint8, device="cuda")
    flg = torch.zeros(F, dtype=torch.uint8, device="cuda")
    ws = torch.empty(mix.workspace_size(F), dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        mix.decode_into(ci, llr, d_o, bits, iters, flg, ws, stream=s)  # warm-up outside capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        mix.decode_into(ci, llr, d_o, bits, iters, flg, ws, stream=torch.cuda.current_stream())
    for rep in range(4):
        nf = synth.mixed_frames([n for n, _ in MIX], F, 100 + rep, MIX_P, 1.5, 5.0)
        llr.copy_(torch.from_numpy(nf.llr))
        ci.copy_(torch.from_numpy(nf.code_idx))
        d_o.copy_(torch.from_numpy(nf.d_o))
        bits.zero_()
        iters.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        eb, ei, ef = mix.decode(ci, llr, d_o)
        torch.cuda.synchronize()
        assert torch.equal(bits, eb) and torch.equal(iters, ei) and torch.equal(flg, ef), rep


# ------------------------------------------------------------ device OSD
@pytest.mark.parametrize("name", ["bch63_36", "bch63_45", "bch127_64", "bch127_78", "bch127_99"])
def test_device_osd_matches_oracle(B, name):
    """Device OSD-p (p = 0, 1, 2) equals the oracle's OSD bit for bit, on
    noisy frames, on integer-valued LLRs (equal reliabilities: ties in the
    ordering and in the candidate costs), and on frames of equal magnitudes
    with random signs and at -3 dB, whose least candidate costs exceed the
    16-bit range the device keeps for large searches."""
    c, p = lib_objects(B, name, 0)
    dec = B.Decoder(c, p, n_branches=1, mode=B.MODE_EXTRINSIC, max_iter=4)
    oc = oracle_code(name)
    fr = synth.frames(name, 200, 1.5, seed=61)
    tied = np.round(fr.llr[:100] / 3.0).astype(np.float32)  # many |L| equal
    tied[:, oc.N:] = 0.0
    rng = np.random.default_rng(64)
    flat = np.zeros_like(fr.llr[:40])
    flat[:, :oc.N] = np.where(rng.random((40, oc.N)) < 0.5, -2.5, 2.5)
    deep = synth.frames(name, 40, -3.0, seed=65).llr
    llr_h = np.concatenate([fr.llr, tied, flat, deep])
    llr_h[5] = 0.0  # all-zero frame: every candidate costs 0
    llr = torch.from_numpy(llr_h).cuda()
    for order in (0, 1, 2):
        bits = torch.zeros((llr_h.shape[0], dec.W64), dtype=torch.int64, device="cuda")
        dec.osd_into(llr, order, bits)
        torch.cuda.synchronize()
        got = B.unpack_bits(bits.cpu().numpy().view(np.uint64), oc.N)
        ref = oracle.osd_batch(oc.G, llr_h, order)
        assert np.array_equal(got, ref), (order, np.nonzero((got != ref).any(1))[0][:10])


def test_device_osd_skip_and_hybrid(B):
    """Frames with skip set are untouched; NMS followed by device OSD on the
    frames whose syndrome stayed nonzero equals the host hybrid."""
    name, rows = "bch127_64", 72
    c, p = lib_objects(B, name, rows)
    dec = B.Decoder(c, p, n_branches=9, max_iter=8)
    fr = synth.frames(name, 700, 2.5, seed=62)
    llr = torch.from_numpy(fr.llr).cuda()
    d_o = torch.from_numpy(fr.d_o).cuda()
    bits, iters, flg, _ = dec.decode(llr, d_o)
    nms = bits.clone()
    dec.osd_into(llr, 2, bits, skip=flg)
    torch.cuda.synchronize()
    fl = flg.cpu().numpy()
    assert (fl == 0).sum() > 20
    b_dev = bits.cpu().numpy().view(np.uint64)
    conv = fl != 0
    assert np.array_equal(b_dev[conv], nms.cpu().numpy().view(np.uint64)[conv])  # skipped frames untouched
    host = B.osd_decode(c, fr.llr, 2, skip=fl.astype(np.uint8), bits=nms.cpu().numpy().view(np.uint64).copy())
    assert np.array_equal(b_dev, host)


def test_mixed_full_size_sampled(B):
    """The mixed workload at its full size: 16,000,000 interleaved frames in one
    call per precision, on per-code launches (the default at this size) and on
    the mixed-code kernel; 200 sampled frames per code against the oracle
    (FP64 with the tie rule for FP32, bit-exact for int8)."""
    names = [n for n, _ in MIX]
    F = 16_000_000
    blocks = 32
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(16) as ex:
        parts = list(ex.map(lambda k: synth.mixed_frames(names, F // blocks, 77, MIX_P, 1.5, 5.0, block=k),
                            range(blocks)))
    code_idx = np.concatenate([p.code_idx for p in parts])
    d_o_h = np.concatenate([p.d_o for p in parts])
    llr = torch.from_numpy(np.concatenate([p.llr for p in parts])).cuda()
    ci = torch.from_numpy(code_idx).cuda()
    d_o = torch.from_numpy(d_o_h).cuda()
    rng = np.random.default_rng(5)
    for precision, flags in ((0, 0), (1, 0), (0, B.MIXED_KERNEL), (1, B.MIXED_KERNEL)):
        objs = [lib_objects(B, n, r) for n, r in MIX]
        decs = [B.Decoder(c, p, n_branches=9, max_iter=8, precision=precision, flags=flags) for c, p in objs]
        assert B.MixedDecoder(decs).kernel_name(F).startswith("mix_") == bool(flags)
        inp = llr
        if precision == B.FIX8:
            inp = torch.empty(llr.shape, dtype=torch.int8, device="cuda")
            for k, (c, _) in enumerate(objs):
                qk = torch.empty(llr.shape, dtype=torch.int8, device="cuda")
                B.quantize_llr(llr, c.N, 4.0, qk)
                sel = ci == k
                inp[sel] = qk[sel]
                del qk, sel
        bits, iters, flg = B.MixedDecoder(decs).decode(ci, inp, d_o)
        torch.cuda.synchronize()
        for k, (name, rows) in enumerate(MIX):
            idx = np.sort(rng.choice(np.nonzero(code_idx == k)[0], 200, replace=False))
            oc = oracle_code(name)
            H = oracle_hopt(name, rows)
            ti = torch.from_numpy(idx).cuda()
            x = inp[ti].cpu().numpy()
            w = B.unpack_bits(bits[ti].cpu().numpy().view(np.uint64)[:, :(oc.N + 63) // 64], oc.N)
            it_h, fl_h = iters[ti].cpu().numpy(), flg[ti].cpu().numpy()
            if precision == 0:
                res = oracle.decode_batch(H, oc.Hstd, x, d_o_h[idx], 9, 0.75, 8, oracle.R1, threads=8, trace=True)
                compare_with_oracle(w, it_h, fl_h, None, *res)
            else:
                ow, oit, ocv = oracle.decode_batch(H, oc.Hstd, x, d_o_h[idx], 9, 0.75, 8, oracle.R1,
                                                   kind=oracle.KIND_FIXED, threads=8)
                assert np.array_equal(w, ow) and np.array_equal(it_h, oit)
                assert np.array_equal(fl_h.astype(bool), ocv)
        del bits, iters, flg, inp


# ------------------------------------------------------------ the mixed-code kernel
def test_mixed_kernel_selection(B):
    """The three codes of the mixed workload in this order have a mixed-code
    kernel per precision, run below the size limit (at any size with
    MIXED_KERNEL); a decoder flagged NO_MIXED_KERNEL, another order or a
    single code runs per-code launches."""
    objs = [lib_objects(B, n, r) for n, r in MIX]
    lim = B.MIXED_KERNEL_MAX_FRAMES
    for precision, suffix in ((0, ""), (1, "_fix8")):
        name = "mix_127_64_m72_127_99_m33_63_36_m122" + suffix
        decs = [B.Decoder(c, p, n_branches=9, max_iter=8, precision=precision) for c, p in objs]
        assert B.MixedDecoder(decs).kernel_name(100) == B.MixedDecoder(decs).kernel_name(lim - 1) == name
        assert B.MixedDecoder(decs).kernel_name(lim) == "per-code"
        assert B.MixedDecoder(decs[::-1]).kernel_name(100) == "per-code"
        assert B.MixedDecoder(decs[:1]).kernel_name(100) == "per-code"
        off = B.Decoder(*objs[0], n_branches=9, max_iter=8, precision=precision, flags=B.NO_MIXED_KERNEL)
        assert B.MixedDecoder([off] + decs[1:]).kernel_name(100) == "per-code"
        on = B.Decoder(*objs[1], n_branches=9, max_iter=8, precision=precision, flags=B.MIXED_KERNEL)
        assert B.MixedDecoder([decs[0], on, decs[2]]).kernel_name(10 ** 8) == name
        assert B.MixedDecoder([off, on, decs[2]]).kernel_name(100) == "per-code"
        with pytest.raises(B.BchError):
            B.Decoder(*objs[0], n_branches=9, max_iter=8, precision=precision,
                      flags=B.MIXED_KERNEL | B.NO_MIXED_KERNEL)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("mix_p", [(0.5, 0.25, 0.25), (0.0, 0.0, 1.0), (0.9, 0.1, 0.0), (0.05, 0.05, 0.9)])
def test_mixed_kernel_equals_per_code_launches(B, precision, mix_p):
    """One launch over every code's frames against one launch per code, on a
    batch large enough for waves to run dry and move between codes' buckets,
    including mixes where a code has no frame, frames whose index names no
    decoder (left untouched) and alpha/I_m that differ per code: identical
    words, iteration counts and flags."""
    F = 200_000
    objs = [lib_objects(B, n, r) for n, r in MIX]
    alphas, its = (0.75, 1.0, 0.55), (8, 6, 8)
    mk = lambda fl: [B.Decoder(c, p, n_branches=9, alpha=a, max_iter=m, precision=precision, flags=fl)
                     for (c, p), a, m in zip(objs, alphas, its)]
    fused, per = B.MixedDecoder(mk(0)), B.MixedDecoder(mk(B.NO_MIXED_KERNEL))
    assert fused.kernel_name(F).startswith("mix_") and per.kernel_name(F) == "per-code"
    probs = [p for p in mix_p]
    mf = synth.mixed_frames([n for n, _ in MIX], F, 71, probs, 1.5, 5.0)
    ci = mf.code_idx.copy()
    ci[::97] = 5  # names no decoder
    llr = torch.from_numpy(mf.llr).cuda()
    if precision:
        q = torch.empty(llr.shape, dtype=torch.int8, device="cuda")
        for k, (c, _) in enumerate(objs):
            qk = torch.empty(llr.shape, dtype=torch.int8, device="cuda")
            B.quantize_llr(llr, c.N, 4.0, qk)
            sel = torch.from_numpy(mf.code_idx == k).cuda()
            q[sel] = qk[sel]
        llr = q
    cid = torch.from_numpy(ci).cuda()
    d_o = torch.from_numpy(mf.d_o).cuda()
    a = fused.decode(cid, llr, d_o)
    b = per.decode(cid, llr, d_o)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    it = a[1].cpu().numpy()
    assert (it[::97] == 0).all() and (it[ci < 3] >= 1).all()


@pytest.mark.parametrize("name,rows", [("bch63_36", 27), ("bch63_36", 47), ("bch63_36", 269), ("bch63_36", 316),
                                       ("bch127_78", 49), ("bch127_78", 65)])
def test_beta_sweep_matrices(B, name, rows):
    """The redundancy sweep's matrices (the paper's (63,36) row counts 27, 47,
    269, 316 and (127,78) at beta = 1, 3) run on specialised kernels and meet
    the parity bar against the oracle (I_m = 4 for length 63, as in the
    paper's list; 8 for length 127)."""
    F = 64 * 3 + 11
    im = 4 if name.startswith("bch63") else 8
    fr, g, o, dec = run_pair(B, name, rows, F, 3.5, 53, 9, oracle.R1, im)
    assert dec.specialized
    compare_with_oracle(*g, *o, onestep=dec.onestep)
