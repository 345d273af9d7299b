"""Throughput of enhanced normalized min-sum decoding of short BCH codes on
one MI355X.

Default workload "fix127" (one "step" = one pass of the whole decode path
over the batch, in both precisions): BCH(127,64) with the optimised 72 x 127
H_o and BCH(127,99) with the optimised 33 x 127 H_o; enhanced NMS with the
9-branch automorphism block (three random cyclic shifts of y, pi_I y and
pi_F y), restart message mode, at most 8 iterations with syndrome stopping,
FP32 (alpha = 0.75) and int8 fixed point (alpha = 3/4 as a shift-add, LLRs
quantised with scale 4); 4,000,000 frames per Eb/N0 point, Eb/N0 = 2.0, 2.5,
..., 5.0 dB; random information bits, BPSK over AWGN, LLR = 2y/sigma^2 (seeded
synthetic frames, resident in HBM before the timed region).  Each code's 7
points go through one decode call per precision (56,000,000 frames per
precision and step in four calls); --launch point makes every point a call
of its own.

Other workloads (--workload): "sweep63", BCH(63,45) and BCH(63,36) at
1.0..6.0 dB, 1,000,000 frames per point, FP32; "mixed", 16,000,000 frames of
BCH(127,64)/(127,99)/(63,36) interleaved per frame (50/25/25 %) at Eb/N0
drawn per frame from U[1.5, 5] dB, decoded in one mixed-code call, FP32 and
int8; "serve", the continuous-batching service with OSD-2; "latency",
decode-call latency against the call size; "alpha", "ablation" and "beta",
experiments of the method.

Prints one JSON line with frames/s (value), information Gbit/s, per-launch
p50/p99 latency, the VALU roofline of the dominant decode kernel (and per
precision), and the CPU oracle decoding distinct frames of every Eb/N0 point
within a time budget: its frame error rate beside the GPU's on the same
frames (Wilson 95% intervals) and its throughput on the host's cores.
"""
from __future__ import annotations

import argparse
import gc
import json
import math
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

# peak of 32-bit vector ALU lane-operations per second: 256 CUs x 128 FP32
# lanes x 2.4 GHz, the published FP32 vector rate of 157.3 TFLOP/s with an FMA
# counted as one lane-operation (two FLOPs)
VALU_PEAK_OPS = 256 * 128 * 2.4e9
HBM_PEAK_BYTES = 8.0e12  # published HBM3E bandwidth of one MI355X
WORKLOADS = {
    # name: (codes with H_o rows, Eb/N0 grid, frames per point, precisions, description)
    "sweep63": ([("bch63_45", 33), ("bch63_36", 122)], "1.0:6.0:0.5", 1_000_000, ["fp32"],
                "BCH(63,45) H_o 33x63 and BCH(63,36) H_o 122x63, enhanced NMS 9 branches, restart "
                "mode, alpha 0.75, max 8 iterations, FP32"),
    "fix127": ([("bch127_64", 72), ("bch127_99", 33)], "2.0:5.0:0.5", 4_000_000, ["fp32", "fix8"],
               "BCH(127,64) H_o 72x127 and BCH(127,99) H_o 33x127, enhanced NMS 9 branches, restart "
               "mode, max 8 iterations, FP32 (alpha 0.75) vs int8 messages (alpha 3/4 shift-add, LLR x 4 "
               "quantised)"),
    "serve": (None, "2.0:5.0", 0, ["fp32"], "serving"),
    "alpha": (None, "", 0, ["fp32"], "alpha sweep"),
    "ablation": (None, "", 0, ["fp32"], "branch-count ablation"),
    "beta": (None, "", 0, ["fp32"], "H_o redundancy sweep"),
    "latency": (None, "", 0, ["fp32"], "decode-call latency"),
    "mixed": ([("bch127_64", 72), ("bch127_99", 33), ("bch63_36", 122)], "1.5:5.0", 16_000_000, ["fp32", "fix8"],
              "mixed-code batch, per frame 50% BCH(127,64) H_o 72x127, 25% BCH(127,99) H_o 33x127, "
              "25% BCH(63,36) H_o 122x63 in one call, enhanced NMS 9 branches, restart mode, max 8 iterations, "
              "FP32 and int8", [0.5, 0.25, 0.25]),
}
FIX_SCALE = 4.0

# HBM traffic of the specialised decode kernels, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs, each scaled by what the same counter reads for a plain 1 GiB
# device copy (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0): bytes per frame of one
# decode call of 28,000,000 frames (one code's seven Eb/N0 points of the
# default workload).  An entry holds only for the kernel
# sources the counters were taken on (a hash of the kernel family's templates
# and of the generator functions that write its row function); any other build
# reports traffic null.
TRAFFIC_B_PER_FRAME = {  # kernel: (fetched, written, family, source hash)
    "spec_bch127_64_m72_b9": (523.11, 90.35, "one_wave", "0a4d801252c7f5af"),
    "spec_bch127_99_m33_b9": (522.03, 88.35, "one_wave", "0a4d801252c7f5af"),
    "spec_bch127_64_m72_b9_fix8_pk16": (135.90, 84.46, "pk16", "80d070ec35864e98"),
    "spec_bch127_99_m33_b9_fix8_pk16": (135.65, 85.67, "pk16", "80d070ec35864e98"),
}
KERNEL_FAMILIES = {
    "one_wave": (["csrc/nms_spec_fp32.inc", "csrc/nms_spec_rot.inc", "csrc/nms_spec_cursor.inc"],
                 ["body_source_ilp", "_min_steps", "syndrome_source", "_sign_masks", "_parity", "_MED3U",
                  "ILP_ROWS", "FOLD_SHIFTS", "FOLD_EXCLUDE", "folded_body_source", "shift_matrices"]),
    "pk16": (["csrc/nms_spec_pk16.inc", "csrc/nms_spec_rot.inc", "csrc/nms_spec_cursor.inc"],
             ["body_source_pk16", "syndrome_source", "_parity", "PK16_GROUP", "FOLD_SHIFTS",
              "folded_body_source", "shift_matrices"]),
}


def kernel_src_hash(family):
    """Hash of the files and generator functions behind a kernel family."""
    import hashlib
    import inspect
    from paper_2412_20828_amd import gen_spec
    pkg = os.path.join(ROOT, "paper_2412_20828_amd")
    files, funcs = KERNEL_FAMILIES[family]
    outer = hashlib.sha256()
    for f in files:
        with open(os.path.join(pkg, f), "rb") as fh:
            outer.update(hashlib.sha256(fh.read()).digest())
    for name in funcs:
        obj = getattr(gen_spec, name)
        text = obj if isinstance(obj, str) else (inspect.getsource(obj) if callable(obj) else repr(obj))
        outer.update(hashlib.sha256(text.encode()).digest())
    return outer.hexdigest()[:16]


V2C_OPS = {1: 0, 2: 2, 3: 1}  # message mode -> v2c arithmetic per edge (restart, memory, extrinsic)


def alg_ops_per_iteration(N, K, M, E, B, mode=1):
    """Algorithmic 32-bit operations of one iteration of one frame: per edge
    7 plus the v2c arithmetic of the message mode (none in restart mode, where
    the v2c message is the gathered input itself; Y - own c2v in the extrinsic
    mode; Y + other c2v sum in the memory mode, counted as S - own + Y), the 7
    being min1/min2/argmin 3, sign 1, c2v select and sign 2, bit-sum add 1;
    per check row 2, per branch coordinate 2 (permutation and merge), plus the
    syndrome test 2 (N-K) ceil(N/64)."""
    per_edge = 7 + V2C_OPS[mode]
    return per_edge * B * E + 2 * B * M + 2 * B * N + 2 * (N - K) * ((N + 63) // 64)


# the coarse complexity account of the paper's Table 2: automorphisms per
# iteration x iterations x rows of the parity-check matrix (x parallel
# decoders), relative to mRRD(1) with (I1, I2, I3) = (15, 50, 1) on the
# 18-row standard matrix of BCH(63,45)
TABLE2_REFERENCE = (1, 15 * 50 * 1, 18)


def table2_complexity(automorphisms, iterations, rows, parallel=1):
    a, i, m = TABLE2_REFERENCE
    return automorphisms * iterations * rows * parallel / (a * i * m)


def gen_point(name, F, ebn0, seed, block_frames=125000):
    nb = (F + block_frames - 1) // block_frames
    sizes = [min(block_frames, F - k * block_frames) for k in range(nb)]
    with ThreadPoolExecutor(min(16, os.cpu_count() or 4)) as ex:
        parts = list(ex.map(lambda k: synth.frames(name, sizes[k], ebn0, seed=seed, block=k), range(nb)))
    return (np.concatenate([p.llr for p in parts]), np.concatenate([p.codewords for p in parts]),
            np.concatenate([p.d_o for p in parts]))


def gen_mixed(names, probs, F, lo, hi, seed, block_frames=500000):
    nb = (F + block_frames - 1) // block_frames
    sizes = [min(block_frames, F - k * block_frames) for k in range(nb)]
    with ThreadPoolExecutor(min(16, os.cpu_count() or 4)) as ex:
        parts = list(ex.map(lambda k: synth.mixed_frames(names, sizes[k], seed, probs, lo, hi, block=k),
                            range(nb)))
    return (np.concatenate([p.llr for p in parts]), np.concatenate([pack(p.codewords) for p in parts]),
            np.concatenate([p.d_o for p in parts]), np.concatenate([p.code_idx for p in parts]))


def pack(bits):
    """[F][n] 0/1 bytes -> [F][2] uint64 words (bit i of word i // 64)."""
    F, n = bits.shape
    padded = np.zeros((F, 128), np.uint8)
    padded[:, :n] = bits
    return np.packbits(padded, axis=1, bitorder="little").view(np.uint64)


# frames per Eb/N0 point kept on the host for the CPU oracle leg
KEEP = 65536


@dataclass
class Sample:
    """The first frames of one Eb/N0 point (or one code of a mixed call) with
    the GPU's outcomes on them, for the oracle decoding the same frames."""
    code: str
    prec: str
    ebn0: object
    x: np.ndarray       # [n][ld] float32 LLRs or int8 quantised LLRs
    d_o: np.ndarray
    words: np.ndarray   # [n][W] uint64 GPU decisions
    iters: np.ndarray
    flags: np.ndarray
    cw: np.ndarray      # [n][2] uint64 transmitted codewords


def wilson(k, n, z=1.96):
    """Wilson score interval of a binomial proportion k / n (95% for z = 1.96)."""
    if n == 0:
        return [0.0, 1.0]
    p = k / n
    den = 1.0 + z * z / n
    c = (p + z * z / (2 * n)) / den
    h = z * math.sqrt(p * (1 - p) / n + z * z / (4.0 * n * n)) / den
    return [max(0.0, c - h), min(1.0, c + h)]


class Item:
    """One launch of the timed step: a single-code decode or a mixed-code one."""

    def __init__(self, label, prec, frames, launch):
        self.label, self.prec, self.frames = label, prec, frames
        self.launch_on = launch          # (stream) -> enqueue the launch on that stream
        self.launch = lambda: launch()   # on the decode stream
        self.graph = None
        self.kernel = "mixed"
        self.stats = None     # () -> (per-point dicts, algorithmic ops, information bits)
        self.sample = None    # () -> [(code name, llr rows, d_o, gpu words, gpu iters)] for the CPU leg


def end_to_end(items, frames, torch, stream):
    """PCIe-inclusive rate of one decode call over the first `frames` frames of
    the first work item: LLRs from pinned host memory to the device, decode,
    decisions / iterations / flags back to pinned host memory, timed with
    events on the decode stream."""
    it = items[0]
    n = min(frames, it.frames)
    dev_in = it.inputs[0][:n]
    host_in = torch.empty(dev_in.shape, dtype=dev_in.dtype, pin_memory=True)
    host_in.copy_(dev_in)
    outs = [o[:n] for o in it.outputs]
    host_out = [torch.empty(o.shape, dtype=o.dtype, pin_memory=True) for o in outs]
    a, b, c, d = (torch.cuda.Event(enable_timing=True) for _ in range(4))
    torch.cuda.synchronize()
    a.record(stream)
    dev_in.copy_(host_in, non_blocking=True)
    b.record(stream)
    it.dec.decode_into(dev_in, it.inputs[1][:n], *outs, workspace=it.ws, stream=stream)
    c.record(stream)
    for h, o in zip(host_out, outs):
        h.copy_(o, non_blocking=True)
    d.record(stream)
    torch.cuda.synchronize()
    tot = a.elapsed_time(d) / 1e3
    return {"launch": it.label, "frames": n, "h2d_ms": a.elapsed_time(b), "decode_ms": b.elapsed_time(c),
            "d2h_ms": c.elapsed_time(d), "frames_per_s": n / tot,
            "bytes_in": dev_in.numel() * dev_in.element_size(),
            "bytes_out": sum(o.numel() * o.element_size() for o in outs)}


def make_decoder(args, B, code, pcm, name, rows, prec):
    """Nine-branch restart-mode decoder of the workloads: the defaults, the
    packed 16-bit layout (--packed16), the generic kernel (--generic), or the
    autotuner's cached layout and grid (--tuned)."""
    precision = B.FIX8 if prec == "fix8" else B.FP32
    flags = (B.FORCE_GENERIC if args.generic else 0) | (B.PACKED16 if args.packed16 and prec == "fix8" else 0)
    flags |= B.CHUNK_BUCKETS if getattr(args, "chunk_buckets", False) else 0
    path = getattr(args, "mixed_path", "fused")
    flags |= {"per-code": B.NO_MIXED_KERNEL, "fused": B.MIXED_KERNEL}.get(path, 0)
    alpha = workload_alpha(args, name, rows)
    if args.tuned and not args.generic:
        from paper_2412_20828_amd import autotune
        return autotune.tuned_decoder(code, pcm, name, rows, alpha=alpha, precision=precision, flags=flags)
    return B.Decoder(code, pcm, n_branches=9, mode=B.MODE_RESTART, alpha=alpha, max_iter=8,
                     precision=precision, flags=flags)


def workload_alpha(args, name, rows):
    """alpha of a code's FP32 decoder: --alpha as a number, or "tuned" (the
    autotuner's cached argmin of the frame error rate, 0.75 when nothing is
    cached).  The fixed-point decoders have alpha = 3/4 built in."""
    if args.alpha == "tuned":
        from paper_2412_20828_amd import autotune
        return autotune.tuned_alpha(name, rows)
    return float(args.alpha)


def build_single(args, B, torch, dev, stream, codes, points, precisions, seed_base):
    """Work items of a single-code sweep.  With --launch code (the default) the
    frames of all Eb/N0 points of a code sit in one array and go through one
    decode call per precision; the per-point statistics are read from slices
    of its outputs.  With --launch point every point is a call of its own."""
    items, mats = [], {}
    for ci, (name, rows) in enumerate(codes):
        d = B.CODE_DEFS[name]
        code = B.Code(d.m, d.prim, d.t)
        pcm = B.Pcm.build(code, target_rows=rows, seed=1)
        mats[name] = pcm
        decs = {prec: make_decoder(args, B, code, pcm, name, rows, prec) for prec in precisions}
        groups = [[pi] for pi in range(len(points))] if args.launch == "point" else [list(range(len(points)))]
        for grp in groups:
            F = args.frames * len(grp)
            ld = 64 if code.N <= 64 else 128
            llr_d = torch.empty((F, ld), dtype=torch.float32, device=dev)
            d_o_d = torch.empty(F, dtype=torch.uint8, device=dev)
            pts = []  # (Eb/N0, first frame, packed codewords, first KEEP LLR rows, their d_o)
            for j, pi in enumerate(grp):
                llr, cw, d_o = gen_point(name, args.frames, points[pi], seed=seed_base + 10 * ci + pi)
                f0 = j * args.frames
                llr_d[f0:f0 + args.frames].copy_(torch.from_numpy(llr))
                d_o_d[f0:f0 + args.frames].copy_(torch.from_numpy(d_o))
                pts.append((points[pi], f0, pack(cw), llr[:KEEP].copy(), d_o[:KEEP].copy()))
                del llr, cw, d_o
            for prec in precisions:
                dec = decs[prec]
                if prec == "fix8":
                    inp = torch.empty(llr_d.shape, dtype=torch.int8, device=dev)
                    B.quantize_llr(llr_d, code.N, FIX_SCALE, inp)
                else:
                    inp = llr_d
                bits = torch.empty((F, dec.W64), dtype=torch.int64, device=dev)
                it = torch.empty(F, dtype=torch.uint8, device=dev)
                fl = torch.empty(F, dtype=torch.uint8, device=dev)
                ws = torch.empty(max(1, dec.workspace_size(F)), dtype=torch.uint8, device=dev)
                label = "%s@%s" % (name, "%g" % points[grp[0]] if len(grp) == 1 else
                                   "%g:%g" % (points[grp[0]], points[grp[-1]]))
                item = Item(label, prec, F,
                            lambda st=stream, dec=dec, inp=inp, d_o_d=d_o_d, bits=bits, it=it, fl=fl, ws=ws:
                            dec.decode_into(inp, d_o_d, bits, it, fl, workspace=ws, stream=st))
                item.inputs, item.outputs = (inp, d_o_d), (bits, it, fl)
                item.dec, item.ws = dec, ws
                item.kernel = dec.kernel_name(F) if dec.specialized else "generic_%s" % prec

                def stats(name=name, prec=prec, code=code, pcm=pcm, bits=bits, it=it, fl=fl, pts=pts):
                    W = bits.cpu().numpy().view(np.uint64)
                    I = it.cpu().numpy().astype(np.int64)
                    C = fl.cpu().numpy().astype(bool)
                    out = []
                    for e, f0, cwp, _, _ in pts:
                        w, iters, conv = W[f0:f0 + len(cwp)], I[f0:f0 + len(cwp)], C[f0:f0 + len(cwp)]
                        err = (w != cwp[:, :w.shape[1]]).any(1)
                        nbit = int(np.bitwise_count(w ^ cwp[:, :w.shape[1]]).sum())
                        out.append({"code": name, "precision": prec, "ebn0": e, "fer": float(err.mean()),
                                    "ber": nbit / (len(err) * code.N), "avg_iters": float(iters.mean()),
                                    "undetected": float((err & conv).mean())})
                    ops = I.sum() * alg_ops_per_iteration(code.N, code.K, pcm.M, pcm.E, 9)
                    return out, float(ops), len(I) * code.K

                def sample(name=name, prec=prec, bits=bits, it=it, fl=fl, pts=pts, inp=inp):
                    W = bits.cpu().numpy().view(np.uint64)
                    I, C = it.cpu().numpy(), fl.cpu().numpy()
                    out = []
                    for e, f0, cwp, lk, dk in pts:
                        n = lk.shape[0]
                        x = lk if prec == "fp32" else inp[f0:f0 + n].cpu().numpy()
                        out.append(Sample(name, prec, e, x, dk, W[f0:f0 + n], I[f0:f0 + n], C[f0:f0 + n], cwp[:n]))
                    return out
                item.stats, item.sample = stats, sample
                items.append(item)
            del llr_d
    return items, mats


def build_mixed(args, B, torch, dev, stream, codes, probs, lohi, precisions, seed):
    names = [n for n, _ in codes]
    objs, mats = [], {}
    for name, rows in codes:
        d = B.CODE_DEFS[name]
        code = B.Code(d.m, d.prim, d.t)
        pcm = B.Pcm.build(code, target_rows=rows, seed=1)
        objs.append((code, pcm))
        mats[name] = pcm
    llr, cwp, d_o, ci = gen_mixed(names, probs, args.frames, lohi[0], lohi[1], seed)
    F = llr.shape[0]
    llr_d = torch.from_numpy(llr).to(dev)
    d_o_d = torch.from_numpy(d_o).to(dev)
    ci_d = torch.from_numpy(ci).to(dev)
    items = []
    for prec in precisions:
        decs = [make_decoder(args, B, c, p, name, rows, prec) for (c, p), (name, rows) in zip(objs, codes)]
        mix = B.MixedDecoder(decs)
        if prec == "fix8":
            inp = torch.empty(llr_d.shape, dtype=torch.int8, device=dev)
            for k, (c, _) in enumerate(objs):
                qk = torch.empty(llr_d.shape, dtype=torch.int8, device=dev)
                B.quantize_llr(llr_d, c.N, FIX_SCALE, qk)
                sel = ci_d == k
                inp[sel] = qk[sel]
                del qk, sel
        else:
            inp = llr_d
        bits = torch.zeros((F, 2), dtype=torch.int64, device=dev)
        it = torch.zeros(F, dtype=torch.uint8, device=dev)
        fl = torch.zeros(F, dtype=torch.uint8, device=dev)
        ws = torch.empty(max(1, mix.workspace_size(F)), dtype=torch.uint8, device=dev)
        item = Item("mixed", prec, F, lambda st=stream, mix=mix, inp=inp, bits=bits, it=it, fl=fl, ws=ws:
                    mix.decode_into(ci_d, inp, d_o_d, bits, it, fl, ws, stream=st))
        # the mixed-code kernel's name, or per-code launches of this precision
        kname = mix.kernel_name(F)
        item.kernel = kname if kname != "per-code" else "per-code_%s" % prec

        def stats(prec=prec, bits=bits, it=it, fl=fl):
            w = bits.cpu().numpy().view(np.uint64)
            iters = it.cpu().numpy().astype(np.int64)
            conv = fl.cpu().numpy().astype(bool)
            err = (w != cwp).any(1)
            pts, ops, info = [], 0.0, 0
            for k, ((name, _), (code, pcm)) in enumerate(zip(codes, objs)):
                sel = ci == k
                if not sel.any():
                    continue
                pts.append({"code": name, "precision": prec, "ebn0": "U[%g,%g]" % tuple(lohi),
                            "frames": int(sel.sum()), "fer": float(err[sel].mean()),
                            "avg_iters": float(iters[sel].mean()), "undetected": float((err & conv)[sel].mean())})
                ops += iters[sel].sum() * alg_ops_per_iteration(code.N, code.K, pcm.M, pcm.E, 9)
                info += int(sel.sum()) * code.K
            return pts, float(ops), info

        def sample(prec=prec, bits=bits, it=it, fl=fl, inp=inp):
            out = []
            W, I, C = bits.cpu().numpy().view(np.uint64), it.cpu().numpy(), fl.cpu().numpy()
            for k, (name, _) in enumerate(codes):
                sel = np.nonzero(ci == k)[0][:KEEP]
                if sel.size == 0:
                    continue
                x = llr[sel].copy() if prec == "fp32" else inp[torch.from_numpy(sel).to(dev)].cpu().numpy()
                out.append(Sample(name, prec, "U[%g,%g]" % tuple(lohi), x, d_o[sel].copy(), W[sel], I[sel], C[sel],
                                  cwp[sel]))
            return out
        item.stats, item.sample = stats, sample
        items.append(item)
    return items, mats


SERVE_CODES = [("bch63_36", 122), ("bch63_45", 33), ("bch127_64", 72), ("bch127_99", 33)]
SERVE_LOADS = [0.1, 0.25, 0.5, 0.75, 0.9, 1.0, 1.2]


def run_serve(args):
    """Serving workload: Poisson arrivals of requests of round(2^(12U))
    frames, code uniform over four, Eb/N0 U[2, 5] dB per request; continuous
    batching on the GPU, OSD-2 (on the device, or on the host with --osd host)
    for frames the NMS stage leaves with a nonzero syndrome.  Saturation is
    measured with every request submitted at once; the offered load is then
    swept over fractions of it."""
    import torch

    from paper_2412_20828_amd import serving
    names = [n for n, _ in SERVE_CODES]
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    eng = serving.Engine(SERVE_CODES, slot_frames=args.slot_frames, n_slots=args.slots, osd_order=2, osd_on=args.osd,
                         osd_threads=max(1, min(16, threads) - 2), tuned=not args.generic,
                         graph=not args.serve_eager)
    t0 = time.time()
    tr = synth.request_trace(args.requests, 5000, len(names), 2.0, 5.0)
    with ThreadPoolExecutor(min(16, os.cpu_count() or 4)) as ex:
        frs = list(ex.map(lambda k: synth.request_frames(names, tr[k], 5000, k), range(len(tr))))
    gen_s = time.time() - t0
    mean_frames = float(np.mean([d.frames for d in tr]))

    def fresh():
        return [serving.Request(code=d.code, llr=f.llr, rid=k) for k, (d, f) in enumerate(zip(tr, frs))]

    # untimed: each warm-up step is three bursts of the whole trace, which
    # replay every slot's graph several times (the first replays of a captured
    # graph, and the first bursts, run slower than the service's steady state)
    for _ in range(3 * args.warmup):
        serving.run_trace(eng, fresh(), [0.0] * len(tr))
    serving.settle_gc()
    done, wall = serving.run_trace(eng, fresh(), [0.0] * len(tr))
    sat = serving.summarize(done, wall)
    sat["launches"] = eng.launches
    sat["hw_queues"] = os.environ.get("GPU_MAX_HW_QUEUES")
    truth = {k: f.codewords for k, f in enumerate(frs)}
    fer_h = np.mean(np.concatenate([(r.bits != pack(truth[r.rid])).any(1) for r in done]))
    fer_n = np.mean(np.concatenate([((r.flags & serving.FLAG_OSD) != 0) | (r.bits != pack(truth[r.rid])).any(1)
                                    for r in done]))
    osd_cost = osd_costs(eng, done, torch)
    serving.settle_gc()
    loads = []
    for frac in SERVE_LOADS:
        rate = frac * sat["frames_per_s"] / mean_frames
        # untimed: the first 256 requests at this load, so that the timed
        # trace starts from the service's steady state at that load (after a
        # burst or an idle gap the first steps take longer)
        serving.run_trace(eng, fresh()[:256], [d.t / rate for d in tr[:256]])
        reqs = fresh()
        gc.collect()
        gc.disable()  # no collection inside the timed trace; one after it
        try:
            done, wall = serving.run_trace(eng, reqs, [d.t / rate for d in tr])
        finally:
            gc.enable()
        row = serving.summarize(done, wall)
        row.update({"offered_fraction": frac, "offered_frames_per_s": rate * mean_frames,
                    "offered_requests_per_s": rate})
        loads.append(row)
        print("load %.2f: %.2fM frames/s p50 %.2f ms p99 %.2f ms" % (frac, row["frames_per_s"] / 1e6,
              row["latency_ms_p50"], row["latency_ms_p99"]), file=sys.stderr, flush=True)
    eng.close()
    ok = [r for r in loads if r["frames_per_s"] >= 0.95 * r["offered_frames_per_s"]]
    res = {
        "metric": "decoded frames/s & info Gbit/s at matched FER vs oracle; p50/p99 latency",
        "value": sat["frames_per_s"], "unit": "frames/s", "n_gpus": 1, "steps": 1, "warmup": args.warmup,
        "ms_per_step": sat["wall_s"] * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "serving: %d requests, Poisson arrivals, round(2^(12U)) frames each, code uniform "
                               "over BCH(63,36) H_o 122x63, (63,45) 33x63, (127,64) 72x127, (127,99) 33x127, "
                               "Eb/N0 U[2, 5] dB per request; enhanced NMS 9 branches, max 8 iterations on the "
                               "GPU (%d slots of %d frames, %s), OSD-2 for NMS failures %s"
                               % (len(tr), args.slots, args.slot_frames,
                                  "each step launched code by code" if args.serve_eager else
                                  "each step one captured graph: one mixed-code kernel, then device OSD"
                                  if args.osd == "device" else "each step one captured graph of the mixed-code "
                                  "kernel", "on the GPU" if args.osd == "device" else
                                  "on %d host threads" % max(1, min(16, threads) - 2)),
                   "mean_request_frames": mean_frames},
        "saturation": sat,
        "info_gbit_s": None,
        "latency_ms": {"request_p50_at_saturation": sat["latency_ms_p50"],
                       "request_p99_at_saturation": sat["latency_ms_p99"]},
        "fer_hybrid": float(fer_h), "fer_nms_only": float(fer_n),
        "load_sweep": loads,
        "osd_us_per_frame": osd_cost,
        "max_sustained_frames_per_s": max([r["frames_per_s"] for r in ok], default=None),
        "roofline": None,
        "input_generation_s": gen_s,
    }
    info = sum(eng.codes[d.code][0].K * d.frames for d in tr)
    res["info_gbit_s"] = info / sat["wall_s"] / 1e9
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_hybrid_baseline(eng, tr, frs, names, args.cpu_seconds, sat["frames_per_s"])
    print(json.dumps(res))


def timed_decode(dec, llr, d_o, torch, reps=2):
    """Event-timed decode of one batch (after one warm-up); returns (words,
    iterations, flags, seconds per decode)."""
    F = llr.shape[0]
    bits = torch.empty((F, dec.W64), dtype=torch.int64, device=llr.device)
    it = torch.empty(F, dtype=torch.uint8, device=llr.device)
    fl = torch.empty(F, dtype=torch.uint8, device=llr.device)
    ws = torch.empty(max(1, dec.workspace_size(F)), dtype=torch.uint8, device=llr.device)
    stream = torch.cuda.current_stream()
    dec.decode_into(llr, d_o, bits, it, fl, workspace=ws, stream=stream)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        dec.decode_into(llr, d_o, bits, it, fl, workspace=ws, stream=stream)
    b.record(stream)
    torch.cuda.synchronize()
    return bits.cpu().numpy().view(np.uint64), it.cpu().numpy(), fl.cpu().numpy(), a.elapsed_time(b) / 1e3 / reps


def run_latency(args):
    """Latency of one decode call against its size: each of the four workload
    codes (9 branches, restart mode, FP32, I_m = 8) at 3 dB, F in {64, 1024,
    16384, 65536} frames per call (the service's batch sizes), 50 timed calls
    after 5 warm-up calls, each timed with events on the decode stream
    (bucketing prepass included).  A call ends when its slowest frame stops,
    so the latency is that of up to 8 iterations; the row names the kernel the
    library picked for the size."""
    import torch

    from paper_2412_20828_amd import binding as B
    stream = torch.cuda.current_stream()
    rows = []
    for ci, (name, rows_h) in enumerate(SERVE_CODES):
        d = B.CODE_DEFS[name]
        code = B.Code(d.m, d.prim, d.t)
        pcm = B.Pcm.build(code, target_rows=rows_h, seed=1)
        dec = B.Decoder(code, pcm, n_branches=9, mode=B.MODE_RESTART, alpha=0.75, max_iter=8)
        fr = synth.frames(name, 65536, 3.0, seed=7000 + ci)
        llr_all, d_o_all = torch.from_numpy(fr.llr).cuda(), torch.from_numpy(fr.d_o).cuda()
        for F in (64, 1024, 16384, 65536):
            llr, d_o = llr_all[:F].contiguous(), d_o_all[:F].contiguous()
            bits = torch.empty((F, dec.W64), dtype=torch.int64, device="cuda")
            it = torch.empty(F, dtype=torch.uint8, device="cuda")
            fl = torch.empty(F, dtype=torch.uint8, device="cuda")
            ws = torch.empty(max(1, dec.workspace_size(F)), dtype=torch.uint8, device="cuda")
            for _ in range(5):
                dec.decode_into(llr, d_o, bits, it, fl, workspace=ws, stream=stream)
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(50)]
            torch.cuda.synchronize()
            for a, b in ev:
                a.record(stream)
                dec.decode_into(llr, d_o, bits, it, fl, workspace=ws, stream=stream)
                b.record(stream)
            torch.cuda.synchronize()
            ms = np.array([a.elapsed_time(b) for a, b in ev])
            rows.append({"code": name, "frames": F, "kernel": dec.kernel_name(F),
                         "latency_ms_p50": float(np.percentile(ms, 50)), "latency_ms_p99": float(np.percentile(ms, 99)),
                         "max_iters": int(it.max().item()), "frames_per_s": F / (float(np.median(ms)) / 1e3)})
            print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    best = min(r["latency_ms_p50"] for r in rows)
    print(json.dumps({"metric": "decoded frames/s & info Gbit/s at matched FER vs oracle; p50/p99 latency",
                      "workload": "latency", "n_gpus": 1, "data": "synthetic", "higher_is_better": False,
                      "vs_baseline": None, "steps": 50, "warmup": 5, "value": best, "unit": "ms",
                      "config": {"workload": "decode-call latency against call size, 9 branches, restart mode, FP32, "
                                             "I_m 8, 3 dB, codes of the service, 64-65536 frames per call"},
                      "rows": rows}))


def run_experiment(args):
    """Experiments of the method on the GPU kernels.

    alpha: the autotuner's alpha search (frame error rate against the
    normalisation factor of eq. 3 at the Eb/N0 where the paper fixes it, 2.6 dB
    for N = 63 and 3.0 dB for N = 127, 9 branches, restart mode, I_m = 8, 10^6
    frames); the argmin stands in for the paper's trained, unprinted values.

    beta: the redundancy factor of H_o (step 5 of Section III-A): rows, edges,
    length-4 cycles, FER, frames/s and VALU fraction for (63,36) at the
    paper's (beta, M_o) list (1, 27), (5, 47), (20, 122), (50, 269), (60, 316)
    at 3.5 dB with I_m = 4 and alpha tuned at 2.6 dB, and for (127,78) at
    beta = 1, 2, 3 (49, 57, 65 rows) at 4 dB; every matrix has a specialised
    kernel.

    ablation: what the automorphism merge buys: plain flooding NMS on the
    standard H (one branch, extrinsic messages), NMS on H_o (one branch,
    restart mode), and the 3- and 9-branch enhanced decoders, at 2, 3 and
    4 dB, 10^6 frames per point: FER, mean iterations and frames/s."""
    import torch

    from paper_2412_20828_amd import binding as B
    dev = torch.device("cuda:0")
    F = args.frames or 1_000_000
    out = {"metric": "decoded frames/s & info Gbit/s at matched FER vs oracle; p50/p99 latency", "n_gpus": 1,
           "data": "synthetic", "higher_is_better": True, "vs_baseline": None, "steps": 1, "warmup": 1}
    rows = []
    if args.workload == "alpha":
        from paper_2412_20828_amd import autotune
        for ci, (name, rows_h) in enumerate([("bch63_45", 33), ("bch63_36", 122), ("bch127_64", 72),
                                             ("bch127_99", 33)]):
            d = B.CODE_DEFS[name]
            code = B.Code(d.m, d.prim, d.t)
            pcm = B.Pcm.build(code, target_rows=rows_h, seed=1)
            e = autotune.search_alpha(code, pcm, name, rows_h, frames=F, seed=6000 + ci, write=args.write_alpha)
            rows.append({"code": name, "rows": rows_h, **e, "cached": args.write_alpha})
        out.update({"workload": "alpha", "config": {"workload": "alpha search: FER of the FP32 9-branch restart-"
                                                               "mode decoder, I_m 8, %d frames, grid 0.50:0.05:1.10 "
                                                               "widened until the argmin is inside" % F}})
    elif args.workload == "beta":
        # the redundancy list of Section III-A: (63,36) at beta = 1, 5, 20, 50, 60
        # with the row counts the paper prints (27, 47, 122, 269, 316), FER at
        # 3.5 dB with I_m = 4 and alpha tuned at 2.6 dB; (127,78) at beta = 1, 2, 3
        # (49, 57, 65 rows: M_o = M_r1 + beta (M - M_r1) with Table 1's
        # M_r1 = 41) at 4 dB with I_m = 8
        from paper_2412_20828_amd import autotune
        for ci, (name, betas, ebn0, im, tune_rows) in enumerate([
                ("bch63_36", [(1, 27), (5, 47), (20, 122), (50, 269), (60, 316)], 3.5, 4, 122),
                ("bch127_78", [(1, 49), (2, 57), (3, 65)], 4.0, 8, 57)]):
            d = B.CODE_DEFS[name]
            code = B.Code(d.m, d.prim, d.t)
            ref = B.Pcm.build(code, target_rows=tune_rows, seed=1)
            alpha = autotune.tuned_alpha(name, tune_rows, max_iter=im, default=float("nan"))
            if alpha != alpha:
                alpha = autotune.search_alpha(code, ref, name, tune_rows, frames=F, max_iter=im,
                                              seed=8100 + ci, write=args.write_alpha)["alpha"]
            llr_h, cw, d_o_h = gen_point(name, F, ebn0, seed=8000 + ci)
            truth = pack(cw)
            llr, d_o = torch.from_numpy(llr_h).to(dev), torch.from_numpy(d_o_h).to(dev)
            for beta, mo in betas:
                pcm = B.Pcm.build(code, target_rows=mo, seed=1)
                dec = B.Decoder(code, pcm, n_branches=9, mode=B.MODE_RESTART, alpha=alpha, max_iter=im)
                w, it, fl, sec = timed_decode(dec, llr, d_o, torch, reps=2)
                st = pcm.stats()
                ops = float(it.astype(np.int64).sum()) * alg_ops_per_iteration(code.N, code.K, pcm.M, pcm.E, 9)
                rows.append({"code": name, "beta": beta, "rows": pcm.M, "edges": pcm.E, "four_cycles": pcm.c4,
                             "row_weights": st["row_range"], "col_weights": st["col_range"],
                             "ebn0": ebn0, "max_iter": im, "alpha": alpha,
                             "fer": float((w != truth[:, :w.shape[1]]).any(1).mean()),
                             "avg_iters": float(it.mean()), "frames_per_s": F / sec,
                             "valu_frac": ops / sec / VALU_PEAK_OPS,
                             "kernel": dec.kernel_name(F) if dec.specialized else "generic"})
        out.update({"workload": "beta", "config": {"workload": "H_o redundancy sweep, 9 branches, restart mode, "
                                                              "%d frames per point" % F}})
    else:
        points = [2.0, 3.0, 4.0]
        for ci, (name, rows_h) in enumerate([("bch63_45", 33), ("bch63_36", 122)]):
            d = B.CODE_DEFS[name]
            code = B.Code(d.m, d.prim, d.t)
            ho = B.Pcm.build(code, target_rows=rows_h, seed=1)
            hs = B.Pcm.standard(code)
            cfgs = [("plain NMS, H_std (%dx63), 1 branch, extrinsic" % hs.M, hs, 1, B.MODE_EXTRINSIC, 0),
                    ("plain NMS, H_std (%dx63), 1 branch, extrinsic, generic kernel" % hs.M, hs, 1,
                     B.MODE_EXTRINSIC, B.FORCE_GENERIC),
                    ("NMS on H_o, 1 branch, restart", ho, 1, B.MODE_RESTART, 0),
                    ("enhanced NMS, 3 branches", ho, 3, B.MODE_RESTART, 0),
                    ("enhanced NMS, 9 branches", ho, 9, B.MODE_RESTART, 0)]
            for pi, e in enumerate(points):
                llr_h, cw, d_o_h = gen_point(name, F, e, seed=7000 + 10 * ci + pi)
                truth = pack(cw)
                llr, d_o = torch.from_numpy(llr_h).to(dev), torch.from_numpy(d_o_h).to(dev)
                for label, pcm, nb, mode, flags in cfgs:
                    dec = B.Decoder(code, pcm, n_branches=nb, mode=mode, alpha=0.75, max_iter=8, flags=flags)
                    w, it, fl, sec = timed_decode(dec, llr, d_o, torch, reps=1)
                    ops = float(it.astype(np.int64).sum()) * alg_ops_per_iteration(code.N, code.K, pcm.M, pcm.E,
                                                                                    nb, mode)
                    rows.append({"code": name, "ebn0": e, "config": label, "kernel": dec.kernel_name(F),
                                 "fer": float((w != truth[:, :w.shape[1]]).any(1).mean()),
                                 "avg_iters": float(it.mean()), "frames_per_s": F / sec,
                                 "valu_frac": ops / sec / VALU_PEAK_OPS})
        out.update({"workload": "ablation", "config": {"workload": "branch-count ablation, alpha 0.75, I_m 8, "
                                                                  "%d frames per point" % F}})
    out["rows"] = rows
    out["value"] = None
    out["unit"] = "frames/s"
    print(json.dumps(out))


def osd_costs(eng, done, torch, cap=2000):
    """Per failed frame: the library's host OSD-2 on one thread, and the
    device OSD-2 (throughput of one launch over the same frames), per code."""
    from paper_2412_20828_amd import binding as B
    from paper_2412_20828_amd import serving
    out = {}
    for k, (code, _) in enumerate(eng.codes):
        rows = [r.llr[np.nonzero(r.flags & serving.FLAG_OSD)[0]] for r in done if r.code == k and r.n_osd]
        if not rows:
            continue
        llr = np.ascontiguousarray(np.concatenate(rows)[:cap])
        n = llr.shape[0]
        t0 = time.time()
        B.osd_decode(code, llr, 2, n_threads=1)
        host = (time.time() - t0) / n * 1e6
        dl = torch.from_numpy(llr).cuda()
        bits = torch.zeros((n, 2), dtype=torch.int64, device="cuda")
        dec = eng.decs[k]
        dec.osd_into(dl, 2, bits)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dec.osd_into(dl, 2, bits)
        b.record()
        torch.cuda.synchronize()
        out[eng.names[k]] = {"frames": n, "host_one_thread_us": host, "device_us": a.elapsed_time(b) * 1e3 / n}
    return out


def cpu_hybrid_baseline(eng, tr, frs, names, budget_s, gpu_fps):
    """The oracle's hybrid (FP64 enhanced NMS, then OSD-2 on the frames whose
    syndrome is nonzero) on a bounded sample of the requests' frames."""
    import oracle
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    mats = {}
    for name, (code, pcm) in zip(names, eng.codes):
        H, Hstd = oracle_matrices(oracle, name, pcm)
        m, p, t = synth.CODES[name]
        mats[name] = (H, Hstd, oracle.Code(m, p, t).G)
    sample = []
    for k in range(len(names)):
        ks = [i for i, d in enumerate(tr) if d.code == k][:16]
        llr = np.concatenate([frs[i].llr for i in ks])[:256]
        d_o = np.concatenate([frs[i].d_o for i in ks])[:256]
        sample.append((names[k], llr, d_o))

    def one_pass():
        n = 0
        for name, llr, d_o in sample:
            H, Hs, G = mats[name]
            c, it, cv = oracle.decode_batch(H, Hs, llr, d_o, 9, 0.75, 8, oracle.R1, threads=threads)
            fail = np.nonzero(~cv.astype(bool))[0]
            if fail.size:
                oracle.osd_batch(G, llr[fail], 2)
            n += llr.shape[0]
        return n
    t0 = time.time()
    n = one_pass()
    pilot = time.time() - t0
    reps = max(1, int(budget_s / max(pilot, 1e-3)) - 1)
    t0 = time.time()
    for _ in range(reps):
        n += one_pass()
    secs = time.time() - t0 + pilot
    return {"value": n / secs, "unit": "frames/s", "cores": threads, "kind": "oracle",
            "sample": "%d frames (up to 256 frames from the first requests of each code, %d passes): FP64 enhanced "
                      "NMS oracle, then the oracle's OSD-2 on its failures (NMS on all cores, OSD serial)"
                      % (n, reps + 1), "seconds": secs, "gpu_over_cpu": gpu_fps / (n / secs)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="fix127", choices=sorted(WORKLOADS))
    ap.add_argument("--frames", type=int, default=0, help="frames per Eb/N0 point (0: the workload's)")
    ap.add_argument("--ebn0", type=str, default="", help="lo:hi:step dB (empty: the workload's)")
    ap.add_argument("--launch", default="code", choices=["code", "point"],
                    help="sweeps: one decode call per code over all its Eb/N0 points, or one per point")
    ap.add_argument("--cpu-seconds", type=float, default=30.0,
                    help="budget of the CPU oracle leg (FP64; the integer oracle gets a third of it)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--generic", action="store_true", help="force the generic (unspecialised) kernel")
    ap.add_argument("--tuned", action="store_true",
                    help="apply the autotuner's cached layouts (frames per wave) and grids")
    ap.add_argument("--precision", default="", choices=["", "fp32", "fix8", "both"],
                    help="override the workload's precisions")
    ap.add_argument("--packed16", action="store_true", help="fixed point: the packed 16-bit kernels (two frames per lane)")
    ap.add_argument("--chunk-buckets", action="store_true",
                    help="decoders with CHUNK_BUCKETS: each XCD decodes its own chunks of the batch first")
    ap.add_argument("--alpha", default="0.75",
                    help='alpha of the FP32 decoders: a number, or "tuned" (the autotuner\'s cached search result)')
    ap.add_argument("--graph", action="store_true",
                    help="capture each launch of the step in a HIP graph once and replay it in the timed loop")
    ap.add_argument("--write-alpha", action="store_true", help="alpha workload: cache the results in tuning.json")
    ap.add_argument("--mixed-path", default="fused", choices=["auto", "fused", "per-code"],
                    help="mixed workload: the mixed-code kernel (one launch, the workload's definition), "
                         "the library's choice by batch size, or one launch per code")
    ap.add_argument("--mix-probs", default="", help="mixed workload: per-code frame probabilities, comma-separated")
    ap.add_argument("--requests", type=int, default=3000, help="requests of the serving workload")
    ap.add_argument("--osd", default="device", choices=["device", "host"], help="serving: where OSD-2 runs")
    ap.add_argument("--slots", type=int, default=3, help="serving: batches in flight (slots)")
    ap.add_argument("--slot-frames", type=int, default=1 << 16, help="serving: frame capacity of a slot")
    ap.add_argument("--serve-eager", action="store_true",
                    help="serving: launch each slot step code by code instead of replaying its captured graph")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (calibrates HBM byte counters) and exit")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        x = torch.ones(args.copy_probe << 18, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe << 20, "copies": 3}))
        return
    if args.gpus != 1:
        print("bench.py: this build measures one GPU; --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.workload == "serve":
        # one hardware queue per stream of the engine (serving.hw_queues),
        # raised before anything starts HIP
        need = min(32, args.slots * (len(SERVE_CODES) + 1) + 1)
        if int(os.environ.get("GPU_MAX_HW_QUEUES", "4")) < need:
            os.environ["GPU_MAX_HW_QUEUES"] = str(need)
        return run_serve(args)
    if args.workload == "latency":
        return run_latency(args)
    if args.workload in ("alpha", "ablation", "beta"):
        return run_experiment(args)

    import torch

    from paper_2412_20828_amd import binding as B

    wl = WORKLOADS[args.workload]
    codes, grid, frames, precisions, wdesc = wl[:5]
    if args.precision:
        precisions = ["fp32", "fix8"] if args.precision == "both" else [args.precision]
        wdesc = wdesc.split(", FP32")[0] + ", precision " + "+".join(precisions)
    if args.alpha != "0.75" and "fp32" in precisions:
        wdesc += "; FP32 alpha %s" % (", ".join("%s %.2f" % (n, workload_alpha(args, n, r)) for n, r in codes)
                                      if args.alpha == "tuned" else args.alpha)
    args.frames = args.frames or frames
    args.ebn0 = args.ebn0 or grid
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    t0 = time.time()
    if args.workload == "mixed":
        lohi = [float(x) for x in args.ebn0.split(":")]
        probs = [float(p) for p in args.mix_probs.split(",")] if args.mix_probs else wl[5]
        if len(probs) != len(codes) or min(probs) < 0 or abs(sum(probs) - 1.0) > 1e-9:
            raise SystemExit("--mix-probs: %d probabilities >= 0 that sum to 1" % len(codes))
        if args.mix_probs:
            wdesc = wdesc.split(" in one call")[0].split(", per frame")[0] + ", per frame " + ", ".join(
                "%g%% %s" % (100 * p, n) for p, (n, _) in zip(probs, codes)) + " in one call"
        items, mats = build_mixed(args, B, torch, dev, stream, codes, probs, lohi, precisions, 4000)
        ebn0_desc = "U[%g, %g] per frame" % tuple(lohi)
    else:
        lo, hi, st = (float(x) for x in args.ebn0.split(":"))
        points = [round(lo + k * st, 3) for k in range(int(round((hi - lo) / st)) + 1)]
        items, mats = build_single(args, B, torch, dev, stream, codes, points, precisions,
                                   {"sweep63": 2000, "fix127": 3000}[args.workload])
        ebn0_desc = args.ebn0
    torch.cuda.synchronize()
    gen_s = time.time() - t0
    total_frames = sum(it.frames for it in items)

    for _ in range(args.warmup):
        for item in items:
            item.launch()
    torch.cuda.synchronize()
    if args.graph:
        # one graph per launch (prepass and persistent kernels of every code),
        # captured on a side stream and replayed on the decode stream
        cap = torch.cuda.Stream()
        for item in items:
            g = torch.cuda.CUDAGraph()
            cap.wait_stream(stream)
            with torch.cuda.stream(cap):
                with torch.cuda.graph(g, stream=cap):
                    item.launch_on(cap)
            stream.wait_stream(cap)
            item.graph = g
        torch.cuda.synchronize()

    def step(events=None):
        for k, item in enumerate(items):
            if events is not None:
                events[k][0].record(stream)
            if args.graph:
                item.graph.replay()
            else:
                item.launch()
            if events is not None:
                events[k][1].record(stream)

    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in items]
          for _ in range(args.steps)]
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for s in range(args.steps):
        step(ev[s])
    stop.record(stream)
    torch.cuda.synchronize()
    elapsed = start.elapsed_time(stop) / 1e3
    launch_ms = np.array([[a.elapsed_time(b) for a, b in evs] for evs in ev])  # [steps][launch]

    e2e = end_to_end(items, args.frames, torch, stream) if args.workload != "mixed" else None

    per_point = []
    ops_total = 0.0
    info_bits = 0
    time_by_prec, frames_by_prec = {}, {}
    by_kernel = {}  # kernel: [seconds per step, ops per step, launches per step, frames per step]
    for k, item in enumerate(items):
        pts, ops, info = item.stats()
        for p in pts:
            p["launch"] = item.label      # the decode call that holds the point
            p["launch_ms"] = float(np.median(launch_ms[:, k]))
        per_point += pts
        ops_total += ops
        info_bits += info
        t_item = launch_ms[:, k].sum() / 1e3 / args.steps
        time_by_prec[item.prec] = time_by_prec.get(item.prec, 0.0) + t_item
        frames_by_prec[item.prec] = frames_by_prec.get(item.prec, 0) + item.frames
        g = by_kernel.setdefault(item.kernel, [0.0, 0.0, 0, 0])
        g[0] += t_item
        g[1] += ops
        g[2] += 1
        g[3] += item.frames

    by_prec_kernel = {}
    for k, item in enumerate(items):
        g = by_prec_kernel.setdefault(item.prec, {}).setdefault(item.kernel, [0.0, 0.0, 0])
        g[0] += launch_ms[:, k].sum() / 1e3 / args.steps
    for kname, (t_k, ops_k, n_k, _) in by_kernel.items():
        for prec in by_prec_kernel:
            if kname in by_prec_kernel[prec]:
                by_prec_kernel[prec][kname][1:] = [ops_k, n_k]
    roof_prec = {}
    for prec, ks in by_prec_kernel.items():
        kd = max(ks, key=lambda n: ks[n][0])
        t_k, ops_k, n_k = ks[kd]
        roof_prec[prec] = {"kernel": kd, "achieved": ops_k / t_k / 1e12, "frac": ops_k / t_k / VALU_PEAK_OPS,
                           "avg_launch_ms": t_k / n_k * 1e3, "algorithmic_ops_per_launch": ops_k / n_k}
    kernel_s = launch_ms.sum() / 1e3 / args.steps
    achieved_all = ops_total / kernel_s
    dom = max(by_kernel, key=lambda n: by_kernel[n][0])
    t_dom, ops_dom, n_dom, fr_dom = by_kernel[dom]
    achieved = ops_dom / t_dom
    traffic = None
    if dom in TRAFFIC_B_PER_FRAME and kernel_src_hash(TRAFFIC_B_PER_FRAME[dom][2]) == TRAFFIC_B_PER_FRAME[dom][3]:
        traffic = sum(TRAFFIC_B_PER_FRAME[dom][:2]) * fr_dom / n_dom
    frames_per_s = total_frames * args.steps / elapsed
    res = {
        "metric": "decoded frames/s & info Gbit/s at matched FER vs oracle; p50/p99 latency",
        "value": frames_per_s,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if precisions == ["fp32"] else "f32+i8",
        "data": "synthetic",
        "config": {"workload": "%s, %d frames per %s, Eb/N0 %s dB%s%s" % (
                       wdesc, args.frames, "step" if args.workload == "mixed" else "point", ebn0_desc,
                       "" if args.workload == "mixed" else
                       ("; one decode call per code over all its points" if args.launch == "code" else
                        "; one decode call per point"),
                       ", each launch replayed from a captured HIP graph" if args.graph else ""),
                   "frames_per_step": total_frames},
        "frames_per_s_by_precision": {p: frames_by_prec[p] / time_by_prec[p] for p in time_by_prec},
        "info_gbit_s": info_bits * args.steps / elapsed / 1e9,
        "latency_ms": {"per_launch_p50": float(np.percentile(launch_ms, 50)),
                       "per_launch_p99": float(np.percentile(launch_ms, 99)),
                       "launch_frames": int(np.median([it.frames for it in items]))},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                     "unit": "Tops/s", "frac": achieved / VALU_PEAK_OPS, "traffic": traffic,
                     "kernel": dom, "launches_per_step": n_dom, "avg_launch_ms": t_dom / n_dom * 1e3,
                     "algorithmic_ops_per_launch": ops_dom / n_dom,
                     "traffic_bytes_per_frame": (list(TRAFFIC_B_PER_FRAME[dom][:2]) if traffic else None),
                     "hbm": ({"achieved_gb_s": traffic / (t_dom / n_dom) / 1e9, "peak_gb_s": HBM_PEAK_BYTES / 1e9,
                              "frac": traffic / (t_dom / n_dom) / HBM_PEAK_BYTES} if traffic else None),
                     "all_kernels": {"achieved": achieved_all / 1e12, "frac": achieved_all / VALU_PEAK_OPS}},
        "roofline_by_precision": roof_prec,
        "points": per_point,
        "input_generation_s": gen_s,
    }
    if e2e:
        res["end_to_end"] = e2e
    if "fix8" in precisions and "fp32" in precisions:
        fer = {(p["code"], p["ebn0"], p["precision"]): p["fer"] for p in per_point}
        res["fix8_fer_loss"] = [{"code": c, "ebn0": e, "fer_fp32": fer[(c, e, "fp32")], "fer_fix8": fer[(c, e, "fix8")]}
                                for (c, e, p) in fer if p == "fp32"]
    if not args.no_cpu:
        samples = [s for it in items for s in it.sample()]
        res["cpu_baseline"] = cpu_baseline(samples, mats, args.cpu_seconds, frames_per_s)
    print(json.dumps(res))


def oracle_matrices(oracle, name, pcm):
    """The oracle's own H_o (same construction parameters as the library's)
    and standard H; refuses to go on if the library's H_o differs."""
    m, p, t = synth.CODES[name]
    oc = oracle.Code(m, p, t)
    H, _, _ = oracle.build_hopt(oc, target_rows=pcm.M, seed=1)
    if not np.array_equal(H, pcm.dense()):
        raise RuntimeError("the library's H_o for %s differs from the oracle's" % name)
    return H, oc.Hstd


def _oracle_pass(oracle, Hs, samples, n_of, threads, kind):
    """Decode the first n_of[k] frames of every sample k with the oracle;
    returns (seconds, frames, per-sample results)."""
    t0 = time.time()
    out = []
    frames = 0
    for k, sm in enumerate(samples):
        H, Hstd = Hs[sm.code]
        n = n_of[k]
        c, it, cv = oracle.decode_batch(H, Hstd, sm.x[:n], sm.d_o[:n], 9, 0.75, 8, oracle.R1, kind=kind,
                                        threads=threads)
        out.append((c, it, cv))
        frames += n
    return time.time() - t0, frames, out


def cpu_baseline(samples, mats, budget_s, gpu_fps):
    """The oracle as it stands, on distinct frames of every Eb/N0 point (the
    first frames of each point, as many as fit the budget) on all host cores:
    the FP64 oracle on the FP32 points (its throughput is the reported
    value), the integer oracle on the fixed-point points (a third of the
    budget).  Per point it puts the oracle's frame error rate beside the
    GPU's on the same frames, each with a Wilson 95% interval, and counts the
    frames whose GPU word, iteration count and flag equal the oracle's."""
    import oracle
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    Hs = {name: oracle_matrices(oracle, name, mats[name]) for name in mats}
    legs = {"fp32": (oracle.KIND_FAST, budget_s), "fix8": (oracle.KIND_FIXED, budget_s / 3.0)}
    report, paired = {}, []
    for prec, (kind, budget) in legs.items():
        sm = [x for x in samples if x.prec == prec]
        if not sm:
            continue
        pilot_n = [min(256, x.x.shape[0]) for x in sm]
        secs, frames, _ = _oracle_pass(oracle, Hs, sm, pilot_n, threads, kind)
        rate = frames / max(secs, 1e-3)
        per = max(256, int(budget * rate / len(sm)))
        n_of = [min(per, x.x.shape[0]) for x in sm]
        secs, frames, res = _oracle_pass(oracle, Hs, sm, n_of, threads, kind)
        match = 0
        for x, n, (c, it, cv) in zip(sm, n_of, res):
            W = (Hs[x.code][0].shape[1] + 63) // 64
            ow = pack(c)[:, :W]
            gw = x.words[:n, :W]
            cw = x.cw[:n, :W]
            same = (gw == ow).all(1) & (x.iters[:n] == it) & (x.flags[:n].astype(bool) == cv)
            match += int(same.sum())
            eo = int((ow != cw).any(1).sum())
            eg = int((gw != cw).any(1).sum())
            paired.append({"code": x.code, "precision": prec, "ebn0": x.ebn0, "frames": n,
                           "oracle_fer": eo / n, "oracle_ci95": wilson(eo, n),
                           "gpu_fer": eg / n, "gpu_ci95": wilson(eg, n), "identical": int(same.sum())})
        report[prec] = {"frames_per_s": frames / secs, "frames": frames, "seconds": secs, "frames_per_point": per,
                        "identical_fraction": match / max(1, frames)}
    fp = report.get("fp32") or next(iter(report.values()))
    # one core: the first FP32 sample, for about a tenth of the budget
    x = next(v for v in samples if v.prec == "fp32") if any(v.prec == "fp32" for v in samples) else samples[0]
    H, Hstd = Hs[x.code]
    kind = oracle.KIND_FAST if x.prec == "fp32" else oracle.KIND_FIXED
    t1 = time.time()
    n1 = 0
    while time.time() - t1 < budget_s / 10:
        oracle.decode_batch(H, Hstd, x.x[:256], x.d_o[:256], 9, 0.75, 8, oracle.R1, kind=kind, threads=1)
        n1 += min(256, x.x.shape[0])
    one = n1 / (time.time() - t1)
    return {"value": fp["frames_per_s"], "unit": "frames/s", "cores": threads, "kind": "oracle",
            "sample": "%d distinct frames: the first %d frames of each of %d Eb/N0 points (or codes of a mixed "
                      "call), FP64 min1/min2 oracle on the same FP32 LLRs as the GPU" % (
                          fp["frames"], fp["frames_per_point"], sum(1 for v in samples if v.prec == "fp32")),
            "seconds": fp["seconds"], "gpu_over_cpu": gpu_fps / fp["frames_per_s"],
            "one_core": {"value": one, "sample": "%d frames of %s at %s dB" % (n1, x.code, x.ebn0)},
            "by_precision": report, "fer_paired": paired}


if __name__ == "__main__":
    main()
