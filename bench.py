"""Throughput of enhanced normalized min-sum decoding of short BCH codes on
one MI355X.

Default workload "sweep63" (one "step" = one pass of the whole decode path
over the batch): BCH(63,45) with the optimised 33 x 63 H_o and BCH(63,36) with the optimised
122 x 63 H_o; enhanced NMS with the 9-branch automorphism block (three random
cyclic shifts of y, pi_I y and pi_F y), restart message mode, alpha = 0.75, at
most 8 iterations with syndrome stopping, FP32; 1,000,000 frames per Eb/N0
point, Eb/N0 = 1.0, 1.5, ..., 6.0 dB; random information bits, BPSK over
AWGN, LLR = 2y/sigma^2 (seeded synthetic frames, resident in HBM before the
timed region).

Other workloads (--workload): "fix127", BCH(127,64) and BCH(127,99) at
2.0..5.0 dB, 4,000,000 frames per point, FP32 and int8 fixed point; "mixed",
16,000,000 frames of BCH(127,64)/(127,99)/(63,36) interleaved per frame
(50/25/25 %) at Eb/N0 drawn per frame from U[1.5, 5] dB, decoded in one
mixed-code call, FP32 and int8.

Prints one JSON line with frames/s (value), information Gbit/s, per-launch
p50/p99 latency, the VALU roofline of the decode kernel and the CPU oracle
timed on a bounded sample of the same frames.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

# peak of 32-bit vector ALU lane-operations per second: 256 CUs x 64 lanes x 2.4 GHz
VALU_PEAK_OPS = 256 * 64 * 2.4e9
WORKLOADS = {
    # name: (codes with H_o rows, Eb/N0 grid, frames per point, precisions, description)
    "sweep63": ([("bch63_45", 33), ("bch63_36", 122)], "1.0:6.0:0.5", 1_000_000, ["fp32"],
                "BCH(63,45) H_o 33x63 and BCH(63,36) H_o 122x63, enhanced NMS 9 branches, restart "
                "mode, alpha 0.75, max 8 iterations, FP32"),
    "fix127": ([("bch127_64", 72), ("bch127_99", 33)], "2.0:5.0:0.5", 4_000_000, ["fp32", "fix8"],
               "BCH(127,64) H_o 72x127 and BCH(127,99) H_o 33x127, enhanced NMS 9 branches, restart "
               "mode, max 8 iterations, FP32 (alpha 0.75) vs int8 messages (alpha 3/4 shift-add, LLR x 4 "
               "quantised)"),
    "mixed": ([("bch127_64", 72), ("bch127_99", 33), ("bch63_36", 122)], "1.5:5.0", 16_000_000, ["fp32", "fix8"],
              "mixed-code batch, per frame 50% BCH(127,64) H_o 72x127, 25% BCH(127,99) H_o 33x127, "
              "25% BCH(63,36) H_o 122x63 in one call, enhanced NMS 9 branches, restart mode, max 8 iterations, "
              "FP32 and int8", [0.5, 0.25, 0.25]),
}
FIX_SCALE = 4.0


def alg_ops_per_iteration(N, K, M, E, B):
    """Algorithmic 32-bit operations of one iteration of one frame: per edge 8
    (v2c 1, min1/min2/argmin 3, sign 1, c2v select and sign 2, bit-sum add 1),
    per check row 2, per branch coordinate 2 (permutation and merge), plus the
    syndrome test 2 (N-K) ceil(N/64)."""
    return 8 * B * E + 2 * B * M + 2 * B * N + 2 * (N - K) * ((N + 63) // 64)


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


class Item:
    """One launch of the timed step: a single-code decode or a mixed-code one."""

    def __init__(self, label, prec, frames, launch):
        self.label, self.prec, self.frames, self.launch = label, prec, frames, launch
        self.stats = None     # () -> (per-point dicts, algorithmic ops, information bits)
        self.sample = None    # () -> [(code name, llr rows, d_o, gpu words, gpu iters)] for the CPU leg


def build_single(args, B, torch, dev, stream, codes, points, precisions, seed_base):
    items, mats = [], {}
    for ci, (name, rows) in enumerate(codes):
        d = B.CODE_DEFS[name]
        code = B.Code(d.m, d.prim, d.t)
        pcm = B.Pcm.build(code, target_rows=rows, seed=1)
        mats[name] = pcm
        decs = {prec: B.Decoder(code, pcm, n_branches=9, mode=B.MODE_RESTART, alpha=0.75, max_iter=8,
                                precision=B.FIX8 if prec == "fix8" else B.FP32,
                                flags=B.FORCE_GENERIC if args.generic else 0) for prec in precisions}
        for pi, e in enumerate(points):
            llr, cw, d_o = gen_point(name, args.frames, e, seed=seed_base + 10 * ci + pi)
            F = llr.shape[0]
            cwp = pack(cw)
            llr_d = torch.from_numpy(llr).to(dev)
            d_o_d = torch.from_numpy(d_o).to(dev)
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
                item = Item("%s@%g" % (name, e), prec, F,
                            lambda dec=dec, inp=inp, d_o_d=d_o_d, bits=bits, it=it, fl=fl, ws=ws:
                            dec.decode_into(inp, d_o_d, bits, it, fl, workspace=ws, stream=stream))

                def stats(name=name, e=e, prec=prec, code=code, pcm=pcm, bits=bits, it=it, fl=fl, cwp=cwp):
                    w = bits.cpu().numpy().view(np.uint64)
                    iters = it.cpu().numpy().astype(np.int64)
                    conv = fl.cpu().numpy().astype(bool)
                    err = (w != cwp[:, :w.shape[1]]).any(1)
                    nbit = int(np.bitwise_count(w ^ cwp[:, :w.shape[1]]).sum())
                    pt = {"code": name, "precision": prec, "ebn0": e, "fer": float(err.mean()),
                          "ber": nbit / (len(err) * code.N), "avg_iters": float(iters.mean()),
                          "undetected": float((err & conv).mean())}
                    ops = iters.sum() * alg_ops_per_iteration(code.N, code.K, pcm.M, pcm.E, 9)
                    return [pt], float(ops), len(err) * code.K

                def sample(name=name, llr=llr[:64].copy(), d_o=d_o[:64].copy(), bits=bits, it=it):
                    return [(name, llr, d_o, bits[:64].cpu().numpy().view(np.uint64), it[:64].cpu().numpy())]
                item.stats, item.sample = stats, (sample if prec == "fp32" else None)
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
        decs = [B.Decoder(c, p, n_branches=9, mode=B.MODE_RESTART, alpha=0.75, max_iter=8,
                          precision=B.FIX8 if prec == "fix8" else B.FP32) for c, p in objs]
        if args.tuned:
            from paper_2412_20828_amd import autotune
            for (name, rows), dec in zip(codes, decs):
                autotune.apply_cached(dec, name, rows)
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
        item = Item("mixed", prec, F, lambda mix=mix, inp=inp, bits=bits, it=it, fl=fl, ws=ws:
                    mix.decode_into(ci_d, inp, d_o_d, bits, it, fl, ws, stream=stream))

        def stats(prec=prec, bits=bits, it=it, fl=fl):
            w = bits.cpu().numpy().view(np.uint64)
            iters = it.cpu().numpy().astype(np.int64)
            conv = fl.cpu().numpy().astype(bool)
            err = (w != cwp).any(1)
            pts, ops, info = [], 0.0, 0
            for k, ((name, _), (code, pcm)) in enumerate(zip(codes, objs)):
                sel = ci == k
                pts.append({"code": name, "precision": prec, "ebn0": "U[%g,%g]" % tuple(lohi),
                            "frames": int(sel.sum()), "fer": float(err[sel].mean()),
                            "avg_iters": float(iters[sel].mean()), "undetected": float((err & conv)[sel].mean())})
                ops += iters[sel].sum() * alg_ops_per_iteration(code.N, code.K, pcm.M, pcm.E, 9)
                info += int(sel.sum()) * code.K
            return pts, float(ops), info

        def sample(bits=bits, it=it):
            out = []
            for k, (name, _) in enumerate(codes):
                sel = np.nonzero(ci == k)[0][:64]
                out.append((name, llr[sel].copy(), d_o[sel].copy(), bits.cpu().numpy().view(np.uint64)[sel],
                            it.cpu().numpy()[sel]))
            return out
        item.stats, item.sample = stats, (sample if prec == "fp32" else None)
        items.append(item)
    return items, mats


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sweep63", choices=sorted(WORKLOADS))
    ap.add_argument("--frames", type=int, default=0, help="frames per Eb/N0 point (0: the workload's)")
    ap.add_argument("--ebn0", type=str, default="", help="lo:hi:step dB (empty: the workload's)")
    ap.add_argument("--cpu-seconds", type=float, default=30.0, help="budget of the CPU oracle leg")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--generic", action="store_true", help="force the generic (unspecialised) kernel")
    ap.add_argument("--tuned", action="store_true", help="apply the autotuner's cached launch shapes")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU; --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2412_20828_amd import binding as B

    wl = WORKLOADS[args.workload]
    codes, grid, frames, precisions, wdesc = wl[:5]
    args.frames = args.frames or frames
    args.ebn0 = args.ebn0 or grid
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    t0 = time.time()
    if args.workload == "mixed":
        lohi = [float(x) for x in args.ebn0.split(":")]
        items, mats = build_mixed(args, B, torch, dev, stream, codes, wl[5], lohi, precisions, 4000)
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

    def step(events=None):
        for k, item in enumerate(items):
            if events is not None:
                events[k][0].record(stream)
            item.launch()
            if events is not None:
                events[k][1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
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

    per_point = []
    ops_total = 0.0
    info_bits = 0
    time_by_prec, frames_by_prec = {}, {}
    for k, item in enumerate(items):
        pts, ops, info = item.stats()
        for p in pts:
            p["launch_ms"] = float(np.median(launch_ms[:, k]))
        per_point += pts
        ops_total += ops
        info_bits += info
        time_by_prec[item.prec] = time_by_prec.get(item.prec, 0.0) + launch_ms[:, k].sum() / 1e3 / args.steps
        frames_by_prec[item.prec] = frames_by_prec.get(item.prec, 0) + item.frames

    kernel_s = launch_ms.sum() / 1e3 / args.steps
    achieved = ops_total / kernel_s
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
        "config": {"workload": "%s, %d frames per %s, Eb/N0 %s dB" % (
                       wdesc, args.frames, "step" if args.workload == "mixed" else "point", ebn0_desc),
                   "frames_per_step": total_frames},
        "frames_per_s_by_precision": {p: frames_by_prec[p] / time_by_prec[p] for p in time_by_prec},
        "info_gbit_s": info_bits * args.steps / elapsed / 1e9,
        "latency_ms": {"per_launch_p50": float(np.percentile(launch_ms, 50)),
                       "per_launch_p99": float(np.percentile(launch_ms, 99)),
                       "launch_frames": int(np.median([it.frames for it in items]))},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                     "unit": "Tops/s", "frac": achieved / VALU_PEAK_OPS, "traffic": None},
        "points": per_point,
        "input_generation_s": gen_s,
    }
    if "fix8" in precisions and "fp32" in precisions:
        fer = {(p["code"], p["ebn0"], p["precision"]): p["fer"] for p in per_point}
        res["fix8_fer_loss"] = [{"code": c, "ebn0": e, "fer_fp32": fer[(c, e, "fp32")], "fer_fix8": fer[(c, e, "fix8")]}
                                for (c, e, p) in fer if p == "fp32"]
    if not args.no_cpu:
        samples = [s for it in items if it.sample is not None for s in it.sample()]
        res["cpu_baseline"] = cpu_baseline(samples, mats, args.cpu_seconds, frames_per_s)
    print(json.dumps(res))


def cpu_baseline(samples, mats, budget_s, gpu_fps):
    """The FP64 oracle (as it stands) on a bounded sample of the same frames,
    on all host cores; also checks that the GPU outcomes on that sample are
    the oracle's (matched FER)."""
    import oracle
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    Hs = {}
    for name in mats:
        m, p, t = synth.CODES[name]
        Hs[name] = (mats[name].dense(), oracle.Code(m, p, t).Hstd)
    # pilot (every sample once) to size the repeat count to the budget
    t0 = time.time()
    for name, l0, d0, _, _ in samples:
        oracle.decode_batch(Hs[name][0], Hs[name][1], l0, d0, 9, 0.75, 8, oracle.R1, threads=threads)
    pilot = max(time.time() - t0, 1e-3)
    reps = max(1, int(budget_s / pilot))
    n = match = total = 0
    t0 = time.time()
    for name, l, d, gw, gi in samples:
        H, Hstd = Hs[name]
        per = l.shape[0]
        c, it, cv = oracle.decode_batch(H, Hstd, np.tile(l, (reps, 1)), np.tile(d, reps), 9, 0.75, 8, oracle.R1,
                                        threads=threads)
        n += per * reps
        W = (H.shape[1] + 63) // 64
        ow = pack(c[:per])[:, :W]
        match += int(((gw[:, :W] == ow).all(1) & (gi == it[:per])).sum())
        total += per
    secs = time.time() - t0
    return {"value": n / secs, "unit": "frames/s", "cores": threads, "kind": "oracle",
            "sample": "%d frames (the first 64 frames of each of %d launches' codes, %d repeats), FP64 "
                      "min1/min2 oracle, same frames as the GPU" % (n, len(samples), reps),
            "seconds": secs, "gpu_over_cpu": gpu_fps / (n / secs),
            "oracle_match_fraction": match / max(1, total)}


if __name__ == "__main__":
    main()
