"""Throughput of enhanced normalized min-sum decoding of short BCH codes on
one MI355X.

Workload (one "step" = one pass of the whole decode path over the batch):
BCH(63,45) with the optimised 33 x 63 H_o and BCH(63,36) with the optimised
122 x 63 H_o; enhanced NMS with the 9-branch automorphism block (three random
cyclic shifts of y, pi_I y and pi_F y), restart message mode, alpha = 0.75, at
most 8 iterations with syndrome stopping, FP32; 1,000,000 frames per Eb/N0
point, Eb/N0 = 1.0, 1.5, ..., 6.0 dB; random information bits, BPSK over
AWGN, LLR = 2y/sigma^2 (seeded synthetic frames, resident in HBM before the
timed region).

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
                "configs[1]: BCH(63,45) H_o 33x63 and BCH(63,36) H_o 122x63, enhanced NMS 9 branches, restart "
                "mode, alpha 0.75, max 8 iterations, FP32"),
    "fix127": ([("bch127_64", 72), ("bch127_99", 33)], "2.0:5.0:0.5", 4_000_000, ["fp32", "fix8"],
               "configs[2]: BCH(127,64) H_o 72x127 and BCH(127,99) H_o 33x127, enhanced NMS 9 branches, restart "
               "mode, max 8 iterations, FP32 (alpha 0.75) vs int8 messages (alpha 3/4 shift-add, LLR x 4 "
               "quantised)"),
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
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU; --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2412_20828_amd import binding as B

    codes, grid, frames, precisions, wdesc = WORKLOADS[args.workload]
    args.frames = args.frames or frames
    args.ebn0 = args.ebn0 or grid
    lo, hi, st = (float(x) for x in args.ebn0.split(":"))
    points = [round(lo + k * st, 3) for k in range(int(round((hi - lo) / st)) + 1)]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    # work items: (code name, ebn0, decoder, device input, d_o, codewords, outputs, host llr, host d_o, precision)
    work = []
    t0 = time.time()
    decoders = {}
    seed_base = {"sweep63": 2000, "fix127": 3000}[args.workload]
    for ci, (name, rows) in enumerate(codes):
        d = B.CODE_DEFS[name]
        code = B.Code(d.m, d.prim, d.t)
        pcm = B.Pcm.build(code, target_rows=rows, seed=1)
        decs = {}
        for prec in precisions:
            decs[prec] = B.Decoder(code, pcm, n_branches=9, mode=B.MODE_RESTART, alpha=0.75, max_iter=8,
                                   precision=B.FIX8 if prec == "fix8" else B.FP32,
                                   flags=B.FORCE_GENERIC if args.generic else 0)
            decoders[(name, prec)] = (code, pcm, decs[prec])
        for pi, e in enumerate(points):
            llr, cw, d_o = gen_point(name, args.frames, e, seed=seed_base + 10 * ci + pi)
            F = llr.shape[0]
            llr_d = torch.from_numpy(llr).to(dev)
            d_o_d = torch.from_numpy(d_o).to(dev)
            for prec in precisions:
                dec = decs[prec]
                if prec == "fix8":
                    inp = torch.empty(llr_d.shape, dtype=torch.int8, device=dev)
                    B.quantize_llr(llr_d, code.N, FIX_SCALE, inp)
                else:
                    inp = llr_d
                out = (torch.empty((F, dec.W64), dtype=torch.int64, device=dev),
                       torch.empty(F, dtype=torch.uint8, device=dev),
                       torch.empty(F, dtype=torch.uint8, device=dev),
                       torch.empty(max(1, dec.workspace_size(F)), dtype=torch.uint8, device=dev))
                work.append((name, e, dec, inp, d_o_d, cw, out, llr[:64].copy(), d_o[:64].copy(), prec))
            del llr, llr_d
    torch.cuda.synchronize()
    gen_s = time.time() - t0
    total_frames = sum(w[3].shape[0] for w in work)

    def step(events=None):
        for k, (name, e, dec, llr, d_o, cw, out, _, _, _) in enumerate(work):
            if events is not None:
                events[k][0].record(stream)
            dec.decode_into(llr, d_o, out[0], out[1], out[2], workspace=out[3], stream=stream)
            if events is not None:
                events[k][1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in work]
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

    # per-point error rates and iteration totals (from the last step's outputs)
    per_point = []
    ops_total = 0.0
    time_by_prec = {}
    frames_by_prec = {}
    for k, (name, e, dec, llr, d_o, cw, out, _, _, prec) in enumerate(work):
        code, pcm, _ = decoders[(name, prec)]
        words = B.unpack_bits(out[0].cpu().numpy().view(np.uint64), code.N)
        iters = out[1].cpu().numpy().astype(np.int64)
        conv = out[2].cpu().numpy().astype(bool)
        err = (words != cw).any(1)
        time_by_prec[prec] = time_by_prec.get(prec, 0.0) + launch_ms[:, k].sum() / 1e3 / args.steps
        frames_by_prec[prec] = frames_by_prec.get(prec, 0) + len(err)
        per_point.append({"code": name, "precision": prec, "ebn0": e, "fer": float(err.mean()),
                          "ber": float((words != cw).mean()), "avg_iters": float(iters.mean()),
                          "undetected": float((err & conv).mean()),
                          "launch_ms": float(np.median(launch_ms[:, k]))})
        ops_total += iters.sum() * alg_ops_per_iteration(code.N, code.K, pcm.M, pcm.E, 9)
    
    kernel_s = launch_ms.sum() / 1e3 / args.steps
    achieved = ops_total / kernel_s
    frames_per_s = total_frames * args.steps / elapsed
    info_bits = sum(w[3].shape[0] * decoders[(w[0], w[9])][0].K for w in work)
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
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%s, %d frames per point, Eb/N0 %s dB" % (wdesc, args.frames, args.ebn0),
                   "frames_per_step": total_frames,
                   "specialised_kernel": {"%s/%s" % n: bool(decoders[n][2].specialized) for n in decoders}},
        "frames_per_s_by_precision": {p: frames_by_prec[p] / time_by_prec[p] for p in time_by_prec},
        "info_gbit_s": info_bits * args.steps / elapsed / 1e9,
        "latency_ms": {"per_launch_p50": float(np.percentile(launch_ms, 50)),
                       "per_launch_p99": float(np.percentile(launch_ms, 99)),
                       "launch_frames": args.frames},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                     "unit": "Tops/s", "frac": achieved / VALU_PEAK_OPS, "traffic": None},
        "points": per_point,
        "input_generation_s": gen_s,
    }
    if len(precisions) > 1:
        fer = {(p["code"], p["ebn0"], p["precision"]): p["fer"] for p in per_point}
        res["fix8_fer_loss"] = [{"code": c, "ebn0": e, "fer_fp32": fer[(c, e, "fp32")], "fer_fix8": fer[(c, e, "fix8")]}
                                for (c, e, p) in fer if p == "fp32"]
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline([w for w in work if w[9] == "fp32"], decoders, args.cpu_seconds,
                                           frames_per_s)
    print(json.dumps(res))


def cpu_baseline(work, decoders, budget_s, gpu_fps):
    """The FP64 oracle (as it stands) on a bounded sample of the same frames,
    on all host cores; also checks that the GPU outcomes on that sample are
    the oracle's (matched FER)."""
    import oracle
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    per = 64
    sample = []
    for (name, e, dec, llr, d_o, cw, out, llr_h, d_o_h, prec) in work:
        sample.append((name, llr_h[:per], d_o_h[:per], out))
    mats = {}
    for (name, prec) in decoders:
        code, pcm, _ = decoders[(name, prec)]
        m, p, t = synth.CODES[name]
        oc = oracle.Code(m, p, t)
        mats[name] = (pcm.dense(), oc.Hstd)
    # pilot (all points once) to size the sample to the budget
    t0 = time.time()
    for name, l0, d0, _ in sample:
        oracle.decode_batch(mats[name][0], mats[name][1], l0, d0, 9, 0.75, 8, oracle.R1, threads=threads)
    pilot = max(time.time() - t0, 1e-3)
    reps = max(1, int(budget_s / pilot))
    n = 0
    match = 0
    t0 = time.time()
    for name, l, d, out in sample:
        H, Hs = mats[name]
        ll = np.tile(l, (reps, 1))
        dd = np.tile(d, reps)
        c, it, cv = oracle.decode_batch(H, Hs, ll, dd, 9, 0.75, 8, oracle.R1, threads=threads)
        n += ll.shape[0]
        from paper_2412_20828_amd import binding as B
        gw = B.unpack_bits(out[0][:per].cpu().numpy().view(np.uint64), H.shape[1])
        gi = out[1][:per].cpu().numpy()
        match += int(((gw == c[:per]).all(1) & (gi == it[:per])).sum())
    secs = time.time() - t0
    return {"value": n / secs, "unit": "frames/s", "cores": threads, "kind": "oracle",
            "sample": "%d frames (first %d frames of each of the %d Eb/N0 points x %d repeats), FP64 "
                      "min1/min2 oracle, same frames as the GPU" % (n, per, len(sample), reps),
            "seconds": secs, "gpu_over_cpu": gpu_fps / (n / secs),
            "oracle_match_fraction": match / (per * len(sample))}


if __name__ == "__main__":
    main()
