"""Autotuner of the specialised decoders' launch shape.

Knob: waves per CU of the persistent grid (the frames per workgroup are fixed
by the kernel: 64 per one-wave workgroup and per three-wave group of the
nine-branch N = 63 kernels, 128 for the packed 16-bit kernels).  The tuner
times every candidate on a synthetic batch of the decoder's own code at a
given Eb/N0 and keeps the fastest; results are cached in tuning.json beside
this file, keyed by (code, rows of H_o, precision, branches, GPU name), and
applied by apply_cached().
"""
from __future__ import annotations

import json
import os
import time

_HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(_HERE, "tuning.json")
WAVES = [0, 2, 3, 4, 6, 8, 9, 12]


def key(code_name: str, rows: int, precision: int, n_branches: int, gpu: str) -> str:
    return "%s/m%d/%s/b%d/%s" % (code_name, rows, "fix8" if precision else "fp32", n_branches, gpu)


def _gpu_name():
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def load():
    if os.path.exists(CACHE):
        with open(CACHE) as fh:
            return json.load(fh)
    return {}


def apply_cached(decoder, code_name: str, rows: int) -> bool:
    entry = load().get(key(code_name, rows, decoder.precision, decoder.n_branches, _gpu_name()))
    if not entry or not decoder.specialized:
        return False
    decoder.set_tuning(entry["waves_per_cu"])
    return True


def default_frames(N: int) -> int:
    """Batch size of the tuning runs: the frames of one Eb/N0 point of the sweep
    (N = 63) and of the 127-bit workloads.  The best grid depends on it: a smaller batch
    favours fewer resident frames, whose drain at the end of the launch is
    shorter."""
    return 1_000_000 if N <= 64 else 4_000_000


def tune(decoder, code_name: str, rows: int, ebn0: float = 3.0, frames: int = 0, reps: int = 3,
         seed: int = 99, write: bool = True):
    """Time every candidate and return the best (also cached when write)."""
    import numpy as np
    import torch

    import synth
    from . import binding as B
    frames = frames or default_frames(decoder.N)
    fr = synth.frames(code_name, frames, ebn0, seed=seed)
    llr = torch.from_numpy(fr.llr).cuda()
    if decoder.precision == B.FIX8:
        q = torch.empty(llr.shape, dtype=torch.int8, device="cuda")
        B.quantize_llr(llr, decoder.N, 4.0, q)
        llr = q
    d_o = torch.from_numpy(fr.d_o).cuda()
    F = frames
    bits = torch.empty((F, decoder.W64), dtype=torch.int64, device="cuda")
    it = torch.empty(F, dtype=torch.uint8, device="cuda")
    fl = torch.empty(F, dtype=torch.uint8, device="cuda")
    # warm the clocks and caches first, so that the first candidate is not
    # timed on a cold GPU
    decoder.set_tuning(0)
    ws = torch.empty(max(1, decoder.workspace_size(F)), dtype=torch.uint8, device="cuda")
    for _ in range(2 * reps):
        decoder.decode_into(llr, d_o, bits, it, fl, workspace=ws)
    torch.cuda.synchronize()
    results = []
    for wv in WAVES:
        decoder.set_tuning(wv)
        ws = torch.empty(max(1, decoder.workspace_size(F)), dtype=torch.uint8, device="cuda")
        decoder.decode_into(llr, d_o, bits, it, fl, workspace=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            decoder.decode_into(llr, d_o, bits, it, fl, workspace=ws)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        results.append((dt, wv))
    results.sort()
    dt, wv = results[0]
    decoder.set_tuning(wv)
    best = {"waves_per_cu": wv, "frames_per_s": F / dt, "ebn0": ebn0, "frames": F,
            "default_frames_per_s": F / next(d for d, w in results if w == 0)}
    if write:
        cache = load()
        cache[key(code_name, rows, decoder.precision, decoder.n_branches, _gpu_name())] = best
        with open(CACHE, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
    return best, results


def main():
    global CACHE
    import argparse
    ap = argparse.ArgumentParser(description="tune the specialised decoders' launch shape")
    ap.add_argument("--codes", default="bch127_64:72,bch127_99:33,bch63_36:122,bch63_45:33")
    ap.add_argument("--precisions", default="fp32,fix8")
    ap.add_argument("--ebn0", type=float, default=3.0)
    ap.add_argument("--frames", type=int, default=0, help="frames per timed launch (0: 10^6 for N = 63, 4 10^6 for N = 127)")
    ap.add_argument("--out", default=CACHE, help="JSON cache to update")
    args = ap.parse_args()
    CACHE = args.out
    from . import binding as B
    for spec in args.codes.split(","):
        name, rows = spec.split(":")
        rows = int(rows)
        d = B.CODE_DEFS[name]
        code = B.Code(d.m, d.prim, d.t)
        pcm = B.Pcm.build(code, target_rows=rows, seed=1)
        for prec in args.precisions.split(","):
            dec = B.Decoder(code, pcm, n_branches=9, max_iter=8, precision=B.FIX8 if prec == "fix8" else B.FP32)
            if not dec.specialized:
                print("%s/%d/%s: no specialised kernel, skipped" % (name, rows, prec), flush=True)
                continue
            best, res = tune(dec, name, rows, ebn0=args.ebn0, frames=args.frames)
            print("%s/%d/%s: best waves %d: %.1fM frames/s (default %.1fM)" % (
                name, rows, prec, best["waves_per_cu"], best["frames_per_s"] / 1e6,
                best["default_frames_per_s"] / 1e6), flush=True)


if __name__ == "__main__":
    main()
