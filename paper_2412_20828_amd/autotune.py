"""Autotuner of the specialised decoders: launch shape and normalisation factor.

The normalisation factor alpha of eq. 3 is the one scalar the method tunes;
the paper trains it as a network weight at one Eb/N0 per block length (2.6 dB
for N = 63, 3.0 dB for N = 127) and fixes it, without printing the values.
search_alpha() stands in for that training: the frame error rate of the FP32
nine-branch decoder on one synthetic batch at that Eb/N0 for every alpha of a
grid, the grid widened by 0.05 steps until the least error rate is inside it,
and the argmin cached per (code, rows of H_o, I_m); tuned_alpha() returns it
(0.75 when nothing is cached).

Launch-shape knobs:
  - frames per wave of the fixed-point decoders: 64 (integers held in 32-bit
    registers) or 128 (the packed 16-bit kernels, two frames per lane);
  - waves per CU of the persistent grid.
The tuner times every candidate on a synthetic batch of the decoder's own
code at a given Eb/N0, at the size of the benchmark's decode calls, and keeps
the fastest; results are cached in tuning.json beside this file, keyed by
(code, rows of H_o, precision, branches, GPU name).  tuned_decoder() builds a
decoder with the cached layout and grid; apply_cached() sets the grid of an
existing decoder.
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
    """Set the cached grid of an existing decoder (only when its layout is the
    cached one)."""
    from . import binding as B
    entry = load().get(key(code_name, rows, decoder.precision, decoder.n_branches, _gpu_name()))
    if not entry or not decoder.specialized:
        return False
    if bool(entry.get("packed16", False)) != bool(decoder.flags & B.PACKED16):
        return False
    decoder.set_tuning(entry["waves_per_cu"])
    return True


def tuned_decoder(code, pcm, code_name: str, rows: int, n_branches=9, mode=None, alpha=0.75, max_iter=8,
                  precision=0, flags=0):
    """A decoder with the cached layout (packed or not) and grid; the
    defaults when nothing is cached."""
    from . import binding as B
    mode = B.MODE_RESTART if mode is None else mode
    entry = load().get(key(code_name, rows, precision, n_branches, _gpu_name()))
    if entry and precision == B.FIX8:
        flags |= B.PACKED16 if entry.get("packed16") else B.UNPACKED16
    dec = B.Decoder(code, pcm, n_branches=n_branches, mode=mode, alpha=alpha, max_iter=max_iter,
                    precision=precision, flags=flags)
    if entry and dec.specialized:
        dec.set_tuning(entry["waves_per_cu"])
    return dec


ALPHA_GRID = [round(0.5 + 0.05 * k, 2) for k in range(13)]  # 0.50 .. 1.10
ALPHA_EBN0 = {63: 2.6, 127: 3.0}  # where the paper fixes alpha, per block length
ALPHA_MAX = 2.0


def alpha_key(code_name: str, rows: int, max_iter: int) -> str:
    return "alpha/%s/m%d/i%d" % (code_name, rows, max_iter)


def tuned_alpha(code_name: str, rows: int, max_iter: int = 8, default: float = 0.75) -> float:
    """The cached alpha of a code's decoder, or default."""
    entry = load().get(alpha_key(code_name, rows, max_iter))
    return float(entry["alpha"]) if entry else default


def search_alpha(code, pcm, code_name: str, rows: int, ebn0: float = None, frames: int = 1_000_000,
                 max_iter: int = 8, seed: int = 6000, grid=None, write: bool = True):
    """Frame error rate of the FP32 nine-branch restart-mode decoder for every
    alpha of the grid on one batch at ebn0 (default: the paper's tuning
    Eb/N0 of the block length); the grid grows by 0.05 at either end while
    the least error rate sits on that end (up to ALPHA_MAX).  Returns the
    entry {alpha, ebn0, frames, max_iter, fer: {alpha: FER}, bracketed}."""
    import numpy as np
    import torch

    import synth
    from . import binding as B
    ebn0 = ALPHA_EBN0.get(code.N, 3.0) if ebn0 is None else ebn0
    grid = sorted(grid or ALPHA_GRID)
    ld = 64 if code.N <= 64 else 128
    llr = torch.empty((frames, ld), dtype=torch.float32, device="cuda")
    d_o = torch.empty(frames, dtype=torch.uint8, device="cuda")
    cw = np.zeros((frames, code.N), np.uint8)
    blk = 250_000
    for k, f0 in enumerate(range(0, frames, blk)):
        q = synth.frames(code_name, min(blk, frames - f0), ebn0, seed=seed, block=k)
        llr[f0:f0 + len(q.d_o)].copy_(torch.from_numpy(q.llr))
        d_o[f0:f0 + len(q.d_o)].copy_(torch.from_numpy(q.d_o))
        cw[f0:f0 + len(q.d_o)] = q.codewords
    padded = np.zeros((frames, 128), np.uint8)
    padded[:, :code.N] = cw
    truth = torch.from_numpy(np.packbits(padded, axis=1, bitorder="little").view(np.int64)).cuda()
    fer = {}

    def run(a):
        dec = B.Decoder(code, pcm, n_branches=9, mode=B.MODE_RESTART, alpha=a, max_iter=max_iter)
        bits, _, _, _ = dec.decode(llr, d_o)
        fer[a] = float((bits != truth[:, :dec.W64]).any(1).float().mean())

    for a in grid:
        run(a)
    while True:
        best = min(fer, key=lambda a: (fer[a], abs(a - 0.75)))
        lo, hi = min(fer), max(fer)
        if best == hi and hi + 0.05 <= ALPHA_MAX + 1e-9:
            run(round(hi + 0.05, 2))
        elif best == lo and lo - 0.05 > 0.0:
            run(round(lo - 0.05, 2))
        else:
            break
    best = min(fer, key=lambda a: (fer[a], abs(a - 0.75)))
    entry = {"alpha": best, "ebn0": ebn0, "frames": frames, "max_iter": max_iter,
             "fer": {"%.2f" % a: fer[a] for a in sorted(fer)},
             "bracketed": min(fer) < best < max(fer)}
    if write:
        cache = load()
        cache[alpha_key(code_name, rows, max_iter)] = entry
        with open(CACHE, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
    return entry


def default_frames(N: int) -> int:
    """Batch size of the tuning runs: the benchmark's decode call of the sweep
    (11 Eb/N0 points of 10^6 frames, N = 63), and one 4 10^6-frame point of
    the 127-bit workloads.  The best choice depends on it: a smaller batch
    favours fewer resident frames, whose drain at the end of the launch is
    shorter (the packed kernels, 128 frames per wave, lose at 10^6 frames and
    win at 11 10^6)."""
    return 11_000_000 if N <= 64 else 4_000_000


def _batch(code_name, N, frames, ebn0, seed, block_frames=500_000):
    """Synthetic frames of one code on the device (generated in blocks)."""
    from concurrent.futures import ThreadPoolExecutor

    import torch

    import synth
    ld = 64 if N <= 64 else 128
    llr = torch.empty((frames, ld), dtype=torch.float32, device="cuda")
    d_o = torch.empty(frames, dtype=torch.uint8, device="cuda")
    starts = list(range(0, frames, block_frames))
    with ThreadPoolExecutor(min(16, os.cpu_count() or 4)) as ex:
        parts = ex.map(lambda k: synth.frames(code_name, min(block_frames, frames - starts[k]), ebn0, seed=seed,
                                              block=k), range(len(starts)))
        for f0, q in zip(starts, parts):
            llr[f0:f0 + len(q.d_o)].copy_(torch.from_numpy(q.llr))
            d_o[f0:f0 + len(q.d_o)].copy_(torch.from_numpy(q.d_o))
    return llr, d_o


def tune(decoder, code_name: str, rows: int, ebn0: float = 3.0, frames: int = 0, reps: int = 3,
         seed: int = 99, write: bool = True, batch=None):
    """Time every grid of one decoder and return the best (also cached when
    write).  batch: (llr FP32 [F][ld], d_o [F]) on the device, else generated."""
    import torch

    from . import binding as B
    if batch is None:
        batch = _batch(code_name, decoder.N, frames or default_frames(decoder.N), ebn0, seed)
    llr, d_o = batch
    if decoder.precision == B.FIX8:
        q = torch.empty(llr.shape, dtype=torch.int8, device="cuda")
        B.quantize_llr(llr, decoder.N, 4.0, q)
        llr = q
    F = llr.shape[0]
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
            "default_frames_per_s": F / next(d for d, w in results if w == 0),
            "packed16": bool(decoder.flags & B.PACKED16)}
    if write:
        cache = load()
        cache[key(code_name, rows, decoder.precision, decoder.n_branches, _gpu_name())] = best
        with open(CACHE, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
    return best, results


def tune_layout(code, pcm, code_name: str, rows: int, precision: int, ebn0: float = 3.0, frames: int = 0,
                reps: int = 3, seed: int = 99, write: bool = True):
    """Time every layout (fixed point: 64 or 128 frames per wave) and grid of
    a nine-branch decoder; cache and return the best entry and every layout's
    (best entry, timings)."""
    from . import binding as B
    cands = [B.UNPACKED16, B.PACKED16] if precision == B.FIX8 else [0]
    batch = None
    out = []
    for fl in cands:
        dec = B.Decoder(code, pcm, n_branches=9, max_iter=8, precision=precision, flags=fl)
        if not dec.specialized:
            continue
        if batch is None:
            batch = _batch(code_name, code.N, frames or default_frames(code.N), ebn0, seed)
        out.append(tune(dec, code_name, rows, ebn0=ebn0, reps=reps, seed=seed, write=False, batch=batch))
    if not out:
        return None, out
    best = dict(max((b for b, _ in out), key=lambda b: b["frames_per_s"]))
    best["default_frames_per_s"] = out[0][0]["default_frames_per_s"]  # the 64-frame layout, default grid
    if write:
        cache = load()
        cache[key(code_name, rows, precision, 9, _gpu_name())] = best
        with open(CACHE, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
    return best, out


def main():
    global CACHE
    import argparse
    ap = argparse.ArgumentParser(description="tune the specialised decoders' launch shape")
    ap.add_argument("--codes", default="bch127_64:72,bch127_99:33,bch63_36:122,bch63_45:33")
    ap.add_argument("--precisions", default="fp32,fix8")
    ap.add_argument("--ebn0", type=float, default=3.0)
    ap.add_argument("--frames", type=int, default=0,
                    help="frames per timed launch (0: 11 10^6 for N = 63, 4 10^6 for N = 127)")
    ap.add_argument("--out", default=CACHE, help="JSON cache to update")
    ap.add_argument("--alpha", action="store_true",
                    help="search alpha (FER argmin at the paper's tuning Eb/N0) instead of the launch shape")
    ap.add_argument("--alpha-frames", type=int, default=1_000_000)
    ap.add_argument("--max-iter", type=int, default=8, help="I_m of the alpha search")
    args = ap.parse_args()
    CACHE = args.out
    from . import binding as B
    if args.alpha:
        for spec in args.codes.split(","):
            name, rows = spec.split(":")
            d = B.CODE_DEFS[name]
            code = B.Code(d.m, d.prim, d.t)
            pcm = B.Pcm.build(code, target_rows=int(rows), seed=1)
            e = search_alpha(code, pcm, name, int(rows), frames=args.alpha_frames, max_iter=args.max_iter)
            print("%s/%s, I_m %d: alpha %.2f (FER %.5f at %.1f dB; 0.75: %.5f)" % (
                name, rows, args.max_iter, e["alpha"], e["fer"]["%.2f" % e["alpha"]], e["ebn0"], e["fer"]["0.75"]),
                flush=True)
        return
    for spec in args.codes.split(","):
        name, rows = spec.split(":")
        rows = int(rows)
        d = B.CODE_DEFS[name]
        code = B.Code(d.m, d.prim, d.t)
        pcm = B.Pcm.build(code, target_rows=rows, seed=1)
        for prec in args.precisions.split(","):
            best, res = tune_layout(code, pcm, name, rows, B.FIX8 if prec == "fix8" else B.FP32,
                                    ebn0=args.ebn0, frames=args.frames)
            if best is None:
                print("%s/%d/%s: no specialised kernel, skipped" % (name, rows, prec), flush=True)
                continue
            print("%s/%d/%s: best %s, waves %d: %.1fM frames/s (default %.1fM)" % (
                name, rows, prec, "128 frames per wave (packed)" if best["packed16"] else "64 frames per wave",
                best["waves_per_cu"], best["frames_per_s"] / 1e6, best["default_frames_per_s"] / 1e6), flush=True)


if __name__ == "__main__":
    main()
