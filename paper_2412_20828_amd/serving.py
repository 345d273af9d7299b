"""Continuous-batching decode service with the hybrid NMS + OSD back end.

Requests (frames of one code, channel LLRs on the host, one cyclic offset per
frame) arrive at any time.  The engine keeps every code's decoder (matrix
and branch tables) resident on the device and owns a fixed set of slots,
each a preallocated batch of pinned host staging, device buffers and a HIP
stream.  Whenever a slot is free, the pending requests are packed into it in
arrival order up to the slot's frame capacity (admission by memory: a slot
never holds more than it was sized for).  Inside the slot each code's frames
are contiguous, and every code present is decoded by its own call on a stream
of the slot's own, so the codes of a batch run side by side on the device
(a batch takes as long as its slowest code, not the sum of its codes).  Slots
run on their own streams too, so the batch of a newly admitted request
overlaps on the device with the batches already in flight.
Frames whose syndrome is still nonzero go to order-p OSD on their channel
LLRs (the hybrid of Section II-B and the complexity account C_t = C_1 +
F_1 C_2 of Section IV), either on the device, enqueued on the slot's stream
right after the decode (osd_on="device"), or on the host when the slot's
results are back (osd_on="host": one library call per code present in the
slot, spread over the OSD threads inside the library, so the interpreter lock
is taken once per call rather than per frame).  A request completes when all
of its frames have a decision.

Every frame decodes exactly as it would alone: the kernel's arithmetic for a
frame depends only on that frame's LLRs and offset, and OSD is deterministic.

With graph=True (the default) a slot's device work is also held as one HIP
graph, captured once per slot when the engine starts: a mixed-code decode over
the slot's whole capacity (frames past the batch carry a code index that names
no decoder, so the prepass skips them; the engine's code set has a mixed-code
kernel, so that is one prepass and one persistent kernel for every code of the
batch) followed by the device OSD of the frames that did not converge.  A step
of at least graph_min_frames frames replays it, with only the copies in and
out, sized by the batch, enqueued beside the replay: one graph launch and
three copies whatever the number of codes in the batch.  A smaller step (and
every step with graph=False) decodes each code present by its own call on a
stream of the slot's own: those calls pick the small-batch kernels, which
spread a frame's nine branches over three waves and so finish a small batch
about three times sooner than the one-wave mixed-code kernel.  The default
limit, 128 frames per CU, is where the per-code calls leave those kernels.

A slot uses 1 + (number of codes) streams (one with graph=True).  HIP maps a
process's streams onto GPU_MAX_HW_QUEUES hardware queues (4 by default), and
streams that share a queue run in submission order, so with too few queues
one slot's copies wait behind another slot's kernels.  A serving process
should set the variable to at least hw_queues(n_slots, n_codes) before HIP
initialises.
"""
from __future__ import annotations

import collections
import gc
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

from . import binding as B

FLAG_CONVERGED = 1
FLAG_OSD = 2


def hw_queues(n_slots: int, n_codes: int) -> int:
    """Hardware queues that give every stream of the engine its own (plus one
    for the default stream), capped at 32."""
    return min(32, n_slots * (n_codes + 1) + 1)


def settle_gc():
    """Collect once and move every object alive now into the collector's
    permanent generation.  Called by a service once its setup is done (engine,
    buffers, inputs): later full collections then scan only the objects made
    while serving, instead of the whole interpreter heap (with torch loaded, a
    full collection otherwise stalls the scheduler loop for tens of ms, which
    the requests in flight at that moment see as latency)."""
    gc.collect()
    gc.freeze()


@dataclass
class Request:
    code: int                  # index into the engine's code list
    llr: np.ndarray            # [F][ld] float32 channel LLRs (host)
    d_o: np.ndarray = None     # [F] uint8 cyclic offsets in [0, d_p), or None: drawn by the engine
    rid: int = 0
    arrival: float = 0.0       # time.perf_counter() at submission (set by submit when 0)
    bits: np.ndarray = None    # [F][2] uint64 decisions (bit i of word i // 64)
    iters: np.ndarray = None   # [F] NMS iterations
    flags: np.ndarray = None   # [F] FLAG_CONVERGED | FLAG_OSD
    t_admit: float = 0.0
    t_gpu: float = 0.0
    t_done: float = 0.0
    n_osd: int = 0

    @property
    def frames(self) -> int:
        return self.llr.shape[0]


@dataclass
class _Slot:
    stream: object          # copies in and out
    event: object           # results back on the host
    copied: object          # inputs on the device
    code_streams: list      # per code: its decode (and device OSD)
    code_done: list         # per code: event after its last kernel
    h_llr: object
    h_do: object
    d_llr: object
    d_do: object
    d_bits: object
    d_iters: object
    d_flags: object
    h_bits: object
    h_iters: object
    h_flags: object
    wss: list               # per code workspace
    h_ci: object = None     # graph mode: code index per frame (pinned), 255 past the batch
    d_ci: object = None
    ws_mix: object = None   # graph mode: workspace of the mixed call
    graph: object = None    # graph mode: the slot's captured decode + OSD
    prev_n: int = 0         # frames of the slot's previous batch (their code bytes are reset)
    n: int = 0              # frames of the batch in flight
    segs: list = field(default_factory=list)      # (first frame, frames) of each code in it
    members: list = field(default_factory=list)   # (request, offset)
    busy: bool = False


class Engine:
    """codes: [(name, rows of H_o)].  slot_frames: capacity of one slot (at
    least the largest request).  osd_order: order of the host OSD stage (None
    disables the hybrid), run on the device (osd_on="device") or on the host
    (osd_on="host": each finished slot's failed frames go to one OSD call per
    code, spread over osd_threads native threads; calls run one at a time on
    a helper thread, so the scheduler never waits for them).  tuned: apply the
    autotuner's cached launch shapes.  graph: replay one captured HIP graph
    per slot step of at least graph_min_frames frames (default 128 per CU;
    see the module notes)."""

    def __init__(self, codes, slot_frames=1 << 16, n_slots=3, osd_order=2, osd_on="device", osd_threads=8,
                 precision=B.FP32, max_iter=8, tuned=True, device="cuda", seed=0, graph=True,
                 graph_min_frames=None):
        import torch
        self.seed = seed  # key of the offsets the engine draws (bch_draw_offsets)
        self.torch = torch
        self.dev = torch.device(device)
        self.names = [n for n, _ in codes]
        self.codes, self.decs = [], []
        for name, rows in codes:
            d = B.CODE_DEFS[name]
            code = B.Code(d.m, d.prim, d.t)
            pcm = B.Pcm.build(code, target_rows=rows, seed=1)
            dec = B.Decoder(code, pcm, n_branches=9, mode=B.MODE_RESTART, alpha=0.75, max_iter=max_iter,
                            precision=precision)
            if not dec.specialized:
                raise B.BchError("%s with %d rows has no specialised kernel" % (name, rows))
            if tuned:
                from . import autotune
                autotune.apply_cached(dec, name, rows)
            self.codes.append((code, pcm))
            self.decs.append(dec)
        if precision != B.FP32:
            raise B.BchError("the service takes FP32 LLRs (quantise per code for int8 decoders)")
        # one-code calls of the mixed entry point: they take the slot's row
        # stride for the decisions, and an all-zero code index
        self.mixes1 = [B.MixedDecoder([d]) for d in self.decs]
        self.cap = slot_frames
        self.ld = B.MixedDecoder(self.decs).ld
        self.d_zero = torch.zeros(slot_frames, dtype=torch.uint8, device=self.dev)
        if osd_on not in ("device", "host"):
            raise B.BchError("osd_on must be 'device' or 'host'")
        self.osd_order = osd_order
        self.osd_on = osd_on
        self.osd_threads = osd_threads
        self.pending = collections.deque()
        self.osd_pool = ThreadPoolExecutor(1) if osd_order is not None and osd_on == "host" else None
        # staging of a step's frames (LLR copies into the pinned buffer and the
        # offset draws), one task per code: numpy's large copies and the
        # library's draw release the interpreter lock, so the codes' parts run
        # side by side instead of on the scheduler thread alone
        self.stage_pool = ThreadPoolExecutor(len(codes))
        self.osd_jobs = []
        ws_bytes = [max(1, m.workspace_size(slot_frames)) for m in self.mixes1]
        self.slots = []
        for _ in range(n_slots):
            pin = dict(pin_memory=True)
            cap, ld = slot_frames, self.ld
            self.slots.append(_Slot(
                stream=torch.cuda.Stream(device=self.dev), event=torch.cuda.Event(), copied=torch.cuda.Event(),
                code_streams=[torch.cuda.Stream(device=self.dev) for _ in self.decs],
                code_done=[torch.cuda.Event() for _ in self.decs],
                h_llr=torch.empty((cap, ld), dtype=torch.float32, **pin),
                h_do=torch.empty(cap, dtype=torch.uint8, **pin),
                d_llr=torch.empty((cap, ld), dtype=torch.float32, device=self.dev),
                d_do=torch.empty(cap, dtype=torch.uint8, device=self.dev),
                d_bits=torch.zeros((cap, 2), dtype=torch.int64, device=self.dev),
                d_iters=torch.empty(cap, dtype=torch.uint8, device=self.dev),
                d_flags=torch.empty(cap, dtype=torch.uint8, device=self.dev),
                h_bits=torch.empty((cap, 2), dtype=torch.int64, **pin),
                h_iters=torch.empty(cap, dtype=torch.uint8, **pin), h_flags=torch.empty(cap, dtype=torch.uint8, **pin),
                wss=[torch.empty(b, dtype=torch.uint8, device=self.dev) for b in ws_bytes]))
        self.mix = B.MixedDecoder(self.decs)
        self.graph = graph
        if graph_min_frames is None:
            graph_min_frames = 128 * torch.cuda.get_device_properties(self.dev).multi_processor_count
        self.graph_min_frames = graph_min_frames
        self.graph_steps = 0
        if graph:
            self._capture_graphs()
        self.launches = 0
        self.frames_launched = 0

    def _slot_device_work(self, s: _Slot, stream):
        """The device work of one slot step over its whole capacity: the
        mixed-code decode, then device OSD of the frames left unconverged."""
        self.mix.decode_into(s.d_ci, s.d_llr, s.d_do, s.d_bits, s.d_iters, s.d_flags, s.ws_mix, stream=stream)
        if self.osd_order is not None and self.osd_on == "device":
            self.mix.osd_into(s.d_ci, s.d_llr, self.osd_order, s.d_bits, skip=s.d_flags, stream=stream)

    def _capture_graphs(self):
        torch = self.torch
        cap = self.cap
        for s in self.slots:
            s.h_ci = torch.full((cap,), 255, dtype=torch.uint8, pin_memory=True)
            s.d_ci = torch.full((cap,), 255, dtype=torch.uint8, device=self.dev)
            s.ws_mix = torch.empty(max(1, self.mix.workspace_size(cap)), dtype=torch.uint8, device=self.dev)
            s.d_llr.zero_()
            s.d_do.zero_()
            # one eager pass outside the capture (first-use set-up of the
            # library), then the capture on the slot's stream
            s.stream.wait_stream(torch.cuda.current_stream(self.dev))
            with torch.cuda.stream(s.stream):
                self._slot_device_work(s, s.stream)
            s.stream.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s.stream):
                self._slot_device_work(s, torch.cuda.current_stream(self.dev))
            s.graph = g
        torch.cuda.synchronize(self.dev)

    # ------------------------------------------------------------ client side
    def submit(self, req: Request):
        if not 0 <= req.code < len(self.decs):
            raise B.BchError("unknown code index %d" % req.code)
        if req.frames > self.cap:
            raise B.BchError("request of %d frames exceeds the slot capacity %d" % (req.frames, self.cap))
        N = self.codes[req.code][0].N
        if req.llr.shape[1] < N:
            raise B.BchError("LLR rows shorter than the code length")
        if req.d_o is not None:
            if req.d_o.shape != (req.frames,):
                raise B.BchError("d_o must hold one offset per frame")
            if req.frames and int(req.d_o.max()) >= B.shift_period(N):
                raise B.BchError("d_o must lie in [0, d_p) = [0, %d)" % B.shift_period(N))
        if not req.arrival:
            req.arrival = time.perf_counter()
        self.pending.append(req)

    def draw_offsets(self, req: Request, out=None):
        """The random offsets of a request that brings none: the library's
        draw keyed by (engine seed, request id), frame uid = index in the
        request, so a request's frames get the same offsets alone and in any
        mix."""
        N = self.codes[req.code][0].N
        if out is None:
            return B.draw_offsets(N, self.seed, req.rid, 0, req.frames)
        return B.draw_offsets(N, self.seed, req.rid, 0, req.frames, out=out)

    def _stage(self, code: int, rs, hl, hd):
        """LLRs and offsets of the requests rs = [(request, offset in the
        slot)] of one code into the slot's pinned staging buffers."""
        drawn = []
        for r, off in rs:
            F, w = r.frames, min(r.llr.shape[1], self.ld)
            hl[off:off + F, :w] = r.llr[:, :w]
            if r.d_o is None:
                drawn.append((r, off))
            else:
                hd[off:off + F] = r.d_o
        if drawn:
            self._draw_segment(code, drawn, hd)

    def _draw_segment(self, code: int, rs, hd):
        """Offsets of the requests rs = [(request, offset in the slot)] of one
        code in one library call (keys = request ids), written into the
        slot's offset bytes hd: in place when the requests lie back to back,
        else through a temporary."""
        N = self.codes[code][0].N
        keys = np.fromiter((r.rid for r, _ in rs), np.uint64, len(rs))
        counts = np.fromiter((r.frames for r, _ in rs), np.int64, len(rs))
        lo, hi = rs[0][1], rs[-1][1] + rs[-1][0].frames
        if hi - lo == int(counts.sum()):
            B.draw_offsets_keys(N, self.seed, keys, counts, out=hd[lo:hi])
            return
        d = B.draw_offsets_keys(N, self.seed, keys, counts)
        o = 0
        for r, off in rs:
            hd[off:off + r.frames] = d[o:o + r.frames]
            o += r.frames

    def busy(self) -> bool:
        return bool(self.pending or self.osd_jobs or any(s.busy for s in self.slots))

    # ------------------------------------------------------------ scheduler
    def poll(self):
        """One scheduler pass: collect finished slots (hand failures to OSD),
        collect finished OSD jobs, then admit pending requests into free slots.
        Returns the requests completed in this pass."""
        done = []
        for s in self.slots:
            if s.busy and s.event.query():
                done += self._finish_slot(s)
        if self.osd_jobs:
            still = []
            for fut, req in self.osd_jobs:
                if fut.done():
                    req.t_done = fut.result()
                    done.append(req)
                else:
                    still.append((fut, req))
            self.osd_jobs = still
        for s in self.slots:
            if not self.pending:
                break
            if not s.busy:
                self._launch(s)
        return done

    def drain(self, sleep=20e-6):
        out = []
        while self.busy():
            new = self.poll()
            out += new
            if not new and sleep:
                time.sleep(sleep)
        return out

    def _launch(self, s: _Slot):
        torch = self.torch
        take, n = [], 0
        while self.pending and n + self.pending[0].frames <= self.cap:
            r = self.pending.popleft()
            take.append(r)
            n += r.frames
        if not take:
            return
        # each code's frames contiguous, requests in arrival order inside it
        counts = [0] * len(self.decs)
        for r in take:
            counts[r.code] += r.frames
        start = [0] * len(self.decs)
        for c in range(1, len(self.decs)):
            start[c] = start[c - 1] + counts[c - 1]
        pos = list(start)
        hl, hd = s.h_llr.numpy(), s.h_do.numpy()
        now = time.perf_counter()
        s.members = []
        per_code = [[] for _ in self.decs]
        for r in take:
            off = pos[r.code]
            r.t_admit = now
            s.members.append((r, off))
            per_code[r.code].append((r, off))
            pos[r.code] += r.frames
        s.n, s.segs = n, list(zip(start, counts))
        futs = [self.stage_pool.submit(self._stage, c, rs, hl, hd) for c, rs in enumerate(per_code) if rs]
        for f in futs:
            f.result()
        if self.graph and n >= self.graph_min_frames:
            # code bytes of this batch, and 255 over what the slot's previous
            # replay used beyond it, so that the replay decodes exactly these
            # frames
            hc = s.h_ci.numpy()
            for c in range(len(self.decs)):
                hc[start[c]:start[c] + counts[c]] = c
            top = max(n, s.prev_n)
            hc[n:top] = 255
            with torch.cuda.stream(s.stream):
                s.d_llr[:n].copy_(s.h_llr[:n], non_blocking=True)
                s.d_do[:n].copy_(s.h_do[:n], non_blocking=True)
                s.d_ci[:top].copy_(s.h_ci[:top], non_blocking=True)
                s.graph.replay()
                s.h_bits[:n].copy_(s.d_bits[:n], non_blocking=True)
                s.h_iters[:n].copy_(s.d_iters[:n], non_blocking=True)
                s.h_flags[:n].copy_(s.d_flags[:n], non_blocking=True)
            s.prev_n = n
            self.graph_steps += 1
            s.event.record(s.stream)
            s.busy = True
            self.launches += 1
            self.frames_launched += n
            return
        with torch.cuda.stream(s.stream):
            s.d_llr[:n].copy_(s.h_llr[:n], non_blocking=True)
            s.d_do[:n].copy_(s.h_do[:n], non_blocking=True)
        s.copied.record(s.stream)
        for c, cnt in enumerate(counts):
            if not cnt:
                continue
            st, seg, m = s.code_streams[c], slice(start[c], start[c] + cnt), self.mixes1[c]
            st.wait_event(s.copied)
            m.decode_into(self.d_zero[:cnt], s.d_llr[seg], s.d_do[seg], s.d_bits[seg], s.d_iters[seg],
                          s.d_flags[seg], s.wss[c], stream=st)
            if self.osd_order is not None and self.osd_on == "device":
                m.osd_into(self.d_zero[:cnt], s.d_llr[seg], self.osd_order, s.d_bits[seg], skip=s.d_flags[seg],
                           stream=st)
            s.code_done[c].record(st)
            s.stream.wait_event(s.code_done[c])
        with torch.cuda.stream(s.stream):
            s.h_bits[:n].copy_(s.d_bits[:n], non_blocking=True)
            s.h_iters[:n].copy_(s.d_iters[:n], non_blocking=True)
            s.h_flags[:n].copy_(s.d_flags[:n], non_blocking=True)
        s.event.record(s.stream)
        s.busy = True
        self.launches += 1
        self.frames_launched += n

    def _finish_slot(self, s: _Slot):
        done = []
        now = time.perf_counter()
        n = s.n
        # one copy of the batch's outputs; the requests get views of it
        bits = s.h_bits.numpy().view(np.uint64)[:n].copy()
        iters = s.h_iters.numpy()[:n].copy()
        flags = s.h_flags.numpy()[:n] & FLAG_CONVERGED
        for c, (st, cnt) in enumerate(s.segs):
            if cnt and self.decs[c].W64 == 1:
                bits[st:st + cnt, 1] = 0  # may hold a longer code's bits from an earlier batch
        conv = np.zeros(n + 1, np.int64)
        np.cumsum(flags, out=conv[1:])
        dev_osd = self.osd_order is not None and self.osd_on == "device"
        if dev_osd:
            flags[flags == 0] = FLAG_OSD  # decided on the device in the same slot
        by_code = {}
        for r, off in s.members:
            F = r.frames
            r.bits, r.iters, r.flags = bits[off:off + F], iters[off:off + F], flags[off:off + F]
            r.t_gpu = now
            r.n_osd = F - int(conv[off + F] - conv[off])
            if r.n_osd and not dev_osd and self.osd_pool is not None:
                by_code.setdefault(r.code, []).append((r, np.flatnonzero(r.flags == 0)))
            else:
                r.t_done = now
                done.append(r)
        for code, segs in by_code.items():
            fut = self.osd_pool.submit(self._osd, code, segs)
            for r, _ in segs:
                self.osd_jobs.append((fut, r))
        s.members = []
        s.busy = False
        return done

    def _osd(self, code: int, segs) -> float:
        """OSD of the failed frames of several requests of one code, in one
        library call over osd_threads native threads; returns the
        completion time."""
        llr = np.concatenate([r.llr[idx] for r, idx in segs])
        out = B.osd_decode(self.codes[code][0], llr, self.osd_order, n_threads=self.osd_threads)
        k = 0
        for r, idx in segs:
            r.bits[idx, :out.shape[1]] = out[k:k + idx.size]
            r.flags[idx] |= FLAG_OSD
            k += idx.size
        return time.perf_counter()

    def close(self):
        if self.osd_pool is not None:
            self.osd_pool.shutdown(wait=True)
        self.stage_pool.shutdown(wait=True)


def decode_alone(engine: Engine, req: Request):
    """Reference path for one request: its code's decoder on its frames alone,
    then host OSD on the failed frames (same back end as the service)."""
    torch = engine.torch
    dec = engine.decs[req.code]
    code = engine.codes[req.code][0]
    llr = torch.from_numpy(np.ascontiguousarray(req.llr)).to(engine.dev)
    d_h = req.d_o if req.d_o is not None else engine.draw_offsets(req)
    d_o = torch.from_numpy(np.ascontiguousarray(d_h)).to(engine.dev)
    bits, iters, flags, _ = dec.decode(llr, d_o)
    torch.cuda.synchronize()
    F = req.frames
    out = np.zeros((F, 2), np.uint64)
    out[:, :dec.W64] = bits.cpu().numpy().view(np.uint64)
    fl = flags.cpu().numpy() & FLAG_CONVERGED
    failed = np.nonzero(fl == 0)[0]
    if failed.size and engine.osd_order is not None:
        out[failed, :dec.W64] = B.osd_decode(code, req.llr[failed], engine.osd_order, n_threads=1)
        fl[failed] |= FLAG_OSD
    return out, iters.cpu().numpy(), fl


def run_trace(engine: Engine, reqs, offsets):
    """Replay requests in real time: request k is submitted offsets[k] seconds
    after the start (all at once when offsets are zero).  Returns the
    completed requests and the wall time from the first submission to the
    last completion."""
    order = np.argsort(np.asarray(offsets), kind="stable")
    t0 = time.perf_counter()
    k = 0
    done = []
    max_busy = 0
    while k < len(order) or engine.busy():
        now = time.perf_counter() - t0
        k0 = k
        while k < len(order) and offsets[order[k]] <= now:
            r = reqs[order[k]]
            r.arrival = t0 + offsets[order[k]]
            engine.submit(r)
            k += 1
        new = engine.poll()
        done += new
        max_busy = max(max_busy, sum(s.busy for s in engine.slots))
        if not new and k == k0:
            time.sleep(20e-6)  # idle: release the interpreter lock to the OSD helper
    wall = max(r.t_done for r in done) - t0
    engine.max_busy_slots = max_busy
    return done, wall


def summarize(done, wall):
    lat = np.array([r.t_done - r.arrival for r in done]) * 1e3
    frames = sum(r.frames for r in done)
    osd = sum(r.n_osd for r in done)
    return {"requests": len(done), "frames": frames, "wall_s": wall, "frames_per_s": frames / wall,
            "latency_ms_p50": float(np.percentile(lat, 50)), "latency_ms_p99": float(np.percentile(lat, 99)),
            "latency_ms_mean": float(lat.mean()), "osd_share": osd / max(1, frames),
            "gpu_latency_ms_p50": float(np.percentile([(r.t_gpu - r.arrival) * 1e3 for r in done], 50))}
