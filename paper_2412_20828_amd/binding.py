"""ctypes binding of libbchnms.so (argument marshalling only).

Device buffers are PyTorch tensors on a HIP device (their data_ptr() is
passed); streams are torch.cuda streams (their cuda_stream handle is passed).
Every decode step runs in the library's HIP kernels; nothing here computes.
The binding refuses to run without the built library.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libbchnms.so")

BCH_OK = 0
BCH_PCM_STD, BCH_PCM_OPT = 0, 1
MODE_RESTART, MODE_MEMORY, MODE_EXTRINSIC = 1, 2, 3
FP32, FIX8 = 0, 1
FORCE_GENERIC = 1
PACKED16 = 2
SMALL_ALWAYS = 4
SMALL_NEVER = 8
UNPACKED16 = 16
NO_MIXED_KERNEL = 32
MIXED_KERNEL = 64
CHUNK_BUCKETS = 128
MIXED_KERNEL_MAX_FRAMES = 3_000_000

SYMBOLS = [
    "bch_last_error", "bch_load_code", "bch_code_info", "bch_code_export", "bch_code_destroy",
    "bch_build_pcm", "bch_pcm_from_dense", "bch_pcm_info", "bch_pcm_export", "bch_pcm_destroy",
    "bch_make_automorphisms", "bch_decoder_create", "bch_decoder_is_specialized",
    "bch_decoder_kernel_name",
    "bch_decoder_destroy", "bch_decode_workspace_size", "bch_nms_decode_batch",
    "bch_syndrome_check", "bch_quantize_llr", "bch_osd_decode", "bch_decoder_set_tuning",
    "bch_mixed_workspace_size", "bch_mixed_decode_batch", "bch_osd_decode_device", "bch_mixed_osd_decode",
    "bch_draw_offsets", "bch_draw_offsets_keys", "bch_pcm_stats", "bch_nms_decode_batch_noalloc", "bch_mixed_kernel_name",
]
MAX_MIX = 8


class BchError(RuntimeError):
    pass


class PcmParams(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("beta", ctypes.c_int), ("target_rows", ctypes.c_int),
                ("Q", ctypes.c_int), ("seed", ctypes.c_uint64), ("sa_steps_per_row", ctypes.c_int),
                ("sa_lambda", ctypes.c_double)]


class DecParams(ctypes.Structure):
    _fields_ = [("n_branches", ctypes.c_int), ("mode", ctypes.c_int), ("alpha", ctypes.c_float),
                ("max_iter", ctypes.c_int), ("precision", ctypes.c_int), ("flags", ctypes.c_int)]


_lib = None


def lib():
    """Load libbchnms.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise BchError("libbchnms.so is not built: run python -m paper_2412_20828_amd.build")
    # torch ships its own libamdhip64.so.7 (same soname as the system one): load
    # it first so that the library binds to torch's HIP runtime; otherwise the
    # process ends up with the system runtime and torch's HSA and sees no GPU
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u32, u64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
    L.bch_last_error.restype = ctypes.c_char_p
    L.bch_load_code.argtypes = [i32, u32, i32, P]
    L.bch_code_info.argtypes = [P, P, P, P]
    L.bch_code_export.argtypes = [P, P, P, P]
    L.bch_code_destroy.argtypes = [P]
    L.bch_code_destroy.restype = None
    L.bch_build_pcm.argtypes = [P, ctypes.POINTER(PcmParams), P]
    L.bch_pcm_from_dense.argtypes = [P, P, i32, P]
    L.bch_pcm_info.argtypes = [P, P, P, P, P, P, P]
    L.bch_pcm_export.argtypes = [P, P, ctypes.c_size_t]
    L.bch_pcm_destroy.argtypes = [P]
    L.bch_pcm_destroy.restype = None
    L.bch_make_automorphisms.argtypes = [i32, i32, i32, P]
    L.bch_draw_offsets.argtypes = [i32, u64, u64, i64, i64, P, i32, P]
    L.bch_draw_offsets_keys.argtypes = [i32, u64, i64, P, P, P]
    L.bch_pcm_stats.argtypes = [P, P, P, P, P]
    L.bch_decoder_create.argtypes = [P, P, ctypes.POINTER(DecParams), P]
    L.bch_decoder_is_specialized.argtypes = [P]
    L.bch_decoder_kernel_name.argtypes = [P, ctypes.c_int64]
    L.bch_decoder_kernel_name.restype = ctypes.c_char_p
    L.bch_decoder_destroy.argtypes = [P]
    L.bch_decoder_destroy.restype = None
    L.bch_decode_workspace_size.argtypes = [P, i64]
    L.bch_decode_workspace_size.restype = ctypes.c_size_t
    L.bch_nms_decode_batch.argtypes = [P, P, i64, i64, P, P, P, P, P, P, ctypes.c_size_t, P]
    L.bch_nms_decode_batch_noalloc.argtypes = [P, P, i64, i64, P, P, P, P, P, P]
    L.bch_syndrome_check.argtypes = [P, P, i64, P, P]
    L.bch_quantize_llr.argtypes = [P, i64, i64, i32, ctypes.c_float, P, i64, P]
    L.bch_osd_decode.argtypes = [P, P, i64, i64, i32, P, P, i32]
    L.bch_decoder_set_tuning.argtypes = [P, i32]
    L.bch_mixed_workspace_size.argtypes = [P, i32, i64]
    L.bch_mixed_workspace_size.restype = ctypes.c_size_t
    L.bch_mixed_decode_batch.argtypes = [P, i32, P, P, i64, i64, P, P, i64, P, P, P, ctypes.c_size_t, P]
    L.bch_mixed_kernel_name.argtypes = [P, i32, ctypes.c_int64]
    L.bch_mixed_kernel_name.restype = ctypes.c_char_p
    L.bch_osd_decode_device.argtypes = [P, P, i64, i64, i32, P, P, i64, P]
    L.bch_mixed_osd_decode.argtypes = [P, i32, P, P, i64, i64, i32, P, P, i64, P]
    _lib = L
    return L


def _check(rc, what):
    if rc != BCH_OK:
        raise BchError("%s failed (%d): %s" % (what, rc, lib().bch_last_error().decode()))


def _np(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise BchError("expected a device tensor")
    if not t.is_contiguous():
        raise BchError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Code:
    def __init__(self, m: int, prim: int, t: int):
        h = ctypes.c_void_p()
        _check(lib().bch_load_code(m, prim, t, ctypes.byref(h)), "bch_load_code")
        self.h = h
        N, K, tt = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().bch_code_info(h, ctypes.byref(N), ctypes.byref(K), ctypes.byref(tt)), "bch_code_info")
        self.N, self.K, self.t, self.m, self.prim = N.value, K.value, tt.value, m, prim

    def export(self):
        g = np.zeros(self.N - self.K + 1, np.uint8)
        G = np.zeros((self.K, self.N), np.uint8)
        H = np.zeros((self.N - self.K, self.N), np.uint8)
        _check(lib().bch_code_export(self.h, _np(g), _np(G), _np(H)), "bch_code_export")
        return g, G, H

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.bch_code_destroy(self.h)
            self.h = None


class Pcm:
    def __init__(self, code: Code, h):
        self.code, self.h = code, h
        M, N, E, c4, mr1, seed = (ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int64(),
                                  ctypes.c_int(), ctypes.c_uint64())
        _check(lib().bch_pcm_info(h, ctypes.byref(M), ctypes.byref(N), ctypes.byref(E), ctypes.byref(c4),
                                  ctypes.byref(mr1), ctypes.byref(seed)), "bch_pcm_info")
        self.M, self.N, self.E, self.c4, self.Mr1, self.seed_used = (M.value, N.value, E.value, c4.value,
                                                                     mr1.value, seed.value)

    @classmethod
    def build(cls, code: Code, kind=BCH_PCM_OPT, beta=2, target_rows=0, Q=4, seed=1,
              sa_steps_per_row=200, sa_lambda=10.0):
        p = PcmParams(kind, beta, target_rows, Q, seed, sa_steps_per_row, sa_lambda)
        h = ctypes.c_void_p()
        _check(lib().bch_build_pcm(code.h, ctypes.byref(p), ctypes.byref(h)), "bch_build_pcm")
        return cls(code, h)

    @classmethod
    def standard(cls, code: Code):
        return cls.build(code, kind=BCH_PCM_STD)

    @classmethod
    def from_dense(cls, code: Code, H):
        H = np.ascontiguousarray(H, dtype=np.uint8)
        h = ctypes.c_void_p()
        _check(lib().bch_pcm_from_dense(code.h, _np(H), H.shape[0], ctypes.byref(h)), "bch_pcm_from_dense")
        return cls(code, h)

    def stats(self) -> dict:
        """Table 1 attributes (bch_pcm_stats)."""
        M, E, c4 = ctypes.c_int(), ctypes.c_int(), ctypes.c_int64()
        w = np.zeros(8, np.float64)
        _check(lib().bch_pcm_stats(self.h, ctypes.byref(M), ctypes.byref(E), ctypes.byref(c4), _np(w)),
               "bch_pcm_stats")
        return {"M": M.value, "E": E.value, "c4": c4.value, "col_range": (int(w[0]), int(w[1])),
                "col_mean": float(w[2]), "col_std": float(w[3]), "row_range": (int(w[4]), int(w[5])),
                "row_mean": float(w[6]), "row_std": float(w[7])}

    def dense(self):
        out = np.zeros((self.M, self.N), np.uint8)
        _check(lib().bch_pcm_export(self.h, _np(out), out.size), "bch_pcm_export")
        return out

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.bch_pcm_destroy(self.h)
            self.h = None


def make_automorphisms(N: int, n_branches: int, d_o: int):
    maps = np.zeros((n_branches, N), np.int16)
    _check(lib().bch_make_automorphisms(N, n_branches, d_o, _np(maps)), "bch_make_automorphisms")
    return maps


def shift_period(N: int) -> int:
    """d_p of the cyclic shifts (Section III-B): 21 for N = 63, 42 for N = 127."""
    return {63: 21, 127: 42}.get(N, N // 3)


def draw_offsets(N: int, seed: int, key_hi: int, frame_base: int, F: int, out=None, stream=None):
    """Per-frame random offsets d_o in [0, d_p) (bch_draw_offsets).  out: a
    device uint8 tensor (drawn on the device, enqueued on stream), a host
    uint8 numpy array of F contiguous bytes, or None (a new numpy array)."""
    if out is None or isinstance(out, np.ndarray):
        d = np.zeros(F, np.uint8) if out is None else out
        if d.dtype != np.uint8 or d.shape != (F,) or not d.flags.c_contiguous:
            raise BchError("host d_o must be F contiguous uint8")
        _check(lib().bch_draw_offsets(N, seed, key_hi, frame_base, F, _np(d), 0, None), "bch_draw_offsets")
        return d
    _check(lib().bch_draw_offsets(N, seed, key_hi, frame_base, F, _dptr(out), 1, _stream(stream)),
           "bch_draw_offsets")
    return out


def draw_offsets_keys(N: int, seed: int, keys, counts, out=None):
    """Offsets of several keys in one host call (bch_draw_offsets_keys): key
    k's counts[k] frames one key after another.  out: a host uint8 numpy array
    of sum(counts) contiguous bytes, or None (a new array)."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    counts = np.ascontiguousarray(counts, dtype=np.int64)
    if keys.shape != counts.shape or keys.ndim != 1:
        raise BchError("keys and counts must be 1-D and of one length")
    F = int(counts.sum())
    d = np.zeros(F, np.uint8) if out is None else out
    if d.dtype != np.uint8 or d.shape != (F,) or not d.flags.c_contiguous:
        raise BchError("d_o must be sum(counts) contiguous uint8")
    _check(lib().bch_draw_offsets_keys(N, seed, keys.size, _np(keys), _np(counts), _np(d)), "bch_draw_offsets_keys")
    return d


class Decoder:
    def __init__(self, code: Code, pcm: Pcm, n_branches=9, mode=MODE_RESTART, alpha=0.75, max_iter=8,
                 precision=FP32, flags=0):
        p = DecParams(n_branches, mode, alpha, max_iter, precision, flags)
        h = ctypes.c_void_p()
        _check(lib().bch_decoder_create(code.h, pcm.h, ctypes.byref(p), ctypes.byref(h)), "bch_decoder_create")
        self.h, self.code, self.pcm = h, code, pcm
        self.N, self.n_branches, self.mode, self.alpha = code.N, n_branches, mode, alpha
        self.max_iter, self.precision, self.flags = max_iter, precision, flags
        self.W64 = (code.N + 63) // 64

    @property
    def specialized(self) -> bool:
        return bool(lib().bch_decoder_is_specialized(self.h))

    def kernel_name(self, F):
        """Name of the kernel a decode of F frames runs."""
        return lib().bch_decoder_kernel_name(self.h, F).decode()

    def set_tuning(self, waves_per_cu: int = 0):
        """Waves per CU of the persistent grid (0: the kernel's default)."""
        _check(lib().bch_decoder_set_tuning(self.h, waves_per_cu), "bch_decoder_set_tuning")
        self.tuning = waves_per_cu

    def workspace_size(self, F: int) -> int:
        return int(lib().bch_decode_workspace_size(self.h, F))

    def decode_into(self, llr, d_o, bits, iters, flags, y_trace=None, workspace=None, stream=None):
        """Enqueue bch_nms_decode_batch on device tensors (no allocation)."""
        F, ld = llr.shape
        ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
        _check(lib().bch_nms_decode_batch(self.h, _dptr(llr), ld, F, _dptr(d_o), _dptr(bits), _dptr(iters),
                                          _dptr(flags), _dptr(y_trace), _dptr(workspace), ws_bytes,
                                          _stream(stream)), "bch_nms_decode_batch")

    def decode_noalloc(self, llr, d_o, bits, iters, flags, y_trace=None, stream=None):
        """Enqueue bch_nms_decode_batch_noalloc (workspace from the library's
        device scratch; nothing allocated)."""
        F, ld = llr.shape
        _check(lib().bch_nms_decode_batch_noalloc(self.h, _dptr(llr), ld, F, _dptr(d_o), _dptr(bits), _dptr(iters),
                                                  _dptr(flags), _dptr(y_trace), _stream(stream)),
               "bch_nms_decode_batch_noalloc")

    def decode(self, llr, d_o=None, trace=False, stream=None):
        """Allocate outputs (and workspace) with torch and decode."""
        import torch
        F, ld = llr.shape
        dev = llr.device
        bits = torch.empty((F, self.W64), dtype=torch.int64, device=dev)
        iters = torch.empty(F, dtype=torch.uint8, device=dev)
        flags = torch.empty(F, dtype=torch.uint8, device=dev)
        tr = None
        if trace:
            tdt = torch.float32 if self.precision == FP32 else torch.int32
            tr = torch.zeros((F, self.max_iter, ld), dtype=tdt, device=dev)
        ws = None
        nws = self.workspace_size(F)
        if nws:
            ws = torch.empty(nws, dtype=torch.uint8, device=dev)
        if d_o is None:
            d_o = torch.zeros(F, dtype=torch.uint8, device=dev)
        elif self.n_branches > 1 and F and int(d_o.max()) >= shift_period(self.N):
            raise BchError("d_o must lie in [0, d_p) = [0, %d)" % shift_period(self.N))
        self.decode_into(llr, d_o, bits, iters, flags, tr, ws, stream)
        return bits, iters, flags, tr

    def osd_into(self, llr, order, bits, skip=None, stream=None):
        """Device OSD-p of the frames whose skip byte is 0 (all frames when
        skip is None); bits [F][>= W64] int64 is written for those frames."""
        F, ld = llr.shape
        _check(lib().bch_osd_decode_device(self.h, _dptr(llr), ld, F, order, _dptr(skip), _dptr(bits),
                                           bits.shape[1], _stream(stream)), "bch_osd_decode_device")

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.bch_decoder_destroy(self.h)
            self.h = None


class MixedDecoder:
    """Frames of several codes interleaved in one batch: one code-keyed
    prepass and one persistent kernel when the library has a mixed-code
    kernel for these matrices, else one of each per code, all enqueued on one
    stream."""

    def __init__(self, decoders):
        if not 1 <= len(decoders) <= MAX_MIX:
            raise BchError("a mix takes 1..%d decoders" % MAX_MIX)
        self.decoders = list(decoders)
        self._arr = (ctypes.c_void_p * len(decoders))(*[d.h.value for d in decoders])
        self.ld = 128 if max(d.N for d in decoders) > 64 else 64
        self.W64 = max(d.W64 for d in decoders)

    def workspace_size(self, F: int) -> int:
        return int(lib().bch_mixed_workspace_size(self._arr, len(self.decoders), F))

    def kernel_name(self, F: int) -> str:
        """The mixed-code kernel a call of F frames runs, or "per-code"."""
        return lib().bch_mixed_kernel_name(self._arr, len(self.decoders), F).decode()

    def decode_into(self, code_idx, llr, d_o, bits, iters, flags, workspace, stream=None):
        F, ld = llr.shape
        ws_bytes = workspace.numel() * workspace.element_size()
        _check(lib().bch_mixed_decode_batch(self._arr, len(self.decoders), _dptr(code_idx), _dptr(llr), ld, F,
                                            _dptr(d_o), _dptr(bits), bits.shape[1], _dptr(iters), _dptr(flags),
                                            _dptr(workspace), ws_bytes, _stream(stream)), "bch_mixed_decode_batch")

    def osd_into(self, code_idx, llr, order, bits, skip=None, stream=None):
        """Device OSD-p of every frame whose skip byte is 0, with its own code."""
        F, ld = llr.shape
        _check(lib().bch_mixed_osd_decode(self._arr, len(self.decoders), _dptr(code_idx), _dptr(llr), ld, F, order,
                                          _dptr(skip), _dptr(bits), bits.shape[1], _stream(stream)),
               "bch_mixed_osd_decode")

    def decode(self, code_idx, llr, d_o, stream=None):
        import torch
        F = llr.shape[0]
        dev = llr.device
        bits = torch.zeros((F, self.W64), dtype=torch.int64, device=dev)
        iters = torch.zeros(F, dtype=torch.uint8, device=dev)
        flags = torch.zeros(F, dtype=torch.uint8, device=dev)
        ws = torch.empty(max(1, self.workspace_size(F)), dtype=torch.uint8, device=dev)
        self.decode_into(code_idx, llr, d_o, bits, iters, flags, ws, stream)
        return bits, iters, flags


def syndrome_check(code: Code, bits, ok, stream=None):
    _check(lib().bch_syndrome_check(code.h, _dptr(bits), bits.shape[0], _dptr(ok), _stream(stream)),
           "bch_syndrome_check")


def quantize_llr(llr, N: int, scale: float, q, stream=None):
    F, ld = llr.shape
    _check(lib().bch_quantize_llr(_dptr(llr), ld, F, N, scale, _dptr(q), q.shape[1], _stream(stream)),
           "bch_quantize_llr")


def osd_decode(code: Code, llr: np.ndarray, order: int, skip=None, bits=None, n_threads=0):
    """Host OSD-p on float32 LLR rows; skip[f] != 0 leaves bits[f] untouched."""
    llr = np.ascontiguousarray(llr, dtype=np.float32)
    F, ld = llr.shape
    W64 = (code.N + 63) // 64
    if bits is None:
        bits = np.zeros((F, W64), np.uint64)
    sk = None if skip is None else np.ascontiguousarray(skip, dtype=np.uint8)
    _check(lib().bch_osd_decode(code.h, _np(llr), ld, F, order, _np(sk) if sk is not None else None,
                                _np(bits), n_threads), "bch_osd_decode")
    return bits


def unpack_bits(words: np.ndarray, N: int) -> np.ndarray:
    """[F][W64] uint64 words -> [F][N] uint8 bits (bit i of word i//64)."""
    w = np.ascontiguousarray(words).view(np.uint64)
    F = w.shape[0]
    out = np.zeros((F, N), np.uint8)
    for i in range(N):
        out[:, i] = ((w[:, i // 64] >> np.uint64(i % 64)) & np.uint64(1)).astype(np.uint8)
    return out


@dataclass(frozen=True)
class CodeDef:
    name: str
    m: int
    prim: int
    t: int


CODE_DEFS = {
    "bch63_36": CodeDef("bch63_36", 6, 0b1000011, 5),
    "bch63_45": CodeDef("bch63_45", 6, 0b1000011, 3),
    "bch127_64": CodeDef("bch127_64", 7, 0b10001001, 10),
    "bch127_78": CodeDef("bch127_78", 7, 0b10001001, 7),
    "bch127_99": CodeDef("bch127_99", 7, 0b10001001, 4),
}
