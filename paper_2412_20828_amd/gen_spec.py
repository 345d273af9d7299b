"""Generator of PCM-specialised decode kernels (stage 2 of the build).

The stage-1 library constructs each matrix the library is built for (the
construction is deterministic); this module then emits, per matrix, the row
function of nms_spec_fp32.inc with the matrix compiled in (static register
indices for every edge) and the syndrome test with the code's standard rows
as constants, plus the lookup table that maps a matrix fingerprint to the
kernel.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

# (code name, target rows of H_o (0: the standard matrix), n_branches, mode
#  (1 restart, 3 extrinsic messages), precision (0 FP32, 1 FIX8), waves per CU
#  of the persistent grid[, variant: 1 = packed 16-bit fixed point, 2 = three
#  waves per 64 frames for N = 127, the kernel for small batches])
SPECS = [
    ("bch63_45", 33, 9, 1, 0, 12),
    ("bch63_36", 122, 9, 1, 0, 12),
    ("bch63_36", 32, 9, 1, 0, 12),
    ("bch127_99", 33, 9, 1, 0, 4),
    ("bch127_64", 72, 9, 1, 0, 4),
    ("bch127_78", 57, 9, 1, 0, 4),
    ("bch63_45", 33, 9, 1, 1, 12),
    ("bch63_36", 122, 9, 1, 1, 12),
    ("bch127_99", 33, 9, 1, 1, 4),
    ("bch127_64", 72, 9, 1, 1, 4),
    # packed 16-bit fixed point, two frames per lane (opt-in variant)
    ("bch63_45", 33, 9, 1, 1, 8, 1),
    ("bch63_36", 122, 9, 1, 1, 8, 1),
    ("bch127_99", 33, 9, 1, 1, 4, 1),
    ("bch127_64", 72, 9, 1, 1, 4, 1),
    # small batches of the 127-bit codes: the branch types of 64 frames on
    # three waves (one workgroup per CU)
    ("bch127_99", 33, 9, 1, 0, 3, 2),
    ("bch127_64", 72, 9, 1, 0, 3, 2),
    ("bch127_78", 57, 9, 1, 0, 3, 2),
    ("bch127_99", 33, 9, 1, 1, 3, 2),
    ("bch127_64", 72, 9, 1, 1, 3, 2),
    # the redundancy sweep of Section III-A: (63,36) at the row counts the
    # paper lists for beta = 1, 5, 50, 60 (27, 47, 269, 316; 122 is beta = 20
    # above), and (127,78) at beta = 1 and 3 with Table 1's M_r1 = 41 (49 and 65
    # rows; 57 is beta = 2 above)
    ("bch63_36", 27, 9, 1, 0, 12),
    ("bch63_36", 47, 9, 1, 0, 12),
    ("bch63_36", 269, 9, 1, 0, 12),
    ("bch63_36", 316, 9, 1, 0, 12),
    ("bch127_78", 49, 9, 1, 0, 4),
    ("bch127_78", 65, 9, 1, 0, 4),
    # branch-count ablation (one and three branches, restart mode)
    ("bch63_45", 33, 3, 1, 0, 8),
    ("bch63_36", 122, 3, 1, 0, 8),
    ("bch63_45", 33, 1, 1, 0, 5),
    ("bch63_36", 122, 1, 1, 0, 4),
    # plain NMS with extrinsic messages on the standard matrices (rows 0):
    # the small configuration of the length-63 codes and the ablation's
    # baseline
    ("bch63_36", 0, 1, 3, 0, 8),
    ("bch63_45", 0, 1, 3, 0, 8),
]
# mixed-code kernels: one persistent launch over frames of these codes, code k
# of a mixed call being the k-th matrix here: the mixed workload's codes (FP32
# and fixed point) and the serving engine's four codes (FP32)
MIXES = [
    ([("bch127_64", 72), ("bch127_99", 33), ("bch63_36", 122)], 0),
    ([("bch127_64", 72), ("bch127_99", 33), ("bch63_36", 122)], 1),
    ([("bch63_36", 122), ("bch63_45", 33), ("bch127_64", 72), ("bch127_99", 33)], 0),
]
# rows whose min searches interleave in the one-wave kernels: one with the
# triple search (its steps hold two independent triples)
ILP_ROWS = 1
# nine-branch kernels compile the three cyclic shifts of a permutation type as
# three row functions, each on the matrix with its columns rotated by s d_p: a
# type then gathers its input once instead of three times, and its sums need
# no register rotation between the shifts
FOLD_SHIFTS = True
# one-wave kernels left unfolded: folded, BCH(127,99)'s 33-row kernels spill
# 33 registers to scratch instead of 3 (measured: 194 B of HBM writes per
# frame instead of 88, for 2.2% less time)
FOLD_EXCLUDE = {("bch127_99", 33)}
# entries whose update steps the packed 16-bit row function interleaves
PK16_GROUP = 4
# edges between scheduling barriers in the extrinsic-message row function
EXT_GROUP = 4
# frames a wave of the one- and three-branch kernels asks its cursor for at
# least: they stop frames nearly every iteration, at rates where one cursor
# atomic per iteration of every wave limits them.  The nine-branch kernels
# take exactly their idle slots (measured: a reserve per workgroup of the
# grouped N = 63 kernels gained nothing)
RESERVE = 64

CODE_DEFS = {
    "bch63_36": (6, 0b1000011, 5),
    "bch63_45": (6, 0b1000011, 3),
    "bch127_64": (7, 0b10001001, 10),
    "bch127_78": (7, 0b10001001, 7),
    "bch127_99": (7, 0b10001001, 4),
}


class _PcmParams(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("beta", ctypes.c_int), ("target_rows", ctypes.c_int),
                ("Q", ctypes.c_int), ("seed", ctypes.c_uint64), ("sa_steps_per_row", ctypes.c_int),
                ("sa_lambda", ctypes.c_double)]


def _matrices(lib, name, rows):
    m, prim, t = CODE_DEFS[name]
    code = ctypes.c_void_p()
    assert lib.bch_load_code(m, prim, t, ctypes.byref(code)) == 0
    N, K = ctypes.c_int(), ctypes.c_int()
    lib.bch_code_info(code, ctypes.byref(N), ctypes.byref(K), None)
    N, K = N.value, K.value
    Hs = np.zeros((N - K, N), np.uint8)
    lib.bch_code_export(code, None, None, Hs.ctypes.data_as(ctypes.c_void_p))
    if rows == 0:  # the standard matrix
        lib.bch_code_destroy(code)
        return Hs.copy(), Hs
    p = _PcmParams(1, 2, rows, 4, 1, 200, 10.0)
    pcm = ctypes.c_void_p()
    assert lib.bch_build_pcm(code, ctypes.byref(p), ctypes.byref(pcm)) == 0
    M = ctypes.c_int()
    lib.bch_pcm_info(pcm, ctypes.byref(M), None, None, None, None, None)
    H = np.zeros((M.value, N), np.uint8)
    lib.bch_pcm_export(pcm, H.ctypes.data_as(ctypes.c_void_p), H.size)
    lib.bch_pcm_destroy(pcm)
    lib.bch_code_destroy(code)
    return H, Hs


def fingerprint(H: np.ndarray) -> int:
    """FNV-1a over N, M and the rows packed as two little-endian 64-bit words
    (the library's pcm_fingerprint)."""
    M, N = H.shape
    h = 1469598103934665603
    mask = (1 << 64) - 1

    def mix(v):
        nonlocal h
        for k in range(8):
            h ^= (v >> (8 * k)) & 0xFF
            h = (h * 1099511628211) & mask

    mix(N)
    mix(M)
    for r in H:
        w0 = sum(1 << i for i in range(min(N, 64)) if r[i])
        w1 = sum(1 << (i - 64) for i in range(64, N) if r[i])
        mix(w0)
        mix(w1)
    return h


# The min1/min2 search runs on the bit patterns of the magnitudes: non-negative
# floats order as their bit patterns, so integer min, min3 and med3 give the
# same values as the float ones, with none of the input canonicalisation the
# compiler adds around a float min.  med3u is a min/max tree that the compiler
# matches to one v_med3_u32 in the entry-by-entry chain; med3i, for the triple
# search, is the float median builtin on the same bit patterns (one
# v_med3_f32: the magnitudes are canonical non-negative floats, never NaN, and
# the kernels keep FP32 denormals, so the float and integer medians are the
# same value).  From the min/max tree the compiler would share a min of the
# same operands between a triple's least value and its median and split the
# median into four instructions; written as inline asm it costs a wait state
# after every use.
_MED3U = """__device__ __forceinline__ uint32_t med3u(uint32_t a, uint32_t b, uint32_t c)
{
    return min(max(a, b), max(min(a, b), c));
}
__device__ __forceinline__ uint32_t med3i(uint32_t a, uint32_t b, uint32_t c)
{
    return __float_as_uint(__builtin_amdgcn_fmed3f(__uint_as_float(a), __uint_as_float(b), __uint_as_float(c)));
}
"""


def _sign_masks(cols, N):
    """Row masks over the sign words S of the 32-bit kernels, which shift the
    sign bits in coordinate by coordinate ((S << 1) | sign): coordinate c of
    word w = c // 32 sits at bit min(N, 32 (w + 1)) - 1 - c."""
    masks = [0] * ((N + 31) // 32)
    for c in cols:
        w = c // 32
        masks[w] |= 1 << (min(N, 32 * (w + 1)) - 1 - c)
    return masks


def _parity(S, masks):
    """Expression whose bit 0 is the parity of the sign bits S & masks: the
    masked words are folded with XOR first (the parity of an XOR is the XOR
    of the parities), so a row costs one popcount however many words N
    takes."""
    terms = ["(%s[%d] & 0x%08xu)" % (S, k, m) for k, m in enumerate(masks) if m]
    return "__builtin_popcount(%s)" % " ^ ".join(terms)


def _min_steps(cols, sfx, val, tree=True, pair_merge=True):
    """Steps (lists of statements) that leave u1<sfx> <= u2<sfx>, the two
    least of the row's values val(c), c in cols (integer form of non-negative
    floats).

    tree=False: one entry per step (u2 = med3(u1, u2, x), u1 = min(u1, x)),
    two instructions per entry and two live values.  tree=True: entries go in
    threes: min3 and med3 of a triple give its least two in two instructions;
    two triples merge into the running pair with u1 = min3(u1, m_a, m_b) and
    u2 = min(med3(u1, m_a, m_b), min3(u2, s_a, s_b)) (the second least of
    three sorted pairs is the middle of their leasts unless the pair holding
    the least has a smaller second): eight instructions per six entries where
    the chain takes twelve, for four more live values (pair_merge=False: one
    triple at a time, five per three).  The two least values of a set do not
    depend on the order they are found in, so every form gives the same
    u1, u2."""
    w = len(cols)
    if w < 2:
        raise ValueError("a check row needs at least two entries")
    v = [val(c) for c in cols]
    u1, u2 = "u1" + sfx, "u2" + sfx
    if not tree:
        steps = [["uint32_t %s = min(%s, %s), %s = max(%s, %s);" % (u1, v[0], v[1], u2, v[0], v[1])]]
        for x in v[2:]:
            steps.append(["%s = med3u(%s, %s, %s); %s = min(%s, %s);" % (u2, u1, u2, x, u1, u1, x)])
        return steps
    n3 = w // 3
    tri = [v[3 * k:3 * k + 3] for k in range(n3)]
    rest = v[3 * n3:]
    steps = []

    def triple(k, x):
        return ["const uint32_t m%s_%d = min(min(%s, %s), %s), s%s_%d = med3i(%s, %s, %s);"
                % (sfx, k, x[0], x[1], x[2], sfx, k, x[0], x[1], x[2])]

    if n3 == 0:
        steps.append(["uint32_t %s = min(%s, %s), %s = max(%s, %s);" % (u1, v[0], v[1], u2, v[0], v[1])])
        rest = v[2:]
    elif n3 == 1 or not pair_merge:
        steps.append(triple(0, tri[0]))
        steps.append(["uint32_t %s = m%s_0, %s = s%s_0;" % (u1, sfx, u2, sfx)])
        for k in range(1, n3):
            steps.append(triple(k, tri[k]))
            steps.append(["%s = med3i(%s, m%s_%d, min(%s, s%s_%d)); %s = min(%s, m%s_%d);"
                          % (u2, u1, sfx, k, u2, sfx, k, u1, u1, sfx, k)])
    else:
        steps.append(triple(0, tri[0]) + triple(1, tri[1]))
        steps.append(["uint32_t %s = min(m%s_0, m%s_1), %s = med3i(m%s_0, m%s_1, min(s%s_0, s%s_1));"
                      % (u1, sfx, sfx, u2, sfx, sfx, sfx, sfx)])
        k = 2
        while k + 1 < n3:
            steps.append(triple(k, tri[k]) + triple(k + 1, tri[k + 1]))
            a, b = k, k + 1
            steps.append(["%s = min(med3i(%s, m%s_%d, m%s_%d), min(min(%s, s%s_%d), s%s_%d)); "
                          "%s = min(min(%s, m%s_%d), m%s_%d);"
                          % (u2, u1, sfx, a, sfx, b, u2, sfx, a, sfx, b, u1, u1, sfx, a, sfx, b)])
            k += 2
        if k < n3:
            steps.append(triple(k, tri[k]))
            steps.append(["%s = med3i(%s, m%s_%d, min(%s, s%s_%d)); %s = min(%s, m%s_%d);"
                          % (u2, u1, sfx, k, u2, sfx, k, u1, u1, sfx, k)])
    for x in rest:
        steps.append(["%s = med3i(%s, %s, %s); %s = min(%s, %s);" % (u2, u1, u2, x, u1, u1, x)])
    return steps


def _forward(cols):
    """Lines of a row's min1 <= min2 search over A[cols] in integer form,
    ending with float m1, m2: the entry-by-entry chain, whose two live values
    suit the kernels that run several waves per SIMD within 168 registers."""
    out = []
    for st in _min_steps(cols, "", lambda c: "__float_as_uint(A[%d])" % c, tree=False):
        out += ["        " + x for x in st]
    out.append("        const float m1 = __uint_as_float(u1), m2 = __uint_as_float(u2);")
    return out


def body_source_ilp(H: np.ndarray, fix8: bool = False, group: int = 1, tree: bool = True,
                    helpers: bool = True) -> str:
    """The row function (accumulating form, FP32 or fixed point) with
    independent work side by side, for kernels that run one wave per SIMD and
    so have no other wave to issue while an instruction waits for its
    predecessor: the min1/min2 searches of `group` consecutive rows
    interleaved step by step (tree: by triples, see _min_steps, whose two
    independent triples per step already give the search its parallel work;
    else entry by entry), and the c2v selections of each row two edges at a
    time, pinned by scheduling barriers.  Every column is still updated by its
    rows in ascending order."""
    M, N = H.shape
    out = ([_MED3U] if helpers else []) + ["__device__ __forceinline__ void body(const float *__restrict__ A, "
                                           "const uint32_t *__restrict__ S, float *__restrict__ T)", "{"]
    for j0 in range(0, M, group):
        rows = list(range(j0, min(M, j0 + group)))
        out.append("    { // rows %s" % ", ".join(map(str, rows)))
        cols = {}
        for r, j in enumerate(rows):
            cs = [int(c) for c in np.nonzero(H[j])[0]]
            cols[r] = cs
            cnt = _parity("S", _sign_masks(cs, N))
            out.append("        const float sg%d = __uint_as_float(0x3f800000u | ((%s) << 31));" % (r, cnt))
        steps = {r: _min_steps(cols[r], "_%d" % r, lambda c: "__float_as_uint(A[%d])" % c, tree=tree) for r in cols}
        for k in range(max(len(st) for st in steps.values())):
            for r in cols:
                if k < len(steps[r]):
                    out += ["        " + x for x in steps[r][k]]
            out.append("        __builtin_amdgcn_sched_barrier(0);")
        for r in cols:
            out.append("        const float m1_%d = __uint_as_float(u1_%d), m2_%d = __uint_as_float(u2_%d);"
                       % (r, r, r, r))
            if fix8:
                out.append("        const float q1_%d = floorf(__builtin_fmaf(m1_%d, 0.75f, 0.5f)), "
                           "q2_%d = floorf(__builtin_fmaf(m2_%d, 0.75f, 0.5f));" % (r, r, r, r))
                out.append("        const float K_%d = __builtin_fmaf(m1_%d, 128.0f, q2_%d);" % (r, r, r))
            else:
                out.append("        const float P_%d = m1_%d + m2_%d;" % (r, r, r))
        for r in cols:
            cs = cols[r]
            for k in range(0, len(cs), 2):
                pair = cs[k:k + 2]
                for q, c in enumerate(pair):
                    if fix8:
                        sel = "__builtin_amdgcn_fmed3f(q1_%d, q2_%d, __builtin_fmaf(A[%d], -128.0f, K_%d))" % (
                            r, r, c, r)
                    else:
                        sel = "__builtin_amdgcn_fmed3f(m1_%d, m2_%d, P_%d - A[%d])" % (r, r, r, c)
                    out.append("        const float t%d_%d = %s;" % (r, k + q, sel))
                for q, c in enumerate(pair):
                    out.append("        T[%d] = __builtin_fmaf(sg%d, t%d_%d, T[%d]);" % (c, r, r, k + q, c))
                out.append("        __builtin_amdgcn_sched_barrier(0);")
        out.append("    }")
    out.append("}")
    return "\n".join(out)


def body_source(H: np.ndarray, accumulate: bool = False, helpers: bool = True) -> str:
    """Row function of the FP32 decoder.  accumulate: add every edge's c2v into
    T (T holds a running sum over branches) instead of overwriting T.
    helpers: emit the med3 helpers in front (once per source)."""
    M, N = H.shape
    out = ([_MED3U] if helpers else []) + ["__device__ __forceinline__ void body(const float *__restrict__ A, "
                                           "const uint32_t *__restrict__ S, float *__restrict__ T)", "{"]
    touched = [False] * N
    for j in range(M):
        cols = [int(c) for c in np.nonzero(H[j])[0]]
        cnt = _parity("S", _sign_masks(cols, N))
        out.append("    { // row %d" % j)
        out.append("        const uint32_t cnt = %s;" % cnt)
        out.append("        const float sg = __uint_as_float(0x3f800000u | (cnt << 31));")
        out += _forward(cols)
        out.append("        const float P = m1 + m2;")
        for c in cols:
            mag = "__builtin_amdgcn_fmed3f(m1, m2, P - A[%d])" % c
            if touched[c] or accumulate:
                out.append("        T[%d] = __builtin_fmaf(sg, %s, T[%d]);" % (c, mag, c))
            else:
                out.append("        T[%d] = sg * %s;" % (c, mag))
                touched[c] = True
        out.append("    }")
    for c in range(N):
        if not touched[c] and not accumulate:
            out.append("    T[%d] = 0.0f;" % c)
    out.append("}")
    return "\n".join(out)


def body_source_fix8(H: np.ndarray, accumulate: bool = False, helpers: bool = True) -> str:
    """Row function of the fixed-point decoder.  A holds the int8-saturated
    magnitudes (integers 0..127 held exactly as floats).  The c2v magnitude is
    (3m + 2) >> 2 = floor(0.75 m + 0.5) of the row's other-entry minimum m;
    with c1, c2 those of min1, min2 and K = c2 + 128 min1, med3(c1, c2,
    K - 128 A) is c2 at the argmin (A = min1) and c1 at every other entry
    (A >= min1 + 1 gives a third argument below 0).  All values are small
    integers, so every step is exact."""
    M, N = H.shape
    out = ([_MED3U] if helpers else []) + ["__device__ __forceinline__ void body(const float *__restrict__ A, "
                                           "const uint32_t *__restrict__ S, float *__restrict__ T)", "{"]
    touched = [False] * N
    for j in range(M):
        cols = [int(c) for c in np.nonzero(H[j])[0]]
        cnt = _parity("S", _sign_masks(cols, N))
        out.append("    { // row %d" % j)
        out.append("        const uint32_t cnt = %s;" % cnt)
        out.append("        const float sg = __uint_as_float(0x3f800000u | (cnt << 31));")
        out += _forward(cols)
        out.append("        const float q1 = floorf(__builtin_fmaf(m1, 0.75f, 0.5f)), "
                   "q2 = floorf(__builtin_fmaf(m2, 0.75f, 0.5f));")
        out.append("        const float K = __builtin_fmaf(m1, 128.0f, q2);")
        for c in cols:
            mag = "__builtin_amdgcn_fmed3f(q1, q2, __builtin_fmaf(A[%d], -128.0f, K))" % c
            if touched[c] or accumulate:
                out.append("        T[%d] = __builtin_fmaf(sg, %s, T[%d]);" % (c, mag, c))
            else:
                out.append("        T[%d] = sg * %s;" % (c, mag))
                touched[c] = True
        out.append("    }")
    for c in range(N):
        if not touched[c] and not accumulate:
            out.append("    T[%d] = 0.0f;" % c)
    out.append("}")
    return "\n".join(out)


def mixed_source(ns, parts, prec, out_dir):
    """Source of one mixed-code kernel: each code's row function and syndrome
    test in a namespace of its own, a traits struct per code, and the
    template.  parts: [(code name, H, Hstd)].  Every code takes the triple
    min1/min2 search of the one-wave kernels."""
    lines = ['#include "mix_launch.h"', "#define SPEC_FIX8 %d" % prec, "#include <hip/hip_runtime.h>",
             "#include <cstdint>", "namespace bch {", "namespace %s {" % ns]
    traits, cases = [], []
    for k, (name, H, Hs) in enumerate(parts):
        M, N = H.shape
        body_path = os.path.join(out_dir, "%s_c%d_body.inc" % (ns, k))
        with open(body_path, "w") as fh:
            fh.write("// generated: %s, H_o %d x %d, %d edges (code %d of %s)\n" % (name, M, N, int(H.sum()), k, ns))
            fh.write(body_source_ilp(H, fix8=bool(prec), group=ILP_ROWS, tree=True))
            fh.write("\n\n" + syndrome_source(Hs) + "\n")
        lines += ["namespace c%d {" % k, '#include "%s"' % os.path.basename(body_path), "}"]
        fn = ("    __device__ static __forceinline__ void body(const float *A, const uint32_t *S, float *T) "
              "{ c%d::body(A, S, T); }" % k)
        traits += ["struct T%d {" % k, "    static constexpr int N = %d;" % N, fn,
                   "    __device__ static __forceinline__ bool syndrome(const uint64_t *w) "
                   "{ return c%d::syndrome_zero(w); }" % k, "};"]
        cases.append("X(%d, T%d)" % (k, k))
    lines += traits + ["}  // namespace %s" % ns, "}  // namespace bch",
                       "#define MIX_NS %s" % ns, "#define MIX_CASES %s" % " ".join(cases),
                       '#include "nms_spec_mixed.inc"']
    src_path = os.path.join(out_dir, ns + ".hip")
    with open(src_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return src_path


def body_source_ext(H: np.ndarray) -> str:
    """Row function of the plain NMS decoder with extrinsic messages
    (nms_spec_ext.inc), in two passes over the rows.  Pass one: for every
    row, v = Y[c] - c2v_old on each edge (the old message rebuilt from the
    row's compressed state), min1/min2 of |v| (the triple search on the bit
    patterns) and the sign parity, and the new compressed state: RA = alpha
    min1, RB = alpha min2, RW = the new messages' sign bits (sign parity x
    sgn(v); the row's i-th edge of w at bit w - 1 - i, as v_alignbit shifts
    them in) with an argmin's edge index + 1 in bits 24-31.  Pass two: every
    row's new message, alpha min2 at the argmin and alpha min1 elsewhere with
    its sign bit, added into T[c], rows in ascending order.  Y is dead once
    pass one ends, so the sums T take its registers instead of living beside
    it.  Ties at min1 give min2 = min1, so every tied edge gets the same
    magnitude whichever is called the argmin (the last one here).  The sign
    of a zero |v| decides only messages of magnitude zero."""
    M, N = H.shape
    out = [_MED3U, "__device__ __forceinline__ void body_ext(const float *__restrict__ Y, float *__restrict__ T, "
           "float *RA, float *RB, uint32_t *RW, float alpha)", "{"]
    for j in range(M):
        cols = [int(c) for c in np.nonzero(H[j])[0]]
        w = len(cols)
        if w > 24 or N > 255:
            raise ValueError("the compressed state holds rows of at most 24 entries")
        out.append("    { // row %d" % j)
        out += _ext_messages(j, cols, "const float v%d = Y[%d] - ")
        vals = ["(__float_as_uint(v%d) & 0x7fffffffu)" % i for i in range(w)]
        for st in _min_steps(list(range(w)), "", lambda i: vals[i]):
            out += ["        " + x for x in st]
        # one v_alignbit per edge: s = (s << 1) | sign of v
        out.append("        uint32_t s = 0u;")
        for i in range(w):
            out.append("        s = __builtin_amdgcn_alignbit(s, __float_as_uint(v%d), 31);" % i)
        out.append("        const uint32_t par = __builtin_popcount(s) & 1u;")
        out.append("        const float am1 = alpha * __uint_as_float(u1), am2 = alpha * __uint_as_float(u2);")
        out.append("        uint32_t kn = 0u;")
        for i in range(w):
            out.append("        kn = (__float_as_uint(v%d) & 0x7fffffffu) == u1 ? %du : kn;" % (i, i + 1))
        out.append("        RA[%d] = am1;" % j)
        out.append("        RB[%d] = am2;" % j)
        out.append("        RW[%d] = (kn << 24) | (s ^ (par ? 0x%xu : 0u));" % (j, (1 << w) - 1))
        # rows in order: every row's v depends only on the inputs, and hoisting
        # them across rows would keep dozens of rows' values live at once
        out.append("        __builtin_amdgcn_sched_barrier(0);")
        out.append("    }")
    for j in range(M):
        cols = [int(c) for c in np.nonzero(H[j])[0]]
        out.append("    { // row %d, new messages" % j)
        out += _ext_messages(j, cols, "T[%d] += ", idx=False, after=M - 1)
        out.append("        __builtin_amdgcn_sched_barrier(0);")
        out.append("    }")
    out.append("}")
    return "\n".join(out)


def _ext_messages(j, cols, lhs, idx=True, after=None):
    """Statements that rebuild row j's messages from its compressed state
    (RA, RB, RW) and apply lhs to each: the message of the row's i-th edge
    (column c) is RB at the argmin, RA elsewhere, with bit w - 1 - i of RW
    as its sign (w edges).  With after = r, the rebuild takes RW[r] and RB[r] as inputs of its
    opaque step, so that it cannot be placed before row r's state is final (the
    compiler otherwise starts the second pass's first rows ahead of the
    first pass's last ones, with both passes' values live at once)."""
    out = ["        const float a = RA[%d], b = RB[%d];" % (j, j),
           # sw opaque: otherwise the compiler folds each edge's shift and
           # mask of it into the loop's phi and carries the row's sign bits in
           # as many registers from one iteration to the next instead of one
           # word; k opaque: compared with inline constants, not folded into
           # byte-select compares whose constant operands it would keep in
           # registers
           "        uint32_t sw = RW[%d], k;" % j,
           ('        __asm__("" : "+v"(sw));' if after is None else
            '        __asm__("" : "+v"(sw) : "v"(RW[%d]), "v"(RB[%d]));' % (after, after)),
           '        __asm__("v_lshrrev_b32 %0, 24, %1" : "=v"(k) : "v"(sw));']
    w = len(cols)
    for i, c in enumerate(cols):
        head = (lhs % (i, c)) if idx else (lhs % c)
        out.append("        %s__uint_as_float(__float_as_uint(k == %du ? b : a) | ((sw << %d) & 0x80000000u));"
                   % (head, i + 1, 32 - w + i))
        # the lane masks of the compares are consumed at once: scheduling
        # barriers every few edges keep the compiler from computing all of a
        # row's compares first and spilling their masks
        if i % EXT_GROUP == EXT_GROUP - 1:
            out.append("        __builtin_amdgcn_sched_barrier(0);")
    return out


def body_source_pk16(H: np.ndarray, B: int) -> str:
    """Row function of the packed 16-bit fixed-point decoder: A, T hold two
    frames per register (v2s), SL / SH their sign bits.  Adds s_j * mag_j(i)
    into T[i] for every entry, mag = q1 + (q2 - q1) e with q = (3m + 2) >> 2
    and e = 1 at an entry equal to min1, 0 elsewhere: the saturating unsigned
    difference (min1 + 1) - A (one packed instruction; every A is min1 or
    more).  Ties at min1 have q2 = q1, so every tied entry gets the same
    magnitude."""
    M, N = H.shape
    colw = H.sum(axis=0)
    if int(colw.max()) * 96 * B > 32767:
        raise ValueError("16-bit accumulators could overflow: column weight %d, %d branches" % (colw.max(), B))
    W32 = (N + 31) // 32
    out = ["__device__ __forceinline__ void body(const v2s *__restrict__ A, const uint32_t *__restrict__ SL, "
           "const uint32_t *__restrict__ SH, v2s *__restrict__ T)", "{"]
    for j in range(M):
        cols = [int(c) for c in np.nonzero(H[j])[0]]
        masks = [0] * W32
        for c in cols:
            masks[c // 32] |= 1 << (c % 32)
        cl, ch = _parity("SL", masks), _parity("SH", masks)
        out.append("    { // row %d" % j)
        out.append("        const uint32_t cl = %s, ch = %s;" % (cl, ch))
        out.append("        const v2s sg = __builtin_bit_cast(v2s, ((cl & 1u) ? 0xffffu : 1u) | "
                   "(((ch & 1u) ? 0xffffu : 1u) << 16));")
        # min1 <= min2 of the row: two running chains over alternate entries,
        # emitted interleaved (independent, so their dependent min / max steps
        # overlap), then one merge (x1, x2), (y1, y2) -> (min(x1, y1),
        # min(max(x1, y1), min(x2, y2))): the same instruction count as one chain
        ca, cb = cols[0::2], cols[1::2]

        def start(ch, tag):
            if len(ch) >= 2:
                return ["v2s %s1 = vmin(A[%d], A[%d]), %s2 = vmax(A[%d], A[%d]);" % (tag, ch[0], ch[1], tag, ch[0], ch[1])], ch[2:]
            return ["v2s %s1 = A[%d], %s2 = (v2s)127;" % (tag, ch[0], tag)], ch[1:]
        la, ra = start(ca, "x")
        lb, rb = start(cb, "y")
        out.append("        " + la[0] + " " + lb[0])
        for k in range(max(len(ra), len(rb))):
            parts = []
            if k < len(ra):
                parts.append("x2 = vmax(x1, vmin(x2, A[%d])); x1 = vmin(x1, A[%d]);" % (ra[k], ra[k]))
            if k < len(rb):
                parts.append("y2 = vmax(y1, vmin(y2, A[%d])); y1 = vmin(y1, A[%d]);" % (rb[k], rb[k]))
            out.append("        " + " ".join(parts))
        out.append("        const v2s m1 = vmin(x1, y1), m2 = vmin(vmax(x1, y1), vmin(x2, y2));")
        out.append("        const v2s q1 = (m1 * (v2s)3 + (v2s)2) >> (v2s)2, q2 = (m2 * (v2s)3 + (v2s)2) >> (v2s)2;")
        out.append("        const v2u m1p = __builtin_bit_cast(v2u, m1) + (v2u)1;")
        out.append("        const v2s sq1 = sg * q1, sdq = sg * (q2 - q1);")
        # the three dependent steps of an entry's update, emitted a group of
        # entries at a time: a packed 16-bit result read by the next
        # instruction costs a wait state, which independent entries fill
        for g0 in range(0, len(cols), PK16_GROUP):
            grp = cols[g0:g0 + PK16_GROUP]
            out.append("        " + " ".join("const v2s e%d = is_min(m1p, A[%d]);" % (c, c) for c in grp))
            out.append("        " + " ".join("T[%d] = sdq * e%d + T[%d];" % (c, c, c) for c in grp))
            out.append("        " + " ".join("T[%d] = T[%d] + sq1;" % (c, c) for c in grp))
        out.append("    }")
    out.append("}")
    return "\n".join(out)


def shift_matrices(H: np.ndarray, dp: int, ns: int = 3):
    """The matrix of each cyclic shift s d_p (s < ns) in the frame of shift 0:
    the row function of branch s reads entry c of the shifted input at index
    (c - s d_p) mod N of the shift-0 input, so its matrix is H with its
    columns rotated left by s d_p.  The rows and their order are H's."""
    return [np.roll(H, -s * dp, axis=1) for s in range(ns)]


def folded_body_source(H: np.ndarray, dp: int, emit) -> str:
    """Three row functions f0::body, f1::body, f2::body, one per cyclic shift
    (see shift_matrices); emit(H_s) returns the source of one."""
    out = []
    for s, Hs in enumerate(shift_matrices(H, dp)):
        out.append("namespace f%d {" % s)
        out.append(emit(Hs))
        out.append("}  // namespace f%d" % s)
    return "\n".join(out)


def syndrome_source(Hs: np.ndarray) -> str:
    Ms, N = Hs.shape
    W64 = (N + 63) // 64
    out = ["__device__ __forceinline__ bool syndrome_zero(const uint64_t *w)", "{", "    uint32_t odd = 0;"]
    for r in range(Ms):
        terms = []
        for k in range(W64):
            mask = sum(1 << (i - 64 * k) for i in range(64 * k, min(N, 64 * k + 64)) if Hs[r, i])
            if mask:
                terms.append("__popcll(w[%d] & 0x%016xull)" % (k, mask))
        out.append("    odd |= %s;" % " + ".join(terms))
    out += ["    return (odd & 1u) == 0;", "}"]
    return "\n".join(out)


def generate(stage1_lib: str, out_dir: str):
    lib = ctypes.CDLL(stage1_lib)
    P = ctypes.c_void_p
    lib.bch_load_code.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_int, P]
    lib.bch_code_info.argtypes = [P, P, P, P]
    lib.bch_code_export.argtypes = [P, P, P, P]
    lib.bch_build_pcm.argtypes = [P, ctypes.POINTER(_PcmParams), P]
    lib.bch_pcm_info.argtypes = [P, P, P, P, P, P, P]
    lib.bch_pcm_export.argtypes = [P, P, ctypes.c_size_t]
    lib.bch_pcm_destroy.argtypes = [P]
    lib.bch_code_destroy.argtypes = [P]
    srcs = []
    entries = []
    decls = []
    mats = {}
    for spec in SPECS:
        name, rows, B, mode, prec, waves = spec[:6]
        variant = spec[6] if len(spec) > 6 else 0
        if (name, rows) not in mats:
            mats[(name, rows)] = _matrices(lib, name, rows)
        H, Hs = mats[(name, rows)]
        M, N = H.shape
        ns = "spec_%s_m%d_b%d%s%s%s" % (name, M, B, "_fix8" if prec else "",
                                         {0: "", 1: "_pk16", 2: "_grp"}[variant], "_ext" if mode == 3 else "")
        body_path = os.path.join(out_dir, ns + "_body.inc")
        regacc = 1 if B > 1 else 0
        pk16 = 1 if prec and regacc and variant == 1 else 0
        # nine branches: three waves (one per automorphism type) share each 64
        # frames; always for N = 63, as the small-batch kernel for N = 127
        group = 1 if regacc and B == 9 and ((N <= 64 and variant == 0) or variant == 2) else 0
        if variant == 1 and not pk16:
            raise ValueError("the packed variant needs fixed point and 3 or 9 branches")
        if variant == 2 and not (group and N > 64):
            raise ValueError("the small-batch variant is for nine branches and N = 127")
        ext = mode == 3
        # every nine-branch kernel folds its shifts but the excluded one-wave ones
        fold = FOLD_SHIFTS and regacc and B == 9 and not ext and (
            group or pk16 or (name, rows) not in FOLD_EXCLUDE)
        dp = {63: 21, 127: 42}.get(N, N // 3)
        if ext and not (B == 1 and prec == 0 and variant == 0):
            raise ValueError("the extrinsic-message kernel is one-branch FP32")
        if not ext and mode != 1:
            raise ValueError("specialised kernels: restart mode, or one-branch extrinsic messages")
        with open(body_path, "w") as fh:
            fh.write("// generated: %s, H %d x %d, %d edges\n" % (name, M, N, int(H.sum())))
            if ext:
                fh.write(body_source_ext(H))
            elif pk16 and fold:
                fh.write(folded_body_source(H, dp, lambda Hs: body_source_pk16(Hs, B)))
            elif pk16:
                fh.write(body_source_pk16(H, B))
            else:
                if fold:
                    # the triple search; in the grouped N = 63 kernels its extra
                    # live values spill some registers, and it still measured
                    # 8% faster than the chain once the shifts were folded
                    fh.write(_MED3U + "\n" + folded_body_source(
                        H, dp, lambda Hs: body_source_ilp(Hs, fix8=bool(prec), group=ILP_ROWS, tree=True,
                                                                helpers=False)))
                elif regacc and N > 64:
                    fh.write(body_source_ilp(H, fix8=bool(prec), group=ILP_ROWS, tree=True))
                else:
                    fh.write(body_source_fix8(H, regacc) if prec else body_source(H, regacc))
            fh.write("\n\n" + syndrome_source(Hs) + "\n")
        src_path = os.path.join(out_dir, ns + ".hip")
        with open(src_path, "w") as fh:
            fh.write('#include "spec_launch.h"\n')
            yg = 1 if N > 64 and not regacc else 0
            fh.write("#define SPEC_N %d\n#define SPEC_B %d\n#define SPEC_NS %s\n#define SPEC_WAVES %d\n"
                     "#define SPEC_Y_GLOBAL %d\n#define SPEC_FIX8 %d\n#define SPEC_REGACC %d\n"
                     % (N, B, ns, waves, yg, prec, regacc))
            fh.write('#define SPEC_BODY "%s"\n' % os.path.basename(body_path))
            if group and N > 64:
                fh.write("#define SPEC_WAVES_PER_SIMD 1\n")
            if ext:
                fh.write("#define SPEC_M %d\n" % M)
            if fold:
                fh.write("#define SPEC_FOLD 1\n")
            if not (pk16 or group):
                fh.write("#define SPEC_RESERVE %d\n" % (RESERVE if ext or B < 9 else 0))
            fh.write('#include "%s"\n' % ("nms_spec_ext.inc" if ext else "nms_spec_pk16.inc" if pk16 else
                                           "nms_spec_group.inc" if group else "nms_spec_fp32.inc"))
        srcs.append(src_path)
        decls.append("namespace %s { hipError_t launch(const SpecLaunch &, int, int, hipStream_t); }" % ns)
        entries.append("    {0x%016xull, %d, %d, %d, %d, %d, %d, %d, %d, %d, %d, \"%s\", &%s::launch}," %
                       (fingerprint(H), N, M, B, mode, prec, variant, waves, 1 if N > 64 and not regacc else 0,
                        128 if pk16 else 64, 3 if group else 1, ns, ns))
    table = "\n".join(decls) + "\nstatic const SpecKernel kSpecKernels[] = {\n" + "\n".join(entries) + \
        "\n    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, nullptr, nullptr}};\n"
    mdecls, mentries = [], []
    for codes, prec in MIXES:
        parts = []
        for name, rows in codes:
            if (name, rows) not in mats:
                mats[(name, rows)] = _matrices(lib, name, rows)
            H, Hs = mats[(name, rows)]
            parts.append((name, H, Hs))
        ns = "mix_" + "_".join("%s_m%d" % (n.replace("bch", ""), r) for n, r in codes) + ("_fix8" if prec else "")
        srcs.append(mixed_source(ns, parts, prec, out_dir))
        mdecls.append("namespace %s { hipError_t launch(const MixLaunch &, int, int, hipStream_t); }" % ns)
        fps = ", ".join("0x%016xull" % fingerprint(H) for _, H, _ in parts)
        mentries.append("    {%d, {%s}, %d, \"%s\", &%s::launch}," % (len(parts), fps, prec, ns, ns))
    table += "\n".join(mdecls) + "\nstatic const MixKernel kMixKernels[] = {\n" + "\n".join(mentries) + \
        "\n    {0, {0}, 0, nullptr, nullptr}};\n"
    return srcs, table
