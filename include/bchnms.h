/*
 * bchnms -- enhanced normalized min-sum (NMS) decoding of short BCH codes on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: G. Li and X. Yu, "Effective Application of Normalized Min-Sum
 * Decoding for Short BCH Codes", arXiv 2412.20828.
 *
 * Conventions for every entry point:
 *   - return value 0 (BCH_OK) on success, a negative BCH_E* code otherwise;
 *     bch_last_error() gives a thread-local description of the last failure;
 *     nothing throws across this interface;
 *   - a binary vector of length N is stored either as N bytes (0/1, "dense")
 *     or packed little-endian in ceil(N/64) 64-bit words (bit i of word i/64
 *     is coordinate i = coefficient of x^i);
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device memory of the current device (any HIP allocation, e.g. a PyTorch
 *     tensor's data_ptr());
 *   - handles (bch_code, bch_pcm, bch_decoder) are created and freed by the
 *     library; they are immutable after creation and may be shared between
 *     threads and streams;
 *   - device buffers passed in are owned by the caller; the library never
 *     allocates device memory inside a decode call (decoders own a small
 *     device copy of their tables, made once at creation);
 *   - calls taking a hipStream_t only enqueue work on that stream; results are
 *     valid once the stream is synchronised.  Argument errors are reported
 *     synchronously; a HIP launch failure returns BCH_EDEVICE.
 */
#ifndef BCHNMS_H
#define BCHNMS_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    BCH_OK = 0,
    BCH_EINVAL = -1,       /* bad argument or shape */
    BCH_ENOMEM = -2,       /* host allocation failed / workspace too small */
    BCH_EDEVICE = -3,      /* HIP runtime error */
    BCH_EUNSUPPORTED = -4, /* outside the supported envelope (N > 127, ...) */
    BCH_ESTATE = -5        /* construction failed (e.g. no full-rank H_o) */
};

typedef struct bch_code_s *bch_code;
typedef struct bch_pcm_s *bch_pcm;
typedef struct bch_decoder_s *bch_decoder;

const char *bch_last_error(void);

/* ------------------------------------------------------------------------
 * Code algebra (system model of Section II; codes of Table 1).
 * Binary primitive narrow-sense BCH code of length N = 2^m - 1 (3 <= m <= 7)
 * over GF(2^m) built from the primitive polynomial prim_poly (bit k = x^k
 * coefficient, e.g. 0x43 = x^6+x+1), designed distance 2t+1.  K follows from
 * the degree of the generator polynomial.  Systematic encoding puts parity in
 * coordinates 0..N-K-1 and the message in N-K..N-1.
 */
int bch_load_code(int m, uint32_t prim_poly, int t, bch_code *out);
int bch_code_info(bch_code code, int *N, int *K, int *t);
/* g: N-K+1 host bytes (coefficients, lowest first); G: K*N host bytes or NULL;
 * Hstd: (N-K)*N host bytes or NULL (rows x^i h~(x), the standard PCM). */
int bch_code_export(bch_code code, uint8_t *g, uint8_t *G, uint8_t *Hstd);
void bch_code_destroy(bch_code code);

/* ------------------------------------------------------------------------
 * Parity-check matrices (Section III-A, the six-step construction of H_o).
 * kind = BCH_PCM_STD: the standard (N-K) x N matrix, other fields ignored.
 * kind = BCH_PCM_OPT: row echelon form, pairwise weight minimisation, Q cyclic
 * passes, redundancy padding (beta (M - M_r1) rows, or up to target_rows rows
 * when target_rows > 0), then simulated annealing on random cyclic row shifts
 * driven by SplitMix64(seed) (sa_steps_per_row * M_o steps, loss = #length-4
 * cycles + sa_lambda * column-weight variance).  The result is validated: every
 * row lies in the dual code and the rank is N-K (otherwise the annealing is
 * repeated with seed+1).  Deterministic for given parameters.
 */
enum { BCH_PCM_STD = 0, BCH_PCM_OPT = 1 };
typedef struct {
    int kind;
    int beta;
    int target_rows;
    int Q;
    uint64_t seed;
    int sa_steps_per_row;
    double sa_lambda;
} bch_pcm_params;

int bch_build_pcm(bch_code code, const bch_pcm_params *params, bch_pcm *out);
/* Import a dense M x N host matrix; re-validated against the code. */
int bch_pcm_from_dense(bch_code code, const uint8_t *H, int M, bch_pcm *out);
/* M rows, N columns, E nonzeros, #length-4 cycles, M_r1 of the construction
 * (0 for imported / standard matrices), seed actually used. */
int bch_pcm_info(bch_pcm pcm, int *M, int *N, int *E, int64_t *c4, int *Mr1,
                 uint64_t *seed_used);
/* Table 1 attributes of a matrix: rows M, nonzeros E, number of length-4
 * cycles c4 (the sum over row pairs of C(shared columns, 2)), and wstats[8] = column weight min, max, mean, population standard
 * deviation, then the same four for the row weights.  Any output may be
 * NULL. */
int bch_pcm_stats(bch_pcm pcm, int *M, int *E, int64_t *c4, double wstats[8]);
int bch_pcm_export(bch_pcm pcm, uint8_t *dense, size_t cap_bytes);
void bch_pcm_destroy(bch_pcm pcm);

/* ------------------------------------------------------------------------
 * Automorphism block (Section III-B).  Writes n_branches x N gather maps to
 * host memory: branch b reads Y_b[j] = y[maps[b*N + j]].  Branch b = 3s + p:
 * type p = identity, interleave (even then odd indices, Y[j] = y[2j mod N]),
 * Frobenius (bit i moves to 2i mod N); followed by the cyclic shift
 * s*d_p + d_o (d_p = 21 for N = 63, 42 for N = 127; s = 0, 1, 2).
 * n_branches = 1 is the identity (plain NMS); 3 uses the three shifts only.
 * d_o is the frame's random offset in [0, d_p), drawn by the caller.
 */
int bch_make_automorphisms(int N, int n_branches, int d_o, int16_t *maps);

/* The random offsets d_o of Section III-B (one per frame, uniform in
 * [0, d_p)), drawn from a counter-based generator so that a frame's offset
 * depends only on the key and its frame uid, never on batch position:
 * d_o[f] = ((x >> 32) * d_p) >> 32 with x the first 64-bit word of
 * Philox4x64-10 (Salmon et al., SC'11) at counter (frame_base + f, 0, 0, 0)
 * under key (seed, key_hi).  d_o: F bytes, on the device (on_device = 1;
 * enqueued on stream) or on the host (on_device = 0; written before return,
 * stream ignored).  BCH_EINVAL for N outside [7, 127], F < 0 or
 * frame_base < 0. */
int bch_draw_offsets(int N, uint64_t seed, uint64_t key_hi, int64_t frame_base, int64_t F, uint8_t *d_o,
                     int on_device, hipStream_t stream);
/* The same draw for several keys in one host call (a service's batch of
 * requests, each keyed by its own id): key k's counts[k] frames, uids 0 to
 * counts[k] - 1, are written to d_o one key after another, so that d_o[o_k + f]
 * equals bch_draw_offsets(N, seed, keys[k], 0, ...)'s byte f, with o_k the
 * sum of the counts before k.  keys, counts and d_o are host memory owned by
 * the caller; BCH_EINVAL for N outside [7, 127], n_keys < 0, a negative
 * count or a NULL pointer with n_keys > 0. */
int bch_draw_offsets_keys(int N, uint64_t seed, int64_t n_keys, const uint64_t *keys, const int64_t *counts,
                          uint8_t *d_o);

/* ------------------------------------------------------------------------
 * Decoder (Algorithm 1 of Section III-B; plain NMS of Section II-A as the
 * one-branch case).
 * mode: how eq. 2 keeps messages across iterations, given that y is replaced
 * by y^(t) after every iteration:
 *   BCH_MODE_RESTART (default): v2c = Y_b (each iteration is one min-sum pass
 *     on the replaced input), y^(t) = y^(t-1) + average;
 *   BCH_MODE_MEMORY: eq. 2 literally, v2c = Y_b + sum of the branch's other
 *     c2v messages of iteration t-1, y^(t) = y^(t-1) + average;
 *   BCH_MODE_EXTRINSIC: v2c = Y_b - the branch's own c2v of iteration t-1,
 *     y^(t) = L + average (one branch: exactly plain flooding NMS).
 * precision: BCH_FP32, or BCH_FIX8 (int8 messages, integer accumulators,
 *   alpha = 3/4 as (3m+2)>>2; input LLRs int8, see bch_quantize_llr).
 */
enum { BCH_MODE_RESTART = 1, BCH_MODE_MEMORY = 2, BCH_MODE_EXTRINSIC = 3 };
enum { BCH_FP32 = 0, BCH_FIX8 = 1 };
enum {
    BCH_DEC_FORCE_GENERIC = 1, /* do not use a PCM-specialised kernel */
    BCH_DEC_PACKED16 = 2,      /* BCH_FIX8: always the packed 16-bit kernel (two frames per
                                  lane, same results), registered for the four workload
                                  matrices of N = 63 and 127.  Without this flag a fixed-point
                                  decode of at least 4,000,000 frames (N = 127) or 8,000,000
                                  (N = 63) runs it where registered, a smaller one the kernel
                                  that holds its integers in 32-bit registers */
    BCH_DEC_SMALL_ALWAYS = 4,  /* N = 127: always use the small-batch kernel (the nine
                                  branches of 64 frames on three waves) where registered */
    BCH_DEC_SMALL_NEVER = 8,   /* N = 127: never use it.  Without either flag a decode of at
                                  most 128 frames per CU uses it, a larger one the kernel
                                  of one wave per 64 frames; the results are the same.
                                  Both flags together, or any other bit, give BCH_EINVAL */
    BCH_DEC_UNPACKED16 = 16,   /* BCH_FIX8: never the packed 16-bit kernel (with
                                  BCH_DEC_PACKED16: BCH_EINVAL) */
    BCH_DEC_NO_MIXED_KERNEL = 32, /* a mixed-code call that includes this decoder runs one
                                   prepass and kernel per code (bch_mixed_decode_batch) */
    BCH_DEC_MIXED_KERNEL = 64,   /* a mixed-code call that includes this decoder runs the
                                   mixed-code kernel at any batch size (where registered and
                                   no decoder of the call has BCH_DEC_NO_MIXED_KERNEL; with
                                   BCH_DEC_NO_MIXED_KERNEL on the same decoder: BCH_EINVAL) */
    BCH_DEC_CHUNK_BUCKETS = 128  /* specialised decodes of at least 1,048,576 frames: the
                                   prepass deals chunks of 65,536 frames round robin to eight
                                   ranges, one per XCD, whose waves decode their own chunks
                                   first, so each output cache line is filled by one XCD and
                                   leaves its L2 whole (HBM writes of the packed 16-bit kernel
                                   on the 127-bit sweep: 83 -> 48 bytes per frame, for about
                                   2% more kernel time).  Same results */
};
typedef struct {
    int n_branches; /* 1, 3 or 9 */
    int mode;
    float alpha;    /* normalisation factor of eq. 3 (FP32 path) */
    int max_iter;   /* I_m, 1..64 */
    int precision;
    int flags;
} bch_dec_params;

/* Builds the device tables for (pcm, params); syndrome stop uses the code's
 * standard PCM (same null space as a full-rank H_o).  May compile nothing: a
 * kernel specialised to this exact PCM is used when the library carries one. */
int bch_decoder_create(bch_code code, bch_pcm pcm, const bch_dec_params *params,
                       bch_decoder *out);
/* 1 if the decoder runs a PCM-specialised kernel, 0 for the generic one. */
int bch_decoder_is_specialized(bch_decoder dec);
/* Name of the kernel a decode of F frames runs ("generic" for the generic
 * kernel, "" for a null decoder); the string is static and owned by the
 * library. */
const char *bch_decoder_kernel_name(bch_decoder dec, int64_t F);
void bch_decoder_destroy(bch_decoder dec);

/* Device workspace (bytes) a decode of F frames needs (0 for some configs). */
size_t bch_decode_workspace_size(bch_decoder dec, int64_t F);

/* Decode F frames.  llr: device [F][ld] float32 (FP32) or int8 (FIX8), first N
 * entries of each row used; d_o: device [F] uint8 random offsets in [0, d_p)
 * (bch_draw_offsets; ignored for one branch; every kernel reduces a larger
 * value modulo d_p, which is how such a frame decodes); bits: device [F][ceil(N/64)] uint64 decoded word; iters: device
 * [F] uint8 iterations run (1..max_iter); flags: device [F] uint8, bit 0 =
 * syndrome satisfied (converged); y_trace: device [F][max_iter][ld] float32 (or
 * int32 for FIX8) per-iteration posteriors y^(t), or NULL (rows past a
 * frame's last iteration are left untouched).  workspace: device, at least
 * bch_decode_workspace_size(dec, F) bytes (may be NULL when that is 0).
 * 0 <= F <= BCH_MAX_FRAMES (BCH_EINVAL otherwise).  Enqueued on stream. */
#define BCH_MAX_FRAMES ((int64_t)1 << 30)
int bch_nms_decode_batch(bch_decoder dec, const void *llr, int64_t ld, int64_t F,
                         const uint8_t *d_o, uint64_t *bits, uint8_t *iters,
                         uint8_t *flags, void *y_trace, void *workspace,
                         size_t ws_bytes, hipStream_t stream);

/* Allocation-free form of bch_nms_decode_batch, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same decode and results, with the
 * workspace taken from a device array that the library holds for each GPU it
 * runs on (BCH_NOALLOC_SCRATCH_BYTES, until the process ends; its address is
 * looked up on the first call on a device).  The call allocates nothing and
 * clears nothing (the bucketing prepass writes every workspace byte it later
 * reads).  A decode whose bch_decode_workspace_size exceeds the scratch (a
 * specialised decoder above 4,194,304 frames, an edge-memory mode of the
 * generic kernel on more than a few frames) returns BCH_EINVAL.  Every call
 * on one GPU shares that GPU's scratch: calls that overlap on one GPU (other
 * streams, other threads) race and must be ordered by the caller. */
#define BCH_NOALLOC_SCRATCH_BYTES ((size_t)17 << 20)
int bch_nms_decode_batch_noalloc(bch_decoder dec, const void *llr, int64_t ld, int64_t F, const uint8_t *d_o,
                                 uint64_t *bits, uint8_t *iters, uint8_t *flags, void *y_trace,
                                 hipStream_t stream);

/* Tuning of a specialised decoder (autotuner hook): waves per CU of the
 * persistent grid (0: the kernel's default; the nine-branch N = 63 kernels
 * run workgroups of three waves, so waves_per_cu / 3 of them per CU).  A
 * decode of F frames never launches more than its frames can occupy.  No
 * effect on the generic kernel.  Not thread-safe against a concurrent
 * decode. */
int bch_decoder_set_tuning(bch_decoder dec, int waves_per_cu);

/* ------------------------------------------------------------------------
 * Mixed-code batch: the frames of up to BCH_MAX_MIX codes interleaved in one
 * array; frame f is decoded by decs[code_idx[f]] (frames with code_idx >=
 * n_codes are left untouched).  Every decoder needs a specialised kernel and
 * all share the precision.  llr: device [F][ld] with ld >= every N; bits:
 * device [F][bits_ld] uint64, bits_ld >= every ceil(N/64); iters, flags: as
 * bch_nms_decode_batch; F <= BCH_MAX_FRAMES.  When the library carries a
 * mixed-code kernel for these decoders' matrices in this order (nine-branch,
 * restart-mode decoders of one precision, none with BCH_DEC_NO_MIXED_KERNEL)
 * and F < BCH_MIXED_KERNEL_MAX_FRAMES (or a decoder has BCH_DEC_MIXED_KERNEL),
 * the call enqueues one prepass that buckets every frame by (code, d_o) and
 * one persistent kernel whose waves take frames of any code (the batching
 * pattern of one launch for a mixed batch); otherwise one prepass and one
 * persistent kernel per code.  The size limit is where the two paths cross
 * over: one launch saves the per-code launch tails, which dominate small
 * batches, while at large batches each code's own kernel is faster (the
 * 63-bit codes' kernels run three waves per SIMD, the mixed kernel one, and
 * large fixed-point calls take the packed 16-bit kernels).  No host synchronisation, no memset: the call
 * can be captured in a HIP graph and replayed.  Per-frame results do not
 * depend on the mix or the path: each frame decodes exactly as alone.
 */
#define BCH_MAX_MIX 8
#define BCH_MIXED_KERNEL_MAX_FRAMES 3000000
size_t bch_mixed_workspace_size(const bch_decoder *decs, int n_codes, int64_t F);
int bch_mixed_decode_batch(const bch_decoder *decs, int n_codes, const uint8_t *code_idx, const void *llr,
                           int64_t ld, int64_t F, const uint8_t *d_o, uint64_t *bits, int64_t bits_ld,
                           uint8_t *iters, uint8_t *flags, void *workspace, size_t ws_bytes,
                           hipStream_t stream);

/* Name of the kernel a mixed call of F frames over decs[0..n_codes) runs:
 * the mixed-code kernel's, or "per-code" ("" for bad arguments); static,
 * owned by the library. */
const char *bch_mixed_kernel_name(const bch_decoder *decs, int n_codes, int64_t F);

/* Syndrome test of eq. 5 with the code's standard PCM: ok[f] = 1 iff
 * H c_f^T = 0.  bits: device [F][ceil(N/64)] uint64; ok: device [F] uint8. */
int bch_syndrome_check(bch_code code, const uint64_t *bits, int64_t F, uint8_t *ok,
                       hipStream_t stream);

/* Fixed-point input: q = clamp(round-half-away(L * scale), -127, 127), the
 * product formed in FP32.  llr: device [F][ld] float32; q: device [F][ldq]
 * int8; columns N..ldq-1 of q are zeroed. */
int bch_quantize_llr(const float *llr, int64_t ld, int64_t F, int N, float scale,
                     int8_t *q, int64_t ldq, hipStream_t stream);

/* Order-p OSD (Section II-B) on the host, the back end of the hybrid decoder:
 * frames with skip[f] != 0 are left alone (skip may be NULL).  llr: host
 * [F][ld] float32 channel LLRs; bits: host [F][ceil(N/64)] uint64, written for
 * every decoded frame.  Runs on n_threads host threads (<= 0: all cores). */
int bch_osd_decode(bch_code code, const float *llr, int64_t ld, int64_t F, int order,
                   const uint8_t *skip, uint64_t *bits, int n_threads);

/* Order-p OSD (Section II-B) on the device: the second stage of the hybrid
 * decoder of Section IV without leaving the GPU.  Same decisions as
 * bch_osd_decode (reliabilities |L| in FP64, positions ordered by decreasing
 * reliability with ties by index, candidates in the order weight 0, 1, 2
 * with the first of least cost kept).  Uses dec's code (its N, K and
 * generator); order 0..2.  llr: device [F][ld] float32 channel LLRs (ld >= N);
 * skip: device [F] uint8 or NULL, frames with skip[f] != 0 are left alone
 * (pass the decoder's flags to run OSD exactly on the frames whose syndrome
 * stayed nonzero); bits: device [F][bits_ld] uint64, written for every other
 * frame.  Enqueued on stream; allocates nothing. */
int bch_osd_decode_device(bch_decoder dec, const float *llr, int64_t ld, int64_t F, int order,
                          const uint8_t *skip, uint64_t *bits, int64_t bits_ld, hipStream_t stream);

/* The same over a mixed-code batch (as bch_mixed_decode_batch): frame f is
 * decoded with decs[code_idx[f]]'s code unless skip[f] != 0 (skip may be
 * NULL); frames with code_idx >= n_codes are left alone.  One launch per code
 * on stream; allocates nothing. */
int bch_mixed_osd_decode(const bch_decoder *decs, int n_codes, const uint8_t *code_idx, const float *llr,
                         int64_t ld, int64_t F, int order, const uint8_t *skip, uint64_t *bits, int64_t bits_ld,
                         hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif
