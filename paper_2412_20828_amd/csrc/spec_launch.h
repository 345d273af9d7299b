// Launch arguments of the PCM-specialised decode kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bch {

struct SpecLaunch {
    const void *llr;       // device [F][ld] float32 (FP32) or int8 (FIX8)
    int64_t ld;
    const int *order;      // frame indices grouped by d_o (bucketing prepass)
    int *bcur;             // per bucket: next slot of order to hand out (atomic)
    const int *bend;       // per bucket: end of its slice of order
    int n_buckets;         // n_ranges x n_offsets
    int n_offsets;         // buckets per frame range: d_p (one: the one-branch decoder)
    int n_ranges;          // frame ranges: bucket r n_offsets + o holds frames of range r with d_o mod d_p = o
    uint64_t *bits;        // [F][bits_ld] (bits_ld >= W64)
    int64_t bits_ld;
    uint8_t *iters;        // [F]
    uint8_t *flags;        // [F]
    void *trace;           // [F][max_iter][ld] float32 / int32, or null
    float *yscratch;       // [grid][N][64] when the kernel keeps y in device memory
    int max_iter;
    float alpha;
};

// Bucketing prepass: groups frames by random offset d_o (reduced modulo d_p;
// all in offset 0 for one branch) and, for large batches of decoders with
// BCH_DEC_CHUNK_BUCKETS, by frame range:
// frame f falls in range (f / 65536) mod R of R = bucket_ranges(F) ranges
// (chunks of 65,536 frames dealt round robin, so every range holds frames
// from the whole batch and the same share of its work), and goes to bucket
// range * n_offsets + d_o mod d_p.  The persistent kernels start the waves
// of XCD x (workgroup index mod 8) on the buckets of range x mod R and move
// to another range only when their own is dry, so each XCD decodes whole
// chunks and writes whole chunks of the outputs, whose cache lines then fill
// in its L2 before they go out to HBM (with frames of every chunk on every
// XCD, each line's bytes would arrive from eight L2s and leave as partial
// writes).  Bucket b is order[cursor[b], end[b]) once the prepass is done;
// the kernels hand out its frames by advancing cursor[b] atomically.
struct BucketWs {
    int *counts;
    int *cursor;
    int *end;
    int *blk_hist;  // [blocks of 2048 frames][d_p] counts, then offsets
    int *order;
};

// frame ranges of a batch of F frames: 8 (one per XCD) from 1,048,576 frames,
// where each bucket still holds thousands of frames, when asked for; 1 else.
// Measured on the 127-bit sweep (28,000,000 frames per call): HBM writes of
// the packed 16-bit kernel 83 -> 48 bytes per frame, kernel time +2%.
constexpr int kRangeXcds = 8;
constexpr int kRangeChunkLog2 = 16;
constexpr int64_t kRangeMinFrames = 1 << 20;
inline int bucket_ranges(int64_t F, bool chunked) { return chunked && F >= kRangeMinFrames ? kRangeXcds : 1; }

// nb: number of buckets
size_t bucket_ws_bytes(int64_t F, int nb);
BucketWs bucket_ws_carve(void *ws, int64_t F, int nb);
// code_idx (may be null): only frames with code_idx[f] == code are taken;
// ranges x dp buckets (x 1 when !use_offsets).
hipError_t launch_bucketing(const uint8_t *d_o, const uint8_t *code_idx, int code, int64_t F, int dp,
                            int use_offsets, int ranges, const BucketWs &w, hipStream_t stream);
// Mixed-code prepass: frame f of code c = code_idx[f] < n_codes goes to bucket
// base[c] + d_o mod dps[c], base[0] = 0, base[c + 1] = base[c] + dps[c] (at
// most 128 buckets); the workspace is carved for that many buckets.
hipError_t launch_bucketing_mixed(const uint8_t *d_o, const uint8_t *code_idx, int n_codes, const int *dps,
                                  int64_t F, const BucketWs &w, hipStream_t stream);

}  // namespace bch
