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
    int n_buckets;
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
// all in bucket 0 for one branch).  Bucket b is order[cursor[b], end[b]) once
// the prepass is done; the persistent kernels hand out its frames by
// advancing cursor[b] atomically.
struct BucketWs {
    int *counts;
    int *cursor;
    int *end;
    int *blk_hist;  // [blocks of 2048 frames][d_p] counts, then offsets
    int *order;
};

size_t bucket_ws_bytes(int64_t F, int dp);
BucketWs bucket_ws_carve(void *ws, int64_t F, int dp);
// code_idx (may be null): only frames with code_idx[f] == code are taken.
hipError_t launch_bucketing(const uint8_t *d_o, const uint8_t *code_idx, int code, int64_t F, int dp,
                            int use_offsets, const BucketWs &w, hipStream_t stream);
// Mixed-code prepass: frame f of code c = code_idx[f] < n_codes goes to bucket
// base[c] + d_o mod dps[c], base[0] = 0, base[c + 1] = base[c] + dps[c] (at
// most 128 buckets); the workspace is carved for that many buckets.
hipError_t launch_bucketing_mixed(const uint8_t *d_o, const uint8_t *code_idx, int n_codes, const int *dps,
                                  int64_t F, const BucketWs &w, hipStream_t stream);

}  // namespace bch
