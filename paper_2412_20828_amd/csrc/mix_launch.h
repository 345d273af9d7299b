// Launch arguments of the mixed-code decode kernels (one persistent kernel
// over frames of several codes, each code's matrix compiled in).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bch {

constexpr int MIX_MAXC = 4;      // codes in one mixed kernel
constexpr int MIX_MAXB = 128;    // buckets: sum over the codes of d_p

struct MixLaunch {
    const void *llr;        // device [F][ld] float32 (FP32) or int8 (fixed point)
    int64_t ld;
    const int *order;       // frame indices grouped by (code, d_o mod d_p)
    int *bcur;              // per bucket: next slot of order to hand out (atomic)
    const int *bend;        // per bucket: end of its slice of order
    const int *counts;      // per bucket: frames (read at start for the work split)
    int n_buckets;
    uint64_t *bits;         // [F][bits_ld]
    int64_t bits_ld;
    uint8_t *iters;         // [F]
    uint8_t *flags;         // [F]
    int n_codes;
    int bbase[MIX_MAXC + 1];  // code k owns buckets [bbase[k], bbase[k + 1])
    float alpha[MIX_MAXC];
    int max_iter[MIX_MAXC];
    float weight[MIX_MAXC];   // work of one frame-iteration, for the start split
};

}  // namespace bch
