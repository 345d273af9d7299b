// Launch interface between the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

#include "bchnms.h"

namespace bch {

struct GenericArgs {
    const void *llr;
    int64_t ld;
    int64_t F;
    const uint8_t *d_o;
    uint64_t *bits;
    uint8_t *iters;
    uint8_t *flags;
    float *trace;          // [F][max_iter][ld_trace] or null
    int64_t ld_trace;
    const uint16_t *rowptr; // [M+1]
    const uint8_t *colp;    // [3][E]: (a_p * column) mod N, a_p = 1, 2, (N+1)/2
    const uint64_t *hsyn;   // [msyn][W64] standard parity-check rows
    int msyn;
    int W64;
    int N, M, E, B, dp, mode, max_iter;
    float alpha;
    float *ws_c2v;          // [B][E][F]   (memory modes)
    float *ws_s;            // [2][B][N][F] (memory mode R2)
};

// Device scratch of the allocation-free decode (one array per GPU, 17 MiB:
// the workspace of a specialised decode of up to 4,194,304 frames).
constexpr size_t kNoAllocScratchBytes = (size_t)17 << 20;
// address of the calling thread's current device's scratch (looked up once per
// device with hipGetSymbolAddress)
hipError_t noalloc_scratch(void **ptr);

hipError_t launch_generic_fp32(const GenericArgs &a, hipStream_t stream);
hipError_t launch_syndrome(const uint64_t *bits, int64_t F, int W64, const uint64_t *hsyn,
                           int msyn, uint8_t *ok, hipStream_t stream);
// d_o[f] = draw_offset(seed, key_hi, base + f, dp) for f < F (device buffer)
hipError_t launch_draw_offsets(uint64_t seed, uint64_t key_hi, int64_t base, int64_t F, int dp, uint8_t *d_o,
                               hipStream_t stream);
hipError_t launch_quantize(const float *llr, int64_t ld, int64_t F, int N, float scale,
                           int8_t *q, int64_t ldq, hipStream_t stream);

struct OsdArgs {
    const float *llr;     // [F][ld] channel LLRs
    int64_t ld;
    int64_t F;
    const uint8_t *skip;  // [F], nonzero: leave the frame alone; or null
    const uint8_t *code_idx;  // [F] or null: only frames with code_idx[f] == code
    int code;
    uint64_t *bits;       // [F][bits_ld]
    int64_t bits_ld;
    const uint32_t *G;    // [K][4] generator rows, bit i of row k = word i / 32, bit i % 32
    int N, K, order;
    int keep_costs;       // set by launch_osd: pass-1 costs in LDS as words (1) or saturated half-words (2)
};

hipError_t launch_osd(const OsdArgs &a, int n_cu, hipStream_t stream);

}  // namespace bch
